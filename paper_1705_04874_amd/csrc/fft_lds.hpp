// Batched in-LDS Stockham FFT for gfx950 (wave64).
//
// The spatial derivatives of the method are taken in the wavenumber domain
// (Sec. II-A), so every time step is a chain of 1-D transforms along x, y and z.
// Each transform here runs on a batch of pencils already staged in LDS: one
// radix-R pass loads R elements per butterfly into registers, applies the
// twiddles and an R-point DFT, and writes them back in Stockham (self-sorting)
// order; a barrier separates the read half and the write half of the pass, so
// one LDS buffer suffices.  Lengths are compile-time: the radix plan (8, 4, 2,
// 3, 5) is unrolled completely.
//
// Conventions: DIR = -1 forward (exp(-2 pi i jk/N)), DIR = +1 inverse without
// the 1/N factor.  Twiddle table tw[e] = exp(-2 pi i e / N), e < N, computed in
// double on the host and rounded to float.
#pragma once
#include <hip/hip_runtime.h>

namespace pstd {

__device__ __forceinline__ float2 c_add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 c_sub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 c_mul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 c_scale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 c_conj(float2 a) { return make_float2(a.x, -a.y); }
// multiply by -i (forward) or +i (inverse)
template <int DIR>
__device__ __forceinline__ float2 c_rot(float2 a)
{
    return DIR < 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
}

// ---------------------------------------------------------------------------
// small DFTs, in place on a[0..R)
template <int R, int DIR> struct Dft;

template <int DIR> struct Dft<2, DIR> {
    static __device__ __forceinline__ void run(float2* a)
    {
        float2 t = a[0];
        a[0] = c_add(t, a[1]);
        a[1] = c_sub(t, a[1]);
    }
};

template <int DIR> struct Dft<4, DIR> {
    static __device__ __forceinline__ void run(float2* a)
    {
        float2 t0 = c_add(a[0], a[2]), t1 = c_sub(a[0], a[2]);
        float2 t2 = c_add(a[1], a[3]), t3 = c_rot<DIR>(c_sub(a[1], a[3]));
        a[0] = c_add(t0, t2);
        a[2] = c_sub(t0, t2);
        a[1] = c_add(t1, t3);
        a[3] = c_sub(t1, t3);
    }
};

template <int DIR> struct Dft<8, DIR> {
    static __device__ __forceinline__ void run(float2* a)
    {
        constexpr float h = 0.70710678118654752440f;
        float2 e[4] = {a[0], a[2], a[4], a[6]};
        float2 o[4] = {a[1], a[3], a[5], a[7]};
        Dft<4, DIR>::run(e);
        Dft<4, DIR>::run(o);
        // o[k] *= W8^k  (W8 = exp(DIR * i pi / 4))
        float2 w1 = c_scale(make_float2(o[1].x + (DIR < 0 ? o[1].y : -o[1].y),
                                        o[1].y + (DIR < 0 ? -o[1].x : o[1].x)), h);
        float2 w2 = c_rot<DIR>(o[2]);
        float2 w3 = c_scale(make_float2(-o[3].x + (DIR < 0 ? o[3].y : -o[3].y),
                                        -o[3].y + (DIR < 0 ? -o[3].x : o[3].x)), h);
        a[0] = c_add(e[0], o[0]);
        a[4] = c_sub(e[0], o[0]);
        a[1] = c_add(e[1], w1);
        a[5] = c_sub(e[1], w1);
        a[2] = c_add(e[2], w2);
        a[6] = c_sub(e[2], w2);
        a[3] = c_add(e[3], w3);
        a[7] = c_sub(e[3], w3);
    }
};

template <int DIR> struct Dft<3, DIR> {
    static __device__ __forceinline__ void run(float2* a)
    {
        constexpr float s3 = 0.86602540378443864676f;
        float2 t = c_add(a[1], a[2]);
        float2 u = c_rot<DIR>(c_scale(c_sub(a[1], a[2]), s3));
        float2 b = make_float2(a[0].x - 0.5f * t.x, a[0].y - 0.5f * t.y);
        a[0] = c_add(a[0], t);
        a[1] = c_add(b, u);
        a[2] = c_sub(b, u);
    }
};

template <int DIR> struct Dft<5, DIR> {
    static __device__ __forceinline__ void run(float2* a)
    {
        constexpr float c1 = 0.30901699437494742410f;   // cos(2 pi / 5)
        constexpr float c2 = -0.80901699437494742410f;  // cos(4 pi / 5)
        constexpr float s1 = 0.95105651629515357212f;   // sin(2 pi / 5)
        constexpr float s2 = 0.58778525229247312917f;   // sin(4 pi / 5)
        float2 t1 = c_add(a[1], a[4]), t2 = c_add(a[2], a[3]);
        float2 t3 = c_sub(a[1], a[4]), t4 = c_sub(a[2], a[3]);
        float2 b1 = make_float2(a[0].x + c1 * t1.x + c2 * t2.x, a[0].y + c1 * t1.y + c2 * t2.y);
        float2 b2 = make_float2(a[0].x + c2 * t1.x + c1 * t2.x, a[0].y + c2 * t1.y + c1 * t2.y);
        float2 d1 = make_float2(s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y);
        float2 d2 = make_float2(s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y);
        float2 r1 = c_rot<DIR>(d1), r2 = c_rot<DIR>(d2);
        a[0] = c_add(a[0], c_add(t1, t2));
        a[1] = c_add(b1, r1);
        a[4] = c_sub(b1, r1);
        a[2] = c_add(b2, r2);
        a[3] = c_sub(b2, r2);
    }
};

// ---------------------------------------------------------------------------
// radix plan: as many 8s as possible, then 4, 2, 3, 5
__host__ __device__ constexpr int plan_radix(int n, int p)
{
    int idx = 0;
    while (n % 8 == 0 && n > 1) {
        if (idx == p) return 8;
        n /= 8;
        ++idx;
    }
    while (n % 4 == 0) {
        if (idx == p) return 4;
        n /= 4;
        ++idx;
    }
    while (n % 2 == 0) {
        if (idx == p) return 2;
        n /= 2;
        ++idx;
    }
    while (n % 3 == 0) {
        if (idx == p) return 3;
        n /= 3;
        ++idx;
    }
    while (n % 5 == 0) {
        if (idx == p) return 5;
        n /= 5;
        ++idx;
    }
    return 0;
}

__host__ __device__ constexpr int plan_passes(int n)
{
    int p = 0;
    while (plan_radix(n, p)) ++p;
    return p;
}

__host__ __device__ constexpr int plan_ns(int n, int p)
{
    int ns = 1;
    for (int i = 0; i < p; ++i) ns *= plan_radix(n, i);
    return ns;
}

__host__ __device__ constexpr bool plan_ok(int n) { return n >= 2 && plan_ns(n, plan_passes(n)) == n; }

// Element (pencil, i) of the LDS batch lives at s[pencil * PS + i * IS].
// COLMAJOR: consecutive threads take consecutive pencils (use when PS == 1,
// i.e. pencils interleaved column-wise); otherwise consecutive elements.
template <int N, int R, int NS, int NPEN, int NT, int DIR, int PS, int IS, bool COLMAJOR>
__device__ __forceinline__ void fft_pass(float2* s, const float2* __restrict__ tw)
{
    constexpr int M = N / R;
    constexpr int NB = NPEN * M;
    constexpr int Q = (NB + NT - 1) / NT;
    constexpr int TS = N / (NS * R);
    float2 a[Q][R];
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int b = t + q * NT;
        if ((NB % NT == 0) || b < NB) {
            const int pen = COLMAJOR ? b % NPEN : b / M;
            const int j = COLMAJOR ? b / NPEN : b - pen * M;
            const int k = j % NS;
#pragma unroll
            for (int r = 0; r < R; ++r) a[q][r] = s[pen * PS + (j + r * M) * IS];
            if (NS > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    float2 w = tw[r * k * TS];
                    if (DIR > 0) w.y = -w.y;
                    a[q][r] = c_mul(a[q][r], w);
                }
            }
            Dft<R, DIR>::run(a[q]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int b = t + q * NT;
        if ((NB % NT == 0) || b < NB) {
            const int pen = COLMAJOR ? b % NPEN : b / M;
            const int j = COLMAJOR ? b / NPEN : b - pen * M;
            const int k = j % NS;
            const int base = (j / NS) * NS * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) s[pen * PS + (base + r * NS) * IS] = a[q][r];
        }
    }
    __syncthreads();
}

template <int N, int P, int NPEN, int NT, int DIR, int PS, int IS, bool COLMAJOR>
struct FftPasses {
    static __device__ __forceinline__ void run(float2* s, const float2* __restrict__ tw)
    {
        if constexpr (P < plan_passes(N)) {
            fft_pass<N, plan_radix(N, P), plan_ns(N, P), NPEN, NT, DIR, PS, IS, COLMAJOR>(s, tw);
            FftPasses<N, P + 1, NPEN, NT, DIR, PS, IS, COLMAJOR>::run(s, tw);
        }
    }
};

// Transform NPEN pencils of length N held in LDS. The caller must have
// synchronised after staging the data; the routine ends with a barrier.
template <int N, int NPEN, int NT, int DIR, int PS, int IS, bool COLMAJOR>
__device__ __forceinline__ void lds_fft(float2* s, const float2* __restrict__ tw)
{
    static_assert(plan_ok(N), "length must factor into 2, 3 and 5");
    FftPasses<N, 0, NPEN, NT, DIR, PS, IS, COLMAJOR>::run(s, tw);
}

}  // namespace pstd
