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

// 16-point DFT as 4 x 4 with constant inner twiddles W16^(n2 k1)
template <int DIR> struct Dft<16, DIR> {
    template <int M>
    static __device__ __forceinline__ float2 w16(float2 a)
    {
        // multiply by exp(DIR * 2 pi i M / 16)
        constexpr float c1 = 0.92387953251128675613f, s1 = 0.38268343236508977173f, h = 0.70710678118654752440f;
        constexpr float cs[8] = {1.f, c1, h, s1, 0.f, -s1, -h, -c1};
        constexpr float sn[8] = {0.f, s1, h, c1, 1.f, c1, h, s1};
        constexpr float c = cs[M % 8] * ((M / 8) % 2 ? -1.f : 1.f);
        constexpr float s = sn[M % 8] * ((M / 8) % 2 ? -1.f : 1.f) * (DIR < 0 ? -1.f : 1.f);
        return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
    }
    static __device__ __forceinline__ void run(float2* a)
    {
        float2 y[4][4];
#pragma unroll
        for (int n2 = 0; n2 < 4; ++n2) {
            y[n2][0] = a[n2];
            y[n2][1] = a[4 + n2];
            y[n2][2] = a[8 + n2];
            y[n2][3] = a[12 + n2];
            Dft<4, DIR>::run(y[n2]);
        }
        y[1][1] = w16<1>(y[1][1]);
        y[1][2] = w16<2>(y[1][2]);
        y[1][3] = w16<3>(y[1][3]);
        y[2][1] = w16<2>(y[2][1]);
        y[2][2] = w16<4>(y[2][2]);
        y[2][3] = w16<6>(y[2][3]);
        y[3][1] = w16<3>(y[3][1]);
        y[3][2] = w16<6>(y[3][2]);
        y[3][3] = w16<9>(y[3][3]);
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            float2 t[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
            Dft<4, DIR>::run(t);
            a[k1] = t[0];
            a[k1 + 4] = t[1];
            a[k1 + 8] = t[2];
            a[k1 + 12] = t[3];
        }
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

// LDS element offset of position i in a pencil: with PAD the row layout gets
// one spare slot every 16 elements, which spreads power-of-two strides over
// all LDS banks.
template <bool PAD>
__device__ __forceinline__ constexpr int lidx(int i)
{
    return PAD ? i + (i >> 4) : i;
}
__host__ __device__ constexpr int padded_len(int n) { return n + (n >> 4) + 1; }

// ---------------------------------------------------------------------------
// radix plan: as many of the largest radix up to MR (16 or 8) as possible, then
// 8, 4, 2, 3, 5
__host__ __device__ constexpr int plan_radix(int n, int p, int mr = 16)
{
    int idx = 0;
    while (mr >= 16 && n % 16 == 0 && n > 1) {
        if (idx == p) return 16;
        n /= 16;
        ++idx;
    }
    while (mr >= 8 && n % 8 == 0 && n > 1) {
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

__host__ __device__ constexpr int plan_passes(int n, int mr = 16)
{
    int p = 0;
    while (plan_radix(n, p, mr)) ++p;
    return p;
}

__host__ __device__ constexpr int plan_ns(int n, int p, int mr = 16)
{
    int ns = 1;
    for (int i = 0; i < p; ++i) ns *= plan_radix(n, i, mr);
    return ns;
}

__host__ __device__ constexpr bool plan_ok(int n) { return n >= 2 && plan_ns(n, plan_passes(n)) == n; }

// the same radices in reverse order (used by inverse transforms that start
// from the register-resident output of a forward transform)
__host__ __device__ constexpr int plan_radix_rev(int n, int p, int mr = 16)
{
    return plan_radix(n, plan_passes(n, mr) - 1 - p, mr);
}
__host__ __device__ constexpr int plan_ns_rev(int n, int p, int mr = 16)
{
    int ns = 1;
    for (int i = 0; i < p; ++i) ns *= plan_radix_rev(n, i, mr);
    return ns;
}

// Loaders that split into fetch (loads only) and finish (arithmetic on the
// loaded values) declare TWO_PHASE; a pass then issues all of a butterfly's
// loads before any of the arithmetic.
template <class Ld, class = void>
struct TwoPhase {
    static constexpr bool value = false;
};
template <class Ld>
struct TwoPhase<Ld, decltype((void)Ld::TWO_PHASE)> {
    static constexpr bool value = Ld::TWO_PHASE;
};
template <class Ld>
__host__ __device__ constexpr bool two_phase() { return TwoPhase<Ld>::value; }

// Element (pencil, i) of the LDS batch lives at s[pencil * PS + i * IS].
// COLMAJOR: consecutive threads take consecutive pencils (use when PS == 1,
// i.e. pencils interleaved column-wise); otherwise consecutive elements.
//
// FROM_G: the pass reads its inputs through the loader ld(pencil, i) instead
// of LDS; TO_G: it hands its outputs to the storer st(pencil, i, value)
// instead of LDS.  The first pass of a transform can so read global memory
// straight into registers and the last pass write registers straight out.
// Twiddles tw[e] = exp(-2 pi i e / N) may live in LDS or global memory.
template <int N, int R, int NS, int NPEN, int NT, int DIR, int PS, int IS, bool COLMAJOR, bool FROM_G, bool TO_G,
          class Ld, class St, bool PAD = false>
__device__ __forceinline__ void fft_pass(float2* s, const float2* tw, const Ld& ld, const St& st)
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
            if constexpr (FROM_G && two_phase<Ld>()) {
                // every load of the butterfly first, then the arithmetic on them
                typename Ld::Raw raw[R];
#pragma unroll
                for (int r = 0; r < R; ++r) raw[r] = ld.fetch(pen, j + r * M);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int r = 0; r < R; ++r) a[q][r] = ld.finish(raw[r], j + r * M);
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if constexpr (FROM_G) a[q][r] = ld(pen, j + r * M);
                    else a[q][r] = s[pen * PS + lidx<PAD>(j + r * M) * IS];
                }
            }
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
    if constexpr (!FROM_G && !TO_G) __syncthreads();
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int b = t + q * NT;
        if ((NB % NT == 0) || b < NB) {
            const int pen = COLMAJOR ? b % NPEN : b / M;
            const int j = COLMAJOR ? b / NPEN : b - pen * M;
            const int k = j % NS;
            const int base = (j / NS) * NS * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if constexpr (TO_G) st(pen, base + r * NS, a[q][r]);
                else s[pen * PS + lidx<PAD>(base + r * NS) * IS] = a[q][r];
            }
        }
    }
    if constexpr (!TO_G) __syncthreads();
}

struct NoLd {
    __device__ float2 operator()(int, int) const { return make_float2(0.f, 0.f); }
};
struct NoSt {
    __device__ void operator()(int, int, float2) const {}
};

template <int N, int P, int NPEN, int NT, int DIR, int PS, int IS, bool COLMAJOR, bool LDG, bool STG, class Ld,
          class St, bool PAD = false>
struct FftPasses {
    static __device__ __forceinline__ void run(float2* s, const float2* tw, const Ld& ld, const St& st)
    {
        constexpr int NP = plan_passes(N);
        if constexpr (P < NP) {
            constexpr bool first = P == 0, last = P == NP - 1;
            fft_pass<N, plan_radix(N, P), plan_ns(N, P), NPEN, NT, DIR, PS, IS, COLMAJOR, LDG && first, STG && last,
                     Ld, St, PAD>(s, tw, ld, st);
            FftPasses<N, P + 1, NPEN, NT, DIR, PS, IS, COLMAJOR, LDG, STG, Ld, St, PAD>::run(s, tw, ld, st);
        }
    }
};

// Transform NPEN pencils of length N held in LDS (in place).  The caller
// synchronises after staging the data; the routine ends with a barrier.
template <int N, int NPEN, int NT, int DIR, int PS, int IS, bool COLMAJOR, bool PAD = false>
__device__ __forceinline__ void lds_fft(float2* s, const float2* tw)
{
    static_assert(plan_ok(N), "length must factor into 2, 3 and 5");
    FftPasses<N, 0, NPEN, NT, DIR, PS, IS, COLMAJOR, false, false, NoLd, NoSt, PAD>::run(s, tw, NoLd{}, NoSt{});
}

// Transform NPEN pencils whose inputs come from ld(pencil, i) (first pass
// reads straight into registers).  With STG the outputs go to st(pencil, i, v)
// and the routine ends WITHOUT a barrier (the caller synchronises before it
// writes the LDS buffer again); otherwise the result is left in LDS followed
// by a barrier.  The caller must make sure the LDS buffer is no longer read
// before the call when the plan has more than one pass.
template <int N, int NPEN, int NT, int DIR, int PS, int IS, bool COLMAJOR, bool STG, class Ld, class St,
          bool PAD = false>
__device__ __forceinline__ void fft_ld(float2* s, const float2* tw, const Ld& ld, const St& st)
{
    static_assert(plan_ok(N), "length must factor into 2, 3 and 5");
    FftPasses<N, 0, NPEN, NT, DIR, PS, IS, COLMAJOR, true, STG, Ld, St, PAD>::run(s, tw, ld, st);
}

// ---------------------------------------------------------------------------
// Register-resident ends.  For a Stockham plan whose last pass has radix RL,
// thread t ends holding, for each of its butterflies b = t + q NT (pencil and
// j from b as in fft_pass), the RL outputs j + r (N / RL).  An inverse run
// with the reversed plan starts from exactly that set, so a forward transform,
// a pointwise multiply and an inverse transform need no LDS round trip in
// between.  reg_coords gives (pencil, element) of a[q][r].
template <int N, int R, int NPEN, int NT, bool COLMAJOR>
__device__ __forceinline__ bool reg_coords(int q, int r, int& pen, int& idx)
{
    constexpr int M = N / R;
    constexpr int NB = NPEN * M;
    const int b = threadIdx.x + q * NT;
    pen = COLMAJOR ? b % NPEN : b / M;
    const int j = COLMAJOR ? b / NPEN : b - pen * M;
    idx = j + r * M;
    return (NB % NT == 0) || b < NB;
}

// One pass of a plan (REV selects the reversed radix order) with the inputs
// in registers (FROM_R) and/or the outputs left in registers (TO_R).
template <int N, int P, bool REV, int NPEN, int NT, int DIR, int PS, int IS, bool COLMAJOR, bool FROM_G, bool FROM_R,
          bool TO_G, bool TO_R, class Ld, class St, class RIn, class ROut, int MR = 16>
__device__ __forceinline__ void fft_pass_r(float2* s, const float2* tw, const Ld& ld, const St& st, RIn& rin,
                                           ROut& rout)
{
    constexpr int R = REV ? plan_radix_rev(N, P, MR) : plan_radix(N, P, MR);
    constexpr int NS = REV ? plan_ns_rev(N, P, MR) : plan_ns(N, P, MR);
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
            for (int r = 0; r < R; ++r) {
                if constexpr (FROM_R) a[q][r] = rin[q][r];
                else if constexpr (FROM_G) a[q][r] = ld(pen, j + r * M);
                else a[q][r] = s[pen * PS + (j + r * M) * IS];
            }
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
    if constexpr (!FROM_G && !FROM_R && !TO_G && !TO_R) __syncthreads();
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int b = t + q * NT;
        if ((NB % NT == 0) || b < NB) {
            const int pen = COLMAJOR ? b % NPEN : b / M;
            const int j = COLMAJOR ? b / NPEN : b - pen * M;
            const int k = j % NS;
            const int base = (j / NS) * NS * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if constexpr (TO_R) rout[q][r] = a[q][r];
                else if constexpr (TO_G) st(pen, base + r * NS, a[q][r]);
                else s[pen * PS + (base + r * NS) * IS] = a[q][r];
            }
        }
    }
    if constexpr (!TO_G && !TO_R) __syncthreads();
}

template <int N, int P, bool REV, int NPEN, int NT, int DIR, int PS, int IS, bool COLMAJOR, bool LDG, bool LDR,
          bool STG, bool STR, class Ld, class St, class RIn, class ROut, int MR = 16>
struct FftPassesR {
    static __device__ __forceinline__ void run(float2* s, const float2* tw, const Ld& ld, const St& st, RIn& rin,
                                               ROut& rout)
    {
        constexpr int NP = plan_passes(N, MR);
        if constexpr (P < NP) {
            constexpr bool first = P == 0, last = P == NP - 1;
            fft_pass_r<N, P, REV, NPEN, NT, DIR, PS, IS, COLMAJOR, LDG && first, LDR && first, STG && last,
                       STR && last, Ld, St, RIn, ROut, MR>(s, tw, ld, st, rin, rout);
            FftPassesR<N, P + 1, REV, NPEN, NT, DIR, PS, IS, COLMAJOR, LDG, LDR, STG, STR, Ld, St, RIn, ROut,
                       MR>::run(s, tw, ld, st, rin, rout);
        }
    }
};

// register array shapes of the first / last pass
template <int N, int NPEN, int NT, int MR = 16>
struct RegShape {
    static constexpr int RL = plan_radix(N, plan_passes(N, MR) - 1, MR);   // forward last = reversed first
    static constexpr int QL = (NPEN * (N / RL) + NT - 1) / NT;
};

// Forward-plan transform from ld(pencil, i) leaving the outputs in registers
// (no trailing barrier: the caller synchronises before it writes s again).
template <int N, int NPEN, int NT, int DIR, int PS, int IS, bool COLMAJOR, class Ld, class ROut, int MR = 16>
__device__ __forceinline__ void fft_g2r(float2* s, const float2* tw, const Ld& ld, ROut& rout)
{
    static_assert(plan_ok(N), "length must factor into 2, 3 and 5");
    float2 dummy[1][1];
    FftPassesR<N, 0, false, NPEN, NT, DIR, PS, IS, COLMAJOR, true, false, false, true, Ld, NoSt, float2[1][1],
               ROut, MR>::run(s, tw, ld, NoSt{}, dummy, rout);
}

// Reversed-plan transform from registers to st(pencil, i, v) (no trailing
// barrier; the caller synchronises before the first pass writes s when s was
// read just before).
template <int N, int NPEN, int NT, int DIR, int PS, int IS, bool COLMAJOR, class RIn, class St, int MR = 16>
__device__ __forceinline__ void fft_r2g(float2* s, const float2* tw, RIn& rin, const St& st)
{
    static_assert(plan_ok(N), "length must factor into 2, 3 and 5");
    float2 dummy[1][1];
    FftPassesR<N, 0, true, NPEN, NT, DIR, PS, IS, COLMAJOR, false, true, true, false, NoLd, St, RIn,
               float2[1][1], MR>::run(s, tw, NoLd{}, st, rin, dummy);
}

}  // namespace pstd
