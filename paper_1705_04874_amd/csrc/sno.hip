// Spectral neural operator surrogate: BF16-MFMA / FP32-accumulate kernels,
// hand-written forward and backward passes, Adam, error head, solver fallback.
//
// Every contraction is one call of a strided, batched GEMM
//   C[b](m, n) = alpha * sum_kb sum_k A[b, kb](m, k) B[b, kb](k, n) + beta * C[b](m, n) + bias(m)
// whose operands are addressed through arbitrary element strides (so
// transposes, the per-mode complex mixing and the weight gradients summed over
// the batch are all the same kernel).  Operands whose k or m/n dimension is
// contiguous (and 16-byte aligned) go through k_gemm_t: a 256-thread block
// computes a BM x BN tile (64 or 128 each), stages 32-deep slices of A and B
// in LDS as BF16 with k contiguous from float4 loads (the next slice's loads
// in flight while the current one is multiplied), and each wave issues
// (BM/32) x (BN/32) MFMA 16x16x32 ops per slice.  Other strides use k_gemm
// (64 x 64 tiles, 16-deep slices, element loads).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "sno.h"

namespace {

typedef short bf4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

thread_local std::string g_serr;

int sfail(int code, const std::string& msg)
{
    g_serr = msg;
    return code;
}

#define S_TRY(expr)                                                                               \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return sfail(e_ == hipErrorOutOfMemory ? PSTD_ENOMEM : PSTD_EDEVICE,                  \
                         std::string(#expr) + ": " + hipGetErrorString(e_));                      \
    } while (0)

// round to nearest even
__device__ __forceinline__ short to_bf16(float f)
{
    unsigned u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

struct GemmP {
    int M, N, K, KB;
    const float* A;
    long sAm, sAk, sAb, sAkb;
    const float* B;
    long sBk, sBn, sBb, sBkb;
    float* C;
    long sCm, sCn, sCb;
    float alpha, beta;
    const float* bias;   // per row, and per batch entry with stride sBiasb
    long sBiasb;
    int nsplit;          // > 1: blockIdx.z splits the (kb, k) slices of one product (batch 1);
    float* part;         // split z writes its partial sum to part + z M N (row-major)
};

__global__ __launch_bounds__(256) void k_gemm(GemmP p)
{
    __shared__ short As[64][16];
    __shared__ short Bs[64][16];
    const int b = blockIdx.z;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    const float* __restrict__ A = p.A + b * p.sAb;
    const float* __restrict__ B = p.B + b * p.sBb;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    f4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    const int am = t >> 2, aq = (t & 3) * 4;      // A tile: row am, k quad aq
    const int bn = t & 63, bq = (t >> 6) * 4;     // B tile: column bn, k quad bq
    for (int kb = 0; kb < p.KB; ++kb) {
        const float* __restrict__ Ak = A + kb * p.sAkb;
        const float* __restrict__ Bk = B + kb * p.sBkb;
        for (int k0 = 0; k0 < p.K; k0 += 16) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int k = k0 + aq + i;
                const float v = (m0 + am < p.M && k < p.K) ? Ak[(long)(m0 + am) * p.sAm + (long)k * p.sAk] : 0.f;
                As[am][aq + i] = to_bf16(v);
                const int kk = k0 + bq + i;
                const float u = (n0 + bn < p.N && kk < p.K) ? Bk[(long)kk * p.sBk + (long)(n0 + bn) * p.sBn] : 0.f;
                Bs[bn][bq + i] = to_bf16(u);
            }
            __syncthreads();
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                for (int ni = 0; ni < 2; ++ni) {
                    const int mr = (w >> 1) * 32 + mi * 16 + (lane & 15);
                    const int nc = (w & 1) * 32 + ni * 16 + (lane & 15);
                    const bf4 av = *reinterpret_cast<const bf4*>(&As[mr][4 * (lane >> 4)]);
                    const bf4 bv = *reinterpret_cast<const bf4*>(&Bs[nc][4 * (lane >> 4)]);
                    acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[mi][ni], 0, 0, 0);
                }
            __syncthreads();
        }
    }
    float* __restrict__ C = p.C + b * p.sCb;
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = m0 + (w >> 1) * 32 + mi * 16 + 4 * (lane >> 4) + i;
                const int col = n0 + (w & 1) * 32 + ni * 16 + (lane & 15);
                if (row < p.M && col < p.N) {
                    float* c = C + (long)row * p.sCm + (long)col * p.sCn;
                    float v = p.alpha * acc[mi][ni][i];
                    if (p.beta != 0.f) v += p.beta * (*c);
                    if (p.bias) v += p.bias[b * p.sBiasb + row];
                    *c = v;
                }
            }
}

// Tiled kernel.  AK: A is k-contiguous (sAk == 1), else m-contiguous
// (sAm == 1); BK: B is k-contiguous (sBk == 1), else n-contiguous (sBn == 1).
// Every float4 the kernel loads is either wholly inside or wholly outside the
// operand (the contiguous extent is a multiple of 4 and the other strides are
// multiples of 4), so the out-of-range ones are zeros.
constexpr int GK = 32;          // k per slice
constexpr int GLD = GK + 8;     // LDS row length in BF16 (80 bytes: conflict-free 16-byte reads)

// One operand's slice: rows [r0, r0 + R) of the m (or n) axis, k [k0, k0 + 32).
// Sub-block sb of 4 rows x 4 k is loaded as 4 float4 and stored as 4 rows of
// 4 BF16 (8 bytes each) into S[row][k].
template <int R, bool KC>
struct Slice {
    static constexpr int NSB = R * GK / 16;          // sub-blocks
    static constexpr int PER = (NSB + 255) / 256;    // per thread
    float4 v[PER][4];
    __device__ __forceinline__ void load(const float* __restrict__ X, long sR, long sK, int nR, int nK, int r0, int k0)
    {
        const int t = threadIdx.x;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int sb = t + q * 256;
            // k-contiguous: 8 neighbouring threads cover one row's 32 k;
            // row-contiguous: R / 4 neighbouring threads cover one k's R rows
            const int rb = KC ? sb / (GK / 4) : sb % (R / 4);
            const int kb = KC ? sb % (GK / 4) : sb / (R / 4);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = r0 + rb * 4 + (KC ? i : 0), k = k0 + kb * 4 + (KC ? 0 : i);
                const bool in = (NSB % 256 == 0 || sb < NSB) && r < nR && k < nK;
                v[q][i] = in ? *reinterpret_cast<const float4*>(X + (long)r * sR + (long)k * sK)
                             : make_float4(0.f, 0.f, 0.f, 0.f);
            }
        }
    }
    __device__ __forceinline__ void store(__bf16 (*S)[GLD]) const
    {
        const int t = threadIdx.x;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int sb = t + q * 256;
            if (NSB % 256 != 0 && sb >= NSB) continue;
            const int rb = KC ? sb / (GK / 4) : sb % (R / 4);
            const int kb = KC ? sb % (GK / 4) : sb / (R / 4);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                // row rb * 4 + i, k kb * 4 .. kb * 4 + 3
                float a, b, c, d;
                if (KC) {
                    a = v[q][i].x; b = v[q][i].y; c = v[q][i].z; d = v[q][i].w;
                } else {
                    const float* e0 = reinterpret_cast<const float*>(&v[q][0]);
                    const float* e1 = reinterpret_cast<const float*>(&v[q][1]);
                    const float* e2 = reinterpret_cast<const float*>(&v[q][2]);
                    const float* e3 = reinterpret_cast<const float*>(&v[q][3]);
                    a = e0[i]; b = e1[i]; c = e2[i]; d = e3[i];
                }
                typedef __bf16 bf4v __attribute__((ext_vector_type(4)));
                bf4v w = {(__bf16)a, (__bf16)b, (__bf16)c, (__bf16)d};
                *reinterpret_cast<bf4v*>(&S[rb * 4 + i][kb * 4]) = w;
            }
        }
    }
};

template <int BM, int BN, bool AK, bool BK>
__global__ __launch_bounds__(256) void k_gemm_t(GemmP p)
{
    constexpr int TM = BM / 32, TN = BN / 32;     // 16 x 16 tiles per wave (2 x 2 waves)
    __shared__ __attribute__((aligned(16))) __bf16 As[BM][GLD];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[BN][GLD];
    const int b = blockIdx.z;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wm = (w >> 1) * (BM / 2), wn = (w & 1) * (BN / 2);
    f4 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    Slice<BM, AK> sa;
    Slice<BN, BK> sb;
    const int nks = (p.K + GK - 1) / GK;
    // slices (kb, k0) of this block: all of them, or with a split its share
    int s_lo = 0, s_hi = p.KB * nks;
    const bool split = p.nsplit > 1;
    const int ab = split ? 0 : b;
    if (split) {
        const long ns = s_hi;
        s_lo = (int)(ns * b / p.nsplit);
        s_hi = (int)(ns * (b + 1) / p.nsplit);
    }
    // A as rows m: stride along the rows sAm, along k sAk; B as rows n: sBn, sBk
    auto load = [&](int s) {
        const int kb = s / nks, k0 = (s - kb * nks) * GK;
        sa.load(p.A + ab * p.sAb + kb * p.sAkb, p.sAm, p.sAk, p.M, p.K, m0, k0);
        sb.load(p.B + ab * p.sBb + kb * p.sBkb, p.sBn, p.sBk, p.N, p.K, n0, k0);
    };
    if (s_lo < s_hi) load(s_lo);
    for (int s = s_lo; s < s_hi; ++s) {
        sa.store(As);
        sb.store(Bs);
        __syncthreads();
        if (s + 1 < s_hi) load(s + 1);
        bf8 av[TM], bv[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) av[i] = *reinterpret_cast<const bf8*>(&As[wm + i * 16 + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
        for (int j = 0; j < TN; ++j) bv[j] = *reinterpret_cast<const bf8*>(&Bs[wn + j * 16 + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    if (split) {
        float* __restrict__ P = p.part + (long)b * p.M * p.N;
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int row = m0 + wm + i * 16 + 4 * (lane >> 4) + q;
                    const int col = n0 + wn + j * 16 + (lane & 15);
                    if (row < p.M && col < p.N) P[(long)row * p.N + col] = acc[i][j][q];
                }
        return;
    }
    float* __restrict__ C = p.C + b * p.sCb;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = m0 + wm + i * 16 + 4 * (lane >> 4) + q;
                const int col = n0 + wn + j * 16 + (lane & 15);
                if (row < p.M && col < p.N) {
                    float* c = C + (long)row * p.sCm + (long)col * p.sCn;
                    float v = p.alpha * acc[i][j][q];
                    if (p.beta != 0.f) v += p.beta * (*c);
                    if (p.bias) v += p.bias[b * p.sBiasb + row];
                    *c = v;
                }
            }
}

// C = alpha * (sum over the splits of the partial products, in split order)
// + beta * C + bias
__global__ __launch_bounds__(256) void k_split_sum(GemmP p)
{
    const long n = (long)p.M * p.N;
    for (long e = blockIdx.x * 256L + threadIdx.x; e < n; e += (long)gridDim.x * 256) {
        const int row = (int)(e / p.N), col = (int)(e - (long)row * p.N);
        float acc = 0.f;
        for (int z = 0; z < p.nsplit; ++z) acc += p.part[(long)z * n + e];
        float* c = p.C + (long)row * p.sCm + (long)col * p.sCn;
        float v = p.alpha * acc;
        if (p.beta != 0.f) v += p.beta * (*c);
        if (p.bias) v += p.bias[row];
        *c = v;
    }
}

// An operand suits the tiled kernel when one of its two dimensions is
// contiguous with an extent that is a multiple of 4 and every other stride
// and the base are 16-byte multiples.
bool tiled_ok(const float* X, long sR, long sK, long sB, long sKB, int nR, int nK, bool& kc)
{
    if ((reinterpret_cast<uintptr_t>(X) & 15) || sB % 4 || sKB % 4) return false;
    if (sK == 1 && sR % 4 == 0 && nK % 4 == 0) {
        kc = true;
        return true;
    }
    if (sR == 1 && sK % 4 == 0 && nR % 4 == 0) {
        kc = false;
        return true;
    }
    return false;
}

template <int BM, int BN>
void launch_tiled(hipStream_t st, const GemmP& p, int batch, bool ak, bool bk)
{
    const dim3 grid((p.N + BN - 1) / BN, (p.M + BM - 1) / BM, batch);
    if (ak && bk) hipLaunchKernelGGL((k_gemm_t<BM, BN, true, true>), grid, dim3(256), 0, st, p);
    else if (ak) hipLaunchKernelGGL((k_gemm_t<BM, BN, true, false>), grid, dim3(256), 0, st, p);
    else if (bk) hipLaunchKernelGGL((k_gemm_t<BM, BN, false, true>), grid, dim3(256), 0, st, p);
    else hipLaunchKernelGGL((k_gemm_t<BM, BN, false, false>), grid, dim3(256), 0, st, p);
}

// ws (ws_floats floats of device memory): where a product of one batch entry
// summed over many kb would leave most compute units idle, its slices are
// split over blocks that write partial sums there, added up in a second pass.
void gemm(hipStream_t st, int batch, int M, int N, int K, int KB, const float* A, long sAm, long sAk, long sAb,
          long sAkb, const float* B, long sBk, long sBn, long sBb, long sBkb, float* C, long sCm, long sCn, long sCb,
          float alpha = 1.f, float beta = 0.f, const float* bias = nullptr, long sBiasb = 0, float* ws = nullptr,
          long ws_floats = 0)
{
    GemmP p{M, N, K, KB, A, sAm, sAk, sAb, sAkb, B, sBk, sBn, sBb, sBkb, C, sCm, sCn, sCb, alpha, beta, bias, sBiasb,
            1, nullptr};
    bool ak = false, bk = false;
    if (M >= 32 && N >= 32 && K >= 16 && tiled_ok(A, sAm, sAk, sAb, sAkb, M, K, ak) &&
        tiled_ok(B, sBn, sBk, sBb, sBkb, N, K, bk)) {
        const long tiles = (long)((N + 63) / 64) * ((M + 63) / 64);
        const long slices = (long)KB * ((K + GK - 1) / GK);
        if (batch == 1 && ws && tiles < 128 && slices >= 32) {
            // at least 8 slices per split, about 512 blocks, within the workspace
            long ns = std::min<long>(std::min<long>(slices / 8, (512 + tiles - 1) / tiles), 256);
            ns = std::min<long>(ns, ws_floats / ((long)M * N));
            if (ns >= 2) {
                p.nsplit = (int)ns;
                p.part = ws;
                launch_tiled<64, 64>(st, p, (int)ns, ak, bk);
                const long n = (long)M * N;
                hipLaunchKernelGGL(k_split_sum, dim3((unsigned)std::min<long>((n + 255) / 256, 2048)), dim3(256), 0,
                                   st, p);
                return;
            }
        }
        // 128-wide tiles where both sides fill them and the grid still has a
        // block per compute unit
        const long big = (long)((N + 127) / 128) * ((M + 127) / 128) * batch;
        if (M >= 128 && N >= 128 && big >= 256) launch_tiled<128, 128>(st, p, batch, ak, bk);
        else if (M >= 128 && (long)((N + 63) / 64) * ((M + 127) / 128) * batch >= 256)
            launch_tiled<128, 64>(st, p, batch, ak, bk);
        else launch_tiled<64, 64>(st, p, batch, ak, bk);
        return;
    }
    hipLaunchKernelGGL(k_gemm, dim3((N + 63) / 64, (M + 63) / 64, batch), dim3(256), 0, st, p);
}

// ---------------------------------------------------------------------------
constexpr float GELU_C = 0.7978845608028654f;   // sqrt(2 / pi)

__device__ __forceinline__ float gelu_f(float x)
{
    return 0.5f * x * (1.f + tanhf(GELU_C * (x + 0.044715f * x * x * x)));
}
__device__ __forceinline__ float gelu_d(float x)
{
    const float th = tanhf(GELU_C * (x + 0.044715f * x * x * x));
    return 0.5f * (1.f + th) + 0.5f * x * (1.f - th * th) * GELU_C * (1.f + 3.f * 0.044715f * x * x);
}

__global__ void k_gelu(const float* __restrict__ z, float* __restrict__ y, long n)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        y[i] = gelu_f(z[i]);
}

__global__ void k_gelu_bwd(const float* __restrict__ dy, const float* __restrict__ z, float* __restrict__ dz, long n)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        dz[i] = dy[i] * gelu_d(z[i]);
}

struct Feat {
    float off[9], inv[9];
    float cyc[SNO_MAX_FOUR];   // Fourier feature frequencies, cycles per window
    int n_four;
};

// lift input A[b][i][t], NA channels: the 3 normalised position features,
// t / T, cos and sin of 2 pi c_f t / T per frequency, and with position
// modulation (NA = 4 + 8 n_four) the products p_k cos, p_k sin for each
// frequency f and position feature k, in the order (f, k, cos / sin)
__device__ __forceinline__ float four_feat(const Feat& f, int q, int sine, int t, int T)
{
    // phase c t / T reduced to [0, 1) turns before the sine and cosine
    const float ph = f.cyc[q] * (float)t / (float)T;
    const float r = 2.f * 3.14159265358979f * (ph - floorf(ph));
    return sine ? sinf(r) : cosf(r);
}

__global__ void k_features(const float* __restrict__ X, Feat f, int B, int T, int NA, float* __restrict__ A)
{
    const int nbase = 4 + 2 * f.n_four;
    const long n = (long)B * NA * T;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        const int t = e % T;
        const int i = (e / T) % NA;
        const int b = e / ((long)NA * T);
        float v;
        if (i < 3) {
            v = (X[b * 9 + i] - f.off[i]) * f.inv[i];
        } else if (i == 3) {
            v = (float)t / (float)T;
        } else if (i < nbase) {
            v = four_feat(f, (i - 4) >> 1, (i - 4) & 1, t, T);
        } else {
            const int j = i - nbase, q = j / 6, k = (j % 6) >> 1;
            v = (X[b * 9 + k] - f.off[k]) * f.inv[k] * four_feat(f, q, j & 1, t, T);
        }
        A[e] = v;
    }
}

// moment features m[b][j] = X[b][3 + j] / scale
__device__ __forceinline__ float mfeat(const float* X, const Feat& f, int b, int j) { return X[b * 9 + 3 + j] * f.inv[3 + j]; }

// The output is linear in the moment features (eq. 2 is linear in its
// source), so the projection's 6 responses are weighted before the product:
// Qm[b][f O + o][h] = sum_j m_bj Q2[(f 6 + j) O + o][h] and bm[b][f O + o] =
// sum_j m_bj q2b[(f 6 + j) O + o], and the output rows of sample b come from
// one product Qm[b] Hq[b] + bm[b] (a sixth of the work of forming all six
// responses and combining them).
__global__ __launch_bounds__(256) void k_qmix(const float* __restrict__ Q2, const float* __restrict__ q2b,
                                              const float* __restrict__ X, Feat f, int B, int FO, int O, int H,
                                              float* __restrict__ Qm, float* __restrict__ bm)
{
    // block rows fo, thread hh (hh = H: the bias); the six response weights
    // of (fo, hh) are read once and applied to every sample
    const int hh = blockIdx.x * 256 + threadIdx.x;
    if (hh > H) return;
    for (int fo = blockIdx.y; fo < FO; fo += gridDim.y) {
        const int fr = fo / O, o = fo - fr * O;
        float q[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            const long row = (long)(fr * 6 + j) * O + o;
            q[j] = hh < H ? Q2[row * H + hh] : q2b[row];
        }
        for (int b = 0; b < B; ++b) {
            float s = 0.f;
#pragma unroll
            for (int j = 0; j < 6; ++j) s += mfeat(X, f, b, j) * q[j];
            if (hh < H) Qm[((long)b * FO + fo) * H + hh] = s;
            else bm[(long)b * FO + fo] = s;
        }
    }
}

// gradients of Q2 and q2b from those of the weighted projection:
// dQ2[(f 6 + j) O + o][h] = sum_b m_bj dQm[b][f O + o][h] (h = H: the bias)
__global__ __launch_bounds__(256) void k_qgrad(const float* __restrict__ dQm, const float* __restrict__ dbm,
                                               const float* __restrict__ X, Feat f, int B, int FO, int O, int H,
                                               float* __restrict__ dQ2, float* __restrict__ dq2b)
{
    // block rows fo, thread hh: each dQm value is read once for all six j
    const int hh = blockIdx.x * 256 + threadIdx.x;
    if (hh > H) return;
    for (int fo = blockIdx.y; fo < FO; fo += gridDim.y) {
        const int fr = fo / O, o = fo - fr * O;
        float s[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        for (int b = 0; b < B; ++b) {
            const float d = hh < H ? dQm[((long)b * FO + fo) * H + hh] : dbm[(long)b * FO + fo];
#pragma unroll
            for (int j = 0; j < 6; ++j) s[j] += mfeat(X, f, b, j) * d;
        }
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            const long row = (long)(fr * 6 + j) * O + o;
            if (hh < H) dQ2[row * H + hh] = s[j];
            else dq2b[row] = s[j];
        }
    }
}

// Travel-time-aligned frames.  shift[b][f][r] = (tau_f - t_ref[f]) / dt with
// tau_f the first-arrival time of the two-point ray from source b's cell
// (X[b][0..2], whole cell indices) to receiver r's through frame f's slowness
// profile over depth (a straight segment where the path stays in one layer,
// is vertical, or crosses a zero slowness); cum[f][k] = h_z (sum_{i<k} s_i +
// s_k / 2) is the depth integral of the slowness from the top to the centre
// of cell k, which the straight segment uses.
struct Rays {
    const int* rec;        // [n_rec][3]
    const double* cum;     // [frames][nz]
    const double* slow;    // [frames][nz]
    double h[3];
    double dt;
    double t_ref[2];
    int nz, n_rec, frames;
};

// sum (all lanes get it) and minimum over the 64 lanes of a wave
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}
__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v = fmin(v, __shfl_xor(v, m, 64));
    return v;
}

// bisection steps for the ray's horizontal slowness: to 2^-32 of the
// smallest slowness, which moves the travel time by at most the horizontal
// distance times that (6e-11 s over a kilometre where the fastest layer runs
// at 4 km/s)
constexpr int RAY_ITERS = 32;

// One wave per (source b, frame f, receiver r); its lanes take the cell
// layers of the path in turn and the sums over layers are wave reductions.
__global__ __launch_bounds__(256) void k_shifts(const float* __restrict__ X, Rays ry, int B, float* __restrict__ shift)
{
    const int lane = threadIdx.x & 63;
    const int n = B * ry.frames * ry.n_rec;
    for (int e = blockIdx.x * 4 + (threadIdx.x >> 6); e < n; e += gridDim.x * 4) {
        const int r = e % ry.n_rec, f = (e / ry.n_rec) % ry.frames, b = e / (ry.n_rec * ry.frames);
        int src[3];
        for (int a = 0; a < 3; ++a) src[a] = (int)rintf(X[b * 9 + a]);
        const double dx = (double)(src[0] - ry.rec[3 * r + 0]) * ry.h[0];
        const double dy = (double)(src[1] - ry.rec[3 * r + 1]) * ry.h[1];
        const int ks = min(max(src[2], 0), ry.nz - 1), kr = ry.rec[3 * r + 2];
        const int k0 = min(ks, kr), k1 = max(ks, kr);
        const double hor = sqrt(dx * dx + dy * dy);
        const double* __restrict__ sl = ry.slow + f * ry.nz;
        double smin = 1e300;
        for (int k = k0 + lane; k <= k1; k += 64) smin = fmin(smin, sl[k]);
        smin = wave_min(smin);
        double tau;
        if (k0 == k1 || hor == 0.0 || !(smin > 0.0)) {
            // straight segment: |d| / |dz| times the depth integral of the
            // slowness (one layer: |d| times its slowness)
            const double dz = (double)(ks - kr) * ry.h[2];
            const double L = sqrt(hor * hor + dz * dz);
            tau = k0 == k1 ? L * sl[ks] : L / fabs(dz) * fabs(ry.cum[f * ry.nz + ks] - ry.cum[f * ry.nz + kr]);
        } else {
            // two-point ray (Snell's law across the cell layers): horizontal
            // slowness p by bisection so that the layers' horizontal runs
            // t p / sqrt(s^2 - p^2) add up to the horizontal distance; layer
            // thickness half a cell at each end, a whole cell between
            double lo = 0.0, hi = smin;
            for (int it = 0; it < RAY_ITERS; ++it) {
                const double p = 0.5 * (lo + hi);
                double run = 0.0;
                for (int k = k0 + lane; k <= k1; k += 64) {
                    const double t = (k == k0 || k == k1 ? 0.5 : 1.0) * ry.h[2];
                    run += t * p / sqrt(sl[k] * sl[k] - p * p);
                }
                if (wave_sum(run) < hor) lo = p;
                else hi = p;
            }
            const double p = 0.5 * (lo + hi);
            double tt = 0.0;
            for (int k = k0 + lane; k <= k1; k += 64) {
                const double t = (k == k0 || k == k1 ? 0.5 : 1.0) * ry.h[2];
                tt += t * sl[k] * sl[k] / sqrt(sl[k] * sl[k] - p * p);
            }
            tau = wave_sum(tt);
        }
        if (lane == 0) shift[e] = (float)((tau - ry.t_ref[f]) / ry.dt);
    }
}

// 4-point Lagrange weights at offsets -1, 0, 1, 2 from floor(x), w = x - floor(x)
__device__ __forceinline__ void lagrange4(float w, float* c)
{
    c[0] = -w * (w - 1.f) * (w - 2.f) * (1.f / 6.f);
    c[1] = (w + 1.f) * (w - 1.f) * (w - 2.f) * 0.5f;
    c[2] = -(w + 1.f) * w * (w - 2.f) * 0.5f;
    c[3] = (w + 1.f) * w * (w - 1.f) * (1.f / 6.f);
}

// Y[b][o][t] = sum_f Yf[b][f O + o](t - shift[b][f][o mod n_rec])
__global__ __launch_bounds__(256) void k_fcomb(const float* __restrict__ Yf, const float* __restrict__ shift, int B,
                                               int F, int O, int n_rec, int T, float* __restrict__ Y)
{
    // block rows (b, o), threads along t
    const long per = (long)O * T;
    for (int row = blockIdx.y; row < B * O; row += gridDim.y) {
        const int b = row / O, o = row - b * O;
        for (int t = blockIdx.x * 256 + threadIdx.x; t < T; t += gridDim.x * 256) {
            float acc = 0.f;
            for (int fr = 0; fr < F; ++fr) {
                const float x = (float)t - shift[(b * F + fr) * n_rec + o % n_rec];
                const float fl = floorf(x);
                float c[4];
                lagrange4(x - fl, c);
                const int i0 = (int)fl - 1;
                const float* u = Yf + ((long)b * F + fr) * per + (long)o * T;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int i = i0 + k;
                    if (i >= 0 && i < T) acc += c[k] * u[i];
                }
            }
            Y[(long)row * T + t] = acc;
        }
    }
}

// dYf[b][f O + o][i] = sum_t dY[b][o][t] w_{t,i}: the transpose of k_fcomb, as a
// gather over the (at most five) t whose interpolation reads sample i
__global__ __launch_bounds__(256) void k_fspread(const float* __restrict__ dY, const float* __restrict__ shift, int B,
                                                 int F, int O, int n_rec, int T, float* __restrict__ dYf)
{
    // block rows ((b F + f) O + o), threads along i
    for (int row = blockIdx.y; row < B * F * O; row += gridDim.y) {
        const int o = row % O, bf = row / O, b = bf / F;
        const float sh = shift[bf * n_rec + o % n_rec];
        const float* __restrict__ g = dY + ((long)b * O + o) * T;
        for (int i = blockIdx.x * 256 + threadIdx.x; i < T; i += gridDim.x * 256) {
            // t - sh in [i - 2, i + 1] reads sample i
            const int t0 = max(0, (int)floorf((float)i - 2.f + sh));
            const int t1 = min(T - 1, (int)ceilf((float)i + 1.f + sh));
            float acc = 0.f;
            for (int t = t0; t <= t1; ++t) {
                const float x = (float)t - sh;
                const float fl = floorf(x);
                const int k = i - (int)fl + 1;
                if (k < 0 || k > 3) continue;
                float c[4];
                lagrange4(x - fl, c);
                acc += c[k] * g[t];
            }
            dYf[(long)row * T + i] = acc;
        }
    }
}

// Per-mode complex channel mixing of the spectral layers (16 modes, width C):
// U[b][c][k] = sum_c' M_k[c][c'] V[b][c'][k] with M_k = Rr_k + i Ri_k
// (forward) or its conjugate transpose (the input gradient), real parts at
// column k and imaginary parts at K + k of each row of 2K.  One block per
// mode stages M_k (rows padded to C + 1, conflict-free) and chunks of up to
// MIX_B samples' V in LDS; FP32 products and sums in a fixed order.
constexpr int MIX_B = 32;
constexpr size_t MIX_LDS_MAX = 64 * 1024;

size_t mix_lds(long C) { return ((size_t)2 * C * (C + 1) + 2 * (size_t)MIX_B * C) * sizeof(float); }

template <bool HERM>
__global__ __launch_bounds__(256) void k_cmix(const float* __restrict__ Rr, const float* __restrict__ Ri,
                                              const float* __restrict__ V, int B, int C, int K,
                                              float* __restrict__ U)
{
    extern __shared__ float sm[];
    const int k = blockIdx.x;
    const int C1 = C + 1;
    float* mr = sm;                     // mr[c][c'] (row stride C + 1)
    float* mi = sm + C * C1;
    float* vr = sm + 2 * C * C1;        // vr[b][c'], b < MIX_B
    float* vi = vr + MIX_B * C;
    const long K2 = 2L * K;
    for (int e = threadIdx.x; e < C * C; e += 256) {
        const int a = e / C, q = e - a * C;
        const float xr = Rr[(long)k * C * C + e], xi = Ri[(long)k * C * C + e];
        if (HERM) {
            mr[q * C1 + a] = xr;
            mi[q * C1 + a] = -xi;
        } else {
            mr[a * C1 + q] = xr;
            mi[a * C1 + q] = xi;
        }
    }
    for (int b0 = 0; b0 < B; b0 += MIX_B) {
        const int nb = min(MIX_B, B - b0);
        __syncthreads();   // M staged / the previous chunk's readers done
        for (int e = threadIdx.x; e < nb * C; e += 256) {
            const long row = (long)(b0 + e / C) * C + (e % C);
            vr[e] = V[row * K2 + k];
            vi[e] = V[row * K2 + K + k];
        }
        __syncthreads();
        for (int e = threadIdx.x; e < nb * C; e += 256) {
            const int b = e / C, c = e - b * C;
            float ur = 0.f, ui = 0.f;
            for (int q = 0; q < C; ++q) {
                const float a = mr[c * C1 + q], bb = mi[c * C1 + q];
                const float xr = vr[b * C + q], xi = vi[b * C + q];
                ur = fmaf(a, xr, fmaf(-bb, xi, ur));
                ui = fmaf(bb, xr, fmaf(a, xi, ui));
            }
            const long row = (long)(b0 + b) * C + c;
            U[row * K2 + k] = ur;
            U[row * K2 + K + k] = ui;
        }
    }
}

// Gradient of the mixing weights, summed over the samples:
// dRr_k[c][c'] = sum_b dUr[b][c] Vr[b][c'] + dUi[b][c] Vi[b][c'],
// dRi_k[c][c'] = sum_b dUi[b][c] Vr[b][c'] - dUr[b][c] Vi[b][c'].
__global__ __launch_bounds__(256) void k_cmix_dw(const float* __restrict__ dU, const float* __restrict__ V, int B,
                                                 int C, int K, float* __restrict__ dRr, float* __restrict__ dRi)
{
    extern __shared__ float sm[];
    const int k = blockIdx.x;
    float* ur = sm;                     // [b][c], b < MIX_B
    float* ui = ur + MIX_B * C;
    float* vr = ui + MIX_B * C;
    float* vi = vr + MIX_B * C;
    const long K2 = 2L * K;
    constexpr int PER = 16;             // outputs per thread and pass
    for (int e0 = 0; e0 < C * C; e0 += 256 * PER) {
        float ar[PER], ai[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) ar[j] = ai[j] = 0.f;
        for (int b0 = 0; b0 < B; b0 += MIX_B) {
            const int nb = min(MIX_B, B - b0);
            __syncthreads();
            for (int e = threadIdx.x; e < nb * C; e += 256) {
                const long row = (long)(b0 + e / C) * C + (e % C);
                ur[e] = dU[row * K2 + k];
                ui[e] = dU[row * K2 + K + k];
                vr[e] = V[row * K2 + k];
                vi[e] = V[row * K2 + K + k];
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                const int e = e0 + j * 256 + threadIdx.x;
                if (e < C * C) {
                    const int c = e / C, q = e - c * C;
                    for (int b = 0; b < nb; ++b) {
                        const float xr = ur[b * C + c], xi = ui[b * C + c];
                        const float yr = vr[b * C + q], yi = vi[b * C + q];
                        ar[j] = fmaf(xr, yr, fmaf(xi, yi, ar[j]));
                        ai[j] = fmaf(xi, yr, fmaf(-xr, yi, ai[j]));
                    }
                }
            }
        }
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int e = e0 + j * 256 + threadIdx.x;
            if (e < C * C) {
                dRr[(long)k * C * C + e] = ar[j];
                dRi[(long)k * C * C + e] = ai[j];
            }
        }
    }
}

// out[r] = sum over b, t of X[b][r][t]  (fixed reduction order)
__global__ __launch_bounds__(256) void k_rowsum(const float* __restrict__ X, int B, int R, int T, float* __restrict__ out)
{
    __shared__ float red[256];
    const int r = blockIdx.x;
    float s = 0.f;
    for (int b = 0; b < B; ++b)
        for (int t = threadIdx.x; t < T; t += 256) s += X[((long)b * R + r) * T + t];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[r] = red[0];
}

// dY = 2 (Y - Yt) / n; block partial sums of (Y - Yt)^2
// dY = 2 w (Y - Yt) / n and per-block partial sums of w (Y - Yt)^2, with w
// = wgt[b][o / n_rec] per sample and component (1 without weights); rows
// (b, o) in a fixed order per block, so the partial sums are reproducible
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ Y, const float* __restrict__ Yt,
                                             const float* __restrict__ wgt, int B, int O, int T, int n_rec,
                                             float* __restrict__ dY, float* __restrict__ part)
{
    __shared__ float red[256];
    float s = 0.f;
    const float g = 2.f / ((float)B * O * T);
    for (int row = blockIdx.x; row < B * O; row += gridDim.x) {
        const int b = row / O, o = row - b * O;
        const float w = wgt ? wgt[b * 4 + o / n_rec] : 1.f;
        const long base = (long)row * T;
        for (int t = threadIdx.x; t < T; t += 256) {
            const float d = Y[base + t] - Yt[base + t];
            dY[base + t] = g * w * d;
            s += w * d * d;
        }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// relative-loss weights of n samples: w[i][c] = 1 / mean square of sample i's
// component c after the output normalisation (0 for an all-zero component)
__global__ __launch_bounds__(256) void k_relw(const float* __restrict__ Y, int n_rec, int T,
                                              const float* __restrict__ scale, float* __restrict__ w)
{
    __shared__ double red[256];
    const int i = blockIdx.x, c = blockIdx.y;
    const long per = (long)n_rec * T;
    const float* __restrict__ y = Y + ((long)i * 4 + c) * per;
    const double inv = 1.0 / (double)scale[c];
    double s = 0.0;
    for (long e = threadIdx.x; e < per; e += 256) {
        const double v = y[e] * inv;
        s += v * v;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) w[i * 4 + c] = red[0] > 0.0 ? (float)((double)per / red[0]) : 0.f;
}

// the batch's weights: wb[b][c] = w[idx[b]][c]
__global__ void k_gather_w(const float* __restrict__ w, const int* __restrict__ idx, int B, float* __restrict__ wb)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < B * 4) wb[e] = w[idx[e / 4] * 4 + e % 4];
}

__global__ void k_sum_parts(const float* __restrict__ part, int np, float* __restrict__ out, float scale)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        float s = 0.f;
        for (int i = 0; i < np; ++i) s += part[i];
        *out = s * scale;
    }
}

// Adam step; omb1 = 1 - b1 and omb2 = 1 - b2 come rounded from double (1 - b2
// formed in float would carry the rounding of b2 = 0.999 into the weight of g^2,
// a 1.3e-5 relative error)
__global__ void k_adam(float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       long n, float lr, float b1, float b2, float omb1, float omb2, float eps, float c1, float c2)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const float mi = b1 * m[i] + omb1 * g[i];
        const float vi = b2 * v[i] + omb2 * g[i] * g[i];
        m[i] = mi;
        v[i] = vi;
        th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// gather a batch: Xb[b] = X[idx[b]], Yb[b][o][t] = Y[idx[b]][o][t] / scale[o / n_rec]
__global__ void k_gather(const float* __restrict__ X, const float* __restrict__ Y, const int* __restrict__ idx, int B,
                         int O, int T, int n_rec, const float* __restrict__ scale, float* __restrict__ Xb,
                         float* __restrict__ Yb)
{
    const long per = (long)O * T;
    const long n = (long)B * per;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        const int b = e / per;
        const long r = e - b * per;
        const int o = r / T;
        Yb[e] = Y[(long)idx[b] * per + r] / scale[o / n_rec];
        if (r < 9) Xb[b * 9 + r] = X[(long)idx[b] * 9 + r];
    }
}

// Y[b][o][t] *= scale[o / n_rec]
__global__ void k_scale_out(float* __restrict__ Y, long n, int O, int T, int n_rec, const float* __restrict__ scale)
{
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        const int o = (e / T) % O;
        Y[e] *= scale[o / n_rec];
    }
}

// per-component sums of squares of Y over samples, receivers and t: block
// (c, j) of SQ_BLOCKS per component writes its share (sample rows j,
// j + SQ_BLOCKS, ...) to ss[c * SQ_BLOCKS + j]; the host adds the shares
constexpr int SQ_BLOCKS = 256;
__global__ __launch_bounds__(256) void k_comp_sumsq(const float* __restrict__ Y, int n, int n_rec, int T,
                                                    double* __restrict__ ss)
{
    __shared__ double red[256];
    const int c = blockIdx.x, j = blockIdx.y;
    double s = 0.0;
    for (long rr = j; rr < (long)n * n_rec; rr += SQ_BLOCKS) {
        const long b = rr / n_rec, r = rr - b * n_rec;
        const float* __restrict__ y = Y + ((b * 4 + c) * n_rec + r) * T;
        for (int i = threadIdx.x; i < T; i += 256) {
            const double v = y[i];
            s += v * v;
        }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) ss[c * SQ_BLOCKS + j] = red[0];
}

// per sample: max over the 4 components of ||Yp - Yt|| / ||Yt|| (any units)
__global__ __launch_bounds__(256) void k_relerr(const float* __restrict__ Yp, const float* __restrict__ Yt, int n_rec,
                                                int T, float* __restrict__ err)
{
    __shared__ float rn[256], rd[256];
    const int b = blockIdx.x;
    const long per = (long)n_rec * T;
    float worst = 0.f;
    for (int c = 0; c < 4; ++c) {
        float sn = 0.f, sd = 0.f;
        const long base = ((long)b * 4 + c) * per;
        for (long i = threadIdx.x; i < per; i += 256) {
            const float d = Yp[base + i] - Yt[base + i];
            sn += d * d;
            sd += Yt[base + i] * Yt[base + i];
        }
        rn[threadIdx.x] = sn;
        rd[threadIdx.x] = sd;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (threadIdx.x < h) {
                rn[threadIdx.x] += rn[threadIdx.x + h];
                rd[threadIdx.x] += rd[threadIdx.x + h];
            }
            __syncthreads();
        }
        worst = fmaxf(worst, sqrtf(rn[0] / fmaxf(rd[0], 1e-30f)));
        __syncthreads();
    }
    if (threadIdx.x == 0) err[b] = worst;
}

// phi[b] = (mean over t of V[b][c][t] for c < C, the 6 moment features, 1)
__global__ __launch_bounds__(256) void k_pool(const float* __restrict__ V, const float* __restrict__ X, Feat f, int C,
                                              int T, float* __restrict__ phi)
{
    __shared__ float red[256];
    const int b = blockIdx.x / C, c = blockIdx.x % C;
    float s = 0.f;
    for (int t = threadIdx.x; t < T; t += 256) s += V[((long)b * C + c) * T + t];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        float* ph = phi + (long)b * (C + 7);
        ph[c] = red[0] / T;
        if (c == 0) {
            for (int j = 0; j < 6; ++j) ph[C + j] = mfeat(X, f, b, j);
            ph[C + 6] = 1.f;
        }
    }
}

// est[b] = exp(sum_j h[j] phi[b][j] + margin)
__global__ void k_head(const float* __restrict__ phi, const float* __restrict__ h, int D, int B, float margin,
                       float* __restrict__ est)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    float s = margin;
    for (int j = 0; j < D; ++j) s += h[j] * phi[(long)b * D + j];
    est[b] = expf(fminf(s, 30.f));
}

__global__ void k_decim(const float* __restrict__ in, long rows, int nt, int decim, float* __restrict__ out)
{
    const int no = nt / decim;
    const long n = rows * no;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        const long r = e / no;
        const int j = e - r * no;
        out[e] = in[r * nt + (long)j * decim];
    }
}

int grid_for(long n) { return (int)std::min<long>((n + 255) / 256, 4096); }
// 256-thread blocks along a row of `len` values, one block row per row (the
// kernels loop over rows past the grid's y limit)
dim3 rows_grid(long len, long rows)
{
    return dim3((unsigned)((len + 255) / 256), (unsigned)std::min<long>(std::max<long>(rows, 1), 65535));
}

}  // namespace

// ===========================================================================
struct sno {
    sno_cfg cfg{};
    int O = 0, NA = 4;   // outputs per time sample, lift input channels
    long np = 0;
    long off_P, off_pb, off_W[16], off_b[16], off_Rr[16], off_Ri[16], off_Q1, off_q1b, off_Q2, off_q2b;
    float *theta = nullptr, *grad = nullptr, *m1 = nullptr, *m2 = nullptr;
    float *Fb = nullptr, *G = nullptr;   // truncated DFT bases
    float *dscale = nullptr;
    float scale[4] = {1, 1, 1, 1};
    std::vector<float> head;
    float head_margin = 0.f;
    float* dhead = nullptr;
    Feat feat{};
    int F = 1;                 // output frames
    int* drec = nullptr;       // ray tables (frames = 2)
    double* dcum = nullptr;
    double* dslow = nullptr;
    Rays rays{};
    int device = 0;
    // workspace for batches of up to bmax samples
    int bmax = 0;
    float *A = nullptr, *Vb = nullptr, *Vh = nullptr, *Z = nullptr, *Uh = nullptr, *Hp = nullptr, *Hq = nullptr,
          *Y = nullptr, *X0 = nullptr, *X1 = nullptr, *X2 = nullptr, *dH = nullptr, *dUh = nullptr, *dVh = nullptr,
          *part = nullptr, *lossd = nullptr, *phi = nullptr, *Xb = nullptr, *Yb = nullptr, *Y6 = nullptr,
          *dY6 = nullptr, *shift = nullptr, *Qm = nullptr, *dQm = nullptr, *bm = nullptr, *dbm = nullptr;
    int* idxd = nullptr;
    // partial sums of the split weight-gradient products
    static constexpr long kws_n = 4L << 20;
    float* kws = nullptr;
    float* wb = nullptr;       // the batch's loss weights [B][4]

    float* V(int l) { return l < cfg.L ? Vb + (long)l * bmax * cfg.C * cfg.T : Z + (long)(cfg.L - 1) * bmax * cfg.C * cfg.T; }
    float* Zl(int l) { return Z + (long)l * bmax * cfg.C * cfg.T; }
    float* Vhl(int l) { return Vh + (long)l * bmax * cfg.C * 2 * cfg.K; }

    void free_ws()
    {
        for (float* p : {A, Vb, Vh, Z, Uh, Hp, Hq, Y, X0, X1, X2, dH, dUh, dVh, part, lossd, phi, Xb, Yb, Y6, dY6, shift,
                         Qm, dQm, bm, dbm, kws, wb})
            (void)hipFree(p);
        (void)hipFree(idxd);
        A = Vb = Vh = Z = Uh = Hp = Hq = Y = X0 = X1 = X2 = dH = dUh = dVh = part = lossd = phi = Xb = Yb = Y6 = dY6 =
            shift = Qm = dQm = bm = dbm = kws = wb = nullptr;
        idxd = nullptr;
        bmax = 0;
    }
    ~sno()
    {
        free_ws();
        for (float* p : {theta, grad, m1, m2, Fb, G, dscale, dhead}) (void)hipFree(p);
        (void)hipFree(drec);
        (void)hipFree(dcum);
        (void)hipFree(dslow);
    }

    int ensure(int B)
    {
        if (B <= bmax) return PSTD_OK;
        free_ws();
        const long C = cfg.C, T = cfg.T, K2 = 2 * cfg.K, H = cfg.H, L = cfg.L;
        auto al = [&](float** p, long n) { return hipMalloc(p, std::max<long>(n, 1) * sizeof(float)); };
        if (al(&A, (long)B * NA * T) || al(&Y6, (long)B * F * O * T) || al(&dY6, (long)B * F * O * T) ||
            al(&shift, (long)B * F * cfg.n_rec) || al(&Qm, (long)B * F * O * H) || al(&dQm, (long)B * F * O * H) ||
            al(&bm, (long)B * F * O) || al(&dbm, (long)B * F * O) || al(&Vb, L * B * C * T) || al(&Vh, L * B * C * K2) || al(&Z, L * B * C * T) ||
            al(&Uh, (long)B * C * K2) || al(&Hp, (long)B * H * T) || al(&Hq, (long)B * H * T) ||
            al(&Y, (long)B * O * T) || al(&X0, (long)B * std::max(C, (long)O) * T) || al(&X1, (long)B * C * T) ||
            al(&X2, (long)B * C * T) || al(&dH, (long)B * H * T) || al(&dUh, (long)B * C * K2) ||
            al(&dVh, (long)B * C * K2) || al(&part, 4096) || al(&lossd, 4) || al(&phi, (long)B * (C + 7)) ||
            al(&Xb, (long)B * 9) || al(&Yb, (long)B * O * T) || al(&kws, kws_n) || al(&wb, (long)B * 4) ||
            hipMalloc(&idxd, B * sizeof(int)))
            return sfail(PSTD_ENOMEM, "surrogate workspace");
        bmax = B;
        return PSTD_OK;
    }
};

namespace {

// lift input channels: position, t / T, cos and sin per frequency, and with
// position modulation the 6 products per frequency
long n_lift(const sno_cfg& c) { return 4 + 2L * c.n_four + (c.pos_mod ? 6L * c.n_four : 0L); }

long layout(sno_cfg c, sno* s)
{
    const int O = 4 * c.n_rec;
    long o = 0;
    auto take = [&](long n) { long r = o; o += n; return r; };
    long P = take((long)c.C * n_lift(c)), pb = take(c.C);
    long W[16], b[16], Rr[16], Ri[16];
    for (int l = 0; l < c.L; ++l) {
        W[l] = take((long)c.C * c.C);
        b[l] = take(c.C);
        Rr[l] = take((long)c.K * c.C * c.C);
        Ri[l] = take((long)c.K * c.C * c.C);
    }
    const long FR = c.frames == 2 ? 2 : 1;
    long Q1 = take((long)c.H * c.C), q1b = take(c.H), Q2 = take(FR * 6L * O * c.H), q2b = take(FR * 6L * O);
    if (s) {
        s->off_P = P;
        s->off_pb = pb;
        for (int l = 0; l < c.L; ++l) {
            s->off_W[l] = W[l];
            s->off_b[l] = b[l];
            s->off_Rr[l] = Rr[l];
            s->off_Ri[l] = Ri[l];
        }
        s->off_Q1 = Q1;
        s->off_q1b = q1b;
        s->off_Q2 = Q2;
        s->off_q2b = q2b;
    }
    return o;
}

bool cfg_ok(const sno_cfg* c)
{
    if (!c || c->n_rec < 1 || c->T < 16 || c->T > 4096 || (c->T & (c->T - 1)) || c->C < 16 || c->C % 16 ||
        c->K < 1 || c->K > c->T / 2 || c->L < 1 || c->L > 16 || c->H < 16 || c->H % 16)
        return false;
    for (int i = 0; i < 9; ++i)
        if (!(c->feat_scale[i] != 0.0) || !std::isfinite(c->feat_off[i]) || !std::isfinite(c->feat_scale[i])) return false;
    for (int i = 3; i < 9; ++i)
        if (c->feat_off[i] != 0.0) return false;
    if (c->n_four < 0 || c->n_four > SNO_MAX_FOUR || (c->pos_mod != 0 && c->pos_mod != 1)) return false;
    for (int f = 0; f < c->n_four; ++f)
        if (!(c->four_cycles[f] > 0.0 && c->four_cycles[f] <= c->T / 2)) return false;
    if (c->frames != 1 && c->frames != 2) return false;
    if (c->frames == 2) {
        if (!c->rec_ijk || !c->slow_p || !c->slow_s || c->nz_slow < 1 || !(c->dt > 0) || !std::isfinite(c->dt))
            return false;
        for (int a = 0; a < 3; ++a)
            if (!(c->h[a] > 0) || !std::isfinite(c->h[a])) return false;
        for (int f = 0; f < 2; ++f)
            if (!std::isfinite(c->t_ref[f])) return false;
        for (int r = 0; r < c->n_rec; ++r)
            if (c->rec_ijk[3 * r + 2] < 0 || c->rec_ijk[3 * r + 2] >= c->nz_slow) return false;
        for (int k = 0; k < c->nz_slow; ++k)
            if (!(c->slow_p[k] >= 0) || !(c->slow_s[k] >= 0) || !std::isfinite(c->slow_p[k]) ||
                !std::isfinite(c->slow_s[k]))
                return false;
    }
    return true;
}

// forward of B samples whose raw features are X (device); leaves the caches in s
void forward(sno* s, hipStream_t st, const float* X, int B)
{
    const sno_cfg& c = s->cfg;
    const long C = c.C, T = c.T, K = c.K, K2 = 2 * K, H = c.H, O = s->O;
    const float* th = s->theta;
    const long NA = s->NA;
    hipLaunchKernelGGL(k_features, dim3(grid_for(B * NA * T)), dim3(256), 0, st, X, s->feat, B, (int)T, (int)NA, s->A);
    gemm(st, B, C, T, NA, 1, th + s->off_P, NA, 1, 0, 0, s->A, T, 1, NA * T, 0, s->V(0), T, 1, C * T, 1.f, 0.f,
         th + s->off_pb);
    for (int l = 0; l < c.L; ++l) {
        float* V = s->V(l);
        float* Vh = s->Vhl(l);
        float* Z = s->Zl(l);
        // truncated DFT along time
        gemm(st, B, C, K2, T, 1, V, T, 1, C * T, 0, s->Fb, K2, 1, 0, 0, Vh, K2, 1, C * K2);
        // complex mixing per mode: batch over modes, samples as columns
        const float* Rr = th + s->off_Rr[l];
        const float* Ri = th + s->off_Ri[l];
        if (mix_lds(C) <= MIX_LDS_MAX) {
            hipLaunchKernelGGL(k_cmix<false>, dim3((unsigned)K), dim3(256), mix_lds(C), st, Rr, Ri, Vh, B, (int)C,
                               (int)K, s->Uh);
        } else {
            gemm(st, K, C, B, C, 1, Rr, C, 1, C * C, 0, Vh, K2, C * K2, 1, 0, s->Uh, K2, C * K2, 1, 1.f, 0.f);
            gemm(st, K, C, B, C, 1, Ri, C, 1, C * C, 0, Vh + K, K2, C * K2, 1, 0, s->Uh, K2, C * K2, 1, -1.f, 1.f);
            gemm(st, K, C, B, C, 1, Ri, C, 1, C * C, 0, Vh, K2, C * K2, 1, 0, s->Uh + K, K2, C * K2, 1, 1.f, 0.f);
            gemm(st, K, C, B, C, 1, Rr, C, 1, C * C, 0, Vh + K, K2, C * K2, 1, 0, s->Uh + K, K2, C * K2, 1, 1.f, 1.f);
        }
        // Z = W V + b + inverse DFT of the mixed modes
        gemm(st, B, C, T, C, 1, th + s->off_W[l], C, 1, 0, 0, V, T, 1, C * T, 0, Z, T, 1, C * T, 1.f, 0.f,
             th + s->off_b[l]);
        gemm(st, B, C, T, K2, 1, s->Uh, K2, 1, C * K2, 0, s->G, T, 1, 0, 0, Z, T, 1, C * T, 1.f, 1.f);
        if (l < c.L - 1)
            hipLaunchKernelGGL(k_gelu, dim3(grid_for(B * C * T)), dim3(256), 0, st, Z, s->V(l + 1), (long)B * C * T);
    }
    gemm(st, B, H, T, C, 1, th + s->off_Q1, C, 1, 0, 0, s->V(c.L), T, 1, C * T, 0, s->Hp, T, 1, H * T, 1.f, 0.f,
         th + s->off_q1b);
    hipLaunchKernelGGL(k_gelu, dim3(grid_for(B * H * T)), dim3(256), 0, st, s->Hp, s->Hq, (long)B * H * T);
    // moment-weighted projection: one frame writes the output directly, two
    // frames go through the per-receiver delays
    const long FO = s->F * O;
    hipLaunchKernelGGL(k_qmix, rows_grid(H + 1, FO), dim3(256), 0, st, th + s->off_Q2, th + s->off_q2b, X, s->feat, B,
                       (int)FO, (int)O, (int)H, s->Qm, s->bm);
    float* Yf = s->F == 1 ? s->Y : s->Y6;
    gemm(st, B, FO, T, H, 1, s->Qm, H, 1, FO * H, 0, s->Hq, T, 1, H * T, 0, Yf, T, 1, FO * T, 1.f, 0.f, s->bm, FO);
    if (s->F == 2) {
        hipLaunchKernelGGL(k_shifts, dim3((unsigned)std::min<long>(((long)B * s->F * c.n_rec + 3) / 4, 4096)),
                           dim3(256), 0, st, X, s->rays, B,
                           s->shift);
        hipLaunchKernelGGL(k_fcomb, rows_grid(T, B * O), dim3(256), 0, st, s->Y6, s->shift, B, s->F, (int)O, c.n_rec,
                           (int)T, s->Y);
    }
}

// gradient of the mean squared error of s->Y against Yt (after the forward of
// the same features X)
void backward(sno* s, hipStream_t st, const float* X, const float* Yt, int B, const float* wgt = nullptr)
{
    const sno_cfg& c = s->cfg;
    const long C = c.C, T = c.T, K = c.K, K2 = 2 * K, H = c.H, O = s->O;
    const float* th = s->theta;
    float* g = s->grad;
    const long nY = (long)B * O * T;
    float* dY = s->X0;
    hipLaunchKernelGGL(k_mse, dim3(256), dim3(256), 0, st, s->Y, Yt, wgt, B, (int)O, (int)T, c.n_rec, dY, s->part);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, st, s->part, 256, s->lossd, 1.f / (float)nY);
    // frame delays (transposed), then the moment-weighted projection:
    // dQm[b] = dYf[b] Hq[b]^T, dbm[b] = row sums of dYf[b], dHq[b] = Qm[b]^T dYf[b],
    // and the 6 responses' gradients weighted back by the moment features
    const long FO = s->F * O;
    float* dYf = dY;
    if (s->F == 2) {
        dYf = s->dY6;
        hipLaunchKernelGGL(k_fspread, rows_grid(T, B * FO), dim3(256), 0, st, dY, s->shift, B, s->F, (int)O, c.n_rec,
                           (int)T, dYf);
    }
    gemm(st, B, FO, H, T, 1, dYf, T, 1, FO * T, 0, s->Hq, 1, T, H * T, 0, s->dQm, H, 1, FO * H);
    hipLaunchKernelGGL(k_rowsum, dim3(B * FO), dim3(256), 0, st, dYf, 1, (int)(B * FO), (int)T, s->dbm);
    hipLaunchKernelGGL(k_qgrad, rows_grid(H + 1, FO), dim3(256), 0, st, s->dQm, s->dbm, X, s->feat, B, (int)FO, (int)O,
                       (int)H, g + s->off_Q2, g + s->off_q2b);
    gemm(st, B, H, T, FO, 1, s->Qm, 1, H, FO * H, 0, dYf, T, 1, FO * T, 0, s->dH, T, 1, H * T);
    hipLaunchKernelGGL(k_gelu_bwd, dim3(grid_for(B * H * T)), dim3(256), 0, st, s->dH, s->Hp, s->dH, (long)B * H * T);
    gemm(st, 1, H, C, T, B, s->dH, T, 1, 0, H * T, s->V(c.L), 1, T, 0, C * T, g + s->off_Q1, C, 1, 0, 1.f, 0.f, nullptr, 0, s->kws, s->kws_n);
    hipLaunchKernelGGL(k_rowsum, dim3(H), dim3(256), 0, st, s->dH, B, (int)H, (int)T, g + s->off_q1b);
    float* bufs[3] = {s->X1, s->X2, s->X0};
    float* dV = bufs[0];
    gemm(st, B, C, T, H, 1, th + s->off_Q1, 1, C, 0, 0, s->dH, T, 1, H * T, 0, dV, T, 1, C * T);
    for (int l = c.L - 1; l >= 0; --l) {
        float* dZ = dV;
        float* other[2];
        int q = 0;
        for (float* b : bufs)
            if (b != dV) other[q++] = b;
        if (l < c.L - 1) {
            dZ = other[0];
            hipLaunchKernelGGL(k_gelu_bwd, dim3(grid_for(B * C * T)), dim3(256), 0, st, dV, s->Zl(l), dZ,
                               (long)B * C * T);
        }
        float* dVn = dZ == dV ? other[0] : other[1];
        float* V = s->V(l);
        float* Vh = s->Vhl(l);
        gemm(st, 1, C, C, T, B, dZ, T, 1, 0, C * T, V, 1, T, 0, C * T, g + s->off_W[l], C, 1, 0, 1.f, 0.f, nullptr, 0, s->kws, s->kws_n);
        hipLaunchKernelGGL(k_rowsum, dim3(C), dim3(256), 0, st, dZ, B, (int)C, (int)T, g + s->off_b[l]);
        // dUh = dZ G^T
        gemm(st, B, C, K2, T, 1, dZ, T, 1, C * T, 0, s->G, 1, T, 0, 0, s->dUh, K2, 1, C * K2);
        // spectral weights: dRr = dUr Vr^T + dUi Vi^T ; dRi = dUi Vr^T - dUr Vi^T  (per mode, summed over samples)
        // dVr = Rr^T dUr + Ri^T dUi ; dVi = -Ri^T dUr + Rr^T dUi
        const float* Rr = th + s->off_Rr[l];
        const float* Ri = th + s->off_Ri[l];
        if (mix_lds(C) <= MIX_LDS_MAX) {
            hipLaunchKernelGGL(k_cmix_dw, dim3((unsigned)K), dim3(256), (size_t)4 * MIX_B * C * sizeof(float), st,
                               s->dUh, Vh, B, (int)C, (int)K, g + s->off_Rr[l], g + s->off_Ri[l]);
            hipLaunchKernelGGL(k_cmix<true>, dim3((unsigned)K), dim3(256), mix_lds(C), st, Rr, Ri, s->dUh, B, (int)C,
                               (int)K, s->dVh);
        } else {
            gemm(st, K, C, C, B, 2, s->dUh, K2, C * K2, 1, K, Vh, C * K2, K2, 1, K, g + s->off_Rr[l], C, 1, C * C);
            gemm(st, K, C, C, B, 1, s->dUh + K, K2, C * K2, 1, 0, Vh, C * K2, K2, 1, 0, g + s->off_Ri[l], C, 1, C * C,
                 1.f, 0.f);
            gemm(st, K, C, C, B, 1, s->dUh, K2, C * K2, 1, 0, Vh + K, C * K2, K2, 1, 0, g + s->off_Ri[l], C, 1, C * C,
                 -1.f, 1.f);
            gemm(st, K, C, B, C, 1, Rr, 1, C, C * C, 0, s->dUh, K2, C * K2, 1, 0, s->dVh, K2, C * K2, 1, 1.f, 0.f);
            gemm(st, K, C, B, C, 1, Ri, 1, C, C * C, 0, s->dUh + K, K2, C * K2, 1, 0, s->dVh, K2, C * K2, 1, 1.f, 1.f);
            gemm(st, K, C, B, C, 1, Ri, 1, C, C * C, 0, s->dUh, K2, C * K2, 1, 0, s->dVh + K, K2, C * K2, 1, -1.f, 0.f);
            gemm(st, K, C, B, C, 1, Rr, 1, C, C * C, 0, s->dUh + K, K2, C * K2, 1, 0, s->dVh + K, K2, C * K2, 1, 1.f, 1.f);
        }
        // dV = W^T dZ + dVh F^T
        gemm(st, B, C, T, C, 1, th + s->off_W[l], 1, C, 0, 0, dZ, T, 1, C * T, 0, dVn, T, 1, C * T);
        gemm(st, B, C, T, K2, 1, s->dVh, K2, 1, C * K2, 0, s->Fb, 1, K2, 0, 0, dVn, T, 1, C * T, 1.f, 1.f);
        dV = dVn;
    }
    const long NA = s->NA;
    gemm(st, 1, C, NA, T, B, dV, T, 1, 0, C * T, s->A, 1, T, 0, NA * T, g + s->off_P, NA, 1, 0, 1.f, 0.f, nullptr, 0, s->kws, s->kws_n);
    hipLaunchKernelGGL(k_rowsum, dim3(C), dim3(256), 0, st, dV, B, (int)C, (int)T, g + s->off_pb);
}

// error head inputs of the last forward (features X): pooled last hidden
// layer and the moment features
void pool(sno* s, hipStream_t st, const float* X, int B)
{
    hipLaunchKernelGGL(k_pool, dim3(B * s->cfg.C), dim3(256), 0, st, s->V(s->cfg.L), X, s->feat, s->cfg.C, s->cfg.T,
                       s->phi);
}

}  // namespace

extern "C" {

long sno_n_params(const sno_cfg* cfg)
{
    if (!cfg_ok(cfg)) return -1;
    return layout(*cfg, nullptr);
}

int sno_create(const sno_cfg* cfg, const float* params, sno** out)
{
    if (!out || !params) return sfail(PSTD_EINVAL, "null argument");
    *out = nullptr;
    if (!cfg_ok(cfg)) return sfail(PSTD_EINVAL, "bad surrogate configuration");
    auto* s = new (std::nothrow) sno();
    if (!s) return sfail(PSTD_ENOMEM, "host allocation");
    s->cfg = *cfg;
    s->cfg.rec_ijk = nullptr;   // the host arrays are copied below, not kept
    s->cfg.slow_p = s->cfg.slow_s = nullptr;
    s->F = cfg->frames;
    s->O = 4 * cfg->n_rec;
    s->NA = n_lift(*cfg);
    s->np = layout(*cfg, s);
    s->feat.n_four = cfg->n_four;
    for (int f = 0; f < cfg->n_four; ++f) s->feat.cyc[f] = (float)cfg->four_cycles[f];
    (void)hipGetDevice(&s->device);
    for (int i = 0; i < 9; ++i) {
        s->feat.off[i] = (float)cfg->feat_off[i];
        s->feat.inv[i] = (float)(1.0 / cfg->feat_scale[i]);
    }
    const long np = s->np;
    const int T = cfg->T, K = cfg->K;
    // DFT bases (double, rounded once): F (T x 2K) = [cos | -sin], G (2K x T)
    std::vector<float> F((size_t)T * 2 * K), G((size_t)2 * K * T);
    for (int j = 0; j < T; ++j)
        for (int k = 0; k < K; ++k) {
            const double a = 2.0 * M_PI * (double)j * k / T;
            const double w = k == 0 ? 1.0 : 2.0;
            F[(size_t)j * 2 * K + k] = (float)std::cos(a);
            F[(size_t)j * 2 * K + K + k] = (float)(-std::sin(a));
            G[(size_t)k * T + j] = (float)(w * std::cos(a) / T);
            G[(size_t)(K + k) * T + j] = (float)(-w * std::sin(a) / T);
        }
    int rc = PSTD_OK;
    if (hipMalloc(&s->theta, np * 4) || hipMalloc(&s->grad, np * 4) || hipMalloc(&s->m1, np * 4) ||
        hipMalloc(&s->m2, np * 4) || hipMalloc(&s->Fb, F.size() * 4) || hipMalloc(&s->G, G.size() * 4) ||
        hipMalloc(&s->dscale, 16) || hipMalloc(&s->dhead, (cfg->C + 7) * 4))
        rc = sfail(PSTD_ENOMEM, "surrogate parameters");
    if (!rc && cfg->frames == 2) {
        // ray tables: receivers, per-frame slowness and its depth integral to
        // each cell centre, h_z (sum_{i<k} s_i + s_k / 2), summed in double
        const int nz = cfg->nz_slow;
        std::vector<double> cum(2 * (size_t)nz), slow(2 * (size_t)nz);
        for (int f = 0; f < 2; ++f) {
            const double* sl = f == 0 ? cfg->slow_p : cfg->slow_s;
            double acc = 0.0;
            for (int k = 0; k < nz; ++k) {
                slow[(size_t)f * nz + k] = sl[k];
                cum[(size_t)f * nz + k] = cfg->h[2] * (acc + 0.5 * sl[k]);
                acc += sl[k];
            }
        }
        if (hipMalloc(&s->drec, (size_t)cfg->n_rec * 3 * sizeof(int)) || hipMalloc(&s->dcum, cum.size() * 8) ||
            hipMalloc(&s->dslow, slow.size() * 8) ||
            hipMemcpy(s->drec, cfg->rec_ijk, (size_t)cfg->n_rec * 3 * sizeof(int), hipMemcpyHostToDevice) ||
            hipMemcpy(s->dcum, cum.data(), cum.size() * 8, hipMemcpyHostToDevice) ||
            hipMemcpy(s->dslow, slow.data(), slow.size() * 8, hipMemcpyHostToDevice))
            rc = sfail(PSTD_ENOMEM, "surrogate ray tables");
        s->rays = Rays{s->drec, s->dcum, s->dslow, {cfg->h[0], cfg->h[1], cfg->h[2]}, cfg->dt,
                       {cfg->t_ref[0], cfg->t_ref[1]}, nz, cfg->n_rec, 2};
    }
    if (!rc && (hipMemcpy(s->theta, params, np * 4, hipMemcpyHostToDevice) ||
                hipMemcpy(s->Fb, F.data(), F.size() * 4, hipMemcpyHostToDevice) ||
                hipMemcpy(s->G, G.data(), G.size() * 4, hipMemcpyHostToDevice) ||
                hipMemcpy(s->dscale, s->scale, 16, hipMemcpyHostToDevice) || hipMemset(s->m1, 0, np * 4) ||
                hipMemset(s->m2, 0, np * 4) || hipMemset(s->grad, 0, np * 4)))
        rc = sfail(PSTD_EDEVICE, "surrogate upload");
    // error head defaults to "always unsure" until trained: exp(30)
    s->head.assign(cfg->C + 7, 0.f);
    s->head[cfg->C + 6] = 30.f;
    if (!rc && hipMemcpy(s->dhead, s->head.data(), (cfg->C + 7) * 4, hipMemcpyHostToDevice))
        rc = sfail(PSTD_EDEVICE, "surrogate upload");
    if (rc) {
        delete s;
        return rc;
    }
    *out = s;
    return PSTD_OK;
}

void sno_destroy(sno* s)
{
    if (!s) return;
    (void)hipSetDevice(s->device);
    (void)hipDeviceSynchronize();
    delete s;
}

int sno_get_params(const sno* s, float* params)
{
    if (!s || !params) return sfail(PSTD_EINVAL, "null argument");
    S_TRY(hipDeviceSynchronize());
    S_TRY(hipMemcpy(params, s->theta, s->np * 4, hipMemcpyDeviceToHost));
    return PSTD_OK;
}

int sno_adam_step(sno* s, const float* grad, long step, double lr, void* hip_stream)
{
    if (!s || !grad || step < 1 || !(lr >= 0) || !std::isfinite(lr)) return sfail(PSTD_EINVAL, "bad arguments");
    hipStream_t st = (hipStream_t)hip_stream;
    const float c1 = (float)(1.0 - std::pow(0.9, (double)step));
    const float c2 = (float)(1.0 - std::pow(0.999, (double)step));
    hipLaunchKernelGGL(k_adam, dim3(grid_for(s->np)), dim3(256), 0, st, s->theta, grad, s->m1, s->m2, s->np, (float)lr,
                       0.9f, 0.999f, (float)(1.0 - 0.9), (float)(1.0 - 0.999), 1e-8f, c1, c2);
    S_TRY(hipGetLastError());
    S_TRY(hipStreamSynchronize(st));
    return PSTD_OK;
}

int sno_get_moments(const sno* s, float* m, float* v)
{
    if (!s || !m || !v) return sfail(PSTD_EINVAL, "null argument");
    S_TRY(hipDeviceSynchronize());
    S_TRY(hipMemcpy(m, s->m1, s->np * 4, hipMemcpyDeviceToHost));
    S_TRY(hipMemcpy(v, s->m2, s->np * 4, hipMemcpyDeviceToHost));
    return PSTD_OK;
}

int sno_get_scale(const sno* s, float* scale4)
{
    if (!s || !scale4) return sfail(PSTD_EINVAL, "null argument");
    std::memcpy(scale4, s->scale, 16);
    return PSTD_OK;
}

int sno_forward(sno* s, const float* X, int n, float* Y, void* hip_stream)
{
    if (!s || !X || !Y || n < 1) return sfail(PSTD_EINVAL, "bad arguments");
    hipStream_t st = (hipStream_t)hip_stream;
    const int bs = 32;
    int rc = s->ensure(std::min(n, bs));
    if (rc) return rc;
    const long per = (long)s->O * s->cfg.T;
    for (int b0 = 0; b0 < n; b0 += bs) {
        const int B = std::min(bs, n - b0);
        forward(s, st, X + (long)b0 * 9, B);
        S_TRY(hipMemcpyAsync(Y + (long)b0 * per, s->Y, B * per * 4, hipMemcpyDeviceToDevice, st));
    }
    S_TRY(hipGetLastError());
    S_TRY(hipStreamSynchronize(st));
    return PSTD_OK;
}

int sno_gradient_weighted(sno* s, const float* X, const float* Yt, const float* w, int n, float* grad, float* loss,
                          void* hip_stream)
{
    if (!s || !X || !Yt || !grad || n < 1) return sfail(PSTD_EINVAL, "bad arguments");
    hipStream_t st = (hipStream_t)hip_stream;
    int rc = s->ensure(n);
    if (rc) return rc;
    forward(s, st, X, n);
    backward(s, st, X, Yt, n, w);
    S_TRY(hipMemcpyAsync(grad, s->grad, s->np * 4, hipMemcpyDeviceToDevice, st));
    float l = 0.f;
    S_TRY(hipMemcpyAsync(&l, s->lossd, 4, hipMemcpyDeviceToHost, st));
    S_TRY(hipGetLastError());
    S_TRY(hipStreamSynchronize(st));
    if (loss) *loss = l;
    return PSTD_OK;
}

int sno_gradient(sno* s, const float* X, const float* Yt, int n, float* grad, float* loss, void* hip_stream)
{
    return sno_gradient_weighted(s, X, Yt, nullptr, n, grad, loss, hip_stream);
}

int sno_train(sno* s, const float* X, const float* Y, int n, const sno_train_cfg* tc, float* loss_curve,
              void* hip_stream)
{
    if (!s || !X || !Y || !tc || tc->epochs < 0 || tc->batch < 1 || !(tc->lr > 0) || tc->n_calib < 0)
        return sfail(PSTD_EINVAL, "bad arguments");
    const int n_fit = n - tc->n_calib;
    if (n_fit < 1) return sfail(PSTD_EINVAL, "no training samples left after the calibration split");
    hipStream_t st = (hipStream_t)hip_stream;
    const sno_cfg& c = s->cfg;
    const int B = std::min(tc->batch, n_fit);
    int rc = s->ensure(std::max(B, 32));
    if (rc) return rc;
    // output normalisation: per-component RMS over the fitting samples
    double* ss = nullptr;
    S_TRY(hipMalloc(&ss, 4 * SQ_BLOCKS * sizeof(double)));
    hipLaunchKernelGGL(k_comp_sumsq, dim3(4, SQ_BLOCKS), dim3(256), 0, st, Y, n_fit, c.n_rec, c.T, ss);
    std::vector<double> hss(4 * SQ_BLOCKS);
    S_TRY(hipMemcpyAsync(hss.data(), ss, hss.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    S_TRY(hipStreamSynchronize(st));
    (void)hipFree(ss);
    for (int k = 0; k < 4; ++k) {
        double sk = 0.0;
        for (int j = 0; j < SQ_BLOCKS; ++j) sk += hss[k * SQ_BLOCKS + j];
        const double rms = std::sqrt(sk / ((double)n_fit * c.n_rec * c.T));
        s->scale[k] = rms > 0 ? (float)rms : 1.f;
    }
    S_TRY(hipMemcpyAsync(s->dscale, s->scale, 16, hipMemcpyHostToDevice, st));
    // relative loss: per-(sample, component) weights of the fitting samples
    float* wfit = nullptr;
    if (tc->rel_loss) {
        S_TRY(hipMalloc(&wfit, (size_t)n_fit * 4 * sizeof(float)));
        hipLaunchKernelGGL(k_relw, dim3(n_fit, 4), dim3(256), 0, st, Y, c.n_rec, c.T, s->dscale, wfit);
    }
    struct FreeW {
        float* p;
        ~FreeW() { (void)hipFree(p); }
    } free_w{wfit};
    // Adam with cosine learning-rate decay
    std::mt19937_64 rng(tc->seed);
    std::vector<int> order(n_fit);
    for (int i = 0; i < n_fit; ++i) order[i] = i;
    const int steps_per_epoch = n_fit / B;
    const long total = (long)steps_per_epoch * tc->epochs;
    long step = 0;
    S_TRY(hipMemsetAsync(s->m1, 0, s->np * 4, st));
    S_TRY(hipMemsetAsync(s->m2, 0, s->np * 4, st));
    std::vector<float> lbuf(steps_per_epoch);
    for (int ep = 0; ep < tc->epochs; ++ep) {
        std::shuffle(order.begin(), order.end(), rng);
        double lsum = 0.0;
        for (int it = 0; it < steps_per_epoch; ++it) {
            S_TRY(hipMemcpyAsync(s->idxd, order.data() + (long)it * B, B * sizeof(int), hipMemcpyHostToDevice, st));
            hipLaunchKernelGGL(k_gather, dim3(grid_for((long)B * s->O * c.T)), dim3(256), 0, st, X, Y, s->idxd, B,
                               s->O, c.T, c.n_rec, s->dscale, s->Xb, s->Yb);
            if (wfit)
                hipLaunchKernelGGL(k_gather_w, dim3((B * 4 + 255) / 256), dim3(256), 0, st, wfit, s->idxd, B, s->wb);
            forward(s, st, s->Xb, B);
            backward(s, st, s->Xb, s->Yb, B, wfit ? s->wb : nullptr);
            ++step;
            const double lr = tc->lr * 0.5 * (1.0 + std::cos(M_PI * (double)(step - 1) / (double)std::max(1L, total)));
            const float c1 = (float)(1.0 - std::pow(0.9, (double)step));
            const float c2 = (float)(1.0 - std::pow(0.999, (double)step));
            hipLaunchKernelGGL(k_adam, dim3(grid_for(s->np)), dim3(256), 0, st, s->theta, s->grad, s->m1, s->m2, s->np,
                               (float)lr, 0.9f, 0.999f, (float)(1.0 - 0.9), (float)(1.0 - 0.999), 1e-8f, c1, c2);
            S_TRY(hipMemcpyAsync(&lbuf[it], s->lossd, 4, hipMemcpyDeviceToHost, st));
        }
        S_TRY(hipGetLastError());
        S_TRY(hipStreamSynchronize(st));
        for (float v : lbuf) lsum += v;
        if (loss_curve) loss_curve[ep] = (float)(lsum / std::max(1, steps_per_epoch));
        if (!std::isfinite(lsum)) return sfail(PSTD_EUNSTABLE, "training diverged");
        if (tc->on_epoch) tc->on_epoch(ep, (float)(lsum / std::max(1, steps_per_epoch)), tc->user);
    }
    // error head: least squares of log(relative error) on the pooled last
    // hidden layer of the calibration samples, plus a one-sided 95 % margin
    const int D = c.C + 7;
    std::vector<float> phis, errs;
    if (tc->n_calib > 1) {
        float* err = nullptr;
        float* Yp = nullptr;
        const long per = (long)s->O * c.T;
        const int bs = std::min(32, s->bmax);
        S_TRY(hipMalloc(&err, tc->n_calib * 4));
        S_TRY(hipMalloc(&Yp, (long)bs * per * 4));
        phis.resize((size_t)tc->n_calib * D);
        errs.resize(tc->n_calib);
        for (int b0 = 0; b0 < tc->n_calib; b0 += bs) {
            const int nb = std::min(bs, tc->n_calib - b0);
            const int i0 = n_fit + b0;
            forward(s, st, X + (long)i0 * 9, nb);
            S_TRY(hipMemcpyAsync(Yp, s->Y, nb * per * 4, hipMemcpyDeviceToDevice, st));
            hipLaunchKernelGGL(k_scale_out, dim3(grid_for(nb * per)), dim3(256), 0, st, Yp, nb * per, s->O, c.T,
                               c.n_rec, s->dscale);
            hipLaunchKernelGGL(k_relerr, dim3(nb), dim3(256), 0, st, Yp, Y + (long)i0 * per, c.n_rec, c.T, err + b0);
            pool(s, st, X + (long)i0 * 9, nb);
            S_TRY(hipMemcpyAsync(phis.data() + (size_t)b0 * D, s->phi, (size_t)nb * D * 4, hipMemcpyDeviceToHost, st));
        }
        S_TRY(hipMemcpyAsync(errs.data(), err, tc->n_calib * 4, hipMemcpyDeviceToHost, st));
        S_TRY(hipGetLastError());
        S_TRY(hipStreamSynchronize(st));
        (void)hipFree(err);
        (void)hipFree(Yp);
        // normal equations (Phi^T Phi + ridge) h = Phi^T log e, Cholesky
        std::vector<double> Ag((size_t)D * D, 0.0), r(D, 0.0);
        for (int i = 0; i < tc->n_calib; ++i) {
            const double le = std::log(std::max(1e-6, (double)errs[i]));
            for (int a = 0; a < D; ++a) {
                r[a] += phis[(size_t)i * D + a] * le;
                for (int bb = 0; bb < D; ++bb) Ag[(size_t)a * D + bb] += (double)phis[(size_t)i * D + a] * phis[(size_t)i * D + bb];
            }
        }
        for (int a = 0; a < D; ++a) Ag[(size_t)a * D + a] += 1e-3 * tc->n_calib;
        std::vector<double> Lc((size_t)D * D, 0.0);
        bool ok = true;
        for (int i = 0; i < D && ok; ++i)
            for (int j = 0; j <= i; ++j) {
                double v = Ag[(size_t)i * D + j];
                for (int k = 0; k < j; ++k) v -= Lc[(size_t)i * D + k] * Lc[(size_t)j * D + k];
                if (i == j) {
                    if (v <= 0) { ok = false; break; }
                    Lc[(size_t)i * D + i] = std::sqrt(v);
                } else {
                    Lc[(size_t)i * D + j] = v / Lc[(size_t)j * D + j];
                }
            }
        if (ok) {
            std::vector<double> yv(D), h(D);
            for (int i = 0; i < D; ++i) {
                double v = r[i];
                for (int k = 0; k < i; ++k) v -= Lc[(size_t)i * D + k] * yv[k];
                yv[i] = v / Lc[(size_t)i * D + i];
            }
            for (int i = D - 1; i >= 0; --i) {
                double v = yv[i];
                for (int k = i + 1; k < D; ++k) v -= Lc[(size_t)k * D + i] * h[k];
                h[i] = v / Lc[(size_t)i * D + i];
            }
            double res = 0.0;
            for (int i = 0; i < tc->n_calib; ++i) {
                double pr = 0.0;
                for (int a = 0; a < D; ++a) pr += h[a] * phis[(size_t)i * D + a];
                const double d = std::log(std::max(1e-6, (double)errs[i])) - pr;
                res += d * d;
            }
            const double sd = std::sqrt(res / std::max(1, tc->n_calib - 1));
            for (int a = 0; a < D; ++a) s->head[a] = (float)h[a];
            s->head_margin = (float)(1.645 * sd);
            S_TRY(hipMemcpy(s->dhead, s->head.data(), D * 4, hipMemcpyHostToDevice));
        }
    }
    return PSTD_OK;
}

int sno_predict(sno* s, const float* X, int n, float* Y, float* est_err, void* hip_stream)
{
    if (!s || !X || !Y || n < 0) return sfail(PSTD_EINVAL, "bad arguments");
    hipStream_t st = (hipStream_t)hip_stream;
    const sno_cfg& c = s->cfg;
    const int bs = 32;
    int rc = s->ensure(bs);
    if (rc) return rc;
    const long per = (long)s->O * c.T;
    for (int b0 = 0; b0 < n; b0 += bs) {
        const int B = std::min(bs, n - b0);
        forward(s, st, X + (long)b0 * 9, B);
        S_TRY(hipMemcpyAsync(Y + (long)b0 * per, s->Y, B * per * 4, hipMemcpyDeviceToDevice, st));
        hipLaunchKernelGGL(k_scale_out, dim3(grid_for(B * per)), dim3(256), 0, st, Y + (long)b0 * per, B * per, s->O,
                           c.T, c.n_rec, s->dscale);
        if (est_err) {
            pool(s, st, X + (long)b0 * 9, B);
            hipLaunchKernelGGL(k_head, dim3((B + 63) / 64), dim3(64), 0, st, s->phi, s->dhead, c.C + 7, B,
                               s->head_margin, est_err + b0);
        }
    }
    S_TRY(hipGetLastError());
    return PSTD_OK;
}

int sno_decimate(const float* in, int n, int n_rec, int nt, int decim, float* out, void* hip_stream)
{
    if (!in || !out || n < 0 || n_rec < 0 || nt < 1 || decim < 1) return sfail(PSTD_EINVAL, "bad arguments");
    const long rows = (long)n * 4 * n_rec;
    const long total = rows * (nt / decim);
    if (total == 0) return PSTD_OK;
    hipLaunchKernelGGL(k_decim, dim3(grid_for(total)), dim3(256), 0, (hipStream_t)hip_stream, in, rows, nt, decim, out);
    S_TRY(hipGetLastError());
    return PSTD_OK;
}

int sno_predict_or_solve(sno* s, pstd3d_ctx* solver, const float* X, const int32_t* src_ijk, const double* m6,
                         const double* wavelet, int nt_w, int decim, int n, double tol, int max_batch, float* Y,
                         float* est_err, int* used, void* hip_stream)
{
    if (!s || !solver || !X || !src_ijk || !m6 || !wavelet || !Y || !est_err || n < 0 || decim < 1 ||
        max_batch < 1 || nt_w < 1)
        return sfail(PSTD_EINVAL, "bad arguments");
    // the solver writes n_shots x 4 x (its receivers) x nt floats into a
    // buffer sized for the surrogate's receivers: they must be the same
    if (pstd3d_n_rec(solver) != s->cfg.n_rec)
        return sfail(PSTD_EINVAL, "the solver's receiver count differs from the surrogate's n_rec");
    hipStream_t st = (hipStream_t)hip_stream;
    int rc = sno_predict(s, X, n, Y, est_err, hip_stream);
    if (rc) return rc;
    std::vector<float> est(n);
    S_TRY(hipMemcpyAsync(est.data(), est_err, (size_t)n * 4, hipMemcpyDeviceToHost, st));
    S_TRY(hipStreamSynchronize(st));
    std::vector<int> redo;
    for (int i = 0; i < n; ++i) {
        const bool r = !(est[i] <= tol);
        if (used) used[i] = r ? 1 : 0;
        if (r) redo.push_back(i);
    }
    if (redo.empty()) return PSTD_OK;
    const int T = s->cfg.T, nrec = s->cfg.n_rec;
    const int nt = decim * T;
    const long per = 4L * nrec * T;
    float *tr = nullptr, *dec = nullptr;
    const int mb = std::min<int>(max_batch, (int)redo.size());
    S_TRY(hipMalloc(&tr, (size_t)mb * 4 * nrec * nt * 4));
    S_TRY(hipMalloc(&dec, (size_t)mb * per * 4));
    for (size_t b0 = 0; b0 < redo.size(); b0 += mb) {
        const int nb = (int)std::min<size_t>(mb, redo.size() - b0);
        std::vector<int32_t> ofs(nb + 1), ijk(3 * nb);
        std::vector<double> mm(6 * nb), wv((size_t)nb * nt_w);
        for (int q = 0; q < nb; ++q) {
            const int i = redo[b0 + q];
            ofs[q] = q;
            for (int a = 0; a < 3; ++a) ijk[3 * q + a] = src_ijk[3 * i + a];
            for (int a = 0; a < 6; ++a) mm[6 * q + a] = m6[6 * i + a];
            std::memcpy(&wv[(size_t)q * nt_w], wavelet, sizeof(double) * nt_w);
        }
        ofs[nb] = nb;
        rc = pstd3d_set_sources(solver, nb, ofs.data(), ijk.data(), mm.data(), wv.data(), nt_w);
        if (!rc) rc = pstd3d_run(solver, nt, tr, hip_stream);
        if (!rc) rc = sno_decimate(tr, nb, nrec, nt, decim, dec, hip_stream);
        for (int q = 0; q < nb && !rc; ++q) {
            const int i = redo[b0 + q];
            if (hipMemcpyAsync(Y + (long)i * per, dec + (long)q * per, per * 4, hipMemcpyDeviceToDevice, st) !=
                hipSuccess)
                rc = sfail(PSTD_EDEVICE, "copy of solver traces");
        }
        if (rc) break;
    }
    (void)hipStreamSynchronize(st);
    (void)hipFree(tr);
    (void)hipFree(dec);
    return rc;
}

const char* sno_last_error(void) { return g_serr.c_str(); }

}  // extern "C"
