// Device kernels of one leapfrog step of the pseudo-spectral elastic solver.
//
// One step (Sec. II-A: FFT-based spatial derivatives, staggered leapfrog):
//   V phase: 6 summed stresses --x FFT (fused in the previous S kernel)-->
//            y FFT --> z FFT * operator * inverse z FFT (9 derivatives) -->
//            inverse y FFT --> [inverse x FFT + velocity update + receivers +
//            x FFT of the 3 summed velocities]
//   S phase: y FFT --> z operator --> inverse y FFT --> [inverse x FFT +
//            stress update + source injection + receivers + x FFT of the 6
//            summed stresses]
// Real fields are [nz][ny][nx]; x-transformed spectra are [nz][ny][ldx]
// complex with kx = 0 .. nx/2 (ldx >= nx/2 + 1, padded to 128-byte rows).
#pragma once
#include "fft_lds.hpp"

namespace pstd {

struct Geo {
    int nx, ny, nz, nxh, ldx, nrows;   // nrows = ny * nz
    long n;                            // cells
    long nspec;                        // complex values per spectrum
    long fstride;                      // floats per shot of split fields (24 n)
    long sstride;                      // complex values per shot of spectra (18 nspec)
};

// material coefficients pre-multiplied by dt (FP64 on the host, stored FP32)
struct Mat {
    const float* dtr[3];   // dt / rho at the vx, vy, vz nodes
    const float* dlam;     // dt * lambda at centres
    const float* dmu2;     // 2 dt * mu at centres
    const float* dmus[3];  // dt * mu at xy, xz, yz shear nodes
};

// PML factors a = exp(-alpha dt / 2) per axis, at integer and half nodes
struct Pml {
    const float* ai[3];
    const float* ah[3];
};

struct Rec {
    const int* ptr;     // [nrows + 1] receivers sorted by row
    const int4* ent;    // {x, row, id, 0}
    int n_rec;
};

struct Inj {
    const int* ptr;     // [n_shots][nrows + 1]
    const int4* ent;    // {x, split field 0..14, coef (float bits), wavelet row}
    const float* wav;   // [n_src_total][nt_w]
    int nt_w;
};

// Outputs of the z kernel: each input spectrum feeds up to three derivatives.
struct PhaseDesc {
    int nin;
    int nout[6];
    int oidx[6][3];
    int axis[6][3];
    int plus[6][3];     // 1: D+, 0: D-
};

struct Ops {
    const float2* sym[3][2];   // per axis, [0] = D-, [1] = D+ : i k exp(-+ i k h/2)
    const float* kap;          // kappa(|k|) / (nx ny nz), [nz][ny][ldx]
};

// device-resident descriptor of the two derivative phases (read with uniform
// loads; kept out of the kernel arguments so runtime indexing stays in memory)
struct ZDesc {
    PhaseDesc ph[2];   // [0] V phase, [1] S phase
    Ops ops;
};

constexpr int rows_for(int nx) { return nx <= 32 ? 16 : nx <= 64 ? 8 : nx <= 160 ? 4 : 2; }
constexpr int tile_for(int n) { return n >= 384 ? 8 : 16; }

// value of real pencil p (= field * ROWS + local row) of a staged spectrum row
__device__ __forceinline__ float2 spec_at(const float2* __restrict__ base, const Geo& g, int rows,
                                          int row0, int p, int k)
{
    const int f = p / rows, r = p - f * rows;
    const int row = row0 + r;
    if (row >= g.nrows) return make_float2(0.f, 0.f);
    return base[f * g.nspec + (long)row * g.ldx + k];
}

// Stage NPI complex pencils, each the Hermitian extension of two half spectra
// (real pencils 2q and 2q+1), so one complex inverse FFT gives both real rows.
template <int NX, int ROWS, int NT, int NPI, int PS>
__device__ __forceinline__ void stage_c2r(float2* s, const float2* __restrict__ src, const Geo& g, int row0)
{
    constexpr int NXH = NX / 2 + 1;
    for (int e = threadIdx.x; e < NPI * NXH; e += NT) {
        const int q = e / NXH, k = e - q * NXH;
        float2 a = spec_at(src, g, ROWS, row0, 2 * q, k);
        float2 b = spec_at(src, g, ROWS, row0, 2 * q + 1, k);
        if (k == 0 || 2 * k == NX) {
            s[q * PS + k] = make_float2(a.x, b.x);
        } else {
            s[q * PS + k] = make_float2(a.x - b.y, a.y + b.x);
            s[q * PS + NX - k] = make_float2(a.x + b.y, b.x - a.y);
        }
    }
}

// Unpack NPO complex forward transforms of paired real rows into half spectra.
template <int NX, int ROWS, int NT, int NPO, int PS>
__device__ __forceinline__ void unstage_r2c(const float2* s, float2* __restrict__ dst, const Geo& g, int row0)
{
    constexpr int NXH = NX / 2 + 1;
    for (int e = threadIdx.x; e < NPO * NXH; e += NT) {
        const int q = e / NXH, k = e - q * NXH;
        const float2 z = s[q * PS + k];
        const float2 zm = s[q * PS + (k == 0 ? 0 : NX - k)];
        const float2 A = make_float2(0.5f * (z.x + zm.x), 0.5f * (z.y - zm.y));
        const float2 B = make_float2(0.5f * (z.y + zm.y), -0.5f * (z.x - zm.x));
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int p = 2 * q + h;
            const int f = p / ROWS, r = p - f * ROWS;
            const int row = row0 + r;
            if (row < g.nrows) dst[f * g.nspec + (long)row * g.ldx + k] = h ? B : A;
        }
    }
}

// real value of pencil p at x (pairs stored as re / im of one complex pencil)
template <int PS>
__device__ __forceinline__ float pencil_val(const float2* s, int p, int x)
{
    const float2 v = s[(p >> 1) * PS + x];
    return (p & 1) ? v.y : v.x;
}

template <int PS>
__device__ __forceinline__ void pencil_set(float2* s, int p, int x, float v)
{
    float* f = reinterpret_cast<float*>(s + (p >> 1) * PS + x);
    f[p & 1] = v;
}

// ---------------------------------------------------------------------------
// V phase tail: inverse x FFT of the 9 stress derivatives, velocity split-PML
// update (eq. 2 second line), receivers vx vy vz, x FFT of the summed v.
template <int NX, int NT>
__global__ __launch_bounds__(NT) void k_vel(Geo g, Mat m, Pml pm, const float2* __restrict__ twx,
                                            float* __restrict__ fields, float2* __restrict__ spec,
                                            Rec rc, float* __restrict__ traces,
                                            const int* __restrict__ stepp, int n0, int ldt)
{
    constexpr int ROWS = rows_for(NX);
    constexpr int PS = NX + 1;
    constexpr int NPI = 9 * ROWS / 2;
    constexpr int NPO = 3 * ROWS / 2;
    constexpr int CPT = (ROWS * NX + NT - 1) / NT;
    __shared__ float2 s[NPI * PS];

    const int shot = blockIdx.y;
    const int row0 = blockIdx.x * ROWS;
    float* __restrict__ F = fields + (long)shot * g.fstride;
    const float2* __restrict__ D9 = spec + (long)shot * g.sstride + 9 * g.nspec;
    float2* __restrict__ S3 = spec + (long)shot * g.sstride + 6 * g.nspec;

    stage_c2r<NX, ROWS, NT, NPI, PS>(s, D9, g, row0);
    __syncthreads();
    lds_fft<NX, NPI, NT, +1, PS, 1, false>(s, twx);

    float vsum[CPT][3];
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
        const int c = threadIdx.x + i * NT;
        vsum[i][0] = vsum[i][1] = vsum[i][2] = 0.f;
        if (c >= ROWS * NX) continue;
        const int r = c / NX, x = c - r * NX;
        const int row = row0 + r;
        if (row >= g.nrows) continue;
        const int y = row % g.ny, z = row / g.ny;
        const long cell = (long)row * NX + x;
        const float axi = pm.ai[0][x], axh = pm.ah[0][x];
        const float ayi = pm.ai[1][y], ayh = pm.ah[1][y];
        const float azi = pm.ai[2][z], azh = pm.ah[2][z];
        // a_d for component c along axis d: half node when c == d
        const float a[3][3] = {{axh, ayi, azi}, {axi, ayh, azi}, {axi, ayi, azh}};
#pragma unroll
        for (int comp = 0; comp < 3; ++comp) {
            const float dtr = m.dtr[comp][cell];
            float acc = 0.f;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const int p = (3 * comp + d) * ROWS + r;
                const float dv = pencil_val<PS>(s, p, x);
                float* f = F + (long)(3 * comp + d) * g.n + cell;
                const float ad = a[comp][d];
                const float v = ad * (ad * (*f) + dtr * dv);
                *f = v;
                acc += v;
            }
            vsum[i][comp] = acc;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
        const int c = threadIdx.x + i * NT;
        if (c >= ROWS * NX) continue;
        const int r = c / NX, x = c - r * NX;
#pragma unroll
        for (int comp = 0; comp < 3; ++comp) pencil_set<PS>(s, comp * ROWS + r, x, vsum[i][comp]);
    }
    __syncthreads();
    // receivers (vx, vy, vz at their staggered nodes, time (n + 1/2) dt)
    {
        const int rend = min(row0 + ROWS, g.nrows);
        const int e0 = rc.ptr[row0], e1 = rc.ptr[rend];
        const int tn = *stepp - n0;
        for (int e = e0 + threadIdx.x; e < e1; e += NT) {
            const int4 q = rc.ent[e];
            const int r = q.y - row0;
#pragma unroll
            for (int comp = 0; comp < 3; ++comp)
                traces[(((long)shot * 4 + 1 + comp) * rc.n_rec + q.z) * ldt + tn] =
                    pencil_val<PS>(s, comp * ROWS + r, q.x);
        }
    }
    lds_fft<NX, NPO, NT, -1, PS, 1, false>(s, twx);
    unstage_r2c<NX, ROWS, NT, NPO, PS>(s, S3, g, row0);
}

// ---------------------------------------------------------------------------
// S phase tail: inverse x FFT of the 9 velocity derivatives, stress split-PML
// update (eq. 2 first line), source injection, receiver p (eq. 3), x FFT of
// the 6 summed stresses.
template <int NX, int NT>
__global__ __launch_bounds__(NT) void k_str(Geo g, Mat m, Pml pm, const float2* __restrict__ twx,
                                            float* __restrict__ fields, float2* __restrict__ spec,
                                            Rec rc, Inj inj, float* __restrict__ traces,
                                            const int* __restrict__ stepp, int n0, int ldt)
{
    constexpr int ROWS = rows_for(NX);
    constexpr int PS = NX + 1;
    constexpr int NPI = 9 * ROWS / 2;
    constexpr int NPO = 6 * ROWS / 2;
    constexpr int CPT = (ROWS * NX + NT - 1) / NT;
    __shared__ float2 s[NPI * PS];

    const int shot = blockIdx.y;
    const int row0 = blockIdx.x * ROWS;
    float* __restrict__ F = fields + (long)shot * g.fstride + 9 * g.n;   // 15 stress parts
    const float2* __restrict__ D9 = spec + (long)shot * g.sstride + 9 * g.nspec;
    float2* __restrict__ S6 = spec + (long)shot * g.sstride;
    const int step = *stepp;
    const int* __restrict__ iptr = inj.ptr + (long)shot * (g.nrows + 1);

    stage_c2r<NX, ROWS, NT, NPI, PS>(s, D9, g, row0);
    __syncthreads();
    lds_fft<NX, NPI, NT, +1, PS, 1, false>(s, twx);

    float ssum[CPT][6];
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
        const int c = threadIdx.x + i * NT;
#pragma unroll
        for (int q = 0; q < 6; ++q) ssum[i][q] = 0.f;
        if (c >= ROWS * NX) continue;
        const int r = c / NX, x = c - r * NX;
        const int row = row0 + r;
        if (row >= g.nrows) continue;
        const int y = row % g.ny, z = row / g.ny;
        const long cell = (long)row * NX + x;
        const float ai[3] = {pm.ai[0][x], pm.ai[1][y], pm.ai[2][z]};
        const float ah[3] = {pm.ah[0][x], pm.ah[1][y], pm.ah[2][z]};
        // derivatives: e0..e2 = D_d^- v_d, e3 = Dy+ vx, e4 = Dx+ vy, e5 = Dz+ vx,
        //              e6 = Dx+ vz, e7 = Dz+ vy, e8 = Dy+ vz
        float e[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) e[q] = pencil_val<PS>(s, q * ROWS + r, x);
        const float dlam = m.dlam[cell], dmu2 = m.dmu2[cell];
        float sp[15];
#pragma unroll
        for (int q = 0; q < 15; ++q) sp[q] = F[(long)q * g.n + cell];
        // normal parts sp[3c + d] (component c, axis d)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc)
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const float coef = cc == d ? dlam + dmu2 : dlam;
                sp[3 * cc + d] = ai[d] * (ai[d] * sp[3 * cc + d] + coef * e[d]);
            }
        // shear parts: 9 sxy(x) <- Dx+ vy, 10 sxy(y) <- Dy+ vx, 11 sxz(x) <- Dx+ vz,
        //              12 sxz(z) <- Dz+ vx, 13 syz(y) <- Dy+ vz, 14 syz(z) <- Dz+ vy
        const float mxy = m.dmus[0][cell], mxz = m.dmus[1][cell], myz = m.dmus[2][cell];
        sp[9] = ah[0] * (ah[0] * sp[9] + mxy * e[4]);
        sp[10] = ah[1] * (ah[1] * sp[10] + mxy * e[3]);
        sp[11] = ah[0] * (ah[0] * sp[11] + mxz * e[6]);
        sp[12] = ah[2] * (ah[2] * sp[12] + mxz * e[5]);
        sp[13] = ah[1] * (ah[1] * sp[13] + myz * e[8]);
        sp[14] = ah[2] * (ah[2] * sp[14] + myz * e[7]);
        // point sources of this shot in this row
        const int j0 = iptr[row], j1 = iptr[row + 1];
        if (j0 != j1 && step < inj.nt_w) {
            for (int j = j0; j < j1; ++j) {
                const int4 q = inj.ent[j];
                if (q.x != x) continue;
                const float val = __int_as_float(q.z) * inj.wav[(long)q.w * inj.nt_w + step];
#pragma unroll
                for (int f = 0; f < 15; ++f)
                    if (q.y == f) sp[f] += val;
            }
        }
#pragma unroll
        for (int q = 0; q < 15; ++q) F[(long)q * g.n + cell] = sp[q];
        ssum[i][0] = sp[0] + sp[1] + sp[2];
        ssum[i][1] = sp[3] + sp[4] + sp[5];
        ssum[i][2] = sp[6] + sp[7] + sp[8];
        ssum[i][3] = sp[9] + sp[10];
        ssum[i][4] = sp[11] + sp[12];
        ssum[i][5] = sp[13] + sp[14];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
        const int c = threadIdx.x + i * NT;
        if (c >= ROWS * NX) continue;
        const int r = c / NX, x = c - r * NX;
#pragma unroll
        for (int q = 0; q < 6; ++q) pencil_set<PS>(s, q * ROWS + r, x, ssum[i][q]);
    }
    __syncthreads();
    {
        const int rend = min(row0 + ROWS, g.nrows);
        const int e0 = rc.ptr[row0], e1 = rc.ptr[rend];
        const int tn = step - n0;
        for (int e = e0 + threadIdx.x; e < e1; e += NT) {
            const int4 q = rc.ent[e];
            const int r = q.y - row0;
            const float tr = pencil_val<PS>(s, 0 * ROWS + r, q.x) + pencil_val<PS>(s, 1 * ROWS + r, q.x) +
                             pencil_val<PS>(s, 2 * ROWS + r, q.x);
            traces[((long)shot * 4 * rc.n_rec + q.z) * ldt + tn] = -tr * (1.0f / 3.0f);
        }
    }
    lds_fft<NX, NPO, NT, -1, PS, 1, false>(s, twx);
    unstage_r2c<NX, ROWS, NT, NPO, PS>(s, S6, g, row0);
}

// ---------------------------------------------------------------------------
// x FFT of sums of consecutive split parts: output f = sum of `cnt[f]` real
// fields starting at in + first[f] * n.  Used to rebuild the stress spectra
// after a state restore and by the derivative test entry.
struct SumDesc {
    int nf;
    int first[9];
    int cnt[9];
};

template <int NX, int NT>
__global__ __launch_bounds__(NT) void k_xfwd(Geo g, const float2* __restrict__ twx, const float* __restrict__ in,
                                             long in_shot_stride, float2* __restrict__ out,
                                             long out_shot_stride, SumDesc sd)
{
    constexpr int ROWS = rows_for(NX);
    constexpr int PS = NX + 1;
    constexpr int NPMAX = 9 * ROWS / 2;
    __shared__ float2 s[NPMAX * PS];
    const int shot = blockIdx.y;
    const int row0 = blockIdx.x * ROWS;
    const float* __restrict__ I = in + (long)shot * in_shot_stride;
    float2* __restrict__ O = out + (long)shot * out_shot_stride;
    const int np = sd.nf * ROWS;
    for (int e = threadIdx.x; e < ((np + 1) / 2) * 2 * NX; e += NT) {
        const int p = e / NX, x = e - p * NX;
        float v = 0.f;
        if (p < np) {
            const int f = p / ROWS, r = p - f * ROWS;
            const int row = row0 + r;
            if (row < g.nrows)
                for (int q = 0; q < sd.cnt[f]; ++q) v += I[(long)(sd.first[f] + q) * g.n + (long)row * NX + x];
        }
        pencil_set<PS>(s, p, x, v);
    }
    __syncthreads();
    // np is a multiple of ROWS (even): np / 2 complex pencils
    if (sd.nf == 3) {
        lds_fft<NX, 3 * ROWS / 2, NT, -1, PS, 1, false>(s, twx);
        unstage_r2c<NX, ROWS, NT, 3 * ROWS / 2, PS>(s, O, g, row0);
    } else {
        lds_fft<NX, 6 * ROWS / 2, NT, -1, PS, 1, false>(s, twx);
        unstage_r2c<NX, ROWS, NT, 6 * ROWS / 2, PS>(s, O, g, row0);
    }
}

// inverse x FFT of 9 spectra to 9 real fields (test entry)
template <int NX, int NT>
__global__ __launch_bounds__(NT) void k_xinv(Geo g, const float2* __restrict__ twx, const float2* __restrict__ in,
                                             float* __restrict__ out)
{
    constexpr int ROWS = rows_for(NX);
    constexpr int PS = NX + 1;
    constexpr int NPI = 9 * ROWS / 2;
    __shared__ float2 s[NPI * PS];
    const int row0 = blockIdx.x * ROWS;
    stage_c2r<NX, ROWS, NT, NPI, PS>(s, in, g, row0);
    __syncthreads();
    lds_fft<NX, NPI, NT, +1, PS, 1, false>(s, twx);
    for (int e = threadIdx.x; e < 9 * ROWS * NX; e += NT) {
        const int p = e / NX, x = e - p * NX;
        const int f = p / ROWS, r = p - f * ROWS;
        const int row = row0 + r;
        if (row < g.nrows) out[(long)f * g.n + (long)row * NX + x] = pencil_val<PS>(s, p, x);
    }
}

// ---------------------------------------------------------------------------
// y FFT (forward or inverse) of `nf` spectra starting at field f0, in place.
// grid: (kx tiles, nz, shots * nf)
template <int NY, int NT, int DIR>
__global__ __launch_bounds__(NT) void k_y(Geo g, const float2* __restrict__ twy, float2* __restrict__ spec,
                                          int f0, int nf)
{
    constexpr int TX = tile_for(NY);
    constexpr int IS = TX + 1;
    __shared__ float2 s[NY * IS];
    const int kx0 = blockIdx.x * TX;
    const int z = blockIdx.y;
    const int shot = blockIdx.z / nf, f = f0 + blockIdx.z % nf;
    float2* __restrict__ base = spec + (long)shot * g.sstride + f * g.nspec + (long)z * NY * g.ldx + kx0;
    const int ncol = min(TX, g.nxh - kx0);
    for (int e = threadIdx.x; e < NY * TX; e += NT) {
        const int y = e / TX, c = e - y * TX;
        s[y * IS + c] = c < ncol ? base[(long)y * g.ldx + c] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    lds_fft<NY, TX, NT, DIR, 1, IS, true>(s, twy);
    for (int e = threadIdx.x; e < NY * TX; e += NT) {
        const int y = e / TX, c = e - y * TX;
        if (c < ncol) base[(long)y * g.ldx + c] = s[y * IS + c];
    }
}

// z FFT, multiply by the staggered derivative symbols and kappa, inverse z
// FFT.  grid: (kx tiles, ny, shots * nin).  Reads spectra `in0 + input`,
// writes the derivative spectra 9.. (deriv block) of the shot.
template <int NZ, int NT>
__global__ __launch_bounds__(NT) void k_z(Geo g, const float2* __restrict__ twz, float2* __restrict__ spec,
                                          int in0, const ZDesc* __restrict__ zd, int phase)
{
    const PhaseDesc& ph = zd->ph[phase];
    const Ops& ops = zd->ops;
    constexpr int TX = tile_for(NZ);
    constexpr int IS = TX + 1;
    __shared__ float2 A[NZ * IS];
    __shared__ float2 B[NZ * IS];
    const int kx0 = blockIdx.x * TX;
    const int ky = blockIdx.y;
    const int shot = blockIdx.z / ph.nin, fi = blockIdx.z % ph.nin;
    const long plane = (long)g.ny * g.ldx;
    float2* __restrict__ sb = spec + (long)shot * g.sstride;
    const float2* __restrict__ in = sb + (in0 + fi) * g.nspec + (long)ky * g.ldx + kx0;
    const int ncol = min(TX, g.nxh - kx0);
    for (int e = threadIdx.x; e < NZ * TX; e += NT) {
        const int z = e / TX, c = e - z * TX;
        A[z * IS + c] = c < ncol ? in[z * plane + c] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    lds_fft<NZ, TX, NT, -1, 1, IS, true>(A, twz);
    const float* __restrict__ kap = ops.kap + (long)ky * g.ldx + kx0;
    for (int o = 0; o < ph.nout[fi]; ++o) {
        const int axis = ph.axis[fi][o], plus = ph.plus[fi][o];
        const float2* __restrict__ sym = ops.sym[axis][plus];
        for (int e = threadIdx.x; e < NZ * TX; e += NT) {
            const int z = e / TX, c = e - z * TX;
            float2 v = make_float2(0.f, 0.f);
            if (c < ncol) {
                const float2 sd = sym[axis == 0 ? kx0 + c : (axis == 1 ? ky : z)];
                v = c_scale(c_mul(sd, A[z * IS + c]), kap[z * plane + c]);
            }
            B[z * IS + c] = v;
        }
        __syncthreads();
        lds_fft<NZ, TX, NT, +1, 1, IS, true>(B, twz);
        float2* __restrict__ out = sb + (9 + ph.oidx[fi][o]) * g.nspec + (long)ky * g.ldx + kx0;
        for (int e = threadIdx.x; e < NZ * TX; e += NT) {
            const int z = e / TX, c = e - z * TX;
            if (c < ncol) out[z * plane + c] = B[z * IS + c];
        }
        __syncthreads();
    }
}

__global__ void k_step_inc(int* stepp)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *stepp += 1;
}

// non-finite check on sampled trace values: flag = 1 if any is not finite
__global__ void k_check_finite(const float* __restrict__ tr, long n, int* __restrict__ flag)
{
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    long stride = (long)gridDim.x * blockDim.x;
    int bad = 0;
    for (; i < n; i += stride) bad |= !isfinite(tr[i]);
    if (bad) *flag = 1;
}

}  // namespace pstd
