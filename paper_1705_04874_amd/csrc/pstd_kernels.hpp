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
// Real fields are [nz][ny][nx].  An x-transformed spectrum (kx = 0 .. nx/2)
// is stored as a main block [nz][ny][ldx] holding kx < nxm (nxm = nx/2 for
// even nx, (nx+1)/2 for odd nx; ldx = nxm rounded up to 16, i.e. 128-byte
// rows) followed, for even nx, by the Nyquist plane kx = nx/2 as [nz][ny].
// The y and z transforms work on 16-column tiles of the main block plus
// tiles of 16 Nyquist pencils, so no tile is left almost empty.
#pragma once
#include "fft_lds.hpp"

namespace pstd {

struct Geo {
    int nx, ny, nz, nxh, ldx, nrows;   // nrows = ny * nz; nxh = nx/2 + 1
    int nxm, has_nyq;                  // main columns, Nyquist plane present
    long n;                            // cells
    long nqoff;                        // offset of the Nyquist plane in a spectrum
    long nspec;                        // complex values per spectrum
    long fstride;                      // floats per shot of split fields (24 n)
    long sstride;                      // complex values per shot of spectra (18 nspec)
    int shot_fast;                     // update kernels' grid is (shots, row blocks)
};

// material coefficients pre-multiplied by dt (FP64 on the host, stored FP32)
struct Mat {
    const float* dtr[3];   // dt / rho at the vx, vy, vz nodes
    const float* dlam;     // dt * lambda at centres
    const float* dmu2;     // 2 dt * mu at centres
    const float* dmus[3];  // dt * mu at xy, xz, yz shear nodes
    // Kelvin-Voigt viscosity (eq. 1-2), only read by the viscous stress
    // update: chi and 2 eta at centres, eta at the shear nodes (not times dt:
    // they multiply the change of a velocity derivative over one step)
    const float* chi;
    const float* eta2;
    const float* etas[3];
};

// PML factors a = exp(-alpha dt / 2) per axis, at integer and half nodes, and
// the multi-axial factors b = a^p: a split part along axis d is damped by
// a_d times b_e of the two other axes e.
struct Pml {
    const float* ai[3];
    const float* ah[3];
    const float* bi[3];
    const float* bh[3];
    // per axis, the indices [flo, fhi] whose four factors are all exactly 1:
    // a cell inside all three ranges is undamped, and there each field keeps
    // its whole value in its first split part (the others stay zero)
    int flo[3] = {0, 0, 0}, fhi[3] = {-1, -1, -1};
};

__device__ __forceinline__ bool undamped(const Pml& pm, int x, int y, int z)
{
    return x >= pm.flo[0] && x <= pm.fhi[0] && y >= pm.flo[1] && y <= pm.fhi[1] && z >= pm.flo[2] &&
           z <= pm.fhi[2];
}

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
    const float* kap;          // kappa(|k|) / (nx ny nz), main block [nz][ny][ldx]
    const float* kapn;         // the same on the Nyquist plane [nz][ny]
    // kappa evaluated in the kernel instead of read from the table (kpoly[phase]
    // = 1): s = (c_ref dt / 2)^2 |k|^2 from the per-axis squares k2[d] (x:
    // 0..nx/2), kappa / (nx ny nz) = sum_n kc[n] s^n, the series of sin(a)/a in
    // s = a^2
    int kpoly[2];
    const float* k2[3];
    float kc[8];
};

// device-resident descriptor of the two derivative phases (read with uniform
// loads; kept out of the kernel arguments so runtime indexing stays in memory)
struct ZDesc {
    PhaseDesc ph[2];   // [0] V phase, [1] S phase
    Ops ops;
};

constexpr int rows_for(int nx) { return nx <= 32 ? 16 : nx <= 64 ? 8 : nx <= 160 ? 4 : 2; }

// Load through a pointer that addresses global memory.  Pointers read from a
// device-resident descriptor are generic to the compiler, and a generic load
// also holds the LDS wait counter, so every LDS wait after it would wait for
// the memory load as well.
__device__ __forceinline__ float gld(const float* p)
{
    return *(const __attribute__((address_space(1))) float*)p;
}
__device__ __forceinline__ float2 gld(const float2* p)
{
    typedef float f2v __attribute__((ext_vector_type(2)));
    const f2v v = *(const __attribute__((address_space(1))) f2v*)p;
    return make_float2(v.x, v.y);
}

// Column-tile widths of the y and z kernels that the library is built with:
// a tile of TX pencils of length N stages N (TX + 1) complex values in LDS
// (at most 64 KB) and, in the z kernel, keeps N TX / NT of them per thread in
// registers twice (spectrum and one derivative), at most 16 each.  y: width 8
// only where 16 does not fit; z: width 8 always (half the LDS of 16, so twice
// the blocks per CU, against 64-byte instead of 128-byte row segments).
constexpr bool y_tile_ok(int n, int tx) { return (long)n * (tx + 1) * 8 + n * 8 <= 65536; }
constexpr bool z_tile_ok(int n, int tx) { return n * tx <= 16 * 256 && (long)n * (tx + 1) * 8 + 3L * n * 8 <= 65536; }
constexpr bool y_tile_built(int n, int tx) { return y_tile_ok(n, tx) && (tx != 8 || !y_tile_ok(n, 16)); }
constexpr bool z_tile_built(int n, int tx) { return z_tile_ok(n, tx); }


// index of spectrum element (row, kx) within one field's spectrum
__device__ __forceinline__ long spec_idx(const Geo& g, int row, int k)
{
    return k < g.nxm ? (long)row * g.ldx + k : g.nqoff + row;
}

// value of real pencil p (= field * ROWS + local row) of a spectrum row.  Rows
// past the grid (only in the last block of a ragged row count) read the last
// row instead: their pencils are transformed on their own and never stored,
// and no branch separates the loads of a pass, so all of them are issued
// before the first wait
__device__ __forceinline__ float2 spec_at(const float2* __restrict__ base, const Geo& g, int rows,
                                          int row0, int p, int k)
{
    const int f = p / rows, r = p - f * rows;
    const int row = min(row0 + r, g.nrows - 1);
    return base[f * g.nspec + spec_idx(g, row, k)];
}

// Loader for an inverse x transform: complex pencil q is the Hermitian
// extension of the half spectra of real pencils 2q and 2q+1 (Z = A + i B), so
// one complex inverse FFT gives both real rows (as real and imaginary parts).
// DC and Nyquist keep only their real parts.
template <int NX, int ROWS>
struct HermLoader {
    const float2* __restrict__ src;
    Geo g;
    int row0;
    // Two phases, so that a pass issues the loads of all its elements before
    // the first wait: fetch() loads the two half-spectrum values at
    // k = min(i, NX - i); finish() combines them branch free with
    // w = sign(2 i - NX) (0 at DC and at the Nyquist bin):
    // Z_i = (a.x + w b.y) + i (b.x - w a.y)
    static constexpr bool TWO_PHASE = true;
    using Raw = float4;
    __device__ float4 fetch(int q, int i) const
    {
        const int k = min(i, NX - i);
        const float2 a = spec_at(src, g, ROWS, row0, 2 * q, k);
        const float2 b = spec_at(src, g, ROWS, row0, 2 * q + 1, k);
        return make_float4(a.x, a.y, b.x, b.y);
    }
    __device__ float2 finish(float4 v, int i) const
    {
        const int sg = (2 * i > NX) - (2 * i < NX);
        const float w = (float)(i == 0 ? 0 : sg);
        return make_float2(fmaf(w, v.w, v.x), fmaf(-w, v.y, v.z));
    }
    __device__ float2 operator()(int q, int i) const { return finish(fetch(q, i), i); }
};

// Unpack NPO complex forward transforms of paired real rows into half spectra.
template <int NX, int ROWS, int NT, int NPO, int PS>
__device__ __forceinline__ void unstage_r2c(const float2* s, float2* __restrict__ dst, const Geo& g, int row0)
{
    constexpr int NXH = NX / 2 + 1;
    for (int e = threadIdx.x; e < NPO * NXH; e += NT) {
        const int q = e / NXH, k = e - q * NXH;
        const float2 z = s[q * PS + lidx<true>(k)];
        const float2 zm = s[q * PS + lidx<true>(k == 0 ? 0 : NX - k)];
        const float2 A = make_float2(0.5f * (z.x + zm.x), 0.5f * (z.y - zm.y));
        const float2 B = make_float2(0.5f * (z.y + zm.y), -0.5f * (z.x - zm.x));
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int p = 2 * q + h;
            const int f = p / ROWS, r = p - f * ROWS;
            const int row = row0 + r;
            if (row < g.nrows) dst[f * g.nspec + spec_idx(g, row, k)] = h ? B : A;
        }
    }
}

// real value of pencil p at x (pairs stored as re / im of one complex pencil)
template <int PS>
__device__ __forceinline__ float pencil_val(const float2* s, int p, int x)
{
    const float2 v = s[(p >> 1) * PS + lidx<true>(x)];
    return (p & 1) ? v.y : v.x;
}

template <int PS>
__device__ __forceinline__ void pencil_set(float2* s, int p, int x, float v)
{
    float* f = reinterpret_cast<float*>(s + (p >> 1) * PS + lidx<true>(x));
    f[p & 1] = v;
}

// Block -> (shot, first row) of the update kernels.  A batch of shots is
// launched on a grid of (shots, row blocks), so that consecutive blocks take
// consecutive shots of one row block and the shots read the model's material
// and PML tables at about the same time and share them in cache; one shot
// (or more row blocks than a grid's y extent holds) on (row blocks, shots).
// The choice is a scalar flag: no division, so shot and row stay scalar.
__device__ __forceinline__ void update_block(const Geo& g, int& shot, int& row0, int rows)
{
    if (g.shot_fast) {
        shot = blockIdx.x;
        row0 = blockIdx.y * rows;
    } else {
        shot = blockIdx.y;
        row0 = blockIdx.x * rows;
    }
}

// Occupancy hint for the velocity update: at power-of-two lengths up to 256
// with 256 or 512 threads (and 512 with 512) the compiler fits it in 96 VGPRs
// without spilling when asked for 5 waves per SIMD (4 otherwise), which
// measured faster; at other lengths the same request spills to scratch or
// cannot be met, so it is not made there.  (The stress update, asked the
// same, measured slightly slower.)
template <int NX, int NT>
constexpr int vel_waves()
{
    return (NX >= 32 && (NX & (NX - 1)) == 0 && NT >= 256 && (NX <= 256 || NT == 512)) ? 5 : 1;
}

// ---------------------------------------------------------------------------
// V phase tail: inverse x FFT of the 9 stress derivatives, velocity split-PML
// update (eq. 2 second line), receivers vx vy vz, x FFT of the summed v.
template <int NX, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(vel_waves<NX, NT>()))) void k_vel(
    Geo g, Mat m, Pml pm, const float2* __restrict__ twx, float* __restrict__ fields, float2* __restrict__ spec,
    Rec rc, float* __restrict__ traces, const int* __restrict__ stepp, int* __restrict__ stepn, int n0, int ldt)
{
    constexpr int ROWS = rows_for(NX);
    constexpr int PS = padded_len(NX);
    constexpr int NPI = 9 * ROWS / 2;
    constexpr int NPO = 3 * ROWS / 2;
    constexpr int CPT = (ROWS * NX + NT - 1) / NT;
    __shared__ float2 s[NPI * PS];
    __shared__ float2 tw[NX];
    // step counters alternate between two words: this step reads one and
    // publishes the next step's index in the other (read by no kernel of
    // this step)
    const int step = *stepp;
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *stepn = step + 1;

    int shot, row0;
    update_block(g, shot, row0, ROWS);
    float* __restrict__ F = fields + (long)shot * g.fstride;
    const float2* __restrict__ D9 = spec + (long)shot * g.sstride + 9 * g.nspec;
    float2* __restrict__ S3 = spec + (long)shot * g.sstride + 6 * g.nspec;

    for (int i = threadIdx.x; i < NX; i += NT) tw[i] = twx[i];
    fft_ld<NX, NPI, NT, +1, PS, 1, false, false, HermLoader<NX, ROWS>, NoSt, true>(s, tw, HermLoader<NX, ROWS>{D9, g, row0}, NoSt{});

    // all loads of the update before any store: the split parts share one
    // base pointer, so interleaved stores would serialise later loads
    float vp[CPT][9], dtr[CPT][3], a[CPT][3][3];
    bool ok[CPT], in[CPT];
    long cell[CPT];
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
        const int c = threadIdx.x + i * NT;
        const int r = c / NX, x = c - r * NX;
        const int row = row0 + r;
        ok[i] = c < ROWS * NX && row < g.nrows;
        const int rr = ok[i] ? row : row0;
        const int y = rr % g.ny, z = rr / g.ny;
        cell[i] = (long)rr * NX + x;
        in[i] = undamped(pm, x, y, z);
        const float axi = pm.ai[0][x], axh = pm.ah[0][x];
        const float ayi = pm.ai[1][y], ayh = pm.ah[1][y];
        const float azi = pm.ai[2][z], azh = pm.ah[2][z];
        const float bxi = pm.bi[0][x], bxh = pm.bh[0][x];
        const float byi = pm.bi[1][y], byh = pm.bh[1][y];
        const float bzi = pm.bi[2][z], bzh = pm.bh[2][z];
        // component c sits half a cell up along axis c; split part d is damped
        // by a_d and by b of the two other axes, all at the component's node
        a[i][0][0] = axh * byi * bzi; a[i][0][1] = ayi * bxh * bzi; a[i][0][2] = azi * bxh * byi;
        a[i][1][0] = axi * byh * bzi; a[i][1][1] = ayh * bxi * bzi; a[i][1][2] = azi * bxi * byh;
        a[i][2][0] = axi * byi * bzh; a[i][2][1] = ayi * bxi * bzh; a[i][2][2] = azh * bxi * byi;
        // an undamped cell reads only the first part of each component
#pragma unroll
        for (int q = 0; q < 9; ++q) vp[i][q] = ok[i] && (q % 3 == 0 || !in[i]) ? F[(long)q * g.n + cell[i]] : 0.f;
#pragma unroll
        for (int comp = 0; comp < 3; ++comp) dtr[i][comp] = ok[i] ? m.dtr[comp][cell[i]] : 0.f;
    }

    float vsum[CPT][3];
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
        const int c = threadIdx.x + i * NT;
        const int r = c / NX, x = c - r * NX;
#pragma unroll
        for (int comp = 0; comp < 3; ++comp) {
            float acc = 0.f;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const int q = 3 * comp + d;
                const float dv = ok[i] ? pencil_val<PS>(s, q * ROWS + r, x) : 0.f;
                const float ad = a[i][comp][d];
                vp[i][q] = ad * (ad * vp[i][q] + dtr[i][comp] * dv);
                acc += vp[i][q];
            }
            vsum[i][comp] = acc;
            // undamped: the parts' factors are 1, their sum is the component
            if (in[i]) vp[i][3 * comp] = acc;
        }
        if (ok[i]) {
#pragma unroll
            for (int q = 0; q < 9; ++q)
                if (q % 3 == 0 || !in[i]) F[(long)q * g.n + cell[i]] = vp[i][q];
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
        const int c = threadIdx.x + i * NT;
        if (c >= ROWS * NX) continue;
        const int r = c / NX, x = c - r * NX;
#pragma unroll
        for (int comp = 0; comp < 3; ++comp) pencil_set<PS>(s, comp * ROWS + r, x, ok[i] ? vsum[i][comp] : 0.f);
    }
    __syncthreads();
    // receivers (vx, vy, vz at their staggered nodes, time (n + 1/2) dt)
    {
        const int rend = min(row0 + ROWS, g.nrows);
        const int e0 = rc.ptr[row0], e1 = rc.ptr[rend];
        const int tn = step - n0;
        for (int e = e0 + threadIdx.x; e < e1; e += NT) {
            const int4 q = rc.ent[e];
            const int r = q.y - row0;
#pragma unroll
            for (int comp = 0; comp < 3; ++comp)
                traces[(((long)shot * 4 + 1 + comp) * rc.n_rec + q.z) * ldt + tn] =
                    pencil_val<PS>(s, comp * ROWS + r, q.x);
        }
    }
    lds_fft<NX, NPO, NT, -1, PS, 1, false, true>(s, tw);
    unstage_r2c<NX, ROWS, NT, NPO, PS>(s, S3, g, row0);
}

// ---------------------------------------------------------------------------
// S phase tail: inverse x FFT of the 9 velocity derivatives, stress split-PML
// update (eq. 2 first line), source injection, receiver p (eq. 3), x FFT of
// the 6 summed stresses.
// the first split part of a stress component (parts 0-8: three per normal
// component, 9-14: two per shear component)
__host__ __device__ constexpr bool first_part(int q) { return q < 9 ? q % 3 == 0 : (q - 9) % 2 == 0; }

// slot of velocity derivative q (order of e[] in k_str) among the nine stored ones
__host__ __device__ constexpr int ep_slot(int q) { return q < 3 ? q : ((q - 3) ^ 1) + 3; }

template <int NX, int NT, bool VISC = false>
__global__ __launch_bounds__(NT) void k_str(Geo g, Mat m, Pml pm, const float2* __restrict__ twx,
                                            float* __restrict__ fields, float2* __restrict__ spec,
                                            Rec rc, Inj inj, float* __restrict__ traces,
                                            const int* __restrict__ stepp, int n0, int ldt)
{
    constexpr int ROWS = rows_for(NX);
    constexpr int PS = padded_len(NX);
    constexpr int NPI = 9 * ROWS / 2;
    constexpr int NPO = 6 * ROWS / 2;
    constexpr int CPT = (ROWS * NX + NT - 1) / NT;
    __shared__ float2 s[NPI * PS];
    __shared__ float2 tw[NX];

    int shot, row0;
    update_block(g, shot, row0, ROWS);
    float* __restrict__ F = fields + (long)shot * g.fstride + 9 * g.n;   // 15 stress parts
    // viscous: the nine velocity derivatives of the previous step, after the 24
    // split parts, in the order D-x vx, D-y vy, D-z vz, Dx+ vy, Dy+ vx, Dx+ vz,
    // Dz+ vx, Dy+ vz, Dz+ vy (e[] below swaps each shear pair)
    float* __restrict__ EP = fields + (long)shot * g.fstride + 24 * g.n;
    const float2* __restrict__ D9 = spec + (long)shot * g.sstride + 9 * g.nspec;
    float2* __restrict__ S6 = spec + (long)shot * g.sstride;
    const int step = *stepp;
    const int* __restrict__ iptr = inj.ptr + (long)shot * (g.nrows + 1);

    for (int i = threadIdx.x; i < NX; i += NT) tw[i] = twx[i];
    fft_ld<NX, NPI, NT, +1, PS, 1, false, false, HermLoader<NX, ROWS>, NoSt, true>(s, tw, HermLoader<NX, ROWS>{D9, g, row0}, NoSt{});

    // every load of every cell of this thread before any arithmetic or store
    // (the split parts share one base pointer, so a store would serialise
    // later loads): split parts, materials, PML factors, source rows
    float sp[CPT][15], mt[CPT][5], fa[CPT][9];
    float ep[VISC ? CPT : 1][9], vm[VISC ? CPT : 1][5];
    int jr[CPT][2];
    bool ok[CPT], in[CPT];
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
        const int c = threadIdx.x + i * NT;
        const int r = c / NX, x = c - r * NX;
        const int row = row0 + r;
        ok[i] = c < ROWS * NX && row < g.nrows;
        const int rr = ok[i] ? row : row0;
        const int y = rr % g.ny, z = rr / g.ny;
        const long cell = (long)rr * NX + x;
        in[i] = undamped(pm, x, y, z);
        // an undamped cell reads only the first part of each component
#pragma unroll
        for (int q = 0; q < 15; ++q) sp[i][q] = first_part(q) || !in[i] ? F[(long)q * g.n + cell] : 0.f;
        mt[i][0] = m.dlam[cell];
        mt[i][1] = m.dmu2[cell];
        mt[i][2] = m.dmus[0][cell];
        mt[i][3] = m.dmus[1][cell];
        mt[i][4] = m.dmus[2][cell];
        const float bxi = pm.bi[0][x], bxh = pm.bh[0][x];
        const float byi = pm.bi[1][y], byh = pm.bh[1][y];
        const float bzi = pm.bi[2][z], bzh = pm.bh[2][z];
        // normal parts (centre nodes): a_d times b of the other two axes
        fa[i][0] = pm.ai[0][x] * byi * bzi;
        fa[i][1] = pm.ai[1][y] * bxi * bzi;
        fa[i][2] = pm.ai[2][z] * bxi * byi;
        // shear parts at their nodes: xy (h,h,i), xz (h,i,h), yz (i,h,h)
        fa[i][3] = pm.ah[0][x] * byh * bzi;   // xy, x part
        fa[i][4] = pm.ah[1][y] * bxh * bzi;   // xy, y part
        fa[i][5] = pm.ah[0][x] * byi * bzh;   // xz, x part
        fa[i][6] = pm.ah[2][z] * bxh * byi;   // xz, z part
        fa[i][7] = pm.ah[1][y] * bxi * bzh;   // yz, y part
        fa[i][8] = pm.ah[2][z] * bxi * byh;   // yz, z part
        jr[i][0] = iptr[rr];
        jr[i][1] = iptr[rr + 1];
        if constexpr (VISC) {
#pragma unroll
            for (int q = 0; q < 9; ++q) ep[i][q] = EP[(long)ep_slot(q) * g.n + cell];
            vm[i][0] = m.chi[cell];
            vm[i][1] = m.eta2[cell];
            vm[i][2] = m.etas[0][cell];
            vm[i][3] = m.etas[1][cell];
            vm[i][4] = m.etas[2][cell];
        }
    }
    __builtin_amdgcn_sched_barrier(0);

    float ssum[CPT][6];
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
        const int c = threadIdx.x + i * NT;
        const int r = c / NX, x = c - r * NX;
        const int row = row0 + r;
#pragma unroll
        for (int q = 0; q < 6; ++q) ssum[i][q] = 0.f;
        if (!ok[i]) continue;
        const long cell = (long)row * NX + x;
        const float dlam = mt[i][0], dmu2 = mt[i][1];
        const float mxy = mt[i][2], mxz = mt[i][3], myz = mt[i][4];
        const float ai[3] = {fa[i][0], fa[i][1], fa[i][2]};
        const float axy_x = fa[i][3], axy_y = fa[i][4], axz_x = fa[i][5], axz_z = fa[i][6];
        const float ayz_y = fa[i][7], ayz_z = fa[i][8];
        // derivatives: e0..e2 = D_d^- v_d, e3 = Dy+ vx, e4 = Dx+ vy, e5 = Dz+ vx,
        //              e6 = Dx+ vz, e7 = Dz+ vy, e8 = Dy+ vz
        float e[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) e[q] = pencil_val<PS>(s, q * ROWS + r, x);
        // viscous terms (eq. 2): chi delta_cd d/dt(div v) + eta d/dt(D v + (D v)^T),
        // d/dt as the change of each derivative over the step
        float de[9];
        if constexpr (VISC) {
#pragma unroll
            for (int q = 0; q < 9; ++q) de[q] = e[q] - ep[i][q];
        }
        // normal parts sp[i][3c + d] (component c, axis d)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc)
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const float coef = cc == d ? dlam + dmu2 : dlam;
                float rhs = coef * e[d];
                if constexpr (VISC) rhs += (cc == d ? vm[i][0] + vm[i][1] : vm[i][0]) * de[d];
                sp[i][3 * cc + d] = ai[d] * (ai[d] * sp[i][3 * cc + d] + rhs);
            }
        // shear parts: 9 sxy(x) <- Dx+ vy, 10 sxy(y) <- Dy+ vx, 11 sxz(x) <- Dx+ vz,
        //              12 sxz(z) <- Dz+ vx, 13 syz(y) <- Dy+ vz, 14 syz(z) <- Dz+ vy
        float sh[6] = {mxy * e[4], mxy * e[3], mxz * e[6], mxz * e[5], myz * e[8], myz * e[7]};
        if constexpr (VISC) {
            sh[0] += vm[i][2] * de[4];
            sh[1] += vm[i][2] * de[3];
            sh[2] += vm[i][3] * de[6];
            sh[3] += vm[i][3] * de[5];
            sh[4] += vm[i][4] * de[8];
            sh[5] += vm[i][4] * de[7];
        }
        sp[i][9] = axy_x * (axy_x * sp[i][9] + sh[0]);
        sp[i][10] = axy_y * (axy_y * sp[i][10] + sh[1]);
        sp[i][11] = axz_x * (axz_x * sp[i][11] + sh[2]);
        sp[i][12] = axz_z * (axz_z * sp[i][12] + sh[3]);
        sp[i][13] = ayz_y * (ayz_y * sp[i][13] + sh[4]);
        sp[i][14] = ayz_z * (ayz_z * sp[i][14] + sh[5]);
        if constexpr (VISC) {
#pragma unroll
            for (int q = 0; q < 9; ++q) EP[(long)ep_slot(q) * g.n + cell] = e[q];
        }
        // point sources of this shot in this row
        const int j0 = jr[i][0], j1 = jr[i][1];
        if (j0 != j1 && step < inj.nt_w) {
            for (int j = j0; j < j1; ++j) {
                const int4 q = inj.ent[j];
                if (q.x != x) continue;
                const float val = __int_as_float(q.z) * inj.wav[(long)q.w * inj.nt_w + step];
#pragma unroll
                for (int f = 0; f < 15; ++f)
                    if (q.y == f) sp[i][f] += val;
            }
        }
        ssum[i][0] = sp[i][0] + sp[i][1] + sp[i][2];
        ssum[i][1] = sp[i][3] + sp[i][4] + sp[i][5];
        ssum[i][2] = sp[i][6] + sp[i][7] + sp[i][8];
        ssum[i][3] = sp[i][9] + sp[i][10];
        ssum[i][4] = sp[i][11] + sp[i][12];
        ssum[i][5] = sp[i][13] + sp[i][14];
        if (in[i]) {
            // undamped: the parts' factors are 1, their sum is the component
            sp[i][0] = ssum[i][0];
            sp[i][3] = ssum[i][1];
            sp[i][6] = ssum[i][2];
            sp[i][9] = ssum[i][3];
            sp[i][11] = ssum[i][4];
            sp[i][13] = ssum[i][5];
        }
#pragma unroll
        for (int q = 0; q < 15; ++q)
            if (first_part(q) || !in[i]) F[(long)q * g.n + cell] = sp[i][q];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
        const int c = threadIdx.x + i * NT;
        if (c >= ROWS * NX) continue;
        const int r = c / NX, x = c - r * NX;
#pragma unroll
        for (int q = 0; q < 6; ++q) pencil_set<PS>(s, q * ROWS + r, x, ok[i] ? ssum[i][q] : 0.f);
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
    lds_fft<NX, NPO, NT, -1, PS, 1, false, true>(s, tw);
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
    constexpr int PS = padded_len(NX);
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
        lds_fft<NX, 3 * ROWS / 2, NT, -1, PS, 1, false, true>(s, twx);
        unstage_r2c<NX, ROWS, NT, 3 * ROWS / 2, PS>(s, O, g, row0);
    } else {
        lds_fft<NX, 6 * ROWS / 2, NT, -1, PS, 1, false, true>(s, twx);
        unstage_r2c<NX, ROWS, NT, 6 * ROWS / 2, PS>(s, O, g, row0);
    }
}

// inverse x FFT of 9 spectra to 9 real fields (test entry)
template <int NX, int NT>
__global__ __launch_bounds__(NT) void k_xinv(Geo g, const float2* __restrict__ twx, const float2* __restrict__ in,
                                             float* __restrict__ out)
{
    constexpr int ROWS = rows_for(NX);
    constexpr int PS = padded_len(NX);
    constexpr int NPI = 9 * ROWS / 2;
    __shared__ float2 s[NPI * PS];
    const int row0 = blockIdx.x * ROWS;
    fft_ld<NX, NPI, NT, +1, PS, 1, false, false, HermLoader<NX, ROWS>, NoSt, true>(s, twx, HermLoader<NX, ROWS>{in, g, row0}, NoSt{});
    for (int e = threadIdx.x; e < 9 * ROWS * NX; e += NT) {
        const int p = e / NX, x = e - p * NX;
        const int f = p / ROWS, r = p - f * ROWS;
        const int row = row0 + r;
        if (row < g.nrows) out[(long)f * g.n + (long)row * NX + x] = pencil_val<PS>(s, p, x);
    }
}

// ---------------------------------------------------------------------------
// Column tile of a y or z transform: element (column c, position i) is at
// base[c * cs + i * is]; columns c >= ncol are outside the array.
struct Tile {
    float2* __restrict__ base;
    long cs, is;
    int ncol;
    // columns past the array read the last column (unconditional load, no
    // branch between the loads of a pass) and give zero
    __device__ float2 operator()(int c, int i) const
    {
        const float2 v = base[min(c, ncol - 1) * cs + i * is];
        return c < ncol ? v : make_float2(0.f, 0.f);
    }
    __device__ void operator()(int c, int i, float2 v) const
    {
        if (c < ncol) base[c * cs + i * is] = v;
    }
};

// y FFT (forward or inverse) of `nf` spectra starting at field f0, in place.
// grid: (main tiles + Nyquist tile, nz, shots * nf).  Main tile bx covers
// columns [TX bx, TX bx + TX) of plane z = by; the Nyquist tile covers the
// Nyquist pencils of planes [TX by, TX by + TX).
template <int NY, int NT, int DIR, int TX>
__global__ __launch_bounds__(NT) void k_y(Geo g, const float2* __restrict__ twy, float2* __restrict__ spec,
                                          int f0, int nf)
{
    constexpr int IS = TX + 1;
    __shared__ float2 s[NY * IS];
    __shared__ float2 tw[NY];
    const int tmain = (g.nxm + TX - 1) / TX;
    const int shot = blockIdx.z / nf, f = f0 + blockIdx.z % nf;
    float2* __restrict__ fb = spec + (long)shot * g.sstride + (long)f * g.nspec;
    Tile t;
    if ((int)blockIdx.x < tmain) {
        const int kx0 = blockIdx.x * TX;
        t = Tile{fb + (long)blockIdx.y * NY * g.ldx + kx0, 1, g.ldx, min(TX, g.nxm - kx0)};
    } else {
        const int z0 = blockIdx.y * TX;
        if (z0 >= g.nz) return;
        t = Tile{fb + g.nqoff + (long)z0 * NY, NY, 1, min(TX, g.nz - z0)};
    }
    for (int i = threadIdx.x; i < NY; i += NT) tw[i] = twy[i];
    fft_ld<NY, TX, NT, DIR, 1, IS, true, true>(s, tw, t, t);
}

// z FFT, multiply by the staggered derivative symbols and kappa, inverse z
// FFT.  grid: (main tiles + Nyquist tile, ny, shots * groups).  Main tile bx
// covers columns [TX bx, +TX) of row ky = by; the Nyquist tile covers the
// Nyquist pencils of rows [TX by, +TX).  A block takes the input spectra
// [fpb g, fpb g + fpb) of its shot (g = blockIdx.z % groups), so that with
// fpb >= the phase's inputs one block applies its tile's kappa and symbols
// (loaded once) to every input field in turn.  For each input it reads
// spectrum `in0 + input`, writes the derivative spectra (9 + output index):
// the forward spectrum stays in registers, each output is multiplied there
// and inverted with the reversed radix plan.  MR caps the radix of the plan
// (16, or 8 for the 512-thread variants, whose threads then all take a
// butterfly of the first pass).
template <int NZ, int NT, int TX, int MR = 16>
__global__ __launch_bounds__(NT) void k_z(Geo g, const float2* __restrict__ twz, float2* __restrict__ spec,
                                          int in0, const ZDesc* __restrict__ zd, int phase, int fpb)
{
    const PhaseDesc& ph = zd->ph[phase];
    const Ops& ops = zd->ops;
    constexpr int IS = TX + 1;
    using RS = RegShape<NZ, TX, NT, MR>;
    constexpr int RL = RS::RL, QL = RS::QL;
    // LDS: the tile, the twiddles, and the D+ symbols along z and of the tile's
    // columns (D- is D+ with the real part negated: i k e^{-i k h/2} =
    // (k sin, k cos) against (-k sin, k cos)); kept under 40 KB at length 256
    // so that four blocks share a CU
    __shared__ float2 s[NZ * IS];
    __shared__ float2 tw[NZ];
    __shared__ float2 symz[NZ];
    __shared__ float2 symc[2][TX];
    __shared__ float kxy2[TX];
    // the forward spectrum is reused by every output of the input field; kept
    // in registers it stays live through the inverse transforms (about a
    // quarter of the kernel's VGPRs), so where it takes at most 16 KB it is
    // parked in thread-private LDS slots instead
    constexpr bool STASH = QL * RL * NT * (int)sizeof(float2) <= 16384;
    __shared__ float2 xs[STASH ? QL * RL * NT : 1];
    const int tmain = (g.nxm + TX - 1) / TX;
    const int groups = (ph.nin + fpb - 1) / fpb;
    const int shot = blockIdx.z / groups, fg = blockIdx.z % groups;
    const int f0 = fg * fpb, f1 = min(ph.nin, f0 + fpb);
    long off, zs;
    const float* kap;
    int ncol, kx0, kxc, ky0, kyc;
    if ((int)blockIdx.x < tmain) {
        kx0 = blockIdx.x * TX;
        kxc = 1;
        ky0 = blockIdx.y;
        kyc = 0;
        off = (long)ky0 * g.ldx + kx0;
        zs = (long)g.ny * g.ldx;
        ncol = min(TX, g.nxm - kx0);
        kap = ops.kap + off;
    } else {
        ky0 = blockIdx.y * TX;
        if (ky0 >= g.ny) return;
        kyc = 1;
        kx0 = g.nx / 2;
        kxc = 0;
        off = g.nqoff + ky0;
        zs = g.ny;
        ncol = min(TX, g.ny - ky0);
        kap = ops.kapn + ky0;
    }
    const bool kpoly = ops.kpoly[phase] != 0;
    for (int i = threadIdx.x; i < NZ; i += NT) {
        tw[i] = twz[i];
        symz[i] = gld(ops.sym[2][1] + i);
    }
    if (kpoly)
        for (int i = threadIdx.x; i < TX; i += NT) {
            const int c = min(i, ncol - 1);
            kxy2[i] = gld(ops.k2[0] + kx0 + kxc * c) + gld(ops.k2[1] + ky0 + kyc * c);
        }
    // x and y D+ symbols of this tile's columns (main tiles: kx0 + c and ky0;
    // Nyquist tile: nx/2 and ky0 + c), so that the multiply loop reads LDS only
    for (int i = threadIdx.x; i < 2 * TX; i += NT) {
        const int ax = i / TX, c = min(i % TX, ncol - 1);
        symc[ax][i % TX] = gld(ops.sym[ax][1] + (ax == 0 ? kx0 + kxc * c : ky0 + kyc * c));
    }
    __syncthreads();
    // kappa of the elements this thread multiplies, once for all the block's inputs
    float kr[QL][RL];
#pragma unroll
    for (int q = 0; q < QL; ++q)
#pragma unroll
        for (int r = 0; r < RL; ++r) {
            int c, z;
            const bool ok = reg_coords<NZ, RL, TX, NT, true>(q, r, c, z);
            float kv;
            if (kpoly) {
                const float sv = kxy2[min(c, TX - 1)] + gld(ops.k2[2] + (ok ? z : 0));
                kv = ops.kc[7];
#pragma unroll
                for (int t = 6; t >= 0; --t) kv = fmaf(kv, sv, ops.kc[t]);
            } else {
                // unconditional load (no branch between the loads) at a valid
                // element: slots past the last butterfly (ok false) carry z >= NZ
                kv = gld(kap + (ok ? z : 0) * zs + min(c, ncol - 1));
            }
            kr[q][r] = (ok && c < ncol) ? kv : 0.f;
        }
    float2* __restrict__ sb = spec + (long)shot * g.sstride;
    for (int fi = f0; fi < f1; ++fi) {
        if (fi > f0) __syncthreads();   // s was read by the previous input's last pass
        const Tile in{sb + (long)(in0 + fi) * g.nspec + off, 1, zs, ncol};
        float2 X[QL][RL];
        fft_g2r<NZ, TX, NT, -1, 1, IS, true, Tile, float2[QL][RL], MR>(s, tw, in, X);
        if constexpr (STASH) {
#pragma unroll
            for (int q = 0; q < QL; ++q)
#pragma unroll
                for (int r = 0; r < RL; ++r) xs[(q * RL + r) * NT + threadIdx.x] = X[q][r];
        }
        for (int o = 0; o < ph.nout[fi]; ++o) {
            const int axis = ph.axis[fi][o], plus = ph.plus[fi][o];
            // symbol table of this output: along z indexed by z, along x or y by column
            const float2* tab = axis == 2 ? symz : symc[axis];
            const bool byz = axis == 2;
            const float sgn = plus ? 1.f : -1.f;
            float2 Y[QL][RL];
#pragma unroll
            for (int q = 0; q < QL; ++q)
#pragma unroll
                for (int r = 0; r < RL; ++r) {
                    int c, z;
                    reg_coords<NZ, RL, TX, NT, true>(q, r, c, z);
                    const float2 s1 = tab[byz ? z : c];
                    const float2 sv = make_float2(sgn * s1.x, s1.y);
                    const float2 xv = STASH ? xs[(q * RL + r) * NT + threadIdx.x] : X[q][r];
                    Y[q][r] = c_scale(c_mul(sv, xv), kr[q][r]);
                }
            __syncthreads();   // s was read by the previous pass
            const Tile out{sb + (long)(9 + ph.oidx[fi][o]) * g.nspec + off, 1, zs, ncol};
            fft_r2g<NZ, TX, NT, +1, 1, IS, true, float2[QL][RL], Tile, MR>(s, tw, Y, out);
        }
    }
}

// The 512-thread z variants: the largest radix (16 or 8) whose first pass
// still gives every thread a butterfly
constexpr int z_maxr(int n, int tx, int nt) { return tx * (n / 16) >= nt ? 16 : 8; }
// at least four values per thread and a radix-8 (or 16) first pass
constexpr bool z512_ok(int n, int tx) { return z_tile_ok(n, tx) && n * tx >= 4 * 512 && n % 8 == 0 && tx * (n / 8) >= 512; }

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
