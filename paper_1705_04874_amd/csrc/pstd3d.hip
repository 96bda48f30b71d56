// Host side of the pstd3d C ABI: model ingest, FP64 operator tables, shot
// state, launch sequencing (eager or HIP-graph), checkpoints.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <new>
#include <vector>

#include "pstd3d.h"
#include "pstd_kernels.hpp"

using namespace pstd;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(e_ == hipErrorOutOfMemory ? PSTD_ENOMEM : PSTD_EDEVICE,             \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                 \
    } while (0)

constexpr int NT = 256;

// ---------------------------------------------------------------------------
// per-length kernel launchers.  Tuning knobs (the autotuner picks one value of
// each per context): the column-tile width of the y and z kernels and the
// threads per block of the two update kernels.
using VelFn = void (*)(dim3, hipStream_t, Geo, Mat, Pml, const float2*, float*, float2*, Rec, float*, const int*,
                       int*, int, int);
using StrFn = void (*)(dim3, hipStream_t, Geo, Mat, Pml, const float2*, float*, float2*, Rec, Inj, float*,
                       const int*, int, int);
struct XFns {
    void (*xfwd)(dim3, hipStream_t, Geo, const float2*, const float*, long, float2*, long, SumDesc);
    void (*xinv)(dim3, hipStream_t, Geo, const float2*, const float2*, float*);
    int rows;
};
struct VelVar {
    VelFn fn;
    int nt;
};
struct StrVar {
    StrFn fn;
    StrFn visc;   // the Kelvin-Voigt variant
    int nt;
};
struct YFns {
    void (*fwd)(dim3, hipStream_t, Geo, const float2*, float2*, int, int);
    void (*inv)(dim3, hipStream_t, Geo, const float2*, float2*, int, int);
    int tile;
};
struct ZFns {
    void (*op)(dim3, hipStream_t, Geo, const float2*, float2*, int, const ZDesc*, int, int);
    int tile;
    int nt;     // threads per block
};
constexpr int MAX_VARIANTS = 8;
constexpr int N_TILES = 4;
constexpr int TILE_CANDIDATES[N_TILES] = {8, 16, 32, 64};
// input fields per block of the z kernels: one, or every input of the phase
constexpr int ZF_VALUES[2] = {1, 6};

// threads per block of the update kernels of length N: 128, 256 and 512,
// none above the cells of a block
constexpr int nt_candidate(int n, int i)
{
    const int cells = rows_for(n) * n;
    const int c[3] = {128, 256, 512};
    const int v = c[i];
    if (v > cells || v % 64 || v > 1024) return 0;
    for (int j = 0; j < i; ++j)
        if (c[j] == v) return 0;
    return v;
}

template <int N>
struct Launch {
    static void xfwd(dim3 gr, hipStream_t st, Geo g, const float2* tw, const float* in, long is, float2* out,
                     long os, SumDesc sd)
    {
        hipLaunchKernelGGL((k_xfwd<N, NT>), gr, dim3(NT), 0, st, g, tw, in, is, out, os, sd);
    }
    static void xinv(dim3 gr, hipStream_t st, Geo g, const float2* tw, const float2* in, float* out)
    {
        hipLaunchKernelGGL((k_xinv<N, NT>), gr, dim3(NT), 0, st, g, tw, in, out);
    }
};

template <int N, int T>
struct LaunchX {
    static void vel(dim3 gr, hipStream_t st, Geo g, Mat m, Pml p, const float2* tw, float* f, float2* s, Rec r,
                    float* tr, const int* sp, int* sn, int n0, int ldt)
    {
        hipLaunchKernelGGL((k_vel<N, T>), gr, dim3(T), 0, st, g, m, p, tw, f, s, r, tr, sp, sn, n0, ldt);
    }
    static void str(dim3 gr, hipStream_t st, Geo g, Mat m, Pml p, const float2* tw, float* f, float2* s, Rec r,
                    Inj in, float* tr, const int* sp, int n0, int ldt)
    {
        hipLaunchKernelGGL((k_str<N, T>), gr, dim3(T), 0, st, g, m, p, tw, f, s, r, in, tr, sp, n0, ldt);
    }
    static void strv(dim3 gr, hipStream_t st, Geo g, Mat m, Pml p, const float2* tw, float* f, float2* s, Rec r,
                     Inj in, float* tr, const int* sp, int n0, int ldt)
    {
        hipLaunchKernelGGL((k_str<N, T, true>), gr, dim3(T), 0, st, g, m, p, tw, f, s, r, in, tr, sp, n0, ldt);
    }
};

template <int N, int I = 0>
void x_variants(VelVar* v, StrVar* s, int& n)
{
    if constexpr (I < 3) {
        constexpr int T = nt_candidate(N, I);
        if constexpr (T > 0) {
            v[n] = VelVar{LaunchX<N, T>::vel, T};
            s[n] = StrVar{LaunchX<N, T>::str, LaunchX<N, T>::strv, T};
            ++n;
        }
        x_variants<N, I + 1>(v, s, n);
    }
}

template <int N, int TX>
struct LaunchYZ {
    static void yf(dim3 gr, hipStream_t st, Geo g, const float2* tw, float2* s, int f0, int nf)
    {
        hipLaunchKernelGGL((k_y<N, NT, -1, TX>), gr, dim3(NT), 0, st, g, tw, s, f0, nf);
    }
    static void yi(dim3 gr, hipStream_t st, Geo g, const float2* tw, float2* s, int f0, int nf)
    {
        hipLaunchKernelGGL((k_y<N, NT, +1, TX>), gr, dim3(NT), 0, st, g, tw, s, f0, nf);
    }
    static void z(dim3 gr, hipStream_t st, Geo g, const float2* tw, float2* s, int in0, const ZDesc* zd, int ph,
                  int fpb)
    {
        hipLaunchKernelGGL((k_z<N, NT, TX>), gr, dim3(NT), 0, st, g, tw, s, in0, zd, ph, fpb);
    }
    static void z512(dim3 gr, hipStream_t st, Geo g, const float2* tw, float2* s, int in0, const ZDesc* zd, int ph,
                     int fpb)
    {
        hipLaunchKernelGGL((k_z<N, 512, TX, z_maxr(N, TX, 512)>), gr, dim3(512), 0, st, g, tw, s, in0, zd, ph, fpb);
    }
};

// the variants of length N: y tiles and z tiles (counts returned)
template <int N, int I = 0>
void yz_variants(YFns* y, int& ny, ZFns* z, int& nz)
{
    if constexpr (I < N_TILES) {
        constexpr int TX = TILE_CANDIDATES[I];
        if constexpr (y_tile_built(N, TX)) y[ny++] = YFns{LaunchYZ<N, TX>::yf, LaunchYZ<N, TX>::yi, TX};
        if constexpr (z_tile_built(N, TX)) z[nz++] = ZFns{LaunchYZ<N, TX>::z, TX, NT};
        if constexpr (z512_ok(N, TX)) z[nz++] = ZFns{LaunchYZ<N, TX>::z512, TX, 512};
        yz_variants<N, I + 1>(y, ny, z, nz);
    }
}

// Grid lengths the library is built for (all factor into 2, 3 and 5).
#define PSTD_LENGTHS(X)                                                                          \
    X(16) X(20) X(24) X(30) X(32) X(40) X(48) X(60) X(64) X(72) X(75) X(80) X(90) X(96) X(100) X(120) X(125) \
    X(128) X(144) X(150) X(160) X(180) X(192) X(200) X(240) X(256) X(288) X(300) X(320) X(360)  \
    X(384) X(400) X(480) X(512)

bool x_fns(int n, XFns* f, VelVar* vv = nullptr, StrVar* sv = nullptr, int* nv = nullptr)
{
    VelVar v[3];
    StrVar t[3];
    int k = 0;
    switch (n) {
#define CASE(N)                                                              \
    case N:                                                                  \
        *f = XFns{Launch<N>::xfwd, Launch<N>::xinv, rows_for(N)};            \
        x_variants<N>(v, t, k);                                              \
        break;
        PSTD_LENGTHS(CASE)
#undef CASE
    default:
        return false;
    }
    if (nv) {
        *nv = k;
        for (int i = 0; i < k; ++i) {
            vv[i] = v[i];
            sv[i] = t[i];
        }
    }
    return true;
}

// all y variants of length n (returns the count; 0: length not built)
int y_variants(int n, YFns* f)
{
    YFns y[MAX_VARIANTS];
    ZFns z[MAX_VARIANTS];
    int ny = 0, nz = 0;
    switch (n) {
#define CASE(N)                             \
    case N:                                 \
        yz_variants<N>(y, ny, z, nz);       \
        break;
        PSTD_LENGTHS(CASE)
#undef CASE
    default:
        return 0;
    }
    for (int i = 0; i < ny; ++i) f[i] = y[i];
    return ny;
}

int z_variants(int n, ZFns* f)
{
    YFns y[MAX_VARIANTS];
    ZFns z[MAX_VARIANTS];
    int ny = 0, nz = 0;
    switch (n) {
#define CASE(N)                             \
    case N:                                 \
        yz_variants<N>(y, ny, z, nz);       \
        break;
        PSTD_LENGTHS(CASE)
#undef CASE
    default:
        return 0;
    }
    for (int i = 0; i < nz; ++i) f[i] = z[i];
    return nz;
}

// V phase: stress spectra (sxx, syy, szz, sxy, sxz, syz) -> 9 derivatives,
// derivative index 3 c + d feeds split part v_c^(d).
PhaseDesc phase_v()
{
    PhaseDesc p{};
    p.nin = 6;
    auto set = [&](int in, int o, int idx, int axis, int plus) {
        p.oidx[in][o] = idx;
        p.axis[in][o] = axis;
        p.plus[in][o] = plus;
        p.nout[in] = o + 1;
    };
    set(0, 0, 0, 0, 1);  // Dx+ sxx -> vx(x)
    set(1, 0, 4, 1, 1);  // Dy+ syy -> vy(y)
    set(2, 0, 8, 2, 1);  // Dz+ szz -> vz(z)
    set(3, 0, 1, 1, 0);  // Dy- sxy -> vx(y)
    set(3, 1, 3, 0, 0);  // Dx- sxy -> vy(x)
    set(4, 0, 2, 2, 0);  // Dz- sxz -> vx(z)
    set(4, 1, 6, 0, 0);  // Dx- sxz -> vz(x)
    set(5, 0, 5, 2, 0);  // Dz- syz -> vy(z)
    set(5, 1, 7, 1, 0);  // Dy- syz -> vz(y)
    return p;
}

// S phase: velocity spectra (vx, vy, vz) -> e0..e8
PhaseDesc phase_s()
{
    PhaseDesc p{};
    p.nin = 3;
    auto set = [&](int in, int o, int idx, int axis, int plus) {
        p.oidx[in][o] = idx;
        p.axis[in][o] = axis;
        p.plus[in][o] = plus;
        p.nout[in] = o + 1;
    };
    set(0, 0, 0, 0, 0);  // Dx- vx
    set(0, 1, 3, 1, 1);  // Dy+ vx
    set(0, 2, 5, 2, 1);  // Dz+ vx
    set(1, 0, 1, 1, 0);  // Dy- vy
    set(1, 1, 4, 0, 1);  // Dx+ vy
    set(1, 2, 7, 2, 1);  // Dz+ vy
    set(2, 0, 2, 2, 0);  // Dz- vz
    set(2, 1, 6, 0, 1);  // Dx+ vz
    set(2, 2, 8, 1, 1);  // Dy+ vz
    return p;
}

template <class T>
int dev_upload(T** dst, const std::vector<T>& h)
{
    size_t bytes = std::max<size_t>(sizeof(T), h.size() * sizeof(T));
    HIP_TRY(hipMalloc(dst, bytes));
    if (!h.empty()) HIP_TRY(hipMemcpy(*dst, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
    return PSTD_OK;
}

// shot state in a caller's workspace: the split fields first, the spectra at
// the next 256-byte boundary
size_t spec_offset(size_t fbytes) { return (fbytes + 255) / 256 * 256; }

double pml_alpha(double pos, int n, int L, double A, double c, double h)
{
    if (L <= 0) return 0.0;
    double depth = std::max((double)L - pos, pos - (double)(n - 1 - L));
    depth = std::min(std::max(depth, 0.0), (double)L);
    double r = depth / L;
    return A * c / h * r * r * r * r;
}

}  // namespace

struct pstd3d_ctx {
    int nx = 0, ny = 0, nz = 0;
    double h[3] = {0, 0, 0}, dt = 0, c_ref = 0, cmax = 0;
    int pml = 0, kspace = 1;
    double pml_A = 0, pml_p = 0;
    int n_rec = 0;
    int device = 0;
    Geo g{};
    XFns xf{};
    // tuning knobs: built variants, forced values (0: autotune), the choice
    VelVar velv[3]{};
    StrVar strv[3]{};
    YFns yv[MAX_VARIANTS]{};   // y variants of length ny
    ZFns zv[MAX_VARIANTS]{};   // z variants of length nz: every built (tile, threads)
    int nzv = 0;
    int ztile[MAX_VARIANTS]{}; // the distinct z tiles (values of PSTD_TUNE_Z)
    int znt[MAX_VARIANTS]{};   // the distinct z thread counts (values of PSTD_TUNE_ZT)
    int nvar[PSTD_TUNE_COUNT] = {};
    int force[PSTD_TUNE_COUNT] = {};
    int sel[PSTD_TUNE_COUNT] = {};
    bool tuned = false;
    bool visc = false;         // Kelvin-Voigt viscosity set (33 state fields)
    int smooth = 0;            // source smoothing for the next set_sources (0 off, 1 Blackman)
    float tune_us[PSTD_TUNE_COUNT][MAX_VARIANTS] = {};   // measured us per launch of each variant
    YFns yf{};                 // the chosen variants
    ZFns zf{};
    int zfpb = 1;              // input fields per z block
    VelVar vel{};
    StrVar str{};

    int knob_value(int k, int i) const
    {
        switch (k) {
        case PSTD_TUNE_Y: return yv[i].tile;
        case PSTD_TUNE_Z: return ztile[i];
        case PSTD_TUNE_VEL: return velv[i].nt;
        case PSTD_TUNE_STR: return strv[i].nt;
        case PSTD_TUNE_ZT: return znt[i];
        default: return ZF_VALUES[i];
        }
    }
    // the built z variant of (tile, threads), or null
    const ZFns* zvar(int tile, int nt) const
    {
        for (int i = 0; i < nzv; ++i)
            if (zv[i].tile == tile && zv[i].nt == nt) return &zv[i];
        return nullptr;
    }
    void apply()
    {
        yf = yv[sel[PSTD_TUNE_Y]];
        const int tile = ztile[sel[PSTD_TUNE_Z]];
        const ZFns* z = zvar(tile, znt[sel[PSTD_TUNE_ZT]]);
        if (!z) {
            // every tile is built with NT threads: the thread knob follows
            z = zvar(tile, NT);
            for (int i = 0; i < nvar[PSTD_TUNE_ZT]; ++i)
                if (znt[i] == NT) sel[PSTD_TUNE_ZT] = i;
        }
        zf = *z;
        zfpb = ZF_VALUES[sel[PSTD_TUNE_ZF]];
        vel = velv[sel[PSTD_TUNE_VEL]];
        str = strv[sel[PSTD_TUNE_STR]];
    }
    StrFn str_fn(const StrVar& v) const { return visc ? v.visc : v.fn; }
    // model-wide device tables
    float* mat = nullptr;      // 8 arrays of n
    float* vmat = nullptr;     // viscous: chi, 2 eta, eta at the 3 shear nodes
    float* pmlb = nullptr;     // ai[3], ah[3] back to back
    float2* tw = nullptr;      // x, y, z twiddles
    float2* sym = nullptr;     // per axis D-, D+
    float* kap = nullptr;
    float* k2tab = nullptr;    // per-axis (c_ref dt / 2)^2 k^2 for the kappa series
    bool kseries_ok = false;   // the series is accurate on this grid
    int* rec_ptr = nullptr;
    int4* rec_ent = nullptr;
    ZDesc* zdesc = nullptr;
    Mat M{};
    Pml P{};
    Ops O{};
    const float2 *twx = nullptr, *twy = nullptr, *twz = nullptr;
    // shots
    int n_shots = 0;
    float* fields = nullptr;
    float2* spec = nullptr;
    bool own_state = true;     // fields and spec allocated here (false: in the caller's workspace)
    char* ws = nullptr;        // caller's workspace for the shot state (pstd3d_set_workspace)
    long ws_bytes = 0;
    int* inj_ptr = nullptr;
    int4* inj_ent = nullptr;
    float* wav = nullptr;
    int nt_w = 0;
    int* stepd = nullptr;
    int* flag = nullptr;
    long step = 0;
    long bytes = 0;
    // per-kernel event timing
    bool prof = false;
    std::vector<hipEvent_t> evpool;
    size_t evused = 0;
    std::vector<std::pair<int, size_t>> evpend;   // (kind, index of start event)
    double prof_ms[PSTD_K_COUNT] = {0};
    long prof_n[PSTD_K_COUNT] = {0};

    ~pstd3d_ctx()
    {
        release_shots();
        release_model();
        for (auto e : evpool) (void)hipEventDestroy(e);
    }

    // record a start event for `kind`; returns the pool index (or -1)
    long ev_begin(int kind, hipStream_t st)
    {
        if (!prof) return -1;
        if (evused + 2 > evpool.size()) {
            for (int i = 0; i < 64; ++i) {
                hipEvent_t e;
                if (hipEventCreate(&e) != hipSuccess) return -1;
                evpool.push_back(e);
            }
        }
        const size_t i = evused;
        evused += 2;
        (void)hipEventRecord(evpool[i], st);
        evpend.push_back({kind, i});
        return (long)i;
    }
    void ev_end(long i, hipStream_t st)
    {
        if (i >= 0) (void)hipEventRecord(evpool[i + 1], st);
    }
    // after the stream has been synchronised: fold the pending pairs in
    void ev_collect()
    {
        for (auto& p : evpend) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, evpool[p.second], evpool[p.second + 1]) == hipSuccess) {
                prof_ms[p.first] += ms;
                prof_n[p.first] += 1;
            }
        }
        evpend.clear();
        evused = 0;
    }

    void release_shots()
    {
        if (own_state) {
            (void)hipFree(fields);
            (void)hipFree(spec);
        }
        own_state = true;
        (void)hipFree(inj_ptr);
        (void)hipFree(inj_ent);
        (void)hipFree(wav);
        fields = nullptr;
        spec = nullptr;
        inj_ptr = nullptr;
        inj_ent = nullptr;
        wav = nullptr;
        n_shots = 0;
    }
    void release_model()
    {
        (void)hipFree(mat);
        (void)hipFree(vmat);
        (void)hipFree(pmlb);
        (void)hipFree(tw);
        (void)hipFree(sym);
        (void)hipFree(kap);
        (void)hipFree(k2tab);
        (void)hipFree(rec_ptr);
        (void)hipFree(rec_ent);
        (void)hipFree(zdesc);
        (void)hipFree(stepd);
        (void)hipFree(flag);
    }
};

namespace {

// device bytes of n_shots shots' state in a workspace (fields, then spectra)
size_t state_bytes(const pstd3d_ctx* c, int n_shots)
{
    const size_t fbytes = (size_t)n_shots * c->g.fstride * sizeof(float);
    return spec_offset(fbytes) + (size_t)n_shots * c->g.sstride * sizeof(float2);
}

int build_model(pstd3d_ctx* c, const pstd3d_model* m)
{
    const int nx = c->nx, ny = c->ny, nz = c->nz;
    const long n = (long)nx * ny * nz;
    const double dt = c->dt;
    auto at = [&](int i, int j, int k) { return (long)i + nx * ((long)j + (long)ny * k); };
    // eq. 4 and staggered averages, in double
    std::vector<double> mu(n);
    for (long q = 0; q < n; ++q) mu[q] = m->rho[q] * m->vs[q] * m->vs[q];
    std::vector<float> hm(8 * n);
    float* dtr[3] = {&hm[0], &hm[n], &hm[2 * n]};
    float* dlam = &hm[3 * n];
    float* dmu2 = &hm[4 * n];
    float* dmus[3] = {&hm[5 * n], &hm[6 * n], &hm[7 * n]};
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const long q = at(i, j, k);
                const int ip = std::min(i + 1, nx - 1), jp = std::min(j + 1, ny - 1), kp = std::min(k + 1, nz - 1);
                const double r0 = m->rho[q];
                dtr[0][q] = (float)(dt / (0.5 * (r0 + m->rho[at(ip, j, k)])));
                dtr[1][q] = (float)(dt / (0.5 * (r0 + m->rho[at(i, jp, k)])));
                dtr[2][q] = (float)(dt / (0.5 * (r0 + m->rho[at(i, j, kp)])));
                const double lam = m->rho[q] * m->vp[q] * m->vp[q] - 2.0 * mu[q];
                dlam[q] = (float)(dt * lam);
                dmu2[q] = (float)(2.0 * dt * mu[q]);
                const long nb[3][4] = {{q, at(ip, j, k), at(i, jp, k), at(ip, jp, k)},
                                       {q, at(ip, j, k), at(i, j, kp), at(ip, j, kp)},
                                       {q, at(i, jp, k), at(i, j, kp), at(i, jp, kp)}};
                for (int p = 0; p < 3; ++p) {
                    double inv = 0.0;
                    bool fluid = false;
                    for (int t = 0; t < 4; ++t) {
                        const double v = mu[nb[p][t]];
                        if (v == 0.0) fluid = true;
                        else inv += 1.0 / v;
                    }
                    dmus[p][q] = fluid ? 0.0f : (float)(dt * 4.0 / inv);
                }
            }
    int rc = dev_upload(&c->mat, hm);
    if (rc) return rc;
    for (int d = 0; d < 3; ++d) c->M.dtr[d] = c->mat + d * n;
    c->M.dlam = c->mat + 3 * n;
    c->M.dmu2 = c->mat + 4 * n;
    for (int p = 0; p < 3; ++p) c->M.dmus[p] = c->mat + (5 + p) * n;

    // PML factors a = exp(-alpha dt/2) and multi-axial factors b = a^p
    const int N[3] = {nx, ny, nz};
    std::vector<float> hp(4 * (nx + ny + nz));
    size_t off[3][4];
    size_t o = 0;
    for (int d = 0; d < 3; ++d)
        for (int kind = 0; kind < 4; ++kind) {
            off[d][kind] = o;
            const double shift = (kind & 1) ? 0.5 : 0.0;
            const double pw = (kind & 2) ? c->pml_p : 1.0;
            for (int i = 0; i < N[d]; ++i)
                hp[o++] = (float)std::exp(-pw * pml_alpha(i + shift, N[d], c->pml, c->pml_A, c->c_ref, c->h[d]) * dt / 2);
        }
    rc = dev_upload(&c->pmlb, hp);
    if (rc) return rc;
    for (int d = 0; d < 3; ++d) {
        c->P.ai[d] = c->pmlb + off[d][0];
        c->P.ah[d] = c->pmlb + off[d][1];
        c->P.bi[d] = c->pmlb + off[d][2];
        c->P.bh[d] = c->pmlb + off[d][3];
        // the undamped index range of this axis: all four factors exactly 1
        // (one interval, the axis minus its two absorbing layers; empty if
        // the flags do not form one)
        auto flat = [&](int i) {
            for (int kind = 0; kind < 4; ++kind)
                if (hp[off[d][kind] + i] != 1.0f) return false;
            return true;
        };
        int lo = 0, hi = N[d] - 1;
        while (lo < N[d] && !flat(lo)) ++lo;
        while (hi >= lo && !flat(hi)) --hi;
        bool one = true;
        for (int i = lo; i <= hi; ++i) one = one && flat(i);
        c->P.flo[d] = one ? lo : 0;
        c->P.fhi[d] = one ? hi : -1;
    }

    // twiddles exp(-2 pi i e / N) per axis
    std::vector<float2> ht;
    size_t toff[3];
    for (int d = 0; d < 3; ++d) {
        toff[d] = ht.size();
        for (int e = 0; e < N[d]; ++e) {
            const double a = -2.0 * M_PI * (double)e / N[d];
            ht.push_back(make_float2((float)std::cos(a), (float)std::sin(a)));
        }
    }
    rc = dev_upload(&c->tw, ht);
    if (rc) return rc;
    c->twx = c->tw + toff[0];
    c->twy = c->tw + toff[1];
    c->twz = c->tw + toff[2];

    // staggered derivative symbols i k exp(+-i k h / 2); x uses kx = 0..nx/2
    auto kval = [](int m, int nn, double h) {
        const int mm = m <= nn / 2 ? m : m - nn;
        return 2.0 * M_PI * mm / (nn * h);
    };
    const int len[3] = {c->g.nxh, ny, nz};
    std::vector<float2> hs;
    size_t soff[3][2];
    for (int d = 0; d < 3; ++d)
        for (int plus = 0; plus < 2; ++plus) {
            soff[d][plus] = hs.size();
            for (int mi = 0; mi < len[d]; ++mi) {
                const double k = kval(mi, N[d], c->h[d]);
                const double a = (plus ? 0.5 : -0.5) * k * c->h[d];
                // i k (cos a + i sin a) = (-k sin a, k cos a)
                hs.push_back(make_float2((float)(-k * std::sin(a)), (float)(k * std::cos(a))));
            }
        }
    rc = dev_upload(&c->sym, hs);
    if (rc) return rc;
    for (int d = 0; d < 3; ++d)
        for (int plus = 0; plus < 2; ++plus) c->O.sym[d][plus] = c->sym + soff[d][plus];

    // k-space correction with the 1/(nx ny nz) of the inverse transform folded
    // in; main block [nz][ny][ldx] (kx < nxm) followed by the Nyquist plane
    const size_t kmain = (size_t)nz * ny * c->g.ldx;
    std::vector<float> hk(kmain + (size_t)nz * ny, 0.0f);
    const double inv_n = 1.0 / (double)n;
    for (int k = 0; k < nz; ++k) {
        const double kz = kval(k, nz, c->h[2]);
        for (int j = 0; j < ny; ++j) {
            const double ky = kval(j, ny, c->h[1]);
            for (int i = 0; i < c->g.nxh; ++i) {
                const double kx = kval(i, nx, c->h[0]);
                const double q = std::sqrt(kx * kx + ky * ky + kz * kz);
                const double arg = 0.5 * c->c_ref * q * dt;
                const double kap = (c->kspace && arg != 0.0) ? std::sin(arg) / arg : 1.0;
                const size_t at = i < c->g.nxm ? ((size_t)k * ny + j) * c->g.ldx + i : kmain + (size_t)k * ny + j;
                hk[at] = (float)(kap * inv_n);
            }
        }
    }
    rc = dev_upload(&c->kap, hk);
    if (rc) return rc;
    c->O.kap = c->kap;
    c->O.kapn = c->kap + kmain;

    // kappa as a power series in s = (c_ref dt / 2)^2 |k|^2 (sin(a)/a = sum_n
    // (-s)^n / (2n+1)!), for the z operator to evaluate instead of reading the
    // table: per-axis squares (x over 0..nx/2) and eight coefficients with the
    // 1/(nx ny nz) folded in.  Offered where s stays <= 4 on the whole grid
    // (the ninth term is then below 2e-10 of kappa).
    const double b2 = 0.25 * c->c_ref * c->c_ref * dt * dt;
    std::vector<float> hk2;
    size_t k2off[3];
    double smax = 0.0;
    for (int d = 0; d < 3; ++d) {
        k2off[d] = hk2.size();
        double mx = 0.0;
        for (int mi = 0; mi < len[d]; ++mi) {
            const double k = kval(mi, N[d], c->h[d]);
            hk2.push_back(c->kspace ? (float)(b2 * k * k) : 0.0f);
            mx = std::max(mx, b2 * k * k);
        }
        smax += mx;
    }
    rc = dev_upload(&c->k2tab, hk2);
    if (rc) return rc;
    for (int d = 0; d < 3; ++d) c->O.k2[d] = c->k2tab + k2off[d];
    double fact = 1.0;
    for (int t = 0; t < 8; ++t) {
        if (t > 0) fact *= (2.0 * t) * (2.0 * t + 1.0);
        c->O.kc[t] = c->kspace ? (float)(((t & 1) ? -1.0 : 1.0) / fact * inv_n) : (t == 0 ? (float)inv_n : 0.0f);
    }
    // The stress phase's operator (3 inputs, 3 outputs each: every input's
    // blocks re-read the table) measured faster with the series, the velocity
    // phase's (6 inputs, 1-2 outputs) with the table.  PSTD_KAPPA=table or
    // series forces one way for both phases.
    c->kseries_ok = !c->kspace || smax <= 4.0;
    const char* km = std::getenv("PSTD_KAPPA");
    const std::string kmode = km ? km : "";
    c->O.kpoly[0] = (c->kseries_ok && kmode == "series") ? 1 : 0;
    c->O.kpoly[1] = (c->kseries_ok && kmode != "table") ? 1 : 0;
    {
        std::vector<ZDesc> zd(1);
        zd[0].ph[0] = phase_v();
        zd[0].ph[1] = phase_s();
        zd[0].ops = c->O;
        rc = dev_upload(&c->zdesc, zd);
        if (rc) return rc;
    }

    // receivers sorted by row
    std::vector<int4> re(c->n_rec);
    for (int r = 0; r < c->n_rec; ++r) {
        const int32_t* q = m->rec_ijk + 3 * r;
        re[r] = make_int4(q[0], q[1] + ny * q[2], r, 0);
    }
    std::stable_sort(re.begin(), re.end(), [](const int4& a, const int4& b) { return a.y < b.y; });
    std::vector<int> rp(c->g.nrows + 1, 0);
    for (auto& e : re) rp[e.y + 1]++;
    for (int r = 0; r < c->g.nrows; ++r) rp[r + 1] += rp[r];
    rc = dev_upload(&c->rec_ptr, rp);
    if (rc) return rc;
    rc = dev_upload(&c->rec_ent, re);
    if (rc) return rc;

    HIP_TRY(hipMalloc(&c->stepd, 2 * sizeof(int)));
    HIP_TRY(hipMemset(c->stepd, 0, 2 * sizeof(int)));
    HIP_TRY(hipMalloc(&c->flag, sizeof(int)));
    c->bytes = (long)(hm.size() * 4 + hp.size() * 4 + ht.size() * 8 + hs.size() * 8 + hk.size() * 4 +
                      rp.size() * 4 + re.size() * 16);
    return PSTD_OK;
}

Rec rec_of(const pstd3d_ctx* c) { return Rec{c->rec_ptr, c->rec_ent, c->n_rec}; }
Inj inj_of(const pstd3d_ctx* c) { return Inj{c->inj_ptr, c->inj_ent, c->wav, c->nt_w}; }

// one leapfrog step of every shot of a context
// Grid of the two update kernels (see update_block): (shots, row blocks) for
// a batch, (row blocks, 1) for one shot.
dim3 update_grid(const pstd3d_ctx* c)
{
    const int nrb = (c->g.nrows + c->xf.rows - 1) / c->xf.rows;
    return c->g.shot_fast ? dim3(c->n_shots, nrb) : dim3(nrb, c->n_shots);
}

// Step n reads the step counter word n & 1 and the velocity kernel writes n + 1
// into the other word.
void enqueue_step(pstd3d_ctx* c, hipStream_t st, float* traces, int n0, int ldt, int parity)
{
    const int* cur = c->stepd + parity;
    int* nxt = c->stepd + (parity ^ 1);
    const Geo& g = c->g;
    const int S = c->n_shots;
    const dim3 gx = update_grid(c);
    const int tyn = (g.nxm + c->yf.tile - 1) / c->yf.tile + g.has_nyq;
    const int tzn = (g.nxm + c->zf.tile - 1) / c->zf.tile + g.has_nyq;
    const int fpb = c->zfpb;
    long e;
    // V phase
    e = c->ev_begin(PSTD_K_YFWD_S, st);
    c->yf.fwd(dim3(tyn, g.nz, S * 6), st, g, c->twy, c->spec, 0, 6);
    c->ev_end(e, st);
    e = c->ev_begin(PSTD_K_ZOP_V, st);
    c->zf.op(dim3(tzn, g.ny, S * ((6 + fpb - 1) / fpb)), st, g, c->twz, c->spec, 0, c->zdesc, 0, fpb);
    c->ev_end(e, st);
    e = c->ev_begin(PSTD_K_YINV_V, st);
    c->yf.inv(dim3(tyn, g.nz, S * 9), st, g, c->twy, c->spec, 9, 9);
    c->ev_end(e, st);
    e = c->ev_begin(PSTD_K_VEL, st);
    c->vel.fn(gx, st, g, c->M, c->P, c->twx, c->fields, c->spec, rec_of(c), traces, cur, nxt, n0, ldt);
    c->ev_end(e, st);
    // S phase
    e = c->ev_begin(PSTD_K_YFWD_V, st);
    c->yf.fwd(dim3(tyn, g.nz, S * 3), st, g, c->twy, c->spec, 6, 3);
    c->ev_end(e, st);
    e = c->ev_begin(PSTD_K_ZOP_S, st);
    c->zf.op(dim3(tzn, g.ny, S * ((3 + fpb - 1) / fpb)), st, g, c->twz, c->spec, 6, c->zdesc, 1, fpb);
    c->ev_end(e, st);
    e = c->ev_begin(PSTD_K_YINV_S, st);
    c->yf.inv(dim3(tyn, g.nz, S * 9), st, g, c->twy, c->spec, 9, 9);
    c->ev_end(e, st);
    e = c->ev_begin(PSTD_K_STR, st);
    c->str_fn(c->str)(gx, st, g, c->M, c->P, c->twx, c->fields, c->spec, rec_of(c), inj_of(c), traces, cur, n0,
                      ldt);
    c->ev_end(e, st);
}

bool len_ok(int n)
{
    XFns a;
    YFns y[MAX_VARIANTS];
    ZFns z[MAX_VARIANTS];
    return x_fns(n, &a) && y_variants(n, y) > 0 && z_variants(n, z) > 0;
}

// variant used before (or without) tuning: tile 16 and 256 threads where
// built, else the first
int default_variant(const pstd3d_ctx* c, int k)
{
    const int want = (k == PSTD_TUNE_Y || k == PSTD_TUNE_Z) ? 16 : k == PSTD_TUNE_ZF ? 1 : 256;
    for (int i = 0; i < c->nvar[k]; ++i)
        if (c->knob_value(k, i) == want) return i;
    return 0;
}

// Autotuner.  Every built variant of every knob runs on this context's own
// state, one warm-up and three timed launches each (HIP events): the y
// inverse of the 9 derivative spectra, the z operator of the velocity phase,
// and the two update kernels with no receivers and no sources; the fastest
// of each knob is kept.  Fields and spectra are overwritten: it runs only
// where the state is cleared afterwards.
int autotune(pstd3d_ctx* c)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int* zero = nullptr;
    auto cleanup = [&]() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)hipFree(zero);
    };
    const Geo& g = c->g;
    const int S = c->n_shots;
    hipError_t he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    if (he == hipSuccess) he = hipMalloc(&zero, (size_t)S * (g.nrows + 1) * sizeof(int));
    if (he == hipSuccess) he = hipMemset(zero, 0, (size_t)S * (g.nrows + 1) * sizeof(int));
    if (he != hipSuccess) {
        cleanup();
        return fail(PSTD_EDEVICE, std::string("autotune setup: ") + hipGetErrorString(he));
    }
    const Rec norec{zero, c->rec_ent, 0};
    const Inj noinj{zero, c->inj_ent, c->wav, 0};
    auto timed = [&](auto&& launch, float* us) -> hipError_t {
        launch();
        hipError_t e = hipEventRecord(e0, nullptr);
        for (int r = 0; r < 3 && e == hipSuccess; ++r) launch();
        if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipGetLastError();
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        *us = ms * 1000.f / 3.f;
        return e;
    };
    const dim3 gx = update_grid(c);
    const int order[PSTD_TUNE_COUNT] = {PSTD_TUNE_Y, PSTD_TUNE_Z, PSTD_TUNE_ZT, PSTD_TUNE_ZF, PSTD_TUNE_VEL,
                                        PSTD_TUNE_STR};
    for (int kk = 0; kk < PSTD_TUNE_COUNT; ++kk) {
        const int k = order[kk];
        int best = -1;
        for (int i = 0; i < c->nvar[k]; ++i) {
            c->tune_us[k][i] = 0.f;
            if (c->force[k] && c->knob_value(k, i) != c->force[k]) continue;
            hipError_t e = hipSuccess;
            if (k == PSTD_TUNE_Y) {
                const YFns v = c->yv[i];
                const int tyn = (g.nxm + v.tile - 1) / v.tile + g.has_nyq;
                e = timed([&] { v.inv(dim3(tyn, g.nz, S * 9), nullptr, g, c->twy, c->spec, 9, 9); }, &c->tune_us[k][i]);
            } else if (k == PSTD_TUNE_Z || k == PSTD_TUNE_ZT || k == PSTD_TUNE_ZF) {
                // the velocity phase's z operator; the other two z knobs at
                // their current choice (the tile knob is tuned first)
                const int tile = k == PSTD_TUNE_Z ? c->ztile[i] : c->ztile[c->sel[PSTD_TUNE_Z]];
                const int nt = k == PSTD_TUNE_ZT ? c->znt[i] : c->znt[c->sel[PSTD_TUNE_ZT]];
                const int fpb = k == PSTD_TUNE_ZF ? ZF_VALUES[i] : ZF_VALUES[c->sel[PSTD_TUNE_ZF]];
                const ZFns* zp = c->zvar(tile, nt);
                if (!zp && k == PSTD_TUNE_ZT) continue;          // no such variant at this tile
                const ZFns v = zp ? *zp : *c->zvar(tile, NT);
                const int tzn = (g.nxm + v.tile - 1) / v.tile + g.has_nyq;
                e = timed([&] { v.op(dim3(tzn, g.ny, S * ((6 + fpb - 1) / fpb)), nullptr, g, c->twz, c->spec, 0,
                                     c->zdesc, 0, fpb); },
                          &c->tune_us[k][i]);
            } else if (k == PSTD_TUNE_VEL) {
                const VelVar v = c->velv[i];
                e = timed([&] { v.fn(gx, nullptr, g, c->M, c->P, c->twx, c->fields, c->spec, norec, nullptr,
                                     c->stepd, c->stepd + 1, 0, 1); }, &c->tune_us[k][i]);
            } else {
                const StrVar v = c->strv[i];
                const StrFn fn = c->str_fn(v);
                e = timed([&] { fn(gx, nullptr, g, c->M, c->P, c->twx, c->fields, c->spec, norec, noinj, nullptr,
                                   c->stepd, 0, 1); }, &c->tune_us[k][i]);
            }
            if (e != hipSuccess) {
                cleanup();
                return fail(PSTD_EDEVICE, std::string("autotune: ") + hipGetErrorString(e));
            }
            if (best < 0 || c->tune_us[k][i] < c->tune_us[k][best]) best = i;
        }
        if (best < 0) {
            cleanup();
            return fail(PSTD_EUNSUPPORTED, "forced tuning value not built for this grid length");
        }
        c->sel[k] = best;
    }
    cleanup();
    c->apply();
    c->tuned = true;
    return PSTD_OK;
}

// In the undamped cells (inside P.flo .. P.fhi on every axis) sum each
// field's split parts into its first part and zero the others: the form the
// update kernels keep there.  fields: one shot's host state [24 + ...][n].
void collapse_undamped(const pstd3d_ctx* c, float* fields)
{
    const long n = (long)c->nx * c->ny * c->nz;
    // first part and part count of the nine fields: vx vy vz sxx syy szz sxy sxz syz
    const int first[9] = {0, 3, 6, 9, 12, 15, 18, 20, 22};
    const int cnt[9] = {3, 3, 3, 3, 3, 3, 2, 2, 2};
    for (int z = c->P.flo[2]; z <= c->P.fhi[2]; ++z)
        for (int y = c->P.flo[1]; y <= c->P.fhi[1]; ++y)
            for (int x = c->P.flo[0]; x <= c->P.fhi[0]; ++x) {
                const long cell = ((long)z * c->ny + y) * c->nx + x;
                for (int f = 0; f < 9; ++f) {
                    float sum = 0.f;
                    for (int k = 0; k < cnt[f]; ++k) sum += fields[(first[f] + k) * n + cell];
                    fields[first[f] * n + cell] = sum;
                    for (int k = 1; k < cnt[f]; ++k) fields[(first[f] + k) * n + cell] = 0.f;
                }
            }
}

// Recompute the x-transformed stress sums from the split fields.
void enqueue_restore_spectra(pstd3d_ctx* c, hipStream_t st)
{
    SumDesc sd{};
    sd.nf = 6;
    const int first[6] = {9, 12, 15, 18, 20, 22};
    const int cnt[6] = {3, 3, 3, 2, 2, 2};
    for (int f = 0; f < 6; ++f) {
        sd.first[f] = first[f];
        sd.cnt[f] = cnt[f];
    }
    const dim3 gx((c->g.nrows + c->xf.rows - 1) / c->xf.rows, c->n_shots);
    c->xf.xfwd(gx, st, c->g, c->twx, c->fields, c->g.fstride, c->spec, c->g.sstride, sd);
}

}  // namespace

// ===========================================================================
extern "C" {

const char* pstd3d_last_error(void) { return g_err.c_str(); }

int pstd3d_create(const pstd3d_model* m, const double d[3], double dt, const pstd3d_pml* pml, pstd3d_ctx** out)
{
    if (!m || !d || !pml || !out) return fail(PSTD_EINVAL, "null argument");
    *out = nullptr;
    const int nx = m->nx, ny = m->ny, nz = m->nz;
    if (nx < 2 || ny < 2 || nz < 2) return fail(PSTD_EINVAL, "grid must be at least 2 cells per axis");
    if (!m->vp || !m->vs || !m->rho) return fail(PSTD_EINVAL, "null model array");
    if (!(d[0] > 0) || !(d[1] > 0) || !(d[2] > 0) || !(dt > 0)) return fail(PSTD_EINVAL, "spacing and dt must be > 0");
    if (pml->thickness < 0 || 2 * pml->thickness > std::min(nx, std::min(ny, nz)) || !(pml->A >= 0) ||
        !(pml->mratio >= 0 && pml->mratio <= 1))
        return fail(PSTD_EINVAL, "bad PML thickness, strength or multi-axial ratio");
    if (!len_ok(nx) || !len_ok(ny) || !len_ok(nz))
        return fail(PSTD_EUNSUPPORTED, "grid length not built (lengths factor into 2, 3, 5; see PSTD_LENGTHS)");
    if (m->n_rec < 0 || (m->n_rec > 0 && !m->rec_ijk)) return fail(PSTD_EINVAL, "bad receivers");
    const long n = (long)nx * ny * nz;
    double cmax = 0.0;
    for (long q = 0; q < n; ++q) {
        const double vp = m->vp[q], vs = m->vs[q], rho = m->rho[q];
        if (!std::isfinite(vp) || !std::isfinite(vs) || !std::isfinite(rho) || !(vp > 0) || !(rho > 0) || !(vs >= 0))
            return fail(PSTD_EINVAL, "model value out of range at cell " + std::to_string(q));
        if (3.0 * vp * vp <= 4.0 * vs * vs) return fail(PSTD_EINVAL, "non-positive bulk modulus at cell " + std::to_string(q));
        cmax = std::max(cmax, vp);
    }
    for (int r = 0; r < m->n_rec; ++r) {
        const int32_t* q = m->rec_ijk + 3 * r;
        if (q[0] < 0 || q[0] >= nx || q[1] < 0 || q[1] >= ny || q[2] < 0 || q[2] >= nz)
            return fail(PSTD_EINVAL, "receiver " + std::to_string(r) + " outside the grid");
    }
    const double c_ref = m->c_ref > 0 ? m->c_ref : cmax;
    const double sh = std::sqrt(1 / (d[0] * d[0]) + 1 / (d[1] * d[1]) + 1 / (d[2] * d[2]));
    if (!m->kspace) {
        if (cmax * dt * sh > 2.0 / M_PI) return fail(PSTD_EUNSTABLE, "CFL: c_max dt sqrt(sum 1/h^2) exceeds 2/pi");
    } else if (c_ref < cmax) {
        const double arg = c_ref * M_PI * sh * dt / 2;
        const double smax = arg >= M_PI / 2 ? 1.0 : std::sin(arg);
        if (cmax / c_ref * smax > 1.0) return fail(PSTD_EUNSTABLE, "k-space scheme unstable: c_ref below c_max");
    }
    auto* c = new (std::nothrow) pstd3d_ctx();
    if (!c) return fail(PSTD_ENOMEM, "host allocation");
    c->nx = nx;
    c->ny = ny;
    c->nz = nz;
    for (int a = 0; a < 3; ++a) c->h[a] = d[a];
    c->dt = dt;
    c->c_ref = c_ref;
    c->cmax = cmax;
    c->pml = pml->thickness;
    c->pml_A = pml->A;
    c->pml_p = pml->mratio;
    c->kspace = m->kspace ? 1 : 0;
    c->n_rec = m->n_rec;
    (void)hipGetDevice(&c->device);
    c->nvar[PSTD_TUNE_Y] = y_variants(ny, c->yv);
    c->nzv = z_variants(nz, c->zv);
    for (int i = 0; i < c->nzv; ++i) {
        bool seen_t = false, seen_n = false;
        for (int j = 0; j < c->nvar[PSTD_TUNE_Z]; ++j) seen_t = seen_t || c->ztile[j] == c->zv[i].tile;
        for (int j = 0; j < c->nvar[PSTD_TUNE_ZT]; ++j) seen_n = seen_n || c->znt[j] == c->zv[i].nt;
        if (!seen_t) c->ztile[c->nvar[PSTD_TUNE_Z]++] = c->zv[i].tile;
        if (!seen_n) c->znt[c->nvar[PSTD_TUNE_ZT]++] = c->zv[i].nt;
    }
    c->nvar[PSTD_TUNE_ZF] = 2;
    x_fns(nx, &c->xf, c->velv, c->strv, &c->nvar[PSTD_TUNE_VEL]);
    c->nvar[PSTD_TUNE_STR] = c->nvar[PSTD_TUNE_VEL];
    for (int k = 0; k < PSTD_TUNE_COUNT; ++k) c->sel[k] = default_variant(c, k);
    c->apply();
    Geo& g = c->g;
    g.nx = nx;
    g.ny = ny;
    g.nz = nz;
    g.nxh = nx / 2 + 1;
    g.has_nyq = nx % 2 == 0;
    g.nxm = g.has_nyq ? nx / 2 : g.nxh;
    g.ldx = (g.nxm + 15) / 16 * 16;
    g.nrows = ny * nz;
    g.n = n;
    g.nqoff = (long)nz * ny * g.ldx;
    // Nyquist plane after the main block; spectra start on 256-byte boundaries
    g.nspec = (g.nqoff + (g.has_nyq ? (long)nz * ny : 0) + 31) / 32 * 32;
    g.fstride = 24 * n;
    g.sstride = 18 * g.nspec;
    int rc = build_model(c, m);
    if (rc) {
        delete c;
        return rc;
    }
    *out = c;
    return PSTD_OK;
}

int pstd3d_set_sources(pstd3d_ctx* c, int n_shots, const int32_t* shot_ofs, const int32_t* src_ijk, const double* m6,
                       const double* wavelet, int nt_w)
{
    if (!c || n_shots < 1 || !shot_ofs || nt_w < 0) return fail(PSTD_EINVAL, "bad arguments");
    if (shot_ofs[0] != 0) return fail(PSTD_EINVAL, "shot_ofs[0] must be 0");
    for (int s = 0; s < n_shots; ++s)
        if (shot_ofs[s + 1] < shot_ofs[s]) return fail(PSTD_EINVAL, "shot_ofs must be non-decreasing");
    const int nsrc = shot_ofs[n_shots];
    if (nsrc > 0 && (!src_ijk || !m6 || (nt_w > 0 && !wavelet))) return fail(PSTD_EINVAL, "null source arrays");
    const int nx = c->nx, ny = c->ny, nz = c->nz;
    for (int q = 0; q < nsrc; ++q) {
        const int32_t* p = src_ijk + 3 * q;
        if (p[0] < 0 || p[0] >= nx || p[1] < 0 || p[1] >= ny || p[2] < 0 || p[2] >= nz)
            return fail(PSTD_EINVAL, "source " + std::to_string(q) + " outside the grid");
        for (int t = 0; t < 6; ++t)
            if (!std::isfinite(m6[6 * q + t])) return fail(PSTD_EINVAL, "non-finite moment tensor");
    }
    HIP_TRY(hipSetDevice(c->device));
    // injection entries per shot: {x, split part, coef, wavelet row}
    const double dV = c->h[0] * c->h[1] * c->h[2];
    const int nrows = c->g.nrows;
    std::vector<int> ptr((size_t)n_shots * (nrows + 1), 0);
    std::vector<int4> ent;
    static const int pair_axes[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    for (int s = 0; s < n_shots; ++s) {
        std::vector<std::pair<long, int4>> es;   // (row, entry)
        const int N[3] = {nx, ny, nz};
        // point source of moment weight * M at cell p: normal components split
        // 1/3 over their split parts, shear components 1/4 on the 4 shear nodes
        // around the centre, 1/2 on each of their two split parts
        auto point = [&](const int* p, const double* M, double weight, int q) {
            for (int cc = 0; cc < 3; ++cc) {
                if (M[cc] == 0.0) continue;
                const float coef = (float)(-c->dt * weight * M[cc] / dV / 3.0);
                for (int d = 0; d < 3; ++d) {
                    int4 e = make_int4(p[0], 3 * cc + d, __builtin_bit_cast(int, coef), q);
                    es.push_back({(long)p[1] + (long)ny * p[2], e});
                }
            }
            for (int pr = 0; pr < 3; ++pr) {
                if (M[3 + pr] == 0.0) continue;
                const float coef = (float)(-c->dt * weight * M[3 + pr] / dV / 8.0);
                const int a0 = pair_axes[pr][0], a1 = pair_axes[pr][1];
                for (int o0 = -1; o0 <= 0; ++o0)
                    for (int o1 = -1; o1 <= 0; ++o1) {
                        int ix[3] = {p[0], p[1], p[2]};
                        ix[a0] = (ix[a0] + o0 + N[a0]) % N[a0];
                        ix[a1] = (ix[a1] + o1 + N[a1]) % N[a1];
                        for (int t = 0; t < 2; ++t) {
                            int4 e = make_int4(ix[0], 9 + 2 * pr + t, __builtin_bit_cast(int, coef), q);
                            es.push_back({(long)ix[1] + (long)ny * ix[2], e});
                        }
                    }
            }
        };
        // Blackman window over [-pi/h, pi/h] on each axis, W(k) = a0 + a1 cos(k h)
        // + a2 cos(2 k h) with (a0, a1, a2) = (0.42, 0.5, 0.08): cos(k h) shifts
        // by one cell, so the smoothed delta is the separable stencil
        // (a2/2, a1/2, a0, a1/2, a2/2) on every axis, periodic at the edges
        const double a0 = 0.42, a1 = 0.5, a2 = 0.08;
        const double st[5] = {a2 / 2, a1 / 2, a0, a1 / 2, a2 / 2};
        for (int q = shot_ofs[s]; q < shot_ofs[s + 1]; ++q) {
            const int32_t* p = src_ijk + 3 * q;
            const double* M = m6 + 6 * q;
            if (!c->smooth) {
                point(p, M, 1.0, q);
                continue;
            }
            for (int dz = -2; dz <= 2; ++dz)
                for (int dy = -2; dy <= 2; ++dy)
                    for (int dx = -2; dx <= 2; ++dx) {
                        const int pp[3] = {((p[0] + dx) % nx + nx) % nx, ((p[1] + dy) % ny + ny) % ny,
                                           ((p[2] + dz) % nz + nz) % nz};
                        point(pp, M, st[dx + 2] * st[dy + 2] * st[dz + 2], q);
                    }
        }
        std::stable_sort(es.begin(), es.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
        int* sp = &ptr[(size_t)s * (nrows + 1)];
        const int base = (int)ent.size();
        for (auto& e : es) sp[e.first + 1]++;
        sp[0] = base;
        for (int r = 0; r < nrows; ++r) sp[r + 1] += sp[r];
        for (auto& e : es) ent.push_back(e.second);
    }
    std::vector<float> w((size_t)nsrc * nt_w);
    for (size_t i = 0; i < w.size(); ++i) w[i] = (float)wavelet[i];

    c->release_shots();
    {
        int ymax = 65535;
        (void)hipDeviceGetAttribute(&ymax, hipDeviceAttributeMaxGridDimY, c->device);
        const int nrb = (c->g.nrows + c->xf.rows - 1) / c->xf.rows;
        c->g.shot_fast = (n_shots > 1 && nrb <= ymax) ? 1 : 0;
    }
    const size_t fbytes = (size_t)n_shots * c->g.fstride * sizeof(float);
    const size_t sbytes = (size_t)n_shots * c->g.sstride * sizeof(float2);
    if (c->ws) {
        const size_t need = state_bytes(c, n_shots);
        if ((long)need > c->ws_bytes)
            return fail(PSTD_EINVAL, "workspace of " + std::to_string(c->ws_bytes) + " bytes is below the " +
                                         std::to_string(need) + " the shots need (pstd3d_workspace_size)");
        c->fields = (float*)c->ws;
        c->spec = (float2*)(c->ws + spec_offset(fbytes));
        c->own_state = false;
    } else {
        HIP_TRY(hipMalloc(&c->fields, fbytes));
        HIP_TRY(hipMalloc(&c->spec, sbytes));
    }
    c->n_shots = n_shots;
    HIP_TRY(hipMemset(c->fields, 0, fbytes));
    HIP_TRY(hipMemset(c->spec, 0, sbytes));
    if (!c->tuned) {
        int trc = autotune(c);
        if (trc) {
            c->release_shots();
            return trc;
        }
        HIP_TRY(hipMemset(c->fields, 0, fbytes));
        HIP_TRY(hipMemset(c->spec, 0, sbytes));
    }
    int rc = dev_upload(&c->inj_ptr, ptr);
    if (rc) return rc;
    rc = dev_upload(&c->inj_ent, ent);
    if (rc) return rc;
    rc = dev_upload(&c->wav, w);
    if (rc) return rc;
    c->nt_w = nt_w;
    c->n_shots = n_shots;
    c->step = 0;
    HIP_TRY(hipMemset(c->stepd, 0, 2 * sizeof(int)));
    HIP_TRY(hipDeviceSynchronize());
    return PSTD_OK;
}

static int check_traces(pstd3d_ctx* c, const float* traces, long count, hipStream_t st)
{
    HIP_TRY(hipMemsetAsync(c->flag, 0, sizeof(int), st));
    if (count > 0) hipLaunchKernelGGL(k_check_finite, dim3(256), dim3(256), 0, st, traces, count, c->flag);
    int h = 0;
    HIP_TRY(hipMemcpyAsync(&h, c->flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (h) return fail(PSTD_EUNSTABLE, "non-finite value in the receiver traces");
    return PSTD_OK;
}

// HIP graph of two consecutive steps of several contexts: each context's two
// steps are captured on its own stream branch (forked from and joined into a
// private origin stream), so independent models run concurrently.
static int capture_pair(pstd3d_ctx* const* ctxs, int n, float* const* traces, const int* n0, int ldt,
                        hipGraphExec_t* out)
{
    hipStream_t origin = nullptr;
    std::vector<hipStream_t> br(n, nullptr);
    std::vector<hipEvent_t> join(n, nullptr);
    hipEvent_t fork = nullptr;
    hipGraph_t graph = nullptr;
    int rc = PSTD_OK;
    auto cleanup = [&]() {
        if (graph) (void)hipGraphDestroy(graph);
        for (auto e : join)
            if (e) (void)hipEventDestroy(e);
        if (fork) (void)hipEventDestroy(fork);
        for (auto s : br)
            if (s) (void)hipStreamDestroy(s);
        if (origin) (void)hipStreamDestroy(origin);
    };
#define CAP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) {                                                          \
            rc = fail(PSTD_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));  \
            cleanup();                                                                   \
            return rc;                                                                   \
        }                                                                                \
    } while (0)
    CAP_TRY(hipStreamCreateWithFlags(&origin, hipStreamNonBlocking));
    CAP_TRY(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
    for (int i = 0; i < n; ++i) {
        CAP_TRY(hipStreamCreateWithFlags(&br[i], hipStreamNonBlocking));
        CAP_TRY(hipEventCreateWithFlags(&join[i], hipEventDisableTiming));
    }
    CAP_TRY(hipStreamBeginCapture(origin, hipStreamCaptureModeThreadLocal));
    hipError_t ce = hipEventRecord(fork, origin);
    for (int i = 0; i < n && ce == hipSuccess; ++i) {
        ce = hipStreamWaitEvent(br[i], fork, 0);
        for (int s = 0; s < 2 && ce == hipSuccess; ++s) enqueue_step(ctxs[i], br[i], traces[i], n0[i], ldt, (n0[i] + s) & 1);
        if (ce == hipSuccess) ce = hipGetLastError();
        if (ce == hipSuccess) ce = hipEventRecord(join[i], br[i]);
        if (ce == hipSuccess) ce = hipStreamWaitEvent(origin, join[i], 0);
    }
    hipError_t ee = hipStreamEndCapture(origin, &graph);
    if (ce != hipSuccess || ee != hipSuccess) {
        rc = fail(PSTD_EDEVICE, std::string("graph capture: ") + hipGetErrorString(ce != hipSuccess ? ce : ee));
        cleanup();
        return rc;
    }
    CAP_TRY(hipGraphInstantiate(out, graph, nullptr, nullptr, 0));
    cleanup();
    return PSTD_OK;
#undef CAP_TRY
}

static bool graphs_enabled()
{
    const char* e = std::getenv("PSTD_GRAPH");
    return !(e && e[0] == '0');
}

// Advance contexts by nt steps: pairs of steps replay one captured graph,
// an odd last step (and runs with event timing) go out eagerly.
static int advance(pstd3d_ctx* const* ctxs, int n, int nt, float* const* traces, hipStream_t st)
{
    std::vector<int> n0(n);
    bool prof = false;
    for (int i = 0; i < n; ++i) {
        n0[i] = (int)ctxs[i]->step;
        prof = prof || ctxs[i]->prof;
    }
    int done = 0;
    if (!prof && graphs_enabled() && nt >= 4) {
        hipGraphExec_t ex = nullptr;
        int rc = capture_pair(ctxs, n, traces, n0.data(), nt, &ex);
        if (rc) return rc;
        for (; done + 2 <= nt; done += 2) {
            hipError_t e = hipGraphLaunch(ex, st);
            if (e != hipSuccess) {
                (void)hipGraphExecDestroy(ex);
                return fail(PSTD_EDEVICE, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
            }
        }
        HIP_TRY(hipStreamSynchronize(st));
        (void)hipGraphExecDestroy(ex);
    }
    for (; done < nt; ++done) {
        for (int i = 0; i < n; ++i) {
            pstd3d_ctx* c = ctxs[i];
            enqueue_step(c, st, traces[i], n0[i], nt, (n0[i] + done) & 1);
            if (c->prof && c->evused >= 4096) {
                HIP_TRY(hipStreamSynchronize(st));
                c->ev_collect();
            }
        }
    }
    HIP_TRY(hipGetLastError());
    for (int i = 0; i < n; ++i) ctxs[i]->step += nt;
    return PSTD_OK;
}

int pstd3d_run(pstd3d_ctx* c, int nt, float* traces_dev, void* hip_stream)
{
    if (!c || nt < 0) return fail(PSTD_EINVAL, "bad arguments");
    if (c->n_shots == 0) return fail(PSTD_EINVAL, "pstd3d_set_sources has not been called");
    if (nt > 0 && c->n_rec > 0 && !traces_dev) return fail(PSTD_EINVAL, "null trace buffer");
    if (c->step + nt > 2147483647L) return fail(PSTD_EINVAL, "step index overflow");
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)hip_stream;
    int rc = advance(&c, 1, nt, &traces_dev, st);
    if (rc) return rc;
    rc = check_traces(c, traces_dev, (long)c->n_shots * 4 * c->n_rec * nt, st);
    if (c->prof) c->ev_collect();
    return rc;
}

int pstd3d_run_many(pstd3d_ctx* const* ctxs, int n, int nt, float* const* traces, void* hip_stream)
{
    if (!ctxs || n < 1 || nt < 0 || !traces) return fail(PSTD_EINVAL, "bad arguments");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    for (int i = 0; i < n; ++i) {
        if (!ctxs[i] || ctxs[i]->n_shots == 0) return fail(PSTD_EINVAL, "context without shots");
        if (nt > 0 && ctxs[i]->n_rec > 0 && !traces[i]) return fail(PSTD_EINVAL, "null trace buffer");
        if (ctxs[i]->device != dev) return fail(PSTD_EINVAL, "contexts must live on the current device");
        if (ctxs[i]->step + nt > 2147483647L) return fail(PSTD_EINVAL, "step index overflow");
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return fail(PSTD_EINVAL, "a context appears twice");
    }
    hipStream_t st = (hipStream_t)hip_stream;
    int rc = advance(ctxs, n, nt, traces, st);
    if (rc) return rc;
    for (int i = 0; i < n; ++i) {
        rc = check_traces(ctxs[i], traces[i], (long)ctxs[i]->n_shots * 4 * ctxs[i]->n_rec * nt, st);
        if (ctxs[i]->prof) ctxs[i]->ev_collect();
        if (rc) return rc;
    }
    return PSTD_OK;
}

int pstd3d_reset(pstd3d_ctx* c, void* hip_stream)
{
    if (!c || c->n_shots == 0) return fail(PSTD_EINVAL, "no shots to reset");
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)hip_stream;
    HIP_TRY(hipMemsetAsync(c->fields, 0, (size_t)c->n_shots * c->g.fstride * sizeof(float), st));
    HIP_TRY(hipMemsetAsync(c->spec, 0, (size_t)c->n_shots * c->g.sstride * sizeof(float2), st));
    HIP_TRY(hipMemsetAsync(c->stepd, 0, 2 * sizeof(int), st));
    c->step = 0;
    return PSTD_OK;
}

int pstd3d_profile(pstd3d_ctx* c, int enable)
{
    if (!c) return fail(PSTD_EINVAL, "null context");
    c->prof = enable != 0;
    for (int k = 0; k < PSTD_K_COUNT; ++k) {
        c->prof_ms[k] = 0;
        c->prof_n[k] = 0;
    }
    c->evpend.clear();
    c->evused = 0;
    return PSTD_OK;
}

int pstd3d_profile_read(const pstd3d_ctx* c, int kind, double* total_ms, long* launches)
{
    if (!c || kind < 0 || kind >= PSTD_K_COUNT || !total_ms || !launches) return fail(PSTD_EINVAL, "bad arguments");
    *total_ms = c->prof_ms[kind];
    *launches = c->prof_n[kind];
    return PSTD_OK;
}

int pstd3d_get_state(pstd3d_ctx* c, int shot, float* fields_host)
{
    if (!c || !fields_host || shot < 0 || shot >= c->n_shots) return fail(PSTD_EINVAL, "bad arguments");
    HIP_TRY(hipSetDevice(c->device));
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(fields_host, c->fields + (size_t)shot * c->g.fstride, c->g.fstride * sizeof(float),
                      hipMemcpyDeviceToHost));
    return PSTD_OK;
}

int pstd3d_set_state(pstd3d_ctx* c, int shot, const float* fields_host, long step)
{
    if (!c || !fields_host || shot < 0 || shot >= c->n_shots || step < 0 || step > 2147483647L)
        return fail(PSTD_EINVAL, "bad arguments");
    HIP_TRY(hipSetDevice(c->device));
    HIP_TRY(hipDeviceSynchronize());
    // undamped cells keep each field's whole value in its first split part
    // (summed in a host copy: the caller's buffer is const)
    std::vector<float> st;
    try {
        st.assign(fields_host, fields_host + c->g.fstride);
    } catch (const std::bad_alloc&) {
        return fail(PSTD_ENOMEM, "pstd3d_set_state: host copy of the state");
    }
    collapse_undamped(c, st.data());
    HIP_TRY(hipMemcpy(c->fields + (size_t)shot * c->g.fstride, st.data(), c->g.fstride * sizeof(float),
                      hipMemcpyHostToDevice));
    enqueue_restore_spectra(c, nullptr);
    const int s32 = (int)step;
    HIP_TRY(hipMemcpy(c->stepd + (s32 & 1), &s32, sizeof(int), hipMemcpyHostToDevice));
    HIP_TRY(hipDeviceSynchronize());
    c->step = step;
    return PSTD_OK;
}

long pstd3d_step(const pstd3d_ctx* c) { return c ? c->step : -1; }

int pstd3d_undamped_range(const pstd3d_ctx* c, int lo[3], int hi[3])
{
    if (!c || !lo || !hi) return fail(PSTD_EINVAL, "bad arguments");
    for (int d = 0; d < 3; ++d) {
        lo[d] = c->P.flo[d];
        hi[d] = c->P.fhi[d];
    }
    return PSTD_OK;
}

int pstd3d_derivs(pstd3d_ctx* c, int phase, const float* in_dev, float* out_dev, void* hip_stream)
{
    if (!c || !in_dev || !out_dev || (phase != 0 && phase != 1)) return fail(PSTD_EINVAL, "bad arguments");
    if (c->n_shots == 0) return fail(PSTD_EINVAL, "pstd3d_set_sources has not been called");
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)hip_stream;
    const Geo& g = c->g;
    SumDesc sd{};
    sd.nf = phase == 0 ? 6 : 3;
    for (int f = 0; f < sd.nf; ++f) {
        sd.first[f] = f;
        sd.cnt[f] = 1;
    }
    const int in0 = phase == 0 ? 0 : 6;
    const dim3 gx((g.nrows + c->xf.rows - 1) / c->xf.rows, 1);
    const int tyn = (g.nxm + c->yf.tile - 1) / c->yf.tile + g.has_nyq;
    const int tzn = (g.nxm + c->zf.tile - 1) / c->zf.tile + g.has_nyq;
    // shot 0 scratch: spectra in0.. and the derivative block
    c->xf.xfwd(gx, st, g, c->twx, in_dev, 0, c->spec + in0 * g.nspec, 0, sd);
    c->yf.fwd(dim3(tyn, g.nz, sd.nf), st, g, c->twy, c->spec, in0, sd.nf);
    c->zf.op(dim3(tzn, g.ny, (sd.nf + c->zfpb - 1) / c->zfpb), st, g, c->twz, c->spec, in0, c->zdesc, phase,
             c->zfpb);
    c->yf.inv(dim3(tyn, g.nz, 9), st, g, c->twy, c->spec, 9, 9);
    c->xf.xinv(gx, st, g, c->twx, c->spec + 9 * g.nspec, out_dev);
    // the stress spectra are part of the state between steps: rebuild them
    enqueue_restore_spectra(c, st);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
    return PSTD_OK;
}

int pstd3d_set_source_smoothing(pstd3d_ctx* c, int window)
{
    if (!c || (window != PSTD_SMOOTH_NONE && window != PSTD_SMOOTH_BLACKMAN)) return fail(PSTD_EINVAL, "bad arguments");
    c->smooth = window;
    return PSTD_OK;
}

int pstd3d_set_viscosity(pstd3d_ctx* c, const double* chi, const double* eta)
{
    if (!c) return fail(PSTD_EINVAL, "null context");
    if (!chi != !eta) return fail(PSTD_EINVAL, "chi and eta must both be given or both be NULL");
    const int nx = c->nx, ny = c->ny, nz = c->nz;
    const long n = (long)nx * ny * nz;
    if (chi)
        for (long q = 0; q < n; ++q)
            if (!std::isfinite(chi[q]) || !std::isfinite(eta[q]) || chi[q] < 0 || eta[q] < 0)
                return fail(PSTD_EINVAL, "viscosities must be finite and >= 0");
    HIP_TRY(hipSetDevice(c->device));
    HIP_TRY(hipDeviceSynchronize());
    c->release_shots();
    c->step = 0;
    (void)hipFree(c->vmat);
    c->vmat = nullptr;
    c->M.chi = c->M.eta2 = nullptr;
    for (int p = 0; p < 3; ++p) c->M.etas[p] = nullptr;
    c->visc = chi != nullptr;
    c->g.fstride = (c->visc ? 33 : 24) * n;
    // the stress knob is timed again on the variant that runs, unless every knob is pinned
    bool pinned = true;
    for (int k = 0; k < PSTD_TUNE_COUNT; ++k) pinned = pinned && c->force[k] != 0;
    c->tuned = pinned;
    if (!c->visc) return PSTD_OK;
    auto at = [&](int i, int j, int k) { return (long)i + nx * ((long)j + (long)ny * k); };
    std::vector<float> hv(5 * n);
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const long q = at(i, j, k);
                const int ip = std::min(i + 1, nx - 1), jp = std::min(j + 1, ny - 1), kp = std::min(k + 1, nz - 1);
                hv[q] = (float)chi[q];
                hv[n + q] = (float)(2.0 * eta[q]);
                const long nb[3][4] = {{q, at(ip, j, k), at(i, jp, k), at(ip, jp, k)},
                                       {q, at(ip, j, k), at(i, j, kp), at(ip, j, kp)},
                                       {q, at(i, jp, k), at(i, j, kp), at(i, jp, kp)}};
                for (int p = 0; p < 3; ++p) {
                    double inv = 0.0;
                    bool zero = false;
                    for (int t = 0; t < 4; ++t) {
                        const double v = eta[nb[p][t]];
                        if (v == 0.0) zero = true;
                        else inv += 1.0 / v;
                    }
                    hv[(2 + p) * n + q] = zero ? 0.0f : (float)(4.0 / inv);
                }
            }
    const int rc = dev_upload(&c->vmat, hv);
    if (rc) {
        c->visc = false;
        c->g.fstride = 24 * n;
        return rc;
    }
    c->M.chi = c->vmat;
    c->M.eta2 = c->vmat + n;
    for (int p = 0; p < 3; ++p) c->M.etas[p] = c->vmat + (2 + p) * n;
    return PSTD_OK;
}

int pstd3d_state_fields(const pstd3d_ctx* c) { return c ? (c->visc ? 33 : 24) : PSTD_EINVAL; }

int pstd3d_set_tuning(pstd3d_ctx* c, const int value[PSTD_TUNE_COUNT])
{
    if (!c || !value) return fail(PSTD_EINVAL, "bad arguments");
    int idx[PSTD_TUNE_COUNT];
    bool all = true;
    for (int k = 0; k < PSTD_TUNE_COUNT; ++k) {
        if (value[k] < 0) return fail(PSTD_EINVAL, "negative tuning value");
        idx[k] = -1;
        if (value[k] == 0) {
            all = false;
            continue;
        }
        for (int i = 0; i < c->nvar[k]; ++i)
            if (c->knob_value(k, i) == value[k]) idx[k] = i;
        if (idx[k] < 0) return fail(PSTD_EUNSUPPORTED, "tuning value not built for this grid length");
    }
    if (idx[PSTD_TUNE_Z] >= 0 && idx[PSTD_TUNE_ZT] >= 0 && !c->zvar(value[PSTD_TUNE_Z], value[PSTD_TUNE_ZT]))
        return fail(PSTD_EUNSUPPORTED, "z threads per block not built for that z tile");
    for (int k = 0; k < PSTD_TUNE_COUNT; ++k) {
        c->force[k] = value[k];
        if (idx[k] >= 0) c->sel[k] = idx[k];
    }
    c->apply();
    c->tuned = all;
    return PSTD_OK;
}

int pstd3d_get_tuning(const pstd3d_ctx* c, int knob, int* chosen, int* values, float* us, int max)
{
    if (!c || knob < 0 || knob >= PSTD_TUNE_COUNT || max < 0 || (max > 0 && (!values || !us)))
        return fail(PSTD_EINVAL, "bad arguments");
    if (chosen) *chosen = c->knob_value(knob, c->sel[knob]);
    for (int i = 0; i < c->nvar[knob] && i < max; ++i) {
        values[i] = c->knob_value(knob, i);
        us[i] = c->tune_us[knob][i];
    }
    return c->nvar[knob];
}

int pstd3d_n_rec(const pstd3d_ctx* c) { return c ? c->n_rec : PSTD_EINVAL; }

long pstd3d_device_bytes(const pstd3d_ctx* c)
{
    if (!c) return 0;
    const long state = c->own_state ? (long)c->n_shots * (c->g.fstride * 4 + c->g.sstride * 8) : 0L;
    return c->bytes + (c->visc ? 20L * c->g.n : 0L) + state;
}

long pstd3d_workspace_size(const pstd3d_ctx* c, int n_shots)
{
    if (!c || n_shots < 1) return fail(PSTD_EINVAL, "bad arguments");
    return (long)state_bytes(c, n_shots);
}

int pstd3d_set_workspace(pstd3d_ctx* c, void* dev_ptr, long bytes)
{
    if (!c || (dev_ptr && bytes <= 0)) return fail(PSTD_EINVAL, "bad arguments");
    if (dev_ptr && ((uintptr_t)dev_ptr % 256) != 0) return fail(PSTD_EINVAL, "workspace must be 256-byte aligned");
    HIP_TRY(hipSetDevice(c->device));
    HIP_TRY(hipDeviceSynchronize());
    c->release_shots();
    c->step = 0;
    c->ws = (char*)dev_ptr;
    c->ws_bytes = dev_ptr ? bytes : 0;
    return PSTD_OK;
}

void pstd3d_destroy(pstd3d_ctx* c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    delete c;
}

}  // extern "C"
