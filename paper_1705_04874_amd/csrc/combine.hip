// seis_combine: superposition of single-event traces (Sec. IV).
//
// out[c][r][m] = sum_e amp[e] * x_e(m dt_out - t_origin[e] - t0[c]), with x_e
// the linear interpolation of trace src_idx[e] (zero outside its samples).
// The host sorts nothing: for each output time tile it lists, in event order,
// the events whose shifted support can touch the tile (a superset is harmless:
// an event outside its support adds exactly 0.0).  Each thread then
// accumulates SPT consecutive output samples of one (component, receiver) in
// double precision, event by event, and rounds once to float.  The input
// position of its first sample costs one division per event, the others
// follow by steps of dt_out / dt_in, and an event that misses the thread's
// samples is skipped (most events of a tile miss most threads).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "pstd3d.h"

namespace {

constexpr int CT = 256;          // threads per block
constexpr int SPT = 8;           // output samples per thread
constexpr int TILE = CT * SPT;   // output samples per block

struct Ev {
    int src;
    double amp;
    double t;
};

__global__ __launch_bounds__(CT) void k_combine(const float* __restrict__ tr, int n_rec, int nt_in, double dt_in,
                                                double ratio, double t00, double t01, double t02, double t03,
                                                const int* __restrict__ tile_ptr, const int* __restrict__ tile_ev,
                                                const Ev* __restrict__ ev, int nt_out, double dt_out,
                                                float* __restrict__ out)
{
#pragma clang fp contract(off)
    const int tile = blockIdx.x;
    const int r = blockIdx.y;
    const int c = blockIdx.z;
    const double t0 = c == 0 ? t00 : c == 1 ? t01 : c == 2 ? t02 : t03;
    const int m0 = tile * TILE + threadIdx.x * SPT;
    double acc[SPT];
#pragma unroll
    for (int s = 0; s < SPT; ++s) acc[s] = 0.0;
    const int e0 = tile_ptr[tile], e1 = tile_ptr[tile + 1];
    for (int j = e0; j < e1; ++j) {
        const Ev E = ev[tile_ev[j]];
        // input position of this thread's first sample; the last one is
        // (SPT - 1) ratio further; nothing to add outside [-1, nt_in)
        const double u0 = ((double)m0 * dt_out - E.t - t0) / dt_in;
        if (u0 + (SPT - 1) * ratio < -1.0 || u0 >= (double)nt_in) continue;
        const float* __restrict__ x = tr + (((long)E.src * 4 + c) * n_rec + r) * nt_in;
#pragma unroll
        for (int s = 0; s < SPT; ++s) {
            const double u = u0 + (double)s * ratio;
            const double fl = floor(u);
            const long i0 = (long)fl;
            const double f = u - fl;
            const long ia = min(max(i0, 0L), (long)nt_in - 1), ib = min(max(i0 + 1, 0L), (long)nt_in - 1);
            const float xa = x[ia], xb = x[ib];
            const double x0 = (i0 >= 0 && i0 < nt_in) ? (double)xa : 0.0;
            const double x1 = (i0 + 1 >= 0 && i0 + 1 < nt_in) ? (double)xb : 0.0;
            acc[s] += E.amp * ((1.0 - f) * x0 + f * x1);
        }
    }
    float* __restrict__ o = out + ((long)c * n_rec + r) * nt_out;
#pragma unroll
    for (int s = 0; s < SPT; ++s)
        if (m0 + s < nt_out) o[m0 + s] = (float)acc[s];
}

thread_local std::string g_cerr;

}  // namespace

extern "C" int seis_combine(const float* tr, int n_src, int n_rec, int nt_in, double dt_in, const double t0[4], int n_ev,
                            const int32_t* src_idx, const double* amp, const double* t_origin, int nt_out,
                            double dt_out, float* out, void* hip_stream)
{
    if (n_src < 1 || n_rec < 0 || nt_in < 1 || nt_out < 0 || n_ev < 0 || !(dt_in > 0) || !(dt_out > 0) || !t0)
        return PSTD_EINVAL;
    if (n_rec == 0 || nt_out == 0) return PSTD_OK;
    if (!tr || !out || (n_ev > 0 && (!src_idx || !amp || !t_origin))) return PSTD_EINVAL;
    for (int e = 0; e < n_ev; ++e) {
        if (src_idx[e] < 0 || src_idx[e] >= n_src) return PSTD_EINVAL;
        if (!std::isfinite(amp[e]) || !std::isfinite(t_origin[e])) return PSTD_EINVAL;
    }
    for (int c = 0; c < 4; ++c)
        if (!std::isfinite(t0[c])) return PSTD_EINVAL;
    const int ntile = (nt_out + TILE - 1) / TILE;
    // per tile: events whose support [t_e + t0_c, t_e + t0_c + nt_in dt_in] meets the
    // tile's time span (widened by one input sample on each side, over all components)
    const double tmin0 = std::min(std::min(t0[0], t0[1]), std::min(t0[2], t0[3]));
    const double tmax0 = std::max(std::max(t0[0], t0[1]), std::max(t0[2], t0[3]));
    std::vector<int> ptr(ntile + 1, 0), list;
    std::vector<std::vector<int>> per(ntile);
    for (int e = 0; e < n_ev; ++e) {
        const double a = t_origin[e] + tmin0 - dt_in;
        const double b = t_origin[e] + tmax0 + (nt_in + 1) * dt_in;
        long first = (long)std::floor(a / dt_out) - 1, last = (long)std::ceil(b / dt_out) + 1;
        first = std::max(first, 0L);
        last = std::min(last, (long)nt_out - 1);
        if (last < first) continue;
        for (long t = first / TILE; t <= last / TILE; ++t) per[t].push_back(e);
    }
    for (int t = 0; t < ntile; ++t) {
        ptr[t + 1] = ptr[t] + (int)per[t].size();
        list.insert(list.end(), per[t].begin(), per[t].end());
    }
    std::vector<Ev> evs(n_ev);
    for (int e = 0; e < n_ev; ++e) evs[e] = Ev{src_idx[e], amp[e], t_origin[e]};
    int *dptr = nullptr, *dlist = nullptr;
    Ev* dev = nullptr;
    auto cleanup = [&]() {
        (void)hipFree(dptr);
        (void)hipFree(dlist);
        (void)hipFree(dev);
    };
    if (hipMalloc(&dptr, ptr.size() * sizeof(int)) != hipSuccess ||
        hipMalloc(&dlist, std::max<size_t>(1, list.size()) * sizeof(int)) != hipSuccess ||
        hipMalloc(&dev, std::max<size_t>(1, evs.size()) * sizeof(Ev)) != hipSuccess) {
        cleanup();
        return PSTD_ENOMEM;
    }
    hipStream_t st = (hipStream_t)hip_stream;
    bool ok = hipMemcpyAsync(dptr, ptr.data(), ptr.size() * sizeof(int), hipMemcpyHostToDevice, st) == hipSuccess;
    if (!list.empty())
        ok = ok && hipMemcpyAsync(dlist, list.data(), list.size() * sizeof(int), hipMemcpyHostToDevice, st) == hipSuccess;
    if (!evs.empty())
        ok = ok && hipMemcpyAsync(dev, evs.data(), evs.size() * sizeof(Ev), hipMemcpyHostToDevice, st) == hipSuccess;
    if (ok) {
        hipLaunchKernelGGL(k_combine, dim3(ntile, n_rec, 4), dim3(CT), 0, st, tr, n_rec, nt_in, dt_in,
                           dt_out / dt_in, t0[0], t0[1], t0[2], t0[3], dptr, dlist, dev, nt_out, dt_out, out);
        ok = hipGetLastError() == hipSuccess && hipStreamSynchronize(st) == hipSuccess;
    }
    cleanup();
    return ok ? PSTD_OK : PSTD_EDEVICE;
}
