// seis_combine: superposition of single-event traces (Sec. IV).
//
// out[c][r][m] = sum_e amp[e] * x_e(m dt_out - t_origin[e] - t0[c]), with x_e
// the linear interpolation of trace src_idx[e] (zero outside its samples).
//
// One block owns one output row (component c, receiver r) over a segment of
// the record and keeps that segment's accumulators in LDS in double precision.
// The events that can touch the segment are grouped by source on the host
// (sources ascending, event order within a source), so the block stages each
// source's input row in LDS once and applies all of that source's events from
// there: every input trace is read from HBM once per segment, and the record
// is written once.  Within an event, output sample m belongs to thread
// m mod NT, so no two threads touch one accumulator and no barrier separates
// the events of a source.
//
// The input position of a sample is u = m (dt_out / dt_in) - (t_origin + t0)/dt_in,
// one fused multiply-add in double; the interpolation weight f = u - floor(u)
// and the two samples around it follow.  The lerp is continuous in u, so the
// rounding of u (a few ulps against the direct quotient) moves the result by
// the same few ulps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "pstd3d.h"

namespace {

constexpr int CT = 1024;           // threads per block
constexpr int SEG_MAX = 12288;     // output samples per segment (96 KiB of double accumulators)
constexpr int STG = 4096;          // input samples staged per chunk (plus one before and one after)

// per-segment work list: groups of events sharing a source
struct Grp {
    int src;
    int e0, e1;    // events [e0, e1) of the segment's event array
    int pad;
};
struct Ev {
    double amp;
    double t;      // origin time
};

// Host-side lists of one call: per segment the source groups, per group its
// events.  The arrays go to the device back to back (offsets in bytes).
struct Plan {
    int nseg = 0, seg_len = 0;
    std::vector<int> seg_ptr;    // [nseg + 1] into grp
    std::vector<Grp> grp;
    std::vector<Ev> ev;
    size_t off_ptr = 0, off_grp = 0, off_ev = 0, bytes = 0;
};

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Build the work lists.  An event can touch output sample m only if
// u(m) lies in (-1, nt_in); the sample range of that is widened by one sample
// on each side (and over all four components' t0): the kernel decides each
// sample exactly, a superset only costs a skipped iteration.
void make_plan(Plan& p, int n_ev, const int32_t* src_idx, const double* amp, const double* t_origin,
               const double t0[4], int nt_in, double dt_in, int nt_out, double dt_out)
{
    p.nseg = (nt_out + SEG_MAX - 1) / SEG_MAX;
    p.seg_len = (nt_out + p.nseg - 1) / p.nseg;
    const double tmin0 = std::min(std::min(t0[0], t0[1]), std::min(t0[2], t0[3]));
    const double tmax0 = std::max(std::max(t0[0], t0[1]), std::max(t0[2], t0[3]));
    // events of each segment in event order, then stably grouped by source
    std::vector<std::vector<int>> per(p.nseg);
    for (int e = 0; e < n_ev; ++e) {
        const double a = t_origin[e] + tmin0 - dt_in;
        const double b = t_origin[e] + tmax0 + nt_in * dt_in;
        const double fd = std::max(0.0, std::floor(a / dt_out) - 1.0);
        const double ld = std::min((double)nt_out - 1.0, std::ceil(b / dt_out) + 1.0);
        if (!(ld >= fd)) continue;
        const long first = (long)fd, last = (long)ld;
        for (long s = first / p.seg_len; s <= last / p.seg_len; ++s) per[s].push_back(e);
    }
    p.seg_ptr.assign(p.nseg + 1, 0);
    p.grp.clear();
    p.ev.clear();
    for (int s = 0; s < p.nseg; ++s) {
        std::vector<int>& L = per[s];
        std::stable_sort(L.begin(), L.end(), [&](int a, int b) { return src_idx[a] < src_idx[b]; });
        for (size_t i = 0; i < L.size();) {
            size_t j = i;
            while (j < L.size() && src_idx[L[j]] == src_idx[L[i]]) ++j;
            Grp g{src_idx[L[i]], (int)p.ev.size(), 0, 0};
            for (size_t k = i; k < j; ++k) p.ev.push_back(Ev{amp[L[k]], t_origin[L[k]]});
            g.e1 = (int)p.ev.size();
            p.grp.push_back(g);
            i = j;
        }
        p.seg_ptr[s + 1] = (int)p.grp.size();
    }
    p.off_ptr = 0;
    p.off_grp = align256(p.seg_ptr.size() * sizeof(int));
    p.off_ev = p.off_grp + align256(std::max<size_t>(1, p.grp.size()) * sizeof(Grp));
    p.bytes = p.off_ev + align256(std::max<size_t>(1, p.ev.size()) * sizeof(Ev));
}

__global__ __launch_bounds__(CT) void k_combine(const float* __restrict__ tr, int n_rec, int nt_in, double dt_in,
                                                double ratio, double t00, double t01, double t02, double t03,
                                                const char* __restrict__ plan, long off_grp, long off_ev,
                                                int seg_len, int nt_out, float* __restrict__ out)
{
#pragma clang fp contract(off)
    __shared__ double acc[SEG_MAX];
    __shared__ float stg[STG + 2];
    const int seg = blockIdx.x;
    const int r = blockIdx.y;
    const int c = blockIdx.z;
    const int tid = threadIdx.x;
    const double t0 = c == 0 ? t00 : c == 1 ? t01 : c == 2 ? t02 : t03;
    const int s0 = seg * seg_len;
    const int s1 = min(s0 + seg_len, nt_out);
    const int* __restrict__ seg_ptr = reinterpret_cast<const int*>(plan);
    const Grp* __restrict__ grp = reinterpret_cast<const Grp*>(plan + off_grp);
    const Ev* __restrict__ ev = reinterpret_cast<const Ev*>(plan + off_ev);
    for (int i = tid; i < s1 - s0; i += CT) acc[i] = 0.0;
    const int g0 = seg_ptr[seg], g1 = seg_ptr[seg + 1];
    // chunks of the input axis: chunk q owns the samples whose left neighbour
    // i0 = floor(u) lies in [a, b), a = q STG - 1, b = a + STG (the last chunk
    // ends at nt_in), and stages x[a .. b] (zero outside the trace)
    const int nchunk = (nt_in + 1 + STG - 1) / STG;
    for (int g = g0; g < g1; ++g) {
        const Grp G = grp[g];
        const float* __restrict__ x = tr + (((long)G.src * 4 + c) * n_rec + r) * nt_in;
        for (int q = 0; q < nchunk; ++q) {
            const int a = q * STG - 1;
            const int b = q == nchunk - 1 ? nt_in : a + STG;
            __syncthreads();   // the previous chunk's readers are done
            for (int i = tid; i <= b - a; i += CT) {
                const int k = a + i;
                stg[i] = (k >= 0 && k < nt_in) ? x[k] : 0.0f;
            }
            __syncthreads();
            for (int e = G.e0; e < G.e1; ++e) {
                const Ev E = ev[e];
                const double be = (E.t + t0) / dt_in;
                // samples with u in [a, b), widened by one on each side (clamped
                // in double first: be may be far outside the record)
                const double lo = fmax((double)s0, floor(((double)a + be) / ratio) - 1.0);
                const double hi = fmin((double)s1, ceil(((double)b + be) / ratio) + 2.0);
                if (!(hi > lo)) continue;
                const long mlo = (long)lo, mhi = (long)hi;
                // sample m belongs to thread m mod CT in every event
                for (long m = mlo - (mlo % CT) + tid; m < mhi; m += CT) {
                    if (m < mlo) continue;
                    const double u = fma((double)m, ratio, -be);
                    const double fl = floor(u);
                    if (fl < (double)a || fl >= (double)b) continue;
                    const int i0 = (int)fl;
                    const double f = u - fl;
                    const double x0 = (double)stg[i0 - a];
                    const double x1 = (double)stg[i0 - a + 1];
                    acc[m - s0] += E.amp * (x0 + f * (x1 - x0));
                }
            }
        }
    }
    __syncthreads();
    float* __restrict__ o = out + ((long)c * n_rec + r) * nt_out;
    for (int i = tid; i < s1 - s0; i += CT) o[s0 + i] = (float)acc[i];
}

thread_local std::string g_cerr;

int cfail(int code, const std::string& msg)
{
    g_cerr = msg;
    return code;
}

int check_args(const float* tr, int n_src, int n_rec, int nt_in, double dt_in, const double t0[4], int n_ev,
               const int32_t* src_idx, const double* amp, const double* t_origin, int nt_out, double dt_out,
               float* out)
{
    if (n_src < 1 || n_rec < 0 || nt_in < 1 || nt_out < 0 || n_ev < 0 || !(dt_in > 0) || !(dt_out > 0) || !t0 ||
        !std::isfinite(dt_in) || !std::isfinite(dt_out))
        return cfail(PSTD_EINVAL, "seis_combine: bad sizes or sampling intervals");
    if (n_rec == 0 || nt_out == 0) return PSTD_OK;
    if (!tr || !out || (n_ev > 0 && (!src_idx || !amp || !t_origin)))
        return cfail(PSTD_EINVAL, "seis_combine: null pointer");
    for (int e = 0; e < n_ev; ++e) {
        if (src_idx[e] < 0 || src_idx[e] >= n_src) return cfail(PSTD_EINVAL, "seis_combine: source index out of range");
        if (!std::isfinite(amp[e]) || !std::isfinite(t_origin[e]))
            return cfail(PSTD_EINVAL, "seis_combine: non-finite amplitude or origin time");
    }
    for (int c = 0; c < 4; ++c)
        if (!std::isfinite(t0[c])) return cfail(PSTD_EINVAL, "seis_combine: non-finite t0");
    return PSTD_OK;
}

// upload the plan to dplan (device, p.bytes) on st and launch; the stream is
// synchronised before returning (the host lists are then free to go)
int launch(const Plan& p, char* dplan, const float* tr, int n_rec, int nt_in, double dt_in, const double t0[4],
           int nt_out, double dt_out, float* out, hipStream_t st)
{
    bool ok = hipMemcpyAsync(dplan + p.off_ptr, p.seg_ptr.data(), p.seg_ptr.size() * sizeof(int),
                             hipMemcpyHostToDevice, st) == hipSuccess;
    if (ok && !p.grp.empty())
        ok = hipMemcpyAsync(dplan + p.off_grp, p.grp.data(), p.grp.size() * sizeof(Grp), hipMemcpyHostToDevice,
                            st) == hipSuccess;
    if (ok && !p.ev.empty())
        ok = hipMemcpyAsync(dplan + p.off_ev, p.ev.data(), p.ev.size() * sizeof(Ev), hipMemcpyHostToDevice, st) ==
             hipSuccess;
    if (ok) {
        hipLaunchKernelGGL(k_combine, dim3(p.nseg, n_rec, 4), dim3(CT), 0, st, tr, n_rec, nt_in, dt_in,
                           dt_out / dt_in, t0[0], t0[1], t0[2], t0[3], dplan, (long)p.off_grp, (long)p.off_ev,
                           p.seg_len, nt_out, out);
        ok = hipGetLastError() == hipSuccess;
    }
    const hipError_t se = hipStreamSynchronize(st);
    if (!ok || se != hipSuccess) return cfail(PSTD_EDEVICE, "seis_combine: HIP launch or copy failed");
    return PSTD_OK;
}

// ---------------------------------------------------------------------------
// Work-list memory of seis_combine_noalloc: one array per device, in the
// library's static device memory.  Host code never uses the array's name as an
// address; it asks the runtime for each device's address once.
constexpr size_t NOALLOC_BYTES = 4u << 20;
__device__ __align__(256) char scratch[NOALLOC_BYTES];
constexpr int MAX_DEVICES = 64;
char* g_scratch_ptr[MAX_DEVICES] = {};
std::mutex g_scratch_mu;

// the address of this device's array, looked up once per device with the
// device current
int scratch_ptr(char** ptr)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES)
        return cfail(PSTD_EDEVICE, "seis_combine_noalloc: no usable current device");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return cfail(PSTD_EDEVICE, std::string("seis_combine_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<char*>(p);
    }
    *ptr = g_scratch_ptr[dev];
    return PSTD_OK;
}

}  // namespace

extern "C" int seis_combine(const float* tr, int n_src, int n_rec, int nt_in, double dt_in, const double t0[4], int n_ev,
                            const int32_t* src_idx, const double* amp, const double* t_origin, int nt_out,
                            double dt_out, float* out, void* hip_stream)
{
    int rc = check_args(tr, n_src, n_rec, nt_in, dt_in, t0, n_ev, src_idx, amp, t_origin, nt_out, dt_out, out);
    if (rc || n_rec == 0 || nt_out == 0) return rc;
    Plan p;
    make_plan(p, n_ev, src_idx, amp, t_origin, t0, nt_in, dt_in, nt_out, dt_out);
    char* dplan = nullptr;
    if (hipMalloc(&dplan, p.bytes) != hipSuccess) return cfail(PSTD_ENOMEM, "seis_combine: hipMalloc failed");
    rc = launch(p, dplan, tr, n_rec, nt_in, dt_in, t0, nt_out, dt_out, out, (hipStream_t)hip_stream);
    (void)hipFree(dplan);
    return rc;
}

extern "C" long seis_combine_noalloc_max_bytes(void) { return (long)NOALLOC_BYTES; }

extern "C" int seis_combine_noalloc(const float* tr, int n_src, int n_rec, int nt_in, double dt_in, const double t0[4],
                                    int n_ev, const int32_t* src_idx, const double* amp, const double* t_origin,
                                    int nt_out, double dt_out, float* out, void* hip_stream)
{
    int rc = check_args(tr, n_src, n_rec, nt_in, dt_in, t0, n_ev, src_idx, amp, t_origin, nt_out, dt_out, out);
    if (rc || n_rec == 0 || nt_out == 0) return rc;
    Plan p;
    make_plan(p, n_ev, src_idx, amp, t_origin, t0, nt_in, dt_in, nt_out, dt_out);
    if (p.bytes > NOALLOC_BYTES)
        return cfail(PSTD_EINVAL, "seis_combine_noalloc: the event lists need " + std::to_string(p.bytes) +
                                      " bytes, more than the " + std::to_string(NOALLOC_BYTES) +
                                      " bytes of its static device memory (use seis_combine)");
    char* dplan = nullptr;
    rc = scratch_ptr(&dplan);
    if (rc) return rc;
    return launch(p, dplan, tr, n_rec, nt_in, dt_in, t0, nt_out, dt_out, out, (hipStream_t)hip_stream);
}

extern "C" const char* seis_combine_last_error(void) { return g_cerr.c_str(); }
