// seis_combine: superposition of single-event traces (Sec. IV).
//
// out[c][r][m] = sum_e amp[e] * x_e(m dt_out - t_origin[e] - t0[c]), with x_e
// the linear interpolation of trace src_idx[e] (zero outside its samples).
//
// One block owns one output row (component c, receiver r) over a segment of
// the record and keeps the segment's sums in registers in double precision.
// The events that can touch the segment are grouped by source on the host
// (sources ascending, event order within a source), so the block stages each
// source's input row in LDS once and applies all of that source's events
// from there: every input trace is read from HBM once per segment and the
// record is written once.
//
// Two kernels share that scheme.  When a whole input trace fits a slot of the
// staging buffer (nt_in + 4 values, two zeros on each side; up to 4 CT),
// k_combine_w stages the rows of several sources between one pair of
// barriers and clamps each sample's index into its slot (an index outside
// the trace lands on the two zero pads at either end, so no sample needs a
// range test).  Its threads own output samples in groups of GQ spread over
// the segment (below), and the host marks per event and component the
// windows of samples it touches, so a wave spends lanes only where an event
// is.  Longer traces go through k_combine, whose threads own SPT consecutive
// samples and which stages one source at a time in chunks of STG samples and
// tests every sample against the chunk.  Blocks of 512 threads (segments of
// 6144 samples) measured faster than 1024: fewer waves wait at each item's
// barriers for the busiest one.
//
// The input position of a sample is u = m (dt_out / dt_in) - (t_origin + t0)/dt_in,
// kept in 32.32 fixed point: the host converts each event's offset
// -(t_origin + t0)/dt_in, a thread converts m (dt_out / dt_in) of its first
// sample once (in double), and each next sample adds the ratio in integers
// (its rounding, 2^-33 of a sample, grows by that much per sample).  The
// integer part picks the two input samples, the fraction f is the
// interpolation weight, the lerp x0 + f (x1 - x0) is formed in float (the
// inputs are float) and added to the double sum.  The lerp is continuous in
// u, so the rounding of u moves the result by as little.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "pstd3d.h"

namespace {

constexpr int CT = 512;            // threads per block
constexpr int SPT = 12;            // output samples per thread
constexpr int SEG_MAX = CT * SPT;  // output samples per segment
constexpr int STG = 4096;          // input samples staged per chunk (plus one before and one after)
// Output samples of k_combine_w go to threads in groups of GQ: group j of
// thread t holds samples s0 + j GSPAN + t GQ + q, q < GQ, so one wave's group
// j covers WSPAN consecutive samples (a window) and its groups lie GSPAN apart.
constexpr int GQ = 4;
constexpr int NGRP = SPT / GQ;
constexpr int GSPAN = CT * GQ;
constexpr int WSPAN = 64 * GQ;
constexpr int NWAVE = CT / 64;
static_assert(NWAVE * NGRP <= 32, "one bit per window of a segment");

// per-segment work list: groups of events sharing a source
struct Grp {
    long long src_off;   // offset of the source's traces in tr: src 4 n_rec nt_in floats
    int e0, e1;          // events [e0, e1) of the plan's event array
};
// one event of a segment: amplitude, and per component the input offset
// (t_origin + t0[c]) / dt_in, the output samples [rng[c][0], rng[c][1]) it can
// touch and the windows of the segment they meet (the chunked kernel reads
// these records)
struct Ev {
    double amp;
    unsigned long long u0[4];   // -(t_origin + t0[c]) / dt_in, 32.32 fixed point
    int rng[4][2];
    unsigned win[4];            // bit w NGRP + j: window j of wave w
};
// the same for one component, as the whole-trace kernel reads it (one
// 32-byte scalar load per event); its plan holds these component-major,
// [4][events]
struct EvC {
    unsigned long long u0;
    double amp;
    unsigned win;
    int lo, hi;
    int pad;
};

// x in 32.32 fixed point modulo 2^64 (two's complement): the integer part in
// the high word, the fraction truncated to 32 bits in the low word.  |x| is
// clamped to 2^52 (a position that far out is never inside a trace, and the
// event ranges keep such positions away from the kernels).
__host__ __device__ inline unsigned long long to_fx(double x)
{
    x = fmin(fmax(x, -4503599627370496.0), 4503599627370496.0);
    const double fl = floor(x);
    const double fr = fmin(floor((x - fl) * 4294967296.0), 4294967295.0);
    return ((unsigned long long)(long long)fl << 32) + (unsigned long long)fr;
}

// Host-side lists of one call: per segment the source groups, per group its
// events.  The arrays go to the device back to back (offsets in bytes).
struct Plan {
    int nseg = 0, seg_len = 0;
    std::vector<int> seg_ptr;    // [nseg + 1] into grp
    std::vector<Grp> grp;
    std::vector<Ev> ev;
    std::vector<EvC> evc;        // [4][ev.size()]
    size_t off_ptr = 0, off_grp = 0, off_ev = 0, bytes = 0;
};

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// bit w NGRP + j set where window j of wave w, [s0 + j GSPAN + w WSPAN, +
// WSPAN), meets the samples [lo, min(hi, s1)) of the segment [s0, s1)
unsigned window_mask(int lo, int hi, int s0, int s1)
{
    hi = std::min(hi, s1);
    unsigned m = 0;
    for (int w = 0; w < NWAVE; ++w)
        for (int j = 0; j < NGRP; ++j) {
            const int a = s0 + j * GSPAN + w * WSPAN;
            if (lo < a + WSPAN && hi > a) m |= 1u << (w * NGRP + j);
        }
    return m;
}

// Build the work lists.  An event can touch output sample m of component c
// only if u(m) lies in (-1, nt_in); that sample range is widened by one
// sample on each side (the kernel decides each sample exactly, a superset
// only costs a skipped iteration).
void make_plan(Plan& p, int n_rec, int n_ev, const int32_t* src_idx, const double* amp, const double* t_origin,
               const double t0[4], int nt_in, double dt_in, int nt_out, double dt_out)
{
    p.nseg = (nt_out + SEG_MAX - 1) / SEG_MAX;
    p.seg_len = (nt_out + p.nseg - 1) / p.nseg;
    const double ratio = dt_out / dt_in;
    std::vector<Ev> all(n_ev);
    std::vector<int> first(n_ev), last(n_ev);
    for (int e = 0; e < n_ev; ++e) {
        Ev& E = all[e];
        E.amp = amp[e];
        double lo_all = 1e300, hi_all = -1e300;
        for (int c = 0; c < 4; ++c) {
            const double be = (t_origin[e] + t0[c]) / dt_in;
            E.u0[c] = to_fx(-be);
            // clamped in double first: the offset may be far outside the record
            const double lo = std::max(0.0, std::floor((be - 1.0) / ratio) - 1.0);
            const double hi = std::min((double)nt_out, std::ceil(((double)nt_in + be) / ratio) + 2.0);
            E.rng[c][0] = (int)std::min(lo, (double)nt_out);
            E.rng[c][1] = hi > lo ? (int)hi : E.rng[c][0];
            if (E.rng[c][1] > E.rng[c][0]) {
                lo_all = std::min(lo_all, (double)E.rng[c][0]);
                hi_all = std::max(hi_all, (double)E.rng[c][1]);
            }
        }
        first[e] = hi_all > lo_all ? (int)lo_all : 1;
        last[e] = hi_all > lo_all ? (int)hi_all - 1 : 0;
    }
    // events of each segment in event order, then stably grouped by source
    std::vector<std::vector<int>> per(p.nseg);
    for (int e = 0; e < n_ev; ++e)
        for (int s = first[e] / p.seg_len; first[e] <= last[e] && s <= last[e] / p.seg_len; ++s) per[s].push_back(e);
    p.seg_ptr.assign(p.nseg + 1, 0);
    p.grp.clear();
    p.ev.clear();
    for (int s = 0; s < p.nseg; ++s) {
        std::vector<int>& L = per[s];
        std::stable_sort(L.begin(), L.end(), [&](int a, int b) { return src_idx[a] < src_idx[b]; });
        for (size_t i = 0; i < L.size();) {
            size_t j = i;
            while (j < L.size() && src_idx[L[j]] == src_idx[L[i]]) ++j;
            Grp g{(long long)src_idx[L[i]] * 4 * n_rec * nt_in, (int)p.ev.size(), 0};
            for (size_t k = i; k < j; ++k) {
                Ev E = all[L[k]];
                const int s0 = s * p.seg_len, s1 = std::min(s0 + p.seg_len, nt_out);
                for (int c = 0; c < 4; ++c) E.win[c] = window_mask(E.rng[c][0], E.rng[c][1], s0, s1);
                p.ev.push_back(E);
            }
            g.e1 = (int)p.ev.size();
            p.grp.push_back(g);
            i = j;
        }
        p.seg_ptr[s + 1] = (int)p.grp.size();
    }
    p.off_ptr = 0;
    p.off_grp = align256(p.seg_ptr.size() * sizeof(int));
    p.off_ev = p.off_grp + align256(std::max<size_t>(1, p.grp.size()) * sizeof(Grp));
    // the whole-trace kernel reads the component-major records, the chunked
    // kernel the per-event ones
    const size_t n = p.ev.size();
    p.evc.clear();
    if (nt_in + 4 <= 4 * CT) {
        p.evc.resize(4 * n);
        for (int c = 0; c < 4; ++c)
            for (size_t i = 0; i < n; ++i) {
                const Ev& E = p.ev[i];
                p.evc[c * n + i] = EvC{E.u0[c], E.amp, E.win[c], E.rng[c][0], E.rng[c][1], 0};
            }
        p.bytes = p.off_ev + align256(std::max<size_t>(1, p.evc.size()) * sizeof(EvC));
    } else {
        p.bytes = p.off_ev + align256(std::max<size_t>(1, n) * sizeof(Ev));
    }
}

// Block -> (segment, receiver, component).  The chip hands consecutive
// blocks to its 8 XCDs in turn, each with its own L2, so the segments of one
// output row (which stage the same source rows) are given block indices 8
// apart: the same XCD, one after the other.  Rows are (c, r) with c slowest;
// blocks past the last row exit.
constexpr int XCDS = 8;

__device__ __forceinline__ bool block_row(int nseg, int n_rec, int& seg, int& r, int& c)
{
    const int L = blockIdx.x;
    const int g = L / (XCDS * nseg), l = L - g * XCDS * nseg;
    seg = l / XCDS;
    const int row = g * XCDS + (l - seg * XCDS);
    if (row >= 4 * n_rec) return false;
    c = row / n_rec;
    r = row - c * n_rec;
    return true;
}

inline unsigned row_blocks(int nseg, int n_rec) { return (unsigned)((4 * n_rec + XCDS - 1) / XCDS * XCDS * nseg); }

// values of the staging buffer each thread loads
constexpr int NPT = (STG + 2 + CT - 1) / CT;
// samples whose positions, loads and sums go together (the loads of a half
// are all issued before the first wait)
constexpr int HALF = SPT / 2;

__global__ __launch_bounds__(CT) __attribute__((amdgpu_waves_per_eu(8))) void k_combine(const float* __restrict__ tr, int nseg, int n_rec, int nt_in, double ratio,
                                                long long ratio_fx, const char* __restrict__ plan, long off_grp,
                                                long off_ev, int seg_len, int nt_out, float* __restrict__ out)
{
    __shared__ float stg[STG + 2];
    int seg, r, c;
    if (!block_row(nseg, n_rec, seg, r, c)) return;
    const int tid = threadIdx.x;
    const int s0 = seg * seg_len;
    const int s1 = min(s0 + seg_len, nt_out);
    const int m0 = s0 + tid * SPT;                 // this thread's samples [m0, m0 + SPT)
    const bool active = m0 < s1;
    const int* __restrict__ seg_ptr = reinterpret_cast<const int*>(plan);
    const Grp* __restrict__ grp = reinterpret_cast<const Grp*>(plan + off_grp);
    const Ev* __restrict__ ev = reinterpret_cast<const Ev*>(plan + off_ev);
    // this block's row (c, r) of source 0; a group adds its source's offset
    const float* __restrict__ rowp = tr + ((long)c * n_rec + r) * nt_in;
    double acc[SPT];
#pragma unroll
    for (int k = 0; k < SPT; ++k) acc[k] = 0.0;
    const int g0 = seg_ptr[seg], g1 = seg_ptr[seg + 1];
    // Work items: (source group, chunk of the input axis).  Chunk q owns the
    // samples whose left neighbour i0 = floor(u) lies in [a, b), a = q STG - 1,
    // b = a + STG (the last chunk ends at nt_in), and stages x[a .. b] (zero
    // outside the trace).  The next item's values are loaded into registers
    // while the current one is computed.
    const int nchunk = (nt_in + 1 + STG - 1) / STG;
    const int nitems = (g1 - g0) * nchunk;
    const double md = (double)m0;
    float pre[NPT];
    auto fetch = [&](int item) {
        const int g = g0 + item / nchunk, q = item % nchunk;
        const int a = q * STG - 1;
        const int b = q == nchunk - 1 ? nt_in : a + STG;
        const float* __restrict__ x = rowp + grp[g].src_off;
#pragma unroll
        for (int j = 0; j < NPT; ++j) {
            const int i = tid + j * CT, k = a + i;
            pre[j] = (i <= b - a && k >= 0 && k < nt_in) ? x[k] : 0.0f;
        }
    };
    if (nitems > 0) fetch(0);
    for (int item = 0; item < nitems; ++item) {
        const int g = g0 + item / nchunk, q = item % nchunk;
        const int a = q * STG - 1;
        const int b = q == nchunk - 1 ? nt_in : a + STG;
        __syncthreads();   // the previous item's readers are done
#pragma unroll
        for (int j = 0; j < NPT; ++j) {
            const int i = tid + j * CT;
            if (i < STG + 2) stg[i] = pre[j];
        }
        __syncthreads();
        if (item + 1 < nitems) fetch(item + 1);
        const Grp G = grp[g];
        for (int e = G.e0; e < G.e1; ++e) {
            const Ev& E = ev[e];
            const int lo = E.rng[c][0], hi = E.rng[c][1];
            if (!active || hi <= m0 || lo >= m0 + SPT) continue;
            const double amp = E.amp;
            // position of this thread's first sample in 32.32 fixed point
            // (from double: m0 (dt_out / dt_in) plus the event's offset; each
            // later sample adds the ratio in integers, 2^-32 of a sample per
            // step), integer part = left neighbour
            const double u0 = fma(md, ratio, (double)(long long)E.u0[c] * 2.3283064365386963e-10);
            const double fl0 = floor(u0);
            long long u = ((long long)fl0 << 32) + (long long)((u0 - fl0) * 4294967296.0);
#pragma unroll
            for (int h = 0; h < SPT; h += HALF) {
                // branch free: the positions of a half, then all its LDS reads,
                // then the arithmetic (a sample outside this chunk's input
                // range reads slot 0 and adds 0 times it)
                int idx[HALF];
                float fr[HALF];
                double w[HALF];
#pragma unroll
                for (int k = 0; k < HALF; ++k) {
                    const int i0 = (int)(u >> 32);
                    const bool in = i0 >= a && i0 < b;
                    idx[k] = in ? i0 - a : 0;
                    fr[k] = (float)(unsigned)(u & 0xffffffffLL) * 2.3283064365386963e-10f;
                    w[k] = in ? amp : 0.0;
                    u += ratio_fx;
                }
                float x0[HALF], x1[HALF];
#pragma unroll
                for (int k = 0; k < HALF; ++k) {
                    x0[k] = stg[idx[k]];
                    x1[k] = stg[idx[k] + 1];
                }
#pragma unroll
                for (int k = 0; k < HALF; ++k)
                    acc[h + k] = fma(w[k], (double)fmaf(fr[k], x1[k] - x0[k], x0[k]), acc[h + k]);
            }
        }
    }
    float* __restrict__ o = out + ((long)c * n_rec + r) * nt_out;
#pragma unroll
    for (int k = 0; k < SPT; ++k)
        if (m0 + k < s1) o[m0 + k] = (float)acc[k];
}

// Whole-trace staging: a slot holds a source row x[-2 .. nt_in + 1] (zeros
// outside the trace), nt_in + 4 values, in VPS CT floats of which each thread
// writes VPS (VPS = 1, 2 or 4: the smallest with nt_in + 4 <= VPS CT); an item
// is NSLOT(VPS) = WPT / VPS slots, staged from WPT registers per thread
// (32 KB of LDS).  The loads are buffer loads whose range is the trace, so
// the positions outside it read zero and staging needs no branch, clamp or
// select.
//
// Output samples go to threads in the groups of GQ described above; the
// host marks per event and component the windows it touches (one bit each),
// and a wave computes only its marked windows.  An event then spends lanes
// on at most one partly covered window of WSPAN samples at either end, where
// runs of SPT samples per thread would waste up to a wave's 64 SPT, and a
// wave that the event misses pays one scalar test for it.
constexpr int WPT = 16;
// buffer resource word 3 for raw 32-bit loads on this chip family
constexpr int BUF_DW3 = 0x00020000;

// fixed-point position of group j's first sample relative to the thread's
// first, plus the slot's two leading pads: to_fx(j GSPAN ratio + 2)
struct GroupPos {
    unsigned long long d[NGRP];
};

__host__ __device__ constexpr int w_slot(int nt_in) { return nt_in + 4; }

template <int VPS>
__global__ __launch_bounds__(CT) __attribute__((amdgpu_waves_per_eu(8))) void k_combine_w(
    const float* __restrict__ tr, int nseg, int n_rec, int nt_in, double ratio, unsigned long long ratio_fx,
    GroupPos gp, const char* __restrict__ plan, long off_grp, long off_ev, int n_evp, int seg_len, int nt_out,
    float* __restrict__ out)
{
    constexpr int NSLOT = WPT / VPS;
    constexpr int S = VPS * CT;      // floats per slot
    extern __shared__ float stw[];   // NSLOT slots of S floats
    int seg, r, c;
    if (!block_row(nseg, n_rec, seg, r, c)) return;
    const int tid = threadIdx.x;
    const int L = w_slot(nt_in);
    const int s0 = seg * seg_len;
    const int s1 = min(s0 + seg_len, nt_out);
    // this wave's bits in the events' window masks (uniform across the wave)
    const int wsh = (__builtin_amdgcn_readfirstlane(tid) / 64) * NGRP;
    const int* __restrict__ seg_ptr = reinterpret_cast<const int*>(plan);
    const Grp* __restrict__ grp = reinterpret_cast<const Grp*>(plan + off_grp);
    const EvC* __restrict__ ev = reinterpret_cast<const EvC*>(plan + off_ev) + (long)c * n_evp;
    // this block's row (c, r) of source 0; a group adds its source's offset
    const float* __restrict__ rowp = tr + ((long)c * n_rec + r) * nt_in;
    double acc[SPT];
#pragma unroll
    for (int k = 0; k < SPT; ++k) acc[k] = 0.0;
    const int g0 = seg_ptr[seg], g1 = seg_ptr[seg + 1];
    // (s0 + t GQ) (dt_out / dt_in) in fixed point; an event adds its offset
    const unsigned long long T = to_fx((double)(s0 + tid * GQ) * ratio);
    // Item q stages the rows of groups [g0 + q NSLOT, g0 + (q + 1) NSLOT); the
    // next item's values are loaded into registers while this one is computed.
    const int nitems = (g1 - g0 + NSLOT - 1) / NSLOT;
    // slot position tid + v CT holds x[tid + v CT - 2]: buffer loads with the
    // trace as the buffer's range return zero outside it (a negative offset
    // is out of range as an unsigned value)
    float pre[WPT];
    // byte offsets of x[tid - 2] and x[tid + 2 CT - 2]; the other loads add
    // constants that fit the instructions' offset field
    const int o0 = (tid - 2) * 4, o2 = o0 + 2 * CT * 4;
    auto fetch = [&](int item) {
        // opaque copies, so the per-load constants stay in the loads'
        // offset fields rather than in registers set up outside the loop
        int b0 = o0, b2 = o2;
        asm volatile("" : "+v"(b0), "+v"(b2));
        const int gb = g0 + item * NSLOT;
#pragma unroll
        for (int sl = 0; sl < NSLOT; ++sl) {
            // a slot past the item's last group is loaded from that group
            // and never read
            const int g = min(gb + sl, g1 - 1);
            const __amdgpu_buffer_rsrc_t rs =
                __builtin_amdgcn_make_buffer_rsrc((void*)(rowp + grp[g].src_off), (short)0, nt_in * 4, BUF_DW3);
#pragma unroll
            for (int v = 0; v < VPS; ++v)
                pre[sl * VPS + v] = __uint_as_float(
                    __builtin_amdgcn_raw_buffer_load_b32(rs, (v < 2 ? b0 : b2) + (v & 1) * CT * 4, 0, 0));
        }
    };
    if (nitems > 0) fetch(0);
    for (int item = 0; item < nitems; ++item) {
        __syncthreads();   // the previous item's readers are done
#pragma unroll
        for (int sl = 0; sl < NSLOT; ++sl)
#pragma unroll
            for (int v = 0; v < VPS; ++v) stw[sl * S + tid + v * CT] = pre[sl * VPS + v];
        __syncthreads();
        if (item + 1 < nitems) fetch(item + 1);
        const int gb = g0 + item * NSLOT;
        const int ng = min(NSLOT, g1 - gb);
        for (int gi = 0; gi < ng; ++gi) {
            const Grp G = grp[gb + gi];
            const float* __restrict__ x = stw + gi * S;
            for (int e = G.e0; e < G.e1; ++e) {
                const EvC E = ev[e];
                // one round trip for the whole record: make its fields live
                // before the test below uses the mask
                asm volatile("" ::"s"(E.u0), "s"(E.amp), "s"(E.win));
                // this wave's windows that the event touches
                const unsigned wm = (E.win >> wsh) & ((1u << NGRP) - 1);
                if (!wm) continue;
                const double amp = E.amp;
                const unsigned long long ue = T + E.u0;
#pragma unroll
                for (int j = 0; j < NGRP; ++j) {
                    if (!(wm >> j & 1)) continue;
                    unsigned long long u = ue + gp.d[j];
                    int idx[GQ];
                    float fr[GQ];
#pragma unroll
                    for (int q = 0; q < GQ; ++q) {
                        // clamped into [0, L - 2] as unsigned (a negative index
                        // becomes L - 2): an index outside the trace reads two
                        // of the zero pads
                        idx[q] = (int)min((unsigned)(u >> 32), (unsigned)(L - 2));
                        fr[q] = (float)(unsigned)u * 2.3283064365386963e-10f;
                        u += ratio_fx;
                    }
                    float x0[GQ], x1[GQ];
#pragma unroll
                    for (int q = 0; q < GQ; ++q) {
                        x0[q] = x[idx[q]];
                        x1[q] = x[idx[q] + 1];
                    }
#pragma unroll
                    for (int q = 0; q < GQ; ++q)
                        acc[j * GQ + q] = fma(amp, (double)fmaf(fr[q], x1[q] - x0[q], x0[q]), acc[j * GQ + q]);
                }
            }
        }
    }
    float* __restrict__ o = out + ((long)c * n_rec + r) * nt_out;
#pragma unroll
    for (int j = 0; j < NGRP; ++j)
#pragma unroll
        for (int q = 0; q < GQ; ++q) {
            const int m = s0 + j * GSPAN + tid * GQ + q;
            if (m < s1) o[m] = (float)acc[j * GQ + q];
        }
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
    if (!(dt_out / dt_in <= 1048576.0) || !(dt_out / dt_in >= 1.0 / 1048576.0))
        return cfail(PSTD_EINVAL, "seis_combine: dt_out / dt_in outside [2^-20, 2^20]");
    // input positions near an event stay within nt_in + 2^25 samples, in int range
    if (nt_in > (1 << 30)) return cfail(PSTD_EINVAL, "seis_combine: nt_in above 2^30");
    if (n_rec == 0 || nt_out == 0) return PSTD_OK;
    {
        // one 1-D launch: blocks x threads must stay below 2^32 work-items
        const long long rows = (4LL * n_rec + XCDS - 1) / XCDS * XCDS;
        const long long nseg = ((long long)nt_out + SEG_MAX - 1) / SEG_MAX;
        if (rows * nseg * CT >= (1LL << 32))
            return cfail(PSTD_EINVAL, "seis_combine: output too large for one call (split the receivers)");
    }
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
    if (ok && !p.evc.empty())
        ok = hipMemcpyAsync(dplan + p.off_ev, p.evc.data(), p.evc.size() * sizeof(EvC), hipMemcpyHostToDevice, st) ==
             hipSuccess;
    else if (ok && !p.ev.empty())
        ok = hipMemcpyAsync(dplan + p.off_ev, p.ev.data(), p.ev.size() * sizeof(Ev), hipMemcpyHostToDevice, st) ==
             hipSuccess;
    if (ok) {
        const double ratio = dt_out / dt_in;
        const long long ratio_fx = (long long)std::llround(ratio * 4294967296.0);
        const int L = w_slot(nt_in);
        const dim3 grid(row_blocks(p.nseg, n_rec));
        const unsigned long long rfx = (unsigned long long)ratio_fx;
        const long og = (long)p.off_grp, oe = (long)p.off_ev;
        const int nev = (int)p.ev.size();
        GroupPos gp;
        for (int j = 0; j < NGRP; ++j) gp.d[j] = to_fx((double)j * GSPAN * ratio + 2.0);
        if (L <= CT) {
            hipLaunchKernelGGL(k_combine_w<1>, grid, dim3(CT), (size_t)WPT * CT * sizeof(float), st, tr, p.nseg,
                               n_rec, nt_in, ratio, rfx, gp, dplan, og, oe, nev, p.seg_len, nt_out, out);
        } else if (L <= 2 * CT) {
            hipLaunchKernelGGL(k_combine_w<2>, grid, dim3(CT), (size_t)WPT * CT * sizeof(float), st, tr, p.nseg,
                               n_rec, nt_in, ratio, rfx, gp, dplan, og, oe, nev, p.seg_len, nt_out, out);
        } else if (L <= 4 * CT) {
            hipLaunchKernelGGL(k_combine_w<4>, grid, dim3(CT), (size_t)WPT * CT * sizeof(float), st, tr, p.nseg,
                               n_rec, nt_in, ratio, rfx, gp, dplan, og, oe, nev, p.seg_len, nt_out, out);
        } else {
            hipLaunchKernelGGL(k_combine, dim3(row_blocks(p.nseg, n_rec)), dim3(CT), 0, st, tr, p.nseg, n_rec, nt_in,
                               ratio, ratio_fx,
                               dplan, (long)p.off_grp, (long)p.off_ev, p.seg_len, nt_out, out);
        }
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
    make_plan(p, n_rec, n_ev, src_idx, amp, t_origin, t0, nt_in, dt_in, nt_out, dt_out);
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
    make_plan(p, n_rec, n_ev, src_idx, amp, t_origin, t0, nt_in, dt_in, nt_out, dt_out);
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
