// Clustered event catalogues (Sec. VI-A): Laplacian of the density (eq. 8)
// on the GPU, interface picking, k-means and the cluster timing rules on the
// host (tens to hundreds of points).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <string>
#include <vector>

#include "seis_catalog.h"

namespace {

thread_local std::string g_cerr;

int cfail(int code, const std::string& msg)
{
    g_cerr = msg;
    return code;
}

// second differences along x, y, z (neighbours past an edge equal the edge
// cell), summed in that order; one thread per cell, x fastest
__global__ void k_laplacian(const float* __restrict__ rho, int nx, int ny, int nz, float* __restrict__ lap)
{
    const long n = (long)nx * ny * nz;
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (long)gridDim.x * blockDim.x) {
        const int x = (int)(c % nx);
        const int y = (int)((c / nx) % ny);
        const int z = (int)(c / ((long)nx * ny));
        const float r0 = rho[c];
        const float xm = rho[c - (x > 0)], xp = rho[c + (x < nx - 1)];
        const float ym = rho[c - (y > 0) * (long)nx], yp = rho[c + (y < ny - 1) * (long)nx];
        const float zm = rho[c - (z > 0) * (long)nx * ny], zp = rho[c + (z < nz - 1) * (long)nx * ny];
        const float lx = (xp - 2.f * r0) + xm;
        const float ly = (yp - 2.f * r0) + ym;
        const float lz = (zp - 2.f * r0) + zm;
        lap[c] = (lx + ly) + lz;
    }
}

__global__ void k_gather_cells(const float* __restrict__ f, int nx, int ny, const int* __restrict__ ijk, int n,
                               float* __restrict__ out)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) out[e] = f[ijk[3 * e] + (long)nx * (ijk[3 * e + 1] + (long)ny * ijk[3 * e + 2])];
}

}  // namespace

extern "C" {

int seis_laplacian(const float* rho_dev, int nx, int ny, int nz, float* lap_dev, void* hip_stream)
{
    if (!rho_dev || !lap_dev || nx < 1 || ny < 1 || nz < 1) return cfail(PSTD_EINVAL, "bad arguments");
    const long n = (long)nx * ny * nz;
    const int grid = (int)std::min<long>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_laplacian, dim3(grid), dim3(256), 0, (hipStream_t)hip_stream, rho_dev, nx, ny, nz, lap_dev);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return cfail(PSTD_EDEVICE, std::string("k_laplacian: ") + hipGetErrorString(e));
    return PSTD_OK;
}

int seis_pick_interfaces(const float* lap_dev, int nx, int ny, int nz, const int32_t* cand_ijk, int n_cand,
                         float threshold, int32_t* keep, void* hip_stream)
{
    if (!lap_dev || n_cand < 0 || (n_cand > 0 && (!cand_ijk || !keep)) || nx < 1 || ny < 1 || nz < 1)
        return cfail(PSTD_EINVAL, "bad arguments");
    if (n_cand == 0) return 0;
    for (int c = 0; c < n_cand; ++c) {
        const int32_t* p = cand_ijk + 3 * c;
        if (p[0] < 0 || p[0] >= nx || p[1] < 0 || p[1] >= ny || p[2] < 0 || p[2] >= nz)
            return cfail(PSTD_EINVAL, "candidate " + std::to_string(c) + " outside the grid");
    }
    hipStream_t st = (hipStream_t)hip_stream;
    int* dijk = nullptr;
    float* dval = nullptr;
    std::vector<float> val(n_cand);
    hipError_t e = hipMalloc(&dijk, sizeof(int) * 3 * n_cand);
    if (e == hipSuccess) e = hipMalloc(&dval, sizeof(float) * n_cand);
    if (e == hipSuccess) e = hipMemcpyAsync(dijk, cand_ijk, sizeof(int) * 3 * n_cand, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_gather_cells, dim3((n_cand + 255) / 256), dim3(256), 0, st, lap_dev, nx, ny, dijk, n_cand,
                           dval);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(val.data(), dval, sizeof(float) * n_cand, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(dijk);
    (void)hipFree(dval);
    if (e != hipSuccess) return cfail(PSTD_EDEVICE, std::string("seis_pick_interfaces: ") + hipGetErrorString(e));
    int kept = 0;
    for (int c = 0; c < n_cand; ++c) {
        keep[c] = std::fabs(val[c]) > threshold ? 1 : 0;
        kept += keep[c];
    }
    return kept;
}

int seis_kmeans(const double* pts, int n, int k, int runs, const int32_t* init_idx, int max_iter, int32_t* labels,
                double* centroids, double* sse)
{
    if (!pts || !init_idx || !labels || !centroids || !sse || n < 1 || k < 1 || k > n || runs < 1 || max_iter < 1)
        return cfail(PSTD_EINVAL, "bad arguments");
    for (int r = 0; r < runs; ++r)
        for (int j = 0; j < k; ++j) {
            const int a = init_idx[r * k + j];
            if (a < 0 || a >= n) return cfail(PSTD_EINVAL, "initial centroid index out of range");
            for (int i = 0; i < j; ++i)
                if (init_idx[r * k + i] == a) return cfail(PSTD_EINVAL, "initial centroid indices must be distinct");
        }
    std::vector<int32_t> lab(n), best_lab(n);
    std::vector<double> cen(3 * k), best_cen(3 * k);
    double best = INFINITY;
    for (int r = 0; r < runs; ++r) {
        for (int j = 0; j < k; ++j)
            for (int a = 0; a < 3; ++a) cen[3 * j + a] = pts[3 * init_idx[r * k + j] + a];
        std::fill(lab.begin(), lab.end(), -1);
        for (int it = 0; it < max_iter; ++it) {
            bool changed = false;
            for (int i = 0; i < n; ++i) {
                int bj = 0;
                double bd = INFINITY;
                for (int j = 0; j < k; ++j) {
                    double d = 0.0;
                    for (int a = 0; a < 3; ++a) {
                        const double t = pts[3 * i + a] - cen[3 * j + a];
                        d += t * t;
                    }
                    if (d < bd) {
                        bd = d;
                        bj = j;
                    }
                }
                if (lab[i] != bj) {
                    lab[i] = bj;
                    changed = true;
                }
            }
            if (!changed) break;
            for (int j = 0; j < k; ++j) {
                double s[3] = {0.0, 0.0, 0.0};
                int cnt = 0;
                for (int i = 0; i < n; ++i)
                    if (lab[i] == j) {
                        for (int a = 0; a < 3; ++a) s[a] += pts[3 * i + a];
                        ++cnt;
                    }
                if (cnt)
                    for (int a = 0; a < 3; ++a) cen[3 * j + a] = s[a] / cnt;
            }
        }
        double tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int a = 0; a < 3; ++a) {
                const double t = pts[3 * i + a] - cen[3 * lab[i] + a];
                tot += t * t;
            }
        if (tot < best) {
            best = tot;
            best_lab = lab;
            best_cen = cen;
        }
    }
    std::copy(best_lab.begin(), best_lab.end(), labels);
    std::copy(best_cen.begin(), best_cen.end(), centroids);
    *sse = best;
    return PSTD_OK;
}

int seis_cluster_catalogue(const int32_t* labels, const double* depth, int n, int k, double t_first,
                           double dt_between, double sigma_within, const double* gauss, double amp_lo,
                           double amp_hi, const double* unif, double* t_origin, double* amp, int32_t* rank)
{
    if (!labels || !depth || !gauss || !unif || !t_origin || !amp || !rank || n < 0 || k < 1)
        return cfail(PSTD_EINVAL, "bad arguments");
    std::vector<double> sum(k, 0.0);
    std::vector<int> cnt(k, 0);
    for (int e = 0; e < n; ++e) {
        if (labels[e] < 0 || labels[e] >= k) return cfail(PSTD_EINVAL, "label out of range");
        sum[labels[e]] += depth[e];
        ++cnt[labels[e]];
    }
    // rank clusters by mean depth, shallowest first (empty clusters last)
    std::vector<int> order(k);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        if ((cnt[a] == 0) != (cnt[b] == 0)) return cnt[b] == 0;
        if (cnt[a] == 0) return false;
        return sum[a] / cnt[a] < sum[b] / cnt[b];
    });
    std::vector<int> rk(k);
    for (int r = 0; r < k; ++r) rk[order[r]] = r;
    for (int e = 0; e < n; ++e) {
        rank[e] = rk[labels[e]];
        t_origin[e] = t_first + rank[e] * dt_between + sigma_within * gauss[e];
        amp[e] = amp_lo + (amp_hi - amp_lo) * unif[e];
    }
    return PSTD_OK;
}

const char* seis_catalog_last_error(void) { return g_cerr.c_str(); }

}  // extern "C"
