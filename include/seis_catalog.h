/*
 * seis_catalog — clustered microseismic event catalogues on top of the solver
 * (arXiv 1705.04874, Sec. VI-A).  Plain C ABI: host or device pointers and
 * sizes only; errors are the PSTD_* codes of pstd3d.h, with the message of the
 * last error on the calling thread in seis_catalog_last_error().
 *
 * The paper keeps, out of its sampled source locations, those that lie on
 * interfaces between rock layers: where the 3-D Laplacian of the density
 * (eq. 8) exceeds a threshold in magnitude (|L| > 0.1).  It groups them into
 * three spatial clusters with k-means, shifts the origin times by 0.3 s
 * between clusters (the cluster nearest the sea floor first) and by a random
 * zero-mean amount with 0.1 s standard deviation within a cluster, and draws
 * the amplitudes uniformly.  The resulting catalogue feeds seis_combine.
 * Every random number is an input (the caller draws them), so a run is
 * reproducible and checkable.
 */
#ifndef SEIS_CATALOG_H
#define SEIS_CATALOG_H

#include <stdint.h>

#include "pstd3d.h"

#ifdef __cplusplus
extern "C" {
#endif

/* L = d2rho/dx2 + d2rho/dy2 + d2rho/dz2 (eq. 8) as second differences per
 * cell (rho[i+1] - 2 rho[i] + rho[i-1] on each axis, summed x, y, z in that
 * order, FP32), the neighbour past a grid edge taken equal to the edge cell.
 * rho_dev, lap_dev: device float [nz][ny][nx] (x fastest); runs on hip_stream. */
int seis_laplacian(const float *rho_dev, int nx, int ny, int nz, float *lap_dev, void *hip_stream);

/* For each of the n_cand candidate cells (host int32 [n_cand][3], i j k),
 * keep[c] (host) = 1 if |L| > threshold at that cell, else 0 (FP32 compare of
 * the device Laplacian lap_dev [nz][ny][nx]).  Returns the number kept or a
 * negative error code. */
int seis_pick_interfaces(const float *lap_dev, int nx, int ny, int nz, const int32_t *cand_ijk, int n_cand,
                         float threshold, int32_t *keep, void *hip_stream);

/* k-means (Lloyd's iterations) of n host points [n][3] into k clusters, FP64.
 * Run r starts from the centroids pts[init_idx[r k + j]] (host int32
 * [runs][k], k distinct indices per run, drawn by the caller), then alternates
 * assignment (nearest centroid by squared Euclidean distance, ties to the
 * lower index) and update (mean of the members; an empty cluster keeps its
 * centroid) until the assignment no longer changes or max_iter iterations.
 * The run with the lowest within-cluster sum of squares wins (the first one on
 * ties).  Outputs (host): labels [n], centroids [k][3], *sse. */
int seis_kmeans(const double *pts, int n, int k, int runs, const int32_t *init_idx, int max_iter, int32_t *labels,
                double *centroids, double *sse);

/* Cluster catalogue (Sec. VI-A).  Clusters are ranked by the mean of depth[]
 * of their members (shallowest, i.e. nearest the sea floor, first); event e
 * of rank-r cluster starts at t_first + r dt_between + sigma_within * gauss[e]
 * and has amplitude amp_lo + (amp_hi - amp_lo) * unif[e] (gauss, unif: host
 * standard-normal and U[0,1) draws, [n]).  Outputs (host, [n]): t_origin,
 * amp, and rank (the cluster's rank). */
int seis_cluster_catalogue(const int32_t *labels, const double *depth, int n, int k, double t_first,
                           double dt_between, double sigma_within, const double *gauss, double amp_lo,
                           double amp_hi, const double *unif, double *t_origin, double *amp, int32_t *rank);

/* Message of the last catalogue error on the calling thread. */
const char *seis_catalog_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
