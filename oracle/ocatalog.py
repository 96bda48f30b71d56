"""Oracle of the clustered event catalogue (Sec. VI-A).  TEST INFRASTRUCTURE ONLY.

 * eq. 8: L = d2rho/dx2 + d2rho/dy2 + d2rho/dz2, as second differences per
   cell, the neighbour past a grid edge taken equal to the edge cell; evaluated
   in float32 in the order x, y, z, because the interface picking (|L| above a
   threshold) is a decision taken in that precision;
 * interface picking: candidate cells with |L| > threshold;
 * k-means: Lloyd's alternation of nearest-centroid assignment and centroid
   means from given initial centroids, best of several runs by the
   within-cluster sum of squares;
 * cluster timing (Sec. VI-A): clusters ranked by mean depth, the shallowest
   (nearest the sea floor) first; origin time = t_first + rank * dt_between +
   sigma * gauss; amplitude = lo + (hi - lo) * unif.
"""
import numpy as np


def laplacian(rho):
    """L of eq. 8 for rho [nz][ny][nx] (float32 in, float32 out)."""
    r = np.asarray(rho, np.float32)
    out = np.empty_like(r)
    nz, ny, nx = r.shape
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                r0 = r[k, j, i]
                xm, xp = r[k, j, max(i - 1, 0)], r[k, j, min(i + 1, nx - 1)]
                ym, yp = r[k, max(j - 1, 0), i], r[k, min(j + 1, ny - 1), i]
                zm, zp = r[max(k - 1, 0), j, i], r[min(k + 1, nz - 1), j, i]
                two = np.float32(2.0)
                lx = (xp - two * r0) + xm
                ly = (yp - two * r0) + ym
                lz = (zp - two * r0) + zm
                out[k, j, i] = (lx + ly) + lz
    return out


def laplacian_fast(rho):
    """The same values as laplacian(), vectorised (float32 throughout)."""
    r = np.asarray(rho, np.float32)
    two = np.float32(2.0)

    def nb(axis, step):
        idx = np.arange(r.shape[axis]) + step
        idx = np.clip(idx, 0, r.shape[axis] - 1)
        return np.take(r, idx, axis=axis)

    lx = (nb(2, +1) - two * r) + nb(2, -1)
    ly = (nb(1, +1) - two * r) + nb(1, -1)
    lz = (nb(0, +1) - two * r) + nb(0, -1)
    return ((lx + ly) + lz).astype(np.float32)


def pick(lap, cand_ijk, threshold):
    """1 where |L| > threshold at candidate (i, j, k), else 0."""
    lap = np.asarray(lap, np.float32)
    c = np.asarray(cand_ijk)
    v = lap[c[:, 2], c[:, 1], c[:, 0]]
    return (np.abs(v) > np.float32(threshold)).astype(np.int32)


def kmeans(pts, k, init_idx, max_iter=100):
    """Best-of-runs Lloyd k-means; returns (labels, centroids, sse)."""
    pts = np.asarray(pts, np.float64)
    n = pts.shape[0]
    best = None
    for run in np.asarray(init_idx).reshape(-1, k):
        cen = pts[run].copy()
        lab = np.full(n, -1)
        for _ in range(max_iter):
            d = ((pts[:, None, :] - cen[None, :, :]) ** 2).sum(axis=2)
            new = np.argmin(d, axis=1)                 # ties: lowest index
            if np.array_equal(new, lab):
                break
            lab = new
            for j in range(k):
                m = lab == j
                if m.any():
                    cen[j] = pts[m].mean(axis=0)
        sse = float(((pts - cen[lab]) ** 2).sum())
        if best is None or sse < best[2]:
            best = (lab.copy(), cen.copy(), sse)
    return best


def catalogue(labels, depth, k, t_first, dt_between, sigma, gauss, lo, hi, unif):
    """(t_origin, amp, rank) of the cluster timing rules."""
    labels = np.asarray(labels)
    depth = np.asarray(depth, np.float64)
    means = []
    for j in range(k):
        m = labels == j
        means.append((0 if m.any() else 1, depth[m].mean() if m.any() else 0.0, j))
    order = [j for _, _, j in sorted(means)]
    rank_of = {j: r for r, j in enumerate(order)}
    rank = np.array([rank_of[int(l)] for l in labels], np.int32)
    t = t_first + rank * dt_between + sigma * np.asarray(gauss, np.float64)
    amp = lo + (hi - lo) * np.asarray(unif, np.float64)
    return t, amp, rank
