"""Pins of the catalogue oracle (oracle/ocatalog.py) against closed forms,
brute force and a library routine:

 * the Laplacian of a quadratic field is 2 (a + b + c) in the interior and of
   a linear field 0; a density step gives +-jump on the two cells beside it;
   the loop and vectorised forms agree bit for bit;
 * k-means from every possible set of initial centroids reaches the global
   optimum of an exhaustive search over all partitions (tiny input), and on
   well separated blobs it finds scikit-learn's partition;
 * the cluster timing rules: ranks follow mean depth, bases dt_between apart.
"""
import itertools

import numpy as np

from oracle import ocatalog


def test_laplacian_closed_forms():
    z, y, x = np.meshgrid(np.arange(9), np.arange(8), np.arange(7), indexing="ij")
    a, b, c = 0.5, 0.25, 2.0
    L = ocatalog.laplacian(a * x * x + b * y * y + c * z * z)
    assert np.all(L[1:-1, 1:-1, 1:-1] == np.float32(2 * (a + b + c)))
    L = ocatalog.laplacian(3.0 * x - 2.0 * y + 0.5 * z + 1.0)
    assert np.all(L[1:-1, 1:-1, 1:-1] == 0.0)
    assert np.all(L[1:-1, 1:-1, 0] == np.float32(3.0))      # x edge: the missing neighbour equals the edge cell
    rho = np.where(z < 4, 1.0, 2.25)
    L = ocatalog.laplacian(rho)
    assert np.all(L[3] == np.float32(1.25)) and np.all(L[4] == np.float32(-1.25))
    assert np.all(L[:3] == 0) and np.all(L[5:] == 0)
    r = np.random.default_rng(0).uniform(1.0, 3.0, (6, 7, 9)).astype(np.float32)
    assert np.array_equal(ocatalog.laplacian(r), ocatalog.laplacian_fast(r))


def test_pick_threshold():
    lap = np.zeros((4, 4, 4), np.float32)
    lap[1, 2, 3] = 0.2
    lap[2, 1, 0] = -0.3
    lap[3, 3, 3] = 0.1
    cand = np.array([[3, 2, 1], [0, 1, 2], [3, 3, 3], [0, 0, 0]])
    assert list(ocatalog.pick(lap, cand, 0.1)) == [1, 1, 0, 0]


def test_kmeans_reaches_the_exhaustive_optimum():
    pts = np.random.default_rng(3).standard_normal((8, 3))
    best = np.inf
    for lab in itertools.product(range(3), repeat=8):
        lab = np.array(lab)
        if len(set(lab)) < 3:
            continue
        sse = sum(((pts[lab == j] - pts[lab == j].mean(axis=0)) ** 2).sum() for j in range(3))
        best = min(best, sse)
    init = np.array(list(itertools.combinations(range(8), 3)))
    lab, cen, sse = ocatalog.kmeans(pts, 3, init)
    assert abs(sse - best) < 1e-12


def test_kmeans_matches_scikit_learn_on_separated_blobs():
    from sklearn.cluster import KMeans
    rng = np.random.default_rng(4)
    centres = np.array([[0, 0, 0], [10, 0, 0], [0, 10, 5]], float)
    pts = np.concatenate([c + rng.standard_normal((20, 3)) for c in centres])
    init = np.stack([rng.choice(60, 3, replace=False) for _ in range(10)])
    lab, _, _ = ocatalog.kmeans(pts, 3, init)
    ref = KMeans(3, n_init=10, random_state=0).fit(pts).labels_
    # same partition up to the naming of the clusters
    assert len({(a, b) for a, b in zip(lab, ref)}) == 3


def test_catalogue_timing_rules():
    labels = np.array([2, 0, 1, 2, 0, 1, 1])
    depth = np.array([90.0, 30.0, 60.0, 95.0, 35.0, 55.0, 65.0])
    g = np.array([0.5, -1.0, 0.0, 2.0, 1.0, -0.5, 0.25])
    u = np.linspace(0, 0.9, 7)
    t, a, r = ocatalog.catalogue(labels, depth, 3, 1.0, 0.3, 0.1, g, 0.5, 1.5, u)
    assert list(r) == [2, 0, 1, 2, 0, 1, 1]                  # cluster 0 shallowest, 2 deepest
    assert np.allclose(t - 0.1 * g, 1.0 + 0.3 * r)
    assert np.allclose(a, 0.5 + u)
