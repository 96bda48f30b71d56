"""Pins of the surrogate oracle (oracle/osno.py) against library routines and calculus.

 * the truncated DFT and its inverse equal numpy's FFT with truncation and
   zero padding (a different implementation of the same definition);
 * the hand-written gradient equals central finite differences of the loss
   for every parameter block (FP64);
 * gelu's derivative equals finite differences;
 * Adam's first step moves every weight by lr * sign(g) (bias correction), and
   three steps equal the recurrence expanded by hand with beta1 = 0.9,
   beta2 = 0.999 (the weights of g1, g2, g3 in m3 and v3, and the bias
   corrections 1 - beta^t written out as numbers);
 * the error head's ridge least squares equals numpy's lstsq of the augmented
   system [Phi; sqrt(ridge n) I] h = [log e; 0], and its margin covers about
   95 % of Gaussian residuals of known spread;
 * the output is linear in the moment-tensor features (the elastic system is
   linear in its source, eq. 2) and does not depend on them otherwise;
 * the Fourier time features are the modes numpy's FFT finds in them.
"""
import math

import numpy as np
import pytest

from oracle import osno
from paper_1705_04874_amd import inputs

D = osno.Dims(n_pos=3, n_mt=6, four=(3.0, 7.5), C=4, T=32, K=5, L=2, H=6, O=5)


def init(d, seed):
    return inputs.sno_init_params(d.C, d.K, d.L, d.H, d.O, osno.n_lift(d), seed, d.n_mt)


def test_truncated_dft_matches_numpy_fft():
    d = osno.Dims(T=64, K=7)
    F, G = osno.dft_bases(d)
    rng = np.random.default_rng(0)
    v = rng.standard_normal((3, d.T))
    vh = v @ F
    ref = np.fft.rfft(v, axis=1)[:, :d.K]
    assert np.abs(vh[:, :d.K] - ref.real).max() < 1e-12
    assert np.abs(vh[:, d.K:] - ref.imag).max() < 1e-12
    spec = np.zeros((3, d.T // 2 + 1), complex)
    spec[:, :d.K] = ref
    back = np.fft.irfft(spec, n=d.T, axis=1)
    assert np.abs(vh @ G - back).max() < 1e-12


def test_gelu_derivative():
    x = np.linspace(-4, 4, 101)
    h = 1e-6
    fd = (osno.gelu(x + h) - osno.gelu(x - h)) / (2 * h)
    assert np.abs(fd - osno.gelu_grad(x)).max() < 1e-8


D_PM = osno.Dims(n_pos=3, n_mt=6, four=(3.0, 7.5), pos_mod=True, C=4, T=32, K=5, L=2, H=6, O=5)


@pytest.mark.parametrize("D", [D, D_PM], ids=["plain", "posmod"])
def test_gradient_matches_finite_differences(D):
    rng = np.random.default_rng(1)
    theta = init(D, 3)
    theta += 0.05 * rng.standard_normal(theta.size)        # break the zero biases / positive R
    src = rng.standard_normal((2, D.n_pos + D.n_mt))
    y = rng.standard_normal((2, D.O, D.T))
    g = osno.grad(theta, src, y, D)
    o = 0
    h = 1e-6
    for name, sh in osno.param_shapes(D):
        n = int(np.prod(sh))
        idx = o + rng.choice(n, size=min(n, 6), replace=False)
        for i in idx:
            tp = theta.copy()
            tm = theta.copy()
            tp[i] += h
            tm[i] -= h
            fd = (osno.loss(tp, src, y, D) - osno.loss(tm, src, y, D)) / (2 * h)
            assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (name, i, fd, g[i])
        o += n
    assert o == theta.size


D_W = osno.Dims(n_pos=3, n_mt=6, four=(3.0, 7.5), C=4, T=32, K=5, L=2, H=6, O=8)


def test_weighted_gradient_matches_finite_differences():
    """Per-(sample, component) loss weights: the gradient still equals
    central finite differences of the weighted loss."""
    rng = np.random.default_rng(6)
    d = D_W
    theta = init(d, 3) + 0.05 * rng.standard_normal(osno.n_params(d))
    src = rng.standard_normal((2, d.n_pos + d.n_mt))
    y = rng.standard_normal((2, d.O, d.T))
    w = rng.uniform(0.2, 5.0, (2, 4))
    g = osno.grad(theta, src, y, d, w=w)
    h = 1e-6
    for i in rng.choice(theta.size, 60, replace=False):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (osno.loss(tp, src, y, d, w=w) - osno.loss(tm, src, y, d, w=w)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])
    # unit weights are the plain loss
    assert osno.loss(theta, src, y, d, w=np.ones((2, 4))) == pytest.approx(osno.loss(theta, src, y, d), rel=1e-14)


def test_relative_weights_give_the_mean_squared_relative_error():
    """With w = 1 / mean square of each target component the weighted loss is
    the mean over samples and components of ||Y - y||^2 / ||y||^2 (receivers
    of a component are the O / 4 consecutive outputs)."""
    rng = np.random.default_rng(7)
    d = D_W
    theta = init(d, 3) + 0.05 * rng.standard_normal(osno.n_params(d))
    src = rng.standard_normal((3, d.n_pos + d.n_mt))
    y = rng.standard_normal((3, d.O, d.T)) * rng.uniform(0.01, 100.0, (3, d.O, 1))
    w = osno.relative_weights(y, d)
    Y = osno.forward(theta, src, d)
    n_rec = d.O // 4
    rel = [np.linalg.norm(Y[b, c * n_rec:(c + 1) * n_rec] - y[b, c * n_rec:(c + 1) * n_rec]) ** 2 /
           np.linalg.norm(y[b, c * n_rec:(c + 1) * n_rec]) ** 2 for b in range(3) for c in range(4)]
    assert osno.loss(theta, src, y, d, w=w) == pytest.approx(np.mean(rel), rel=1e-12)
    z = y.copy()
    z[1, 2 * n_rec:3 * n_rec] = 0.0
    assert osno.relative_weights(z, d)[1, 2] == 0.0


def test_adam_first_step():
    theta = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -1e-3, 2.0])
    t, m, v = osno.adam(theta, g, np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.allclose(t, theta - 0.01 * np.sign(g), atol=1e-7)


def test_output_is_linear_in_the_moment_tensor():
    rng = np.random.default_rng(4)
    theta = init(D, 5) + 0.05 * rng.standard_normal(osno.n_params(D))
    pos = rng.standard_normal((1, D.n_pos))
    m1, m2 = rng.standard_normal((2, D.n_mt))
    y = lambda m: osno.forward(theta, np.concatenate([pos, m[None]], axis=1), D)
    np.testing.assert_allclose(y(2.0 * m1 - 0.5 * m2), 2.0 * y(m1) - 0.5 * y(m2), rtol=1e-12, atol=1e-12)
    assert np.abs(y(np.zeros(D.n_mt))).max() == 0.0


def test_fourier_features_have_their_frequencies():
    d = osno.Dims(four=(4.0, 11.0), T=64)
    A = osno.features(np.zeros((1, 9)), d)[0]
    for f, c in enumerate(d.four):
        sp = np.fft.rfft(A[d.n_pos + 1 + 2 * f])
        assert np.argmax(np.abs(sp)) == int(c) and abs(sp[int(c)].real - d.T / 2) < 1e-9
        sp = np.fft.rfft(A[d.n_pos + 2 + 2 * f])
        assert np.argmax(np.abs(sp)) == int(c) and abs(sp[int(c)].imag + d.T / 2) < 1e-9


def test_position_modulated_features_shift_the_phase():
    """With position modulation a linear map of the lift input can move the
    phase of a time feature with the source position: cos(w t - a p) is, to
    first order in p, cos(w t) + a p sin(w t); the product channels carry
    exactly p cos and p sin at each frequency (order frequency, position,
    cos / sin), and are zero at p = 0."""
    d = osno.Dims(four=(4.0, 11.0), pos_mod=True, T=64)
    rng = np.random.default_rng(4)
    src = np.concatenate([rng.uniform(-1, 1, (2, 3)), np.zeros((2, 6))], axis=1)
    src[1, :3] = 0.0
    A = osno.features(src, d)
    base = d.n_pos + 1 + 2 * len(d.four)
    assert A.shape[1] == base + 2 * d.n_pos * len(d.four)
    t = np.arange(d.T) / d.T
    for f, c in enumerate(d.four):
        for k in range(d.n_pos):
            p = src[0, k]
            np.testing.assert_allclose(A[0, base + 2 * (3 * f + k)], p * np.cos(2 * np.pi * c * t), atol=1e-15)
            np.testing.assert_allclose(A[0, base + 2 * (3 * f + k) + 1], p * np.sin(2 * np.pi * c * t), atol=1e-15)
    assert not A[1, base:].any()
    # first-order phase shift through the product channels
    a, f = 0.05, 1
    p = src[0, 0]
    lin = A[0, d.n_pos + 1 + 2 * f] + a * A[0, base + 2 * (3 * f + 0) + 1]
    exact = np.cos(2 * np.pi * d.four[f] * t - a * p)
    assert np.abs(lin - exact).max() <= (a * p) ** 2


def test_adam_three_steps_equal_the_hand_expanded_recurrence():
    rng = np.random.default_rng(4)
    n = 7
    theta0 = rng.standard_normal(n)
    g = rng.standard_normal((3, n))
    lr = 1e-2
    th, m, v = theta0.copy(), np.zeros(n), np.zeros(n)
    for t in range(3):
        th, m, v = osno.adam(th, g[t], m, v, t + 1, lr)
    # m3 = 0.1 (0.81 g1 + 0.9 g2 + g3); v3 = 0.001 (0.998001 g1^2 + 0.999 g2^2 + g3^2)
    m3 = 0.081 * g[0] + 0.09 * g[1] + 0.1 * g[2]
    v3 = 0.000998001 * g[0] ** 2 + 0.000999 * g[1] ** 2 + 0.001 * g[2] ** 2
    assert np.abs(m - m3).max() < 1e-15 and np.abs(v - v3).max() < 1e-15
    # bias corrections 1 - 0.9^t = 0.1, 0.19, 0.271 and 1 - 0.999^t = 0.001, 0.001999, 0.002997001
    m1, v1 = 0.1 * g[0], 0.001 * g[0] ** 2
    m2, v2 = 0.09 * g[0] + 0.1 * g[1], 0.000999 * g[0] ** 2 + 0.001 * g[1] ** 2
    want = theta0.copy()
    for mm, vv, c1, c2 in [(m1, v1, 0.1, 0.001), (m2, v2, 0.19, 0.001999), (m3, v3, 0.271, 0.002997001)]:
        want = want - lr * (mm / c1) / (np.sqrt(vv / c2) + 1e-8)
    assert np.abs(th - want).max() < 1e-13
    # a wrong beta2 (0.99) is far off after three steps
    th2, m2_, v2_ = theta0.copy(), np.zeros(n), np.zeros(n)
    for t in range(3):
        th2, m2_, v2_ = osno.adam(th2, g[t], m2_, v2_, t + 1, lr, b2=0.99)
    assert np.abs(th2 - want).max() > 1e-5


def test_error_head_fit_equals_lstsq_of_the_augmented_system():
    rng = np.random.default_rng(6)
    n, D = 200, 9
    phi = rng.standard_normal((n, D))
    err = np.exp(phi @ rng.standard_normal(D) * 0.3 - 3.0 + 0.2 * rng.standard_normal(n))
    err[:3] = [0.0, 1e-9, 1e-7]                       # clamped at 1e-6
    ridge = 1e-3
    h, margin = osno.error_head_fit(phi, err, ridge)
    y = np.log(np.maximum(1e-6, err))
    aug = np.concatenate([phi, math.sqrt(ridge * n) * np.eye(D)])
    ref = np.linalg.lstsq(aug, np.concatenate([y, np.zeros(D)]), rcond=None)[0]
    assert np.abs(h - ref).max() < 1e-10 * np.abs(ref).max()
    res = y - phi @ ref
    assert margin == pytest.approx(1.645 * np.sqrt(res @ res / (n - 1)), rel=1e-12)


def test_error_head_margin_covers_95_percent_of_gaussian_residuals():
    rng = np.random.default_rng(8)
    n, D, sigma = 4000, 5, 0.4
    phi = np.concatenate([np.ones((n, 1)), rng.standard_normal((n, D - 1))], axis=1)
    h_true = np.array([-4.0, 0.5, -0.3, 0.2, 0.1])
    err = np.exp(phi @ h_true + sigma * rng.standard_normal(n))
    h, margin = osno.error_head_fit(phi, err, ridge=1e-6)
    assert np.abs(h - h_true).max() < 0.05
    assert margin == pytest.approx(1.645 * sigma, rel=0.05)
    est = osno.error_head_predict(phi, h, margin)
    cover = float(np.mean(err <= est))
    assert 0.93 < cover < 0.97


# ---------------------------------------------------------------------------
# travel-time-aligned frames
def test_delay_by_whole_samples_is_a_zero_filled_shift():
    rng = np.random.default_rng(10)
    u = rng.standard_normal((3, 40))
    for n in (0, 1, 7, -5, 39, 45, -45):
        want = np.zeros_like(u)
        for t in range(40):
            if 0 <= t - n < 40:
                want[:, t] = u[:, t - n]
        assert np.abs(osno.delay(u, float(n)) - want).max() < 1e-14, n


def test_delay_is_exact_for_cubics_away_from_the_edges():
    t = np.arange(64, dtype=np.float64)
    coef = (0.3, -1.2, 0.05, -0.002)
    poly = lambda x: coef[0] + coef[1] * x + coef[2] * x ** 2 + coef[3] * x ** 3
    for delta in (0.37, -2.81, 5.5, 11.999):
        got = osno.delay(poly(t), delta)
        inner = slice(int(math.ceil(delta)) + 3, 64 + int(math.floor(delta)) - 3) if delta > 0 else \
            slice(3, 64 + int(math.floor(delta)) - 3)
        assert np.abs(got[inner] - poly(t[inner] - delta)).max() < 1e-9 * np.abs(poly(t)).max(), delta
    # a quartic is not reproduced: the interpolation is cubic, not higher
    q = (t / 10.0) ** 4
    assert np.abs(osno.delay(q, 0.5)[10:50] - ((t[10:50] - 0.5) / 10.0) ** 4).max() > 1e-6


def test_delay_transpose_is_the_adjoint():
    rng = np.random.default_rng(12)
    u, v = rng.standard_normal((2, 50))
    for delta in (0.0, 0.25, -3.7, 12.6):
        lhs = float(np.dot(osno.delay(u, delta), v))
        rhs = float(np.dot(u, osno.delay_transpose(v, delta)))
        assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs)), delta


def test_straight_ray_times():
    h = (10.0, 12.5, 8.0)
    # homogeneous: distance / speed, in any direction, and the same both ways
    slow = np.full(40, 1 / 2500.0)
    for a, b in [((3, 4, 30), (10, 2, 5)), ((0, 0, 0), (7, 9, 0)), ((5, 5, 2), (5, 5, 38))]:
        d = math.sqrt(sum(((a[k] - b[k]) * h[k]) ** 2 for k in range(3)))
        assert osno.straight_ray_time(a, b, slow, h) == pytest.approx(d / 2500.0, rel=1e-14)
        assert osno.straight_ray_time(a, b, slow, h) == osno.straight_ray_time(b, a, slow, h)
    # layered: the oblique ray against a fine quadrature of the slowness along the segment
    rng = np.random.default_rng(3)
    slow = 1.0 / rng.uniform(1800, 4200, 40)
    a, b = np.array([2, 30, 33]), np.array([17, 3, 6])
    pa, pb = a * np.array(h), b * np.array(h)
    s = (np.arange(400000) + 0.5) / 400000
    pts = pa[None, :] + s[:, None] * (pb - pa)[None, :]
    k = np.floor(pts[:, 2] / h[2] + 0.5).astype(int)       # cell k spans [(k - 1/2) h, (k + 1/2) h)
    quad = np.mean(slow[k]) * np.linalg.norm(pb - pa)
    assert osno.straight_ray_time(a, b, slow, h) == pytest.approx(quad, rel=1e-4)
    # vertical ray: half of each end cell plus the cells between
    assert osno.straight_ray_time((1, 1, 4), (1, 1, 9), slow, h) == pytest.approx(
        h[2] * (0.5 * slow[4] + slow[5:9].sum() + 0.5 * slow[9]), rel=1e-14)


def test_ray_time_reduces_to_the_straight_segment():
    """Homogeneous medium: the two-point ray is the straight segment; a
    vertical path, a path within one layer and a path through a zero
    slowness (fluid S) are the straight segment by construction."""
    h = (10.0, 12.5, 8.0)
    slow = np.full(40, 1 / 2500.0)
    for a, b in [((3, 4, 30), (10, 2, 5)), ((0, 0, 3), (7, 9, 20)), ((5, 5, 2), (25, 1, 38))]:
        d = math.sqrt(sum(((a[k] - b[k]) * h[k]) ** 2 for k in range(3)))
        assert osno.ray_time(a, b, slow, h) == pytest.approx(d / 2500.0, rel=1e-12)
    rng = np.random.default_rng(4)
    slow = 1.0 / rng.uniform(1800, 4200, 40)
    assert osno.ray_time((1, 1, 4), (1, 1, 9), slow, h) == osno.straight_ray_time((1, 1, 4), (1, 1, 9), slow, h)
    assert osno.ray_time((1, 1, 7), (9, 4, 7), slow, h) == osno.straight_ray_time((1, 1, 7), (9, 4, 7), slow, h)
    s0 = slow.copy()
    s0[10] = 0.0
    assert osno.ray_time((1, 1, 4), (9, 1, 19), s0, h) == osno.straight_ray_time((1, 1, 4), (9, 1, 19), s0, h)


def test_ray_time_two_media_against_fermat():
    """Two homogeneous media: the first-arrival time is the minimum over the
    crossing point x of s1 sqrt(x^2 + D1^2) + s2 sqrt((X - x)^2 + D2^2)
    (Fermat), found here by a bounded scalar minimisation."""
    from scipy.optimize import minimize_scalar
    h = (10.0, 10.0, 10.0)
    slow = np.where(np.arange(60) < 25, 1 / 1800.0, 1 / 3600.0)
    for a, b in [((0, 0, 10), (30, 0, 45)), ((2, 3, 5), (40, 20, 55)), ((0, 0, 24), (12, 5, 26))]:
        X = math.hypot((a[0] - b[0]) * h[0], (a[1] - b[1]) * h[1])
        k0, k1 = min(a[2], b[2]), max(a[2], b[2])
        # thickness in each medium: half a cell at each end, whole cells between
        th = np.array([0.5] + [1.0] * (k1 - k0 - 1) + [0.5]) * h[2]
        ks = np.arange(k0, k1 + 1)
        D1, D2 = th[ks < 25].sum(), th[ks >= 25].sum()
        f = lambda x: math.sqrt(x * x + D1 * D1) / 1800.0 + math.sqrt((X - x) ** 2 + D2 * D2) / 3600.0
        best = minimize_scalar(f, bounds=(0.0, X), method="bounded", options={"xatol": 1e-10})
        t = osno.ray_time(a, b, slow, h)
        assert t == pytest.approx(best.fun, rel=1e-9)
        assert t == pytest.approx(osno.ray_time(b, a, slow, h), rel=1e-13)
        assert t < osno.straight_ray_time(a, b, slow, h)


def test_ray_time_is_the_least_time_path_through_many_layers():
    """Forty layers of random slowness: the ray time equals the least time
    over all paths straight within each layer (horizontal runs r_i summing to
    the horizontal distance; time sum s_i sqrt(r_i^2 + t_i^2)), minimised
    numerically without Snell's law, and is below the straight segment's."""
    from scipy.optimize import minimize
    rng = np.random.default_rng(5)
    h = (10.0, 12.5, 8.0)
    slow = 1.0 / rng.uniform(1800, 4200, 60)
    for a, b in [((2, 30, 45), (17, 3, 6)), ((0, 0, 50), (30, 10, 12))]:
        X = math.hypot((a[0] - b[0]) * h[0], (a[1] - b[1]) * h[1])
        th, sl = osno.ray_layers(a, b, slow, h)
        n = th.size

        def T(r):
            return float(np.sum(sl * np.sqrt(r * r + th * th)))

        def J(r):
            return sl * r / np.sqrt(r * r + th * th)

        r0 = np.full(n, X / n)
        res = minimize(T, r0, jac=J, method="SLSQP",
                       constraints=[{"type": "eq", "fun": lambda r: np.sum(r) - X, "jac": lambda r: np.ones(n)}],
                       bounds=[(0.0, X)] * n, options={"ftol": 1e-15, "maxiter": 2000})
        t = osno.ray_time(a, b, slow, h)
        assert t == pytest.approx(res.fun, rel=1e-8)
        assert t <= T(r0) and t < osno.straight_ray_time(a, b, slow, h)


D_FR = osno.Dims(n_pos=3, n_mt=6, four=(3.0, 7.5), C=4, T=32, K=5, L=2, H=6, O=8, frames=2)


def test_gradient_with_aligned_frames_matches_finite_differences():
    rng = np.random.default_rng(21)
    d = D_FR
    theta = init_frames(d, 4) + 0.05 * rng.standard_normal(osno.n_params(d))
    src = rng.standard_normal((2, 9))
    shift = rng.uniform(-4.0, 9.0, (2, 2, d.O // 4))
    y = rng.standard_normal((2, d.O, d.T))
    g = osno.grad(theta, src, y, d, shift=shift)
    idx = rng.choice(theta.size, 60, replace=False)
    idx = np.concatenate([idx, np.arange(theta.size - 2 * d.n_mt * d.O, theta.size, 97)])   # q2b of both frames
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (osno.loss(tp, src, y, d, shift) - osno.loss(tm, src, y, d, shift)) / (2 * h)
        assert abs(fd - g[i]) < 1e-6 * max(1.0, abs(fd)) + 1e-9, i


def test_aligned_frames_delay_each_receiver_by_its_shift():
    """With the network's trunk fixed, delaying frame f of receiver r by one
    more sample delays that receiver's frame-f contribution by exactly one
    sample, and the output stays linear in the moment tensor."""
    rng = np.random.default_rng(22)
    d = D_FR
    theta = init_frames(d, 5) + 0.05 * rng.standard_normal(osno.n_params(d))
    src = rng.standard_normal((1, 9))
    shift = rng.uniform(0.0, 3.0, (1, 2, d.O // 4))
    base = osno.forward(theta, src, d, shift=shift)
    sh2 = shift.copy()
    sh2[0, 1, 1] += 1.0                                   # frame S of receiver 1
    moved = osno.forward(theta, src, d, shift=sh2)
    one = shift.copy()
    one[0, 0, :] = 1e6                                    # frame P pushed out of the window
    s_only = osno.forward(theta, src, d, shift=one)
    sh3 = one.copy()
    sh3[0, 1, 1] += 1.0
    s_moved = osno.forward(theta, src, d, shift=sh3)
    for o in range(d.O):
        if o % (d.O // 4) == 1:
            assert np.abs(s_moved[0, o, 1:] - s_only[0, o, :-1]).max() < 1e-12
        else:
            assert np.abs(moved[0, o] - base[0, o]).max() == 0.0
    m2 = src.copy()
    m2[0, 3:] *= -2.5
    assert np.abs(osno.forward(theta, m2, d, shift=shift) + 2.5 * base).max() < 1e-12 * np.abs(base).max()


def init_frames(d, seed):
    return inputs.sno_init_params(d.C, d.K, d.L, d.H, d.frames * d.O, osno.n_lift(d), seed, d.n_mt)
