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
