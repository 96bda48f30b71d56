"""Pins of the surrogate oracle (oracle/osno.py) against library routines and calculus.

 * the truncated DFT and its inverse equal numpy's FFT with truncation and
   zero padding (a different implementation of the same definition);
 * the hand-written gradient equals central finite differences of the loss
   for every parameter block (FP64);
 * gelu's derivative equals finite differences;
 * Adam's first step moves every weight by lr * sign(g) (bias correction);
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
