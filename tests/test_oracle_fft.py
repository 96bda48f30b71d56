"""Pins of the oracle's own FFT against brute-force DFTs and exact identities.

The spatial derivatives of the method are taken by FFT / IFFT (Sec. II-A); the
oracle's transform must therefore be right on every length the solver uses
(products of 2, 3 and 5) before anything built on it can be trusted.
"""
import numpy as np
import pytest

import oracle


def brute_dft(x, sign=-1):
    n = x.size
    j = np.arange(n)
    return np.exp(sign * 2j * np.pi * np.outer(j, j) / n) @ x


def smooth_lengths(limit):
    return [n for n in range(1, limit + 1)
            if all(p in (2, 3, 5) for p in _factors(n))]


def _factors(n):
    f, p = [], 2
    while n > 1:
        while n % p == 0:
            f.append(p)
            n //= p
        p += 1
    return f


@pytest.mark.parametrize("n", smooth_lengths(64) + [7, 11, 13, 49])
def test_fft_matches_brute_force_dft(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    ref = brute_dft(x)
    got = oracle.fft(x)
    assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
    inv = oracle.fft(x, inverse=True)
    assert np.abs(inv - brute_dft(x, +1) / n).max() <= 1e-12 * max(1.0, np.abs(x).max())


@pytest.mark.parametrize("n", [1, 2, 6, 30, 64, 75, 125, 128, 384])
def test_fft_roundtrip_and_parseval(n):
    rng = np.random.default_rng(1000 + n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    X = oracle.fft(x)
    back = oracle.fft(X, inverse=True)
    assert np.abs(back - x).max() < 1e-13 * np.sqrt(n)
    # Parseval: sum |x|^2 = (1/n) sum |X|^2
    assert abs(np.vdot(x, x).real - np.vdot(X, X).real / n) < 1e-12 * np.vdot(x, x).real


def test_fft_impulse_and_single_tone():
    n = 60
    e = np.zeros(n, complex)
    e[7] = 1.0
    X = oracle.fft(e)
    k = np.arange(n)
    assert np.abs(X - np.exp(-2j * np.pi * 7 * k / n)).max() < 1e-13
    tone = np.exp(2j * np.pi * 11 * k / n)
    T = oracle.fft(tone)
    expect = np.zeros(n, complex)
    expect[11] = n
    assert np.abs(T - expect).max() < 1e-11


def test_fft3_is_separable_brute_force():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((4, 5, 6)) + 1j * rng.standard_normal((4, 5, 6))   # [z][y][x]
    ref = a.copy()
    for ax in range(3):
        ref = np.apply_along_axis(brute_dft, ax, ref)
    got = oracle.fft3(a)
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
    back = oracle.fft3(got, inverse=True)
    assert np.abs(back - a).max() < 1e-13
