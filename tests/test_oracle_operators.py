"""Pins of the oracle's staggered spectral derivative operators.

The derivative operators act in the wavenumber domain (Sec. II-A) on a grid
staggered in space.  For a sampled sinusoid of any wavenumber below Nyquist the
staggered operator is exact: D^+ of cos(k x) sampled at integer nodes equals the
analytic derivative at the half nodes x + h/2, and D^- takes half nodes back to
integer nodes.  At the Nyquist wavenumber the staggered symbol is real
(-pi/h for D^+, +pi/h for D^-).  With the k-space correction on, every mode is
scaled by sinc(c |k| dt / 2).
"""
import math

import numpy as np
import pytest

import oracle

SHAPE = (6, 10, 8)          # [z][y][x]
H = (10.0, 12.5, 8.0)       # dx, dy, dz (different on purpose)


def grid(half_axis=None):
    nz, ny, nx = SHAPE
    z, y, x = np.meshgrid(np.arange(nz) * H[2], np.arange(ny) * H[1], np.arange(nx) * H[0],
                          indexing="ij")
    c = [x, y, z]
    if half_axis is not None:
        c[half_axis] = c[half_axis] + 0.5 * H[half_axis]
    return c


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("sign", [+1, -1])
def test_derivative_of_sinusoids_is_exact(axis, sign):
    n = SHAPE[2 - axis]
    L = n * H[axis]
    for m in range(0, n // 2):
        k = 2 * math.pi * m / L
        phi = 0.37
        src = grid(None if sign > 0 else axis)
        dst = grid(axis if sign > 0 else None)
        f = np.cos(k * src[axis] + phi)
        want = -k * np.sin(k * dst[axis] + phi)
        got = oracle.deriv(f, axis, sign, h=H)
        assert np.abs(got - want).max() < 1e-12 * max(1.0, k * 10), (axis, sign, m)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_nyquist_symbol_is_real(axis):
    n = SHAPE[2 - axis]
    idx = np.indices(SHAPE)[2 - axis]
    f = (-1.0) ** idx
    hp = oracle.deriv(f, axis, +1, h=H)
    hm = oracle.deriv(f, axis, -1, h=H)
    assert np.abs(hp - (-math.pi / H[axis]) * f).max() < 1e-12
    assert np.abs(hm - (+math.pi / H[axis]) * f).max() < 1e-12
    assert n % 2 == 0


def test_mixed_mode_with_kspace_correction():
    c, dt = 3000.0, 1.3e-3
    nz, ny, nx = SHAPE
    mx, my, mz = 2, 3, 1
    k = np.array([2 * math.pi * mx / (nx * H[0]), 2 * math.pi * my / (ny * H[1]),
                  2 * math.pi * mz / (nz * H[2])])
    kn = np.linalg.norm(k)
    kap = math.sin(0.5 * c * kn * dt) / (0.5 * c * kn * dt)
    x, y, z = grid()
    f = np.sin(k[0] * x + k[1] * y + k[2] * z)
    for axis in range(3):
        xh, yh, zh = grid(axis)
        want = kap * k[axis] * np.cos(k[0] * xh + k[1] * yh + k[2] * zh)
        got = oracle.deriv(f, axis, +1, h=H, kspace=1, c_ref=c, dt=dt)
        assert np.abs(got - want).max() < 1e-12 * kn


def test_adjoint_identity():
    """D^- = -(D^+)^T in the Euclidean inner product (the property that makes the
    discrete energy exact)."""
    rng = np.random.default_rng(0)
    f = rng.standard_normal(SHAPE)
    g = rng.standard_normal(SHAPE)
    for axis in range(3):
        lhs = np.sum(g * oracle.deriv(f, axis, +1, h=H, kspace=1, c_ref=2000, dt=1e-3))
        rhs = -np.sum(f * oracle.deriv(g, axis, -1, h=H, kspace=1, c_ref=2000, dt=1e-3))
        assert abs(lhs - rhs) < 1e-11 * abs(lhs)
