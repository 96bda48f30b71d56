"""Pins of the oracle's trace superposition (Sec. IV).

 * brute force: a direct pure-Python evaluation of the definition on tiny inputs;
 * the paper's integer-shift procedure (double the record, shift each trace by a
   whole number of samples, zero-pad, add; Case 2) is the special case of
   whole-sample shifts with equal input / output sampling;
 * physics: combining single-source traces equals one solver run with all the
   sources at once, delayed and scaled (linearity and time translation of eq. 2).
"""
import math

import numpy as np

import oracle
from paper_1705_04874_amd import inputs


def brute(tr, t0, src, amp, to, nt_out, dt_in, dt_out):
    n_src, _, n_rec, nt_in = tr.shape
    out = np.zeros((4, n_rec, nt_out))
    for c in range(4):
        for r in range(n_rec):
            for m in range(nt_out):
                acc = 0.0
                for e in range(len(src)):
                    u = (m * dt_out - to[e] - t0[c]) / dt_in
                    i0 = math.floor(u)
                    f = u - i0
                    x = tr[src[e], c, r]
                    x0 = float(x[i0]) if 0 <= i0 < nt_in else 0.0
                    x1 = float(x[i0 + 1]) if 0 <= i0 + 1 < nt_in else 0.0
                    acc += amp[e] * ((1 - f) * x0 + f * x1)
                out[c, r, m] = acc
    return out


def test_combine_matches_brute_force():
    rng = np.random.default_rng(0)
    tr = rng.standard_normal((3, 4, 2, 25)).astype(np.float32)
    t0 = np.array([0.001, 0.0005, 0.0005, 0.0005])
    src = np.array([0, 2, 1, 2, 0], np.int32)
    amp = rng.lognormal(0, 1, 5)
    to = rng.uniform(-0.005, 0.03, 5)
    got = oracle.combine(tr, t0, src, amp, to, 40, 1e-3, 0.7e-3)
    want = brute(tr, t0, src, amp, to, 40, 1e-3, 0.7e-3)
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-13)


def test_integer_shift_is_paper_shift_and_add():
    rng = np.random.default_rng(1)
    nt = 50
    tr = rng.standard_normal((4, 4, 3, nt)).astype(np.float32)
    dt = 1e-3
    src = np.array([3, 1, 1, 0, 2, 3], np.int32)
    amp = rng.uniform(0.5, 2.0, src.size)
    shifts = rng.integers(0, nt, src.size)          # less than the signal length
    got = oracle.combine(tr, np.zeros(4), src, amp, shifts * dt, 2 * nt, dt, dt)
    rec = np.zeros((4, 3, 2 * nt))                  # doubled record, zero padded
    for e in range(src.size):
        rec[..., shifts[e]:shifts[e] + nt] += amp[e] * tr[src[e]].astype(np.float64)
    np.testing.assert_allclose(got, rec, rtol=0, atol=1e-12)


def test_combine_equals_joint_simulation():
    """Superposed single-event records equal one run with all events at once."""
    shape = (16, 14, 18)
    vp = np.full(shape, 2800.0)
    vs = np.full(shape, 1600.0)
    rho = np.full(shape, 2200.0)
    vp[:4], vs[:4], rho[:4] = 1500.0, 0.0, 1000.0
    h = (10.0, 10.0, 10.0)
    dt = 0.8e-3
    nt = 70
    rec = inputs.receiver_block(4, 14, 5, 9, 4)
    w = inputs.ricker(30.0, dt, nt)
    pos = np.array([[8, 7, 10], [5, 9, 12], [11, 6, 9]])
    mts = [inputs.double_couple(0.3, 0.7, 1.1, 1000.0), inputs.explosive(700.0),
           inputs.clvd(400.0)]
    singles = []
    for p, m in zip(pos, mts):
        s = oracle.Solver(vp, vs, rho, h, dt, pml=4, kspace=1, rec=rec)
        s.set_sources(p[None], m[None], w[None])
        singles.append(s.run(nt))
    singles = np.stack(singles).astype(np.float32)
    src = np.array([0, 1, 2, 1], np.int32)
    amp = np.array([1.5, 0.5, 2.0, 1.25])
    lag = np.array([3, 11, 0, 25])
    joint = oracle.Solver(vp, vs, rho, h, dt, pml=4, kspace=1, rec=rec)
    wav = np.stack([np.concatenate([np.zeros(l), w[:nt - l]]) for l in lag])
    joint.set_sources(pos[src], np.stack([a * mts[s] for a, s in zip(amp, src)]), wav)
    ref = joint.run(nt)
    got = oracle.combine(singles, np.zeros(4), src, amp, lag * dt, nt, dt, dt)
    for c in range(4):
        err = np.linalg.norm(got[c] - ref[c]) / np.linalg.norm(ref[c])
        assert err < 1e-6, (c, err)   # single-event traces were stored in FP32
