"""Pins of the oracle's perfectly matched layer (Sec. II-B reserves grid points
at the edges for an absorbing layer; the split-field profile is a reading of
this build: alpha_d = (A c_ref / h_d) (depth / L)^4, depth measured from the
layer's inner edge at integer and half nodes, a = exp(-alpha dt / 2) applied
before and after the update, and the multi-axial factor b = a^p of the two
other axes).

 * One step of uniform fields: every derivative of a uniform field is zero, so
   one step multiplies each split part by exactly (a_d b_e b_f)^2 at its own
   node; the test reads that factor off every cell of every part and compares
   it with the profile written out from the reading above, with anisotropic
   spacing, an explicit c_ref, p = 0 and p = 0.1.
 * Reflection (the physical pin): an explosion near the +x face of a grid with
   the PML against the same run on a grid three times longer in x, whose own
   faces are too far away to be heard in the window; the difference is what
   the small grid's x faces send back.  It stays below -40 dB of the direct
   wave's energy, while a layer with a quarter of the absorption (A = 0.5,
   the control) reflects far more.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1705_04874_amd import inputs

# split part -> (component node offsets per axis, axis the part belongs to)
# velocity parts v_c^(d): the node of v_c is half a cell up along c
# normal stress parts s_cc^(d): cell centre; shear s_cd^(d) at the (c, d) shear node
PARTS = []
for c in range(3):
    for d in range(3):
        PARTS.append((tuple(0.5 if a == c else 0.0 for a in range(3)), d))          # v_c^(d)
for c in range(3):
    for d in range(3):
        PARTS.append(((0.0, 0.0, 0.0), d))                                          # s_cc^(d)
for (c, e) in [(0, 1), (0, 2), (1, 2)]:
    node = tuple(0.5 if a in (c, e) else 0.0 for a in range(3))
    PARTS.append((node, c))                                                         # s_ce^(c)
    PARTS.append((node, e))                                                         # s_ce^(e)


def alpha(s, n, L, A, c_ref, h):
    """Absorption at node coordinate s (cells) of an axis of n cells."""
    depth = min(max(max(L - s, s - (n - 1 - L)), 0.0), float(L))
    return A * c_ref / h * (depth / L) ** 4


def expected_factor(node, d, idx, N, L, A, p, c_ref, h, dt):
    """(a_d b_e b_f)^2 of a split part along axis d at grid index idx."""
    f = 1.0
    for ax in range(3):
        al = alpha(idx[ax] + node[ax], N[ax], L, A, c_ref, h[ax])
        f *= math.exp(-(1.0 if ax == d else p) * al * dt / 2)
    return f * f


@pytest.mark.parametrize("p", [0.0, 0.1])
def test_one_step_of_uniform_fields_damps_each_part_by_its_profile(p):
    shape = (16, 18, 20)                    # [z][y][x]
    N = (20, 18, 16)
    h = (10.0, 12.5, 8.0)
    L, A, c_ref, dt = 5, 2.0, 3500.0, 0.6e-3
    vp, vs, rho = [np.full(shape, v) for v in (3000.0, 1700.0, 2300.0)]
    s = oracle.Solver(vp, vs, rho, h, dt, pml=L, pml_A=A, pml_p=p, kspace=1, c_ref=c_ref)
    s.set_sources(np.zeros((0, 3)), np.zeros((0, 6)), np.zeros((0, 1)))
    kk, jj, ii = np.meshgrid(np.arange(N[2]), np.arange(N[1]), np.arange(N[0]), indexing="ij")
    # velocity parts from (v uniform, sigma = 0); stress parts from (sigma uniform, v = 0):
    # in each case the fields the checked parts feed back from stay zero for one step
    for first, last in [(0, 9), (9, 24)]:
        st = np.zeros((24,) + shape)
        st[first:last] = 1.0
        s.set_state(st)
        s.step = 0
        s.run(1)
        got = s.get_state()
        for f in range(first, last):
            node, d = PARTS[f]
            want = np.vectorize(lambda i, j, k: expected_factor(node, d, (i, j, k), N, L, A, p, c_ref, h, dt))(
                ii, jj, kk)
            assert np.abs(got[f] - want).max() < 1e-12, (f, np.abs(got[f] - want).max())
        # the profile is not trivial: the deepest node is damped strongly, the interior not at all
        assert got[first:last].min() < 0.7 and got[first:last].max() == pytest.approx(1.0, abs=1e-12)
    s.close()


def reflection_db(A, L=6, nt=220):
    """Energy of (small grid - 3x longer grid) over the direct wave's, in dB, at
    three receivers between an explosion and the +x face of the small grid."""
    ny = nz = 4 * L
    nx = 6 * L
    f0, dt = 30.0, 1e-3
    offs = [L // 2, L, 2 * L - 3]
    out = []
    for n in (nx, 3 * nx):
        m = inputs.homogeneous(n, ny, nz, 3000.0, 1700.0, 2400.0)
        sx = n // 2
        rec = np.array([[sx + o, ny // 2, nz // 2] for o in offs], np.int32)
        s = oracle.Solver(m.vp, m.vs, m.rho, (10.0, 10.0, 10.0), dt, pml=L, pml_A=A, pml_p=0.1, kspace=1, rec=rec)
        s.set_sources(np.array([[sx, ny // 2, nz // 2]]), inputs.explosive(1000.0)[None],
                      inputs.ricker(f0, dt, nt)[None])
        out.append(s.run(nt))
        s.close()
    small, big = out
    d = small - big
    return [10 * math.log10(np.sum(d[:, i] ** 2) / np.sum(big[:, i] ** 2)) for i in range(len(offs))]


def test_pml_reflection_is_below_minus_40_db():
    db = reflection_db(2.0)
    assert max(db) < -40.0, db
    # control: a quarter of the absorption is plainly visible to the same measure
    weak = reflection_db(0.5)
    assert max(weak) > -30.0, weak
    assert all(w > x + 15.0 for w, x in zip(weak, db)), (weak, db)


def test_undamped_cells_need_only_the_sum_of_their_split_parts():
    """Where every factor of the split update is exactly 1 the parts of a field
    evolve without damping and only their sum enters the physics: summing them
    into the first part there (the form the GPU keeps) and zeroing the others
    leaves every field of the oracle's run unchanged to FP64 rounding over
    further steps, and those cells are exactly the box [L, n - 2 - L] on every
    axis of the profile above (at L - 1 and n - 1 - L a half node is damped)."""
    from tests import physics
    nz, ny, nx = 22, 20, 26
    L, A, dt = 5, 2.0, 0.8e-3
    N = (nx, ny, nz)
    rng = np.random.default_rng(9)
    vp = 2500.0 + 300.0 * rng.random((nz, ny, nx))
    vs = vp / 1.8
    rho = 2000.0 + 100.0 * rng.random((nz, ny, nx))
    c_ref = float(vp.max())
    # undamped along an axis: the integer and the half node of the index both have alpha = 0
    flat = [np.array([alpha(i, n, L, A, c_ref, 10.0) == 0.0 and alpha(i + 0.5, n, L, A, c_ref, 10.0) == 0.0
                      for i in range(n)]) for n in N]
    lo = tuple(int(np.argmax(f)) for f in flat)
    hi = tuple(int(len(f) - 1 - np.argmax(f[::-1])) for f in flat)
    assert lo == (L, L, L) and hi == (nx - 2 - L, ny - 2 - L, nz - 2 - L)
    assert all(f[l:h + 1].all() and not f[:l].any() and not f[h + 1:].any() for f, l, h in zip(flat, lo, hi))
    mask = physics.undamped_mask((nz, ny, nx), lo, hi)
    m6 = inputs.random_dc(rng, 1000.0)[None]

    def solver():
        s = oracle.Solver(vp, vs, rho, (10.0, 10.0, 10.0), dt, pml=L, pml_A=A, pml_p=0.1, kspace=1, c_ref=c_ref,
                          rec=np.array([[nx // 2, ny // 2, 3], [L + 1, ny // 2, nz // 2]], np.int32))
        s.set_sources(np.array([[nx // 2 + 2, ny // 2 - 1, nz // 2]]), m6, inputs.ricker(40.0, dt, 120)[None])
        return s

    a = solver()
    a.run(40)
    st = a.get_state()
    b = solver()
    b.set_state(physics.collapse_undamped(st, mask))
    b.step = 40
    assert np.abs(st[1][mask]).max() > 0           # the uncollapsed state does split the interior
    tra, trb = a.run(60), b.run(60)
    sa, sb = physics.summed(a.get_state()), physics.summed(b.get_state())
    for fa, fb in zip(sa, sb):
        assert np.abs(fa - fb).max() <= 1e-12 * np.abs(fa).max()
    assert np.abs(tra - trb).max() <= 1e-12 * np.abs(tra).max()
    a.close()
    b.close()
