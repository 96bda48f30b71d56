"""Closed forms used to pin the solvers (shared by the oracle tests and the GPU tests).

Nothing here calls either solver; it only writes down textbook physics:
exact discrete plane waves of the staggered leapfrog scheme, the discrete
energy, and the homogeneous whole-space response to an explosive point source.
"""
import math

import numpy as np

# state order: v[c][d] (9), normal s[c][d] (9), shear xy(x,y) xz(x,z) yz(y,z) (6)
V_FIRST = {0: 0, 1: 3, 2: 6}            # first split part of vx, vy, vz
N_FIRST = {0: 9, 1: 12, 2: 15}          # sxx, syy, szz
S_FIRST = {(0, 1): 18, (0, 2): 20, (1, 2): 22}


def node_coords(shape, h, offset):
    """Physical coordinates (x, y, z) of the nodes of a field offset by
    `offset` cells (e.g. (0.5, 0, 0) for vx)."""
    nz, ny, nx = shape
    z, y, x = np.meshgrid((np.arange(nz) + offset[2]) * h[2], (np.arange(ny) + offset[1]) * h[1],
                          (np.arange(nx) + offset[0]) * h[0], indexing="ij")
    return x, y, z


OFFSETS = {
    "vx": (0.5, 0, 0), "vy": (0, 0.5, 0), "vz": (0, 0, 0.5),
    "sxx": (0, 0, 0), "syy": (0, 0, 0), "szz": (0, 0, 0),
    "sxy": (0.5, 0.5, 0), "sxz": (0.5, 0, 0.5), "syz": (0, 0.5, 0.5),
}


def plane_wave_state(shape, h, dt, m, wave, vp, vs, rho, n, kspace, c_ref, amp=1e-3, phase=0.3):
    """Exact state (v^{n-1/2}, s^n) of a periodic plane P or S wave of the
    staggered leapfrog scheme in a homogeneous medium.

    For a single Fourier mode the staggered operators are exact derivatives
    times kappa, so the discrete system is the continuous one with k -> kappa k
    and omega -> (2/dt) sin(omega dt / 2).  Hence sin(omega dt/2) = (c dt/2)|k| kappa
    and the stress / velocity amplitudes satisfy the continuous impedance
    relations: P: s_ij = -(V/vp)(lam d_ij + 2 mu k_i k_j); S (polarisation e):
    s_ij = -(mu V/vs)(k_i e_j + e_i k_j).
    """
    nz, ny, nx = shape
    N = (nx, ny, nz)
    k = np.array([2 * math.pi * m[a] / (N[a] * h[a]) for a in range(3)])
    kn = np.linalg.norm(k)
    khat = k / kn
    mu = rho * vs * vs
    lam = rho * vp * vp - 2 * mu
    if kspace:
        x = 0.5 * c_ref * kn * dt
        kap = math.sin(x) / x
    else:
        kap = 1.0
    if wave == "P":
        c = vp
        e = khat
        S = -(amp / vp) * (lam * np.eye(3) + 2 * mu * np.outer(khat, khat))
    else:
        c = vs
        t = np.array([1.0, 0.0, 0.0]) if abs(khat[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
        e = np.cross(khat, t)
        e /= np.linalg.norm(e)
        S = -(mu * amp / vs) * (np.outer(khat, e) + np.outer(e, khat))
    omega = 2.0 / dt * math.asin(0.5 * c * dt * kn * kap)
    state = np.zeros((24,) + tuple(shape))
    tv = (n - 0.5) * dt
    ts = n * dt
    names = ["vx", "vy", "vz"]
    for a in range(3):
        x, y, z = node_coords(shape, h, OFFSETS[names[a]])
        state[V_FIRST[a]] = amp * e[a] * np.cos(k[0] * x + k[1] * y + k[2] * z - omega * tv + phase)
    for a, nm in zip(range(3), ["sxx", "syy", "szz"]):
        x, y, z = node_coords(shape, h, OFFSETS[nm])
        state[N_FIRST[a]] = S[a, a] * np.cos(k[0] * x + k[1] * y + k[2] * z - omega * ts + phase)
    for (a, b), nm in zip([(0, 1), (0, 2), (1, 2)], ["sxy", "sxz", "syz"]):
        x, y, z = node_coords(shape, h, OFFSETS[nm])
        state[S_FIRST[(a, b)]] = S[a, b] * np.cos(k[0] * x + k[1] * y + k[2] * z - omega * ts + phase)
    return state


def summed(state):
    """(vx, vy, vz, sxx, syy, szz, sxy, sxz, syz) from the 24 split parts."""
    v = [state[3 * c:3 * c + 3].sum(0) for c in range(3)]
    s = [state[9 + 3 * c:9 + 3 * c + 3].sum(0) for c in range(3)]
    sh = [state[18:20].sum(0), state[20:22].sum(0), state[22:24].sum(0)]
    return v + s + sh


# first split part and part count of vx vy vz sxx syy szz sxy sxz syz
FIELD_PARTS = [("vx", 0, 3), ("vy", 3, 3), ("vz", 6, 3), ("sxx", 9, 3), ("syy", 12, 3), ("szz", 15, 3),
               ("sxy", 18, 2), ("sxz", 20, 2), ("syz", 22, 2)]


def undamped_mask(shape, lo, hi):
    """Boolean [nz][ny][nx]: the cells with lo[d] <= index <= hi[d] on every
    axis d = (x, y, z), where the absorbing layer leaves the split update
    undamped."""
    nz, ny, nx = shape
    mx = (np.arange(nx) >= lo[0]) & (np.arange(nx) <= hi[0])
    my = (np.arange(ny) >= lo[1]) & (np.arange(ny) <= hi[1])
    mz = (np.arange(nz) >= lo[2]) & (np.arange(nz) <= hi[2])
    return mz[:, None, None] & my[None, :, None] & mx[None, None, :]


def collapse_undamped(state, mask):
    """The split state as the GPU keeps it: in the cells of `mask` each field's
    parts summed into its first part and the others zero (state [F][...] with
    the 24 split parts first; mask of the trailing shape)."""
    st = np.array(state, dtype=np.float64, copy=True)
    for _, f0, n in FIELD_PARTS:
        tot = st[f0:f0 + n][:, mask].sum(axis=0)
        st[f0][mask] = tot
        for k in range(1, n):
            st[f0 + k][mask] = 0.0
    return st


def split_errors(got, ref):
    """Per field: (name, rel-L2 of the field (sum of its parts), largest
    rel-L2 of one part on the scale of the field's norm) of got against ref."""
    out = []
    for name, f0, n in FIELD_PARTS:
        fr = ref[f0:f0 + n].sum(axis=0)
        nf = float(np.linalg.norm(fr))
        ef = float(np.linalg.norm(got[f0:f0 + n].astype(np.float64).sum(axis=0) - fr)) / nf
        ep = max(float(np.linalg.norm(got[f0 + k].astype(np.float64) - ref[f0 + k])) / nf for k in range(n))
        out.append((name, ef, ep))
    return out


def staggered_materials(vp, vs, rho):
    """rho at velocity nodes, lam/mu at centres and mu at shear nodes, with the
    same averaging reading the solvers take (arithmetic rho, harmonic mu)."""
    mu = rho * vs * vs
    lam = rho * vp * vp - 2 * mu

    def up(a, axis):
        # neighbour one cell up along `axis` (array axes are z, y, x), clamped
        ax = 2 - axis
        idx = np.arange(a.shape[ax]) + 1
        idx[-1] = a.shape[ax] - 1
        return np.take(a, idx, axis=ax)

    rho_n = [0.5 * (rho + up(rho, d)) for d in range(3)]
    mus = []
    for (a, b) in [(0, 1), (0, 2), (1, 2)]:
        q = [mu, up(mu, a), up(mu, b), up(up(mu, a), b)]
        fluid = np.any([qq == 0 for qq in q], axis=0)
        with np.errstate(divide="ignore"):
            hm = 4.0 / sum(1.0 / np.where(qq == 0, 1.0, qq) for qq in q)
        mus.append(np.where(fluid, 0.0, hm))
    return rho_n, lam, mu, mus


def discrete_energy(before, after, vp, vs, rho, dV=1.0):
    """E^n = 1/2 sum rho_c v^{n-1/2} v^{n+1/2} + 1/2 s^n C^{-1} s^n, the quantity the
    lossless staggered leapfrog scheme conserves exactly."""
    rho_n, lam, mu, mus = staggered_materials(vp, vs, rho)
    vb = summed(before)
    va = summed(after)
    ek = 0.5 * sum(np.sum(rho_n[c] * vb[c] * va[c]) for c in range(3))
    sxx, syy, szz = vb[3], vb[4], vb[5]
    solid = mu > 0
    tr = sxx + syy + szz
    with np.errstate(divide="ignore", invalid="ignore"):
        e_solid = (sxx ** 2 + syy ** 2 + szz ** 2 - lam / (3 * lam + 2 * mu) * tr ** 2) / (4 * mu)
        e_fluid = sxx ** 2 / (2 * lam)
    en = np.sum(np.where(solid, e_solid, e_fluid))
    es = 0.0
    for p in range(3):
        sh = vb[6 + p]
        with np.errstate(divide="ignore", invalid="ignore"):
            es += np.sum(np.where(mus[p] > 0, sh ** 2 / (2 * mus[p]), 0.0))
    return (ek + en + es) * dV


def explosion_pressure(t, r, m0, vp, vs, rho, f0):
    """Whole-space pressure from an explosive point source with moment rate
    m0 * w(t) (w a Ricker wavelet): p = m0 K w'(t - r/vp) / (4 pi rho vp^4 r),
    K = lam + 2 mu / 3 (Aki & Richards, Sec. 4.2)."""
    from paper_1705_04874_amd.inputs import ricker_derivative
    K = rho * vp * vp - 4.0 / 3.0 * rho * vs * vs
    return m0 * K * ricker_derivative(f0, t - r / vp) / (4 * math.pi * rho * vp ** 4 * r)


def explosion_radial_velocity(t, r, m0, vp, rho, f0):
    """Whole-space radial particle velocity from an explosive point source with
    moment rate m0 * w(t) (w a Ricker wavelet): the time derivative of the
    displacement u_r = m0 / (4 pi rho vp^2) [S(tau) / r^2 + S'(tau) / (vp r)],
    tau = t - r / vp, S' = w (Aki & Richards, Sec. 4.2), i.e.
    v_r = m0 / (4 pi rho vp^2) [w(tau) / r^2 + w'(tau) / (vp r)]: a near-field
    term in 1/r^2 and a far-field term in 1/r."""
    from paper_1705_04874_amd.inputs import ricker_derivative, ricker_value
    tau = t - r / vp
    return m0 / (4 * math.pi * rho * vp * vp) * (ricker_value(f0, tau) / (r * r) +
                                                 ricker_derivative(f0, tau) / (vp * r))
