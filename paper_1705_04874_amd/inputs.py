"""Seeded synthetic inputs: velocity models, receivers, sources, wavelets, events.

This module is shared by the FP64 CPU oracle (tests) and the GPU path. It holds
no arithmetic of the solver itself (no Lame parameters, no staggered material
averages, no operators): only the recipes that describe the workloads.

The workloads follow the structure of the paper's marine setting (Sec. II-B):
a water column over rock, a plane of four-component sensors on the seabed
(where the shear speed first becomes non-zero), point sources in the rock, and
explosive / double-couple / CLVD mechanisms (Sec. V-A, eq. 6-7). The paper's
Marmousi2-derived models are not available; layered models with a seeded,
Gaussian-correlated perturbation stand in for them.

Index convention: arrays are [nz][ny][nx] (x fastest), z = 0 at the sea
surface and growing downward; a cell index is (i, j, k) = (x, y, z).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


# ----------------------------------------------------------------------------
# wavelets
# ----------------------------------------------------------------------------
def ricker(f0: float, dt: float, nt: int, t0: float | None = None) -> np.ndarray:
    """Ricker wavelet sampled at the stress-update midpoints t = (n + 1/2) dt.

    w(t) = (1 - 2 pi^2 f0^2 (t - t0)^2) exp(-pi^2 f0^2 (t - t0)^2), t0 = 1.5 / f0.
    Used as a moment-rate function (unit 1/s): the source adds
    -dt * w[n] * M / dV to the stress at the source cell in step n.
    """
    if t0 is None:
        t0 = 1.5 / f0
    t = (np.arange(nt, dtype=np.float64) + 0.5) * dt - t0
    a = (math.pi * f0 * t) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def ricker_derivative(f0: float, t: np.ndarray, t0: float | None = None) -> np.ndarray:
    """d/dt of the Ricker wavelet above, evaluated at arbitrary times t."""
    if t0 is None:
        t0 = 1.5 / f0
    tau = np.asarray(t, dtype=np.float64) - t0
    b = (math.pi * f0) ** 2
    return (-6.0 * b * tau + 4.0 * b * b * tau ** 3) * np.exp(-b * tau * tau)


def ricker_value(f0: float, t: np.ndarray, t0: float | None = None) -> np.ndarray:
    if t0 is None:
        t0 = 1.5 / f0
    tau = np.asarray(t, dtype=np.float64) - t0
    a = (math.pi * f0 * tau) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


# ----------------------------------------------------------------------------
# moment tensors, order (xx, yy, zz, xy, xz, yz), unit N*m
# ----------------------------------------------------------------------------
def explosive(m0: float) -> np.ndarray:
    """Isotropic source: equal diagonal entries (Sec. V-A)."""
    return np.array([m0, m0, m0, 0.0, 0.0, 0.0])


def clvd(m0: float) -> np.ndarray:
    """CLVD as diag(1, 1, -2) (eq. 7; the printed -2*sigma_zz read as -2 M0)."""
    return np.array([m0, m0, -2.0 * m0, 0.0, 0.0, 0.0])


def dc_xy(m0: float) -> np.ndarray:
    """The double couple of eq. 7: a single symmetric tau_xy couple."""
    return np.array([0.0, 0.0, 0.0, m0, 0.0, 0.0])


def double_couple(strike: float, dip: float, rake: float, m0: float) -> np.ndarray:
    """Double-couple tensor from fault angles (radians).

    Aki & Richards (Box 4.4) with x = north, y = east, z = down mapped onto
    the grid's x, y, z axes. Trace is zero.
    """
    s, d, r = strike, dip, rake
    sd, cd, s2d, c2d = math.sin(d), math.cos(d), math.sin(2 * d), math.cos(2 * d)
    sr, cr = math.sin(r), math.cos(r)
    ss, cs, s2s, c2s = math.sin(s), math.cos(s), math.sin(2 * s), math.cos(2 * s)
    mxx = -m0 * (sd * cr * s2s + s2d * sr * ss * ss)
    mxy = m0 * (sd * cr * c2s + 0.5 * s2d * sr * s2s)
    mxz = -m0 * (cd * cr * cs + c2d * sr * ss)
    myy = m0 * (sd * cr * s2s - s2d * sr * cs * cs)
    myz = -m0 * (cd * cr * ss - c2d * sr * cs)
    mzz = m0 * s2d * sr
    return np.array([mxx, myy, mzz, mxy, mxz, myz])


def random_dc(rng: np.random.Generator, m0: float) -> np.ndarray:
    """Uniform random strike in [0, 2pi), dip in [0, pi/2], rake in [-pi, pi)."""
    strike = rng.uniform(0.0, 2 * math.pi)
    dip = rng.uniform(0.0, 0.5 * math.pi)
    rake = rng.uniform(-math.pi, math.pi)
    return double_couple(strike, dip, rake, m0)


def dc_plus_iso(rng: np.random.Generator, m0: float, iso_frac: float = 0.2) -> np.ndarray:
    """M = M0 (0.8 * unit DC + 0.2 * I) for iso_frac = 0.2."""
    dc = random_dc(rng, 1.0)
    return m0 * ((1.0 - iso_frac) * dc + iso_frac * explosive(1.0))


# ----------------------------------------------------------------------------
# velocity models
# ----------------------------------------------------------------------------
@dataclass
class Model:
    vp: np.ndarray      # [nz][ny][nx] m/s
    vs: np.ndarray      # [nz][ny][nx] m/s
    rho: np.ndarray     # [nz][ny][nx] kg/m^3

    @property
    def shape(self):
        return self.vp.shape  # (nz, ny, nx)


def homogeneous(nx, ny, nz, vp, vs, rho) -> Model:
    shp = (nz, ny, nx)
    return Model(np.full(shp, float(vp)), np.full(shp, float(vs)), np.full(shp, float(rho)))


def two_layer(n=32, water_cells=8, water=(1500.0, 0.0, 1000.0), rock=(2500.0, 1200.0, 2200.0)) -> Model:
    m = homogeneous(n, n, n, *rock)
    m.vp[:water_cells] = water[0]
    m.vs[:water_cells] = water[1]
    m.rho[:water_cells] = water[2]
    return m


def gardner(vp: np.ndarray) -> np.ndarray:
    """Gardner's density relation rho = 310 vp^0.25 (kg/m^3, vp in m/s)."""
    return 310.0 * np.power(vp, 0.25)


def correlated_field(shape, corr_cells: float, seed: int) -> np.ndarray:
    """Zero-mean Gaussian field with correlation ~exp(-r^2/L^2), max |.| = 1.

    White Gaussian noise filtered by a Gaussian kernel exp(-2 r^2 / L^2).
    """
    rng = np.random.default_rng(seed)
    white = rng.standard_normal(shape)
    spec = np.fft.rfftn(white)
    ks = [np.fft.fftfreq(n) for n in shape[:-1]] + [np.fft.rfftfreq(shape[-1])]
    kk = np.meshgrid(*ks, indexing="ij")
    k2 = sum(k * k for k in kk) * (2 * math.pi) ** 2
    # Fourier transform of exp(-2 r^2/L^2) is proportional to exp(-k^2 L^2 / 8)
    spec *= np.exp(-k2 * corr_cells ** 2 / 8.0)
    f = np.fft.irfftn(spec, s=shape, axes=tuple(range(len(shape))))
    f -= f.mean()
    return f / np.abs(f).max()


def layered(nx, ny, nz, water_cells, n_layers=6, vp_top=2000.0, vp_bot=4000.0,
            vs_ratio=1.8, perturb=0.05, corr_cells=5.0, seed=0) -> Model:
    """Water over flat sediment layers with a correlated +-perturb on vp.

    Layer l (0-based) of n_layers has vp = vp_top + l (vp_bot - vp_top)/(n_layers - 1);
    vs = vp / vs_ratio; rho from Gardner. The perturbation multiplies vp in the
    sediment only, after which vs and rho are recomputed from the perturbed vp.
    Water: vp 1500, vs 0, rho 1000.
    """
    shp = (nz, ny, nx)
    vp = np.full(shp, 1500.0)
    thick = (nz - water_cells) // n_layers
    for l in range(n_layers):
        z0 = water_cells + l * thick
        z1 = nz if l == n_layers - 1 else z0 + thick
        vp[z0:z1] = vp_top + l * (vp_bot - vp_top) / (n_layers - 1)
    if perturb > 0:
        delta = correlated_field(shp, corr_cells, seed) * perturb
        vp[water_cells:] *= 1.0 + delta[water_cells:]
    vs = vp / vs_ratio
    rho = gardner(vp)
    vp[:water_cells] = 1500.0
    vs[:water_cells] = 0.0
    rho[:water_cells] = 1000.0
    return Model(vp, vs, rho)


# ----------------------------------------------------------------------------
# receivers / sources / events
# ----------------------------------------------------------------------------
def receiver_block(x0, x1, y0, y1, z) -> np.ndarray:
    """All (i, j, z) with x0 <= i < x1, y0 <= j < y1, x fastest: int32 [n][3]."""
    jj, ii = np.meshgrid(np.arange(y0, y1), np.arange(x0, x1), indexing="ij")
    out = np.stack([ii.ravel(), jj.ravel(), np.full(ii.size, z)], axis=1)
    return out.astype(np.int32)


def receiver_line_x(x0, x1, y, z) -> np.ndarray:
    return receiver_block(x0, x1, y, y + 1, z)


def latin_hypercube(n: int, lo, hi, rng: np.random.Generator) -> np.ndarray:
    """n points in the box [lo, hi) with one point per stratum on each axis."""
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    d = lo.size
    u = np.empty((n, d))
    for a in range(d):
        perm = rng.permutation(n)
        u[:, a] = (perm + rng.uniform(size=n)) / n
    return lo + u * (hi - lo)


@dataclass
class Events:
    src_idx: np.ndarray    # int32 [n_ev]
    amp: np.ndarray        # float64 [n_ev]
    t_origin: np.ndarray   # float64 [n_ev] seconds


def event_catalogue(n_ev: int, n_src: int, window_s: float, sigma: float, seed: int) -> Events:
    """Events pick a source uniformly (with replacement), amplitude ~ LogNormal(0, sigma),
    origin time ~ U[0, window)."""
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n_src, size=n_ev).astype(np.int32)
    amp = rng.lognormal(0.0, sigma, size=n_ev)
    t = rng.uniform(0.0, window_s, size=n_ev)
    return Events(src, amp, t)


# ----------------------------------------------------------------------------
# workload configurations
# ----------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    model: Model
    d: tuple            # (dx, dy, dz) metres
    dt: float
    nt: int
    pml: int
    pml_A: float
    kspace: int
    c_ref: float        # <= 0: max vp of the model
    rec: np.ndarray     # int32 [n_rec][3]
    # shots: list of point sources per shot
    src_ijk: np.ndarray          # int32 [n_src_total][3]
    src_m: np.ndarray            # float64 [n_src_total][6]
    shot_ofs: np.ndarray         # int32 [n_shots + 1]
    wavelet: np.ndarray          # float64 [n_src_total][nt_w]
    meta: dict = field(default_factory=dict)
    pml_p: float = 0.1           # multi-axial PML ratio
    smooth: int = 0              # source smoothing: 0 point sources, 1 Blackman window in k-space
    chi: np.ndarray = None       # Kelvin-Voigt viscosities per cell (None: lossless)
    eta: np.ndarray = None

    @property
    def n_shots(self):
        return int(self.shot_ofs.size - 1)

    @property
    def cells(self):
        nz, ny, nx = self.model.shape
        return nx * ny * nz


DV_UNIT_MOMENT = 1000.0  # N*m: 1 Pa over a 10 m cube cell


def two_layer_workload() -> Workload:
    """Two layers, 32^3, dx 10 m, dt 1 ms, 300 steps, 8-cell PML, explosive at (16,16,24),
    30 Hz Ricker, 16 receivers on the seabed line x = 8..23, y = 16, z = 8."""
    m = two_layer(32, 8)
    nt = 300
    dt = 1e-3
    rec = receiver_line_x(8, 24, 16, 8)
    return Workload("two_layer_32x32x32", m, (10.0, 10.0, 10.0), dt, nt, 8, 2.0, 1, 0.0, rec,
                    np.array([[16, 16, 24]], np.int32), explosive(DV_UNIT_MOMENT)[None, :],
                    np.array([0, 1], np.int32), ricker(30.0, dt, nt)[None, :])


def layered128_model(seed=0) -> Model:
    return layered(128, 128, 128, water_cells=20, seed=seed)


def layered128_workload(seed_model=0, seed_src=1, nt=2000) -> Workload:
    """128^3, dx 10 m, dt 0.8 ms, 16-cell PML, water over the top 20 cells, 6 layers,
    one random DC at (64, 64, z ~ U{24..104}), 25 Hz Ricker, 64x64 seabed receivers."""
    m = layered128_model(seed_model)
    rng = np.random.default_rng(seed_src)
    z = int(rng.integers(24, 105))
    mt = random_dc(rng, DV_UNIT_MOMENT)
    dt = 0.8e-3
    rec = receiver_block(32, 96, 32, 96, 20)
    return Workload("layered_128x128x128", m, (10.0, 10.0, 10.0), dt, nt, 16, 2.0, 1, 0.0, rec,
                    np.array([[64, 64, z]], np.int32), mt[None, :], np.array([0, 1], np.int32),
                    ricker(25.0, dt, nt)[None, :], meta={"src_z": z})


def layered384_workload(seed_model=0, seed_src=1, nt=4000) -> Workload:
    """384x384x256, same family scaled in z (water 40 cells, 6 x 36 layers), 20-cell PML,
    one random DC laterally centred, 128x128 seabed receivers at z = 40."""
    m = layered(384, 384, 256, water_cells=40, seed=seed_model)
    rng = np.random.default_rng(seed_src)
    z = int(rng.integers(48, 209))
    mt = random_dc(rng, DV_UNIT_MOMENT)
    dt = 0.8e-3
    rec = receiver_block(128, 256, 128, 256, 40)
    return Workload("layered_384x384x256", m, (10.0, 10.0, 10.0), dt, nt, 20, 2.0, 1, 0.0, rec,
                    np.array([[192, 192, z]], np.int32), mt[None, :], np.array([0, 1], np.int32),
                    ricker(25.0, dt, nt)[None, :], meta={"src_z": z})


def layered128_shots(n_shots=64, seed_model=0, seed_src=2, nt=2000) -> Workload:
    """n_shots single-source shots on the 128^3 layered model: positions uniform in the
    500 m cube centred at (64, 64, 70) (x, y in [39, 89), z in [45, 95)), tensors
    0.8 DC + 0.2 ISO, 25 Hz Ricker, 64x64 seabed receivers."""
    m = layered128_model(seed_model)
    rng = np.random.default_rng(seed_src)
    ijk = np.stack([rng.integers(39, 89, n_shots), rng.integers(39, 89, n_shots),
                    rng.integers(45, 95, n_shots)], axis=1).astype(np.int32)
    mts = np.stack([dc_plus_iso(rng, DV_UNIT_MOMENT) for _ in range(n_shots)])
    dt = 0.8e-3
    rec = receiver_block(32, 96, 32, 96, 20)
    w = np.repeat(ricker(25.0, dt, nt)[None, :], n_shots, axis=0)
    return Workload(f"layered_128x128x128_shots{n_shots}", m, (10.0, 10.0, 10.0), dt, nt, 16, 2.0, 1,
                    0.0, rec, ijk, mts, np.arange(n_shots + 1, dtype=np.int32), w)


def ragged_models(n_models=24, seed=5, nt=2000):
    """Uneven grids for the multi-model batch: (nx = ny) from {64..160} x nz from {64..128},
    including 64^3 and 160x160x128; each with one centred DC source."""
    rng = np.random.default_rng(seed)
    lat = [64, 80, 96, 120, 128, 144, 160]
    dep = [64, 80, 96, 128]
    sizes = [(64, 64, 64), (160, 160, 128)]
    while len(sizes) < n_models:
        n = int(rng.choice(lat))
        sizes.append((n, n, int(rng.choice(dep))))
    out = []
    dt = 0.8e-3
    for mi, (nx, ny, nz) in enumerate(sizes):
        water = max(4, round(20 * nz / 128))
        m = layered(nx, ny, nz, water_cells=water, seed=100 + mi)
        mt = random_dc(rng, DV_UNIT_MOMENT)
        zs = water + (nz - water) // 2
        half = min(32, (nx - 2 * 16) // 2)
        rec = receiver_block(nx // 2 - half, nx // 2 + half, ny // 2 - half, ny // 2 + half, water)
        out.append(Workload(f"ragged_{nx}x{ny}x{nz}", m, (10.0, 10.0, 10.0), dt, nt, 16, 2.0, 1, 0.0,
                            rec, np.array([[nx // 2, ny // 2, zs]], np.int32), mt[None, :],
                            np.array([0, 1], np.int32), ricker(25.0, dt, nt)[None, :]))
    return out


# ----------------------------------------------------------------------------
# surrogate initial weights (random numbers the training starts from)
# ----------------------------------------------------------------------------
def sno_param_shapes(C: int, K: int, L: int, H: int, O: int, n_lift: int, n_mt: int = 6):
    """(name, shape) of the surrogate's flat parameter vector, in the order of
    include/sno.h: P, pb, {W_l, b_l, Rr_l, Ri_l}, Q1, q1b, Q2, q2b."""
    s = [("P", (C, n_lift)), ("pb", (C,))]
    for l in range(L):
        s += [(f"W{l}", (C, C)), (f"b{l}", (C,)), (f"Rr{l}", (K, C, C)), (f"Ri{l}", (K, C, C))]
    s += [("Q1", (H, C)), ("q1b", (H,)), ("Q2", (n_mt * O, H)), ("q2b", (n_mt * O,))]
    return s


def sno_init_params(C: int, K: int, L: int, H: int, O: int, n_lift: int, seed: int, n_mt: int = 6) -> np.ndarray:
    """Seeded initial weights (float64 flat vector): uniform(+-1/sqrt(fan_in)) for
    the pointwise maps, uniform(0, 1) / C^2 for the spectral weights, zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, sh in sno_param_shapes(C, K, L, H, O, n_lift, n_mt):
        if name.startswith(("Rr", "Ri")):
            parts.append(rng.uniform(0.0, 1.0, sh) / (C * C))
        elif len(sh) == 2:
            lim = 1.0 / np.sqrt(sh[1])
            parts.append(rng.uniform(-lim, lim, sh))
        else:
            parts.append(np.zeros(sh))
    return np.concatenate([p.ravel() for p in parts])


def sno_fourier_cycles(n: int, lo: float, hi: float) -> tuple:
    """n Fourier feature frequencies (cycles per window) evenly spaced in [lo, hi]."""
    return tuple(float(v) for v in np.linspace(lo, hi, n)) if n > 0 else ()


def paper_shaped_workload(nt=2000, seed_model=0) -> Workload:
    """The paper's simulation shape (Sec. III-A): 125 x 75 x 300 cells (the paper's
    301 rounded to a 2-3-5 length), dx = dy = 12.5 m, dz = 10 m, dt = 0.5 ms,
    2000 steps, 10-cell PML; water over the top 57 cells, 6 perturbed sediment
    layers below; one explosive source of initial pressure 1 Pa (Sec. III-A,
    as a one-sample moment-rate wavelet w[0] = 1/dt with M = 1 Pa x dx dy dz,
    smoothed by the Blackman window in k-space as in Sec. II-A);
    four-component receivers at every (x, y) of the seabed plane z = 57
    (9375 receivers)."""
    nx, ny, nz, water = 125, 75, 300, 57
    m = layered(nx, ny, nz, water_cells=water, seed=seed_model)
    d = (12.5, 12.5, 10.0)
    dt = 0.5e-3
    rec = receiver_block(0, nx, 0, ny, water)
    dv = d[0] * d[1] * d[2]
    w = np.zeros((1, nt))
    w[0, 0] = 1.0 / dt
    return Workload("paper_shaped_125x75x300", m, d, dt, nt, 10, 2.0, 1, 0.0, rec,
                    np.array([[nx // 2, ny // 2, 200]], np.int32), explosive(dv)[None, :],
                    np.array([0, 1], np.int32), w, smooth=1)


def cluster_draws(n: int, k: int, runs: int, seed: int):
    """Random numbers of the clustered catalogue: k distinct initial-centroid
    indices per k-means run (int32 [runs][k]), standard normals and U[0, 1)
    draws per event."""
    rng = np.random.default_rng(seed)
    init = np.stack([rng.choice(n, size=k, replace=False) for _ in range(runs)]).astype(np.int32)
    return init, rng.standard_normal(n), rng.uniform(size=n)


def depth_slowness(model: Model):
    """Mean slowness per depth cell, P and S (s/m): the depth profile a
    travel-time-aligned surrogate uses; 0 for S where the layer is fluid."""
    slow_p = (1.0 / model.vp).mean(axis=(1, 2))
    with np.errstate(divide="ignore"):
        inv_s = np.where(model.vs > 0, 1.0 / np.where(model.vs > 0, model.vs, 1.0), 0.0)
    return slow_p, inv_s.mean(axis=(1, 2))


def straight_ray_reference_times(slow_p, slow_s, src, rec, h):
    """P and S straight-ray times (s) between two cell centres through depth
    profiles of slowness: |d| / |dz| times the depth integral of the slowness
    from centre to centre (|d| times the slowness of the layer for a
    horizontal segment).  Reference times of the aligned surrogate frames."""
    d = np.array([(src[a] - rec[a]) * h[a] for a in range(3)], np.float64)
    L = float(np.linalg.norm(d))
    k0, k1 = int(min(src[2], rec[2])), int(max(src[2], rec[2]))
    out = []
    for sl in (slow_p, slow_s):
        if k0 == k1:
            out.append(L * sl[k0])
        else:
            integ = h[2] * (0.5 * sl[k0] + sl[k0 + 1:k1].sum() + 0.5 * sl[k1])
            out.append(L / abs(d[2]) * integ)
    return tuple(out)
