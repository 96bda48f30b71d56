"""FP64 oracle of the spectral neural operator surrogate (test infrastructure only).

The paper names a learned proxy of the forward simulation as future work
(Sec. VII); the surrogate here maps a point source (position and moment tensor)
to four-component receiver traces with a Fourier neural operator along time.
The elastic system is linear in the source term (eq. 2; the superposition of
Sec. IV rests on it), so the output is a linear combination of six responses
weighted by the moment-tensor components, and the network sees the position
only:

  lift:     V0 = P A + pb,   A = [position broadcast; t_j / T;
                                  cos, sin(2 pi c_f t_j / T) for the Fourier
                                  feature frequencies c_f (cycles per window)]
  layer l:  Vh = V F                  truncated DFT, F = [cos | -sin](2 pi j k / T), k < K
            U_k = R_l[k] Vh_k         complex C x C mixing per retained mode k
            U  = Uh G                 inverse DFT of the K modes of a real signal
            Z  = W_l V + b_l + U
            V  = gelu(Z)  (no activation after the last layer)
  project:  Y6 = Q2 gelu(Q1 V + q1b) + q2b                     (frames x 6 O x T)
  output:   Y[o](t) = sum_f sum_j m_j Y6[f][j O + o](t - shift[f][r(o)]),
            m = the 6 moment-tensor features, r(o) = o mod n_rec the receiver

With one frame and no shift this is a plain operator along time.  With two
frames the network's time axis is a travel-time-aligned one: frame P (S) of
receiver r is delayed by the straight-ray P (S) travel time from the source to
r minus a reference time, so the direct arrivals sit at fixed frame times for
every source and the network only has to learn their amplitudes and shapes.
The delay is fractional: the delayed series is the 4-point Lagrange (cubic)
interpolation of the frame, zero outside its samples.

gelu(x) = x/2 (1 + tanh(sqrt(2/pi) (x + 0.044715 x^3))).  Loss: mean squared
error over the batch and all outputs.  Gradients are written out by hand
(reverse mode), each step the transpose of its forward step.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class Dims:
    n_pos: int = 3         # position features (broadcast along time)
    n_mt: int = 6          # moment-tensor features (the output is linear in them)
    four: tuple = ()       # Fourier time features: frequencies in cycles per window
    pos_mod: bool = False  # also each position feature times each cos / sin feature
    C: int = 64            # width
    T: int = 1024          # time samples
    K: int = 16            # retained modes
    L: int = 4             # Fourier layers
    H: int = 128           # projection hidden width
    O: int = 256           # outputs per time sample (4 components x 64 receivers)
    frames: int = 1        # output frames: 1 (plain time axis) or 2 (P- and S-aligned, shifted per receiver)


def n_lift(d: Dims):
    """Input channels of the lift: position, t / T, cos and sin per frequency,
    and with position modulation n_pos x (cos, sin) products per frequency."""
    return d.n_pos + 1 + 2 * len(d.four) + (2 * d.n_pos * len(d.four) if d.pos_mod else 0)


def param_shapes(d: Dims):
    """Ordered (name, shape) list; the flat parameter vector follows this order."""
    s = [("P", (d.C, n_lift(d))), ("pb", (d.C,))]
    for l in range(d.L):
        s += [(f"W{l}", (d.C, d.C)), (f"b{l}", (d.C,)), (f"Rr{l}", (d.K, d.C, d.C)), (f"Ri{l}", (d.K, d.C, d.C))]
    s += [("Q1", (d.H, d.C)), ("q1b", (d.H,)), ("Q2", (d.frames * d.n_mt * d.O, d.H)),
          ("q2b", (d.frames * d.n_mt * d.O,))]
    return s


def n_params(d: Dims):
    return sum(int(np.prod(sh)) for _, sh in param_shapes(d))


def unflatten(theta, d: Dims):
    out, o = {}, 0
    for name, sh in param_shapes(d):
        n = int(np.prod(sh))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(sh)
        o += n
    return out


def flatten(p, d: Dims):
    return np.concatenate([np.asarray(p[name], np.float64).ravel() for name, _ in param_shapes(d)])


def dft_bases(d: Dims):
    """F (T x 2K): [cos | -sin](2 pi j k / T); G (2K x T): inverse of the K modes
    of a real signal, [w_k cos / T ; -w_k sin / T], w_0 = 1, w_k = 2."""
    j = np.arange(d.T)[:, None]
    k = np.arange(d.K)[None, :]
    ang = 2 * math.pi * j * k / d.T
    F = np.concatenate([np.cos(ang), -np.sin(ang)], axis=1)
    w = np.where(np.arange(d.K) == 0, 1.0, 2.0)[None, :]
    G = np.concatenate([(w * np.cos(ang)).T, (-w * np.sin(ang)).T], axis=0) / d.T
    return F, G


def gelu(x):
    c = math.sqrt(2 / math.pi)
    return 0.5 * x * (1 + np.tanh(c * (x + 0.044715 * x ** 3)))


def gelu_grad(x):
    c = math.sqrt(2 / math.pi)
    u = c * (x + 0.044715 * x ** 3)
    th = np.tanh(u)
    return 0.5 * (1 + th) + 0.5 * x * (1 - th * th) * c * (1 + 3 * 0.044715 * x * x)


def features(src, d: Dims):
    """A (B x n_lift x T): the position features of src (B x (n_pos + n_mt))
    broadcast along time, t_j = j / T, then cos and sin of 2 pi c_f t_j / T."""
    src = np.asarray(src, np.float64)
    B = src.shape[0]
    t = np.arange(d.T) / d.T
    A = np.empty((B, n_lift(d), d.T))
    A[:, :d.n_pos, :] = src[:, :d.n_pos, None]
    A[:, d.n_pos, :] = t
    for f, c in enumerate(d.four):
        A[:, d.n_pos + 1 + 2 * f, :] = np.cos(2 * math.pi * c * t)
        A[:, d.n_pos + 2 + 2 * f, :] = np.sin(2 * math.pi * c * t)
    if d.pos_mod:
        # products with the position features, order (frequency, position, cos / sin)
        base = d.n_pos + 1 + 2 * len(d.four)
        for f, c in enumerate(d.four):
            for k in range(d.n_pos):
                A[:, base + 2 * (d.n_pos * f + k), :] = src[:, k, None] * np.cos(2 * math.pi * c * t)
                A[:, base + 2 * (d.n_pos * f + k) + 1, :] = src[:, k, None] * np.sin(2 * math.pi * c * t)
    return A


def moments(src, d: Dims):
    """The n_mt moment-tensor features of src (B x n_mt)."""
    return np.asarray(src, np.float64)[:, d.n_pos:d.n_pos + d.n_mt]


def forward(theta, src, d: Dims, keep=False, shift=None):
    p = unflatten(theta, d)
    F, G = dft_bases(d)
    A = features(src, d)
    V = np.einsum("ci,bit->bct", p["P"], A) + p["pb"][None, :, None]
    cache = {"A": A, "V": [V], "Vh": [], "Z": []}
    for l in range(d.L):
        Vh = V @ F                                              # B x C x 2K
        Vr, Vi = Vh[..., :d.K], Vh[..., d.K:]
        Rr, Ri = p[f"Rr{l}"], p[f"Ri{l}"]                       # K x C x C
        Ur = np.einsum("koc,bck->bok", Rr, Vr) - np.einsum("koc,bck->bok", Ri, Vi)
        Ui = np.einsum("koc,bck->bok", Ri, Vr) + np.einsum("koc,bck->bok", Rr, Vi)
        U = np.concatenate([Ur, Ui], axis=2) @ G                # B x C x T
        Z = np.einsum("oc,bct->bot", p[f"W{l}"], V) + p[f"b{l}"][None, :, None] + U
        V = gelu(Z) if l < d.L - 1 else Z
        cache["Vh"].append(Vh)
        cache["Z"].append(Z)
        cache["V"].append(V)
    Hp = np.einsum("hc,bct->bht", p["Q1"], V) + p["q1b"][None, :, None]
    Hq = gelu(Hp)
    Y6 = np.einsum("oh,bht->bot", p["Q2"], Hq) + p["q2b"][None, :, None]
    Y6 = Y6.reshape(Y6.shape[0], d.frames, d.n_mt, d.O, d.T)
    m = moments(src, d)
    # each frame's rows are delayed by their receiver's shift, then combined
    Yf = Y6 if shift is None else frame_shift(Y6, shift, d)
    Y = np.einsum("bj,bfjot->bot", m, Yf)
    cache.update(Hp=Hp, Hq=Hq, m=m)
    return (Y, cache) if keep else Y


def element_weights(w, d: Dims):
    """Per-element loss weights from per-(sample, component) ones: w [B][4]
    -> [B][O][1] (output o belongs to component o // n_rec); None -> 1."""
    if w is None:
        return 1.0
    n_rec = d.O // 4
    w = np.asarray(w, np.float64)
    return w[:, np.arange(d.O) // n_rec][:, :, None]


def relative_weights(y, d: Dims):
    """w[b][c] = 1 / mean square of target b's component c: with these the
    weighted mean squared error is the mean over samples and components of
    the squared relative L2 error (0 for an all-zero component)."""
    n_rec = d.O // 4
    ms = np.mean(np.asarray(y, np.float64).reshape(y.shape[0], 4, n_rec * d.T) ** 2, axis=2)
    return np.where(ms > 0, 1.0 / np.where(ms > 0, ms, 1.0), 0.0)


def loss(theta, src, y, d: Dims, shift=None, w=None):
    """Mean over all outputs of w (Y - y)^2; w [B][4] per sample and
    component, or None for the plain mean squared error."""
    Y = forward(theta, src, d, shift=shift)
    return float(np.mean(element_weights(w, d) * (Y - y) ** 2))


def grad(theta, src, y, d: Dims, shift=None, w=None):
    """Gradient of loss() with respect to the flat parameters."""
    p = unflatten(theta, d)
    F, G = dft_bases(d)
    Y, c = forward(theta, src, d, keep=True, shift=shift)
    g = {}
    dY = 2.0 * element_weights(w, d) * (Y - y) / Y.size
    dYf = np.broadcast_to(c["m"][:, None, :, None, None] * dY[:, None, None, :, :],
                          (Y.shape[0], d.frames, d.n_mt, d.O, d.T))
    if shift is not None:
        dYf = frame_shift_transpose(dYf, shift, d)
    dY6 = np.ascontiguousarray(dYf).reshape(Y.shape[0], d.frames * d.n_mt * d.O, d.T)
    g["Q2"] = np.einsum("bot,bht->oh", dY6, c["Hq"])
    g["q2b"] = dY6.sum(axis=(0, 2))
    dHq = np.einsum("oh,bot->bht", p["Q2"], dY6)
    dHp = dHq * gelu_grad(c["Hp"])
    g["Q1"] = np.einsum("bht,bct->hc", dHp, c["V"][-1])
    g["q1b"] = dHp.sum(axis=(0, 2))
    dV = np.einsum("hc,bht->bct", p["Q1"], dHp)
    for l in reversed(range(d.L)):
        Z = c["Z"][l]
        dZ = dV * gelu_grad(Z) if l < d.L - 1 else dV
        Vin = c["V"][l]
        g[f"W{l}"] = np.einsum("bot,bct->oc", dZ, Vin)
        g[f"b{l}"] = dZ.sum(axis=(0, 2))
        dUh = dZ @ G.T                                          # B x C x 2K
        dUr, dUi = dUh[..., :d.K], dUh[..., d.K:]
        Vh = c["Vh"][l]
        Vr, Vi = Vh[..., :d.K], Vh[..., d.K:]
        g[f"Rr{l}"] = np.einsum("bok,bck->koc", dUr, Vr) + np.einsum("bok,bck->koc", dUi, Vi)
        g[f"Ri{l}"] = np.einsum("bok,bck->koc", dUi, Vr) - np.einsum("bok,bck->koc", dUr, Vi)
        Rr, Ri = p[f"Rr{l}"], p[f"Ri{l}"]
        dVr = np.einsum("koc,bok->bck", Rr, dUr) + np.einsum("koc,bok->bck", Ri, dUi)
        dVi = -np.einsum("koc,bok->bck", Ri, dUr) + np.einsum("koc,bok->bck", Rr, dUi)
        dV = np.einsum("oc,bot->bct", p[f"W{l}"], dZ) + np.concatenate([dVr, dVi], axis=2) @ F.T
    g["P"] = np.einsum("bct,bit->ci", dV, c["A"])
    g["pb"] = dV.sum(axis=(0, 2))
    return flatten(g, d)


def adam(theta, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (step counts from 1); returns the new (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------------------
# Error head (a reading of this build: the paper leaves the proxy as future
# work, Sec. VII): least squares of the log relative error on per-sample
# features phi with a ridge, and a one-sided 95 % margin of the residuals.
def error_head_fit(phi, err, ridge=1e-3):
    """Fit h minimising |Phi h - log e|^2 + ridge n |h|^2 (e clamped below at
    1e-6), by the normal equations; margin = 1.645 * the residual standard
    deviation (n - 1 in the denominator).  Returns (h, margin)."""
    phi = np.asarray(phi, np.float64)
    n, D = phi.shape
    y = np.log(np.maximum(1e-6, np.asarray(err, np.float64)))
    A = phi.T @ phi + ridge * n * np.eye(D)
    h = np.linalg.solve(A, phi.T @ y)
    res = y - phi @ h
    sd = math.sqrt(float(res @ res) / max(1, n - 1))
    return h, 1.645 * sd


def error_head_predict(phi, h, margin):
    """Estimated relative error of each sample: exp(phi h + margin)."""
    return np.exp(np.asarray(phi, np.float64) @ h + margin)


# ---------------------------------------------------------------------------
# Travel-time-aligned output frames
def lagrange4(w):
    """Weights of the 4-point Lagrange interpolation at offsets -1, 0, 1, 2
    from the sample left of the point, w in [0, 1): exact for cubics."""
    return np.array([-w * (w - 1) * (w - 2) / 6.0, (w + 1) * (w - 1) * (w - 2) / 2.0,
                     -(w + 1) * w * (w - 2) / 2.0, (w + 1) * w * (w - 1) / 6.0])


def delay(u, delta):
    """u(t - delta) for t = 0 .. T-1 (delta in samples): 4-point Lagrange
    interpolation of u, samples outside [0, T) taken as zero."""
    T = u.shape[-1]
    out = np.zeros(u.shape[:-1] + (T,))
    for t in range(T):
        x = t - delta
        i = math.floor(x)
        w = lagrange4(x - i)
        for k in range(4):
            j = i - 1 + k
            if 0 <= j < T:
                out[..., t] += w[k] * u[..., j]
    return out


def delay_transpose(v, delta):
    """The transpose of delay(., delta): scatters each v(t) onto the four
    samples its interpolation read, with the same weights."""
    T = v.shape[-1]
    out = np.zeros(v.shape[:-1] + (T,))
    for t in range(T):
        x = t - delta
        i = math.floor(x)
        w = lagrange4(x - i)
        for k in range(4):
            j = i - 1 + k
            if 0 <= j < T:
                out[..., j] += w[k] * v[..., t]
    return out


def frame_shift(Y6, shift, d: Dims):
    """Y6 (B x frames x n_mt x O x T) with row (f, j, o) delayed by shift[b][f][o mod n_rec]."""
    n_rec = d.O // 4
    out = np.empty_like(Y6)
    for b in range(Y6.shape[0]):
        for f in range(d.frames):
            for o in range(d.O):
                out[b, f, :, o] = delay(Y6[b, f, :, o], shift[b][f][o % n_rec])
    return out


def frame_shift_transpose(dY, shift, d: Dims):
    n_rec = d.O // 4
    out = np.empty(dY.shape)
    for b in range(dY.shape[0]):
        for f in range(d.frames):
            for o in range(d.O):
                out[b, f, :, o] = delay_transpose(dY[b, f, :, o], shift[b][f][o % n_rec])
    return out


def straight_ray_time(src, rec, slow, h):
    """Travel time along the straight segment between two cell centres
    (cell indices src, rec = (i, j, k)) through a medium whose slowness
    depends on depth only: slow[k] (s/m) in the cells of depth index k, each
    h[2] thick and centred on k h[2].  Along the segment the path length per
    unit depth is constant (|d| / |dz|), so the time is that ratio times the
    depth integral of the slowness, which from centre to centre is
    h[2] (slow[k0] / 2 + sum of the cells strictly between + slow[k1] / 2);
    a horizontal segment stays in one cell layer: |d| slow[k]."""
    d = np.array([(src[a] - rec[a]) * h[a] for a in range(3)], np.float64)
    L = float(np.linalg.norm(d))
    k0, k1 = int(min(src[2], rec[2])), int(max(src[2], rec[2]))
    if k0 == k1:
        return L * slow[k0]
    integral = 0.5 * slow[k0] + 0.5 * slow[k1]
    for k in range(k0 + 1, k1):
        integral += slow[k]
    integral *= h[2]
    return L / abs(d[2]) * integral


def ray_layers(src, rec, slow, h):
    """The cell layers a path between two cell centres crosses: thickness
    (half a cell at each end, whole cells between, times h[2]) and slowness
    of each, from the shallower end down."""
    k0, k1 = int(min(src[2], rec[2])), int(max(src[2], rec[2]))
    th = [0.5 * h[2]] + [h[2]] * (k1 - k0 - 1) + [0.5 * h[2]]
    return np.array(th, np.float64), np.array([slow[k] for k in range(k0, k1 + 1)], np.float64)


def ray_time(src, rec, slow, h, iters=64):
    """First-arrival time of the two-point ray between two cell centres
    through a medium whose slowness depends on depth only (Snell's law across
    the cell layers of ray_layers).  A ray of horizontal slowness p crosses a
    layer of thickness t and slowness s (p < s) with horizontal run
    t p / sqrt(s^2 - p^2) in time t s^2 / sqrt(s^2 - p^2); the run is 0 at
    p = 0 and grows without bound as p approaches the smallest slowness of
    the layers, so the p whose total run equals the horizontal distance is
    found by bisection (iters halvings of [0, min s)).  A path within one
    layer, a vertical path, and a path through a layer of zero slowness (the
    fluid in an S profile) take the straight segment."""
    k0, k1 = int(min(src[2], rec[2])), int(max(src[2], rec[2]))
    X = float(np.hypot((src[0] - rec[0]) * h[0], (src[1] - rec[1]) * h[1]))
    if k0 == k1 or X == 0.0 or min(slow[k] for k in range(k0, k1 + 1)) <= 0.0:
        return straight_ray_time(src, rec, slow, h)
    th, sl = ray_layers(src, rec, slow, h)
    lo, hi = 0.0, float(sl.min())
    for _ in range(iters):
        p = 0.5 * (lo + hi)
        run = float(np.sum(th * p / np.sqrt(sl * sl - p * p)))
        if run < X:
            lo = p
        else:
            hi = p
    p = 0.5 * (lo + hi)
    return float(np.sum(th * sl * sl / np.sqrt(sl * sl - p * p)))


def frame_shifts(src_ijk, rec_ijk, slows, h, dt, t_ref):
    """shift[b][f][r] = (ray time of frame f from source b to receiver r -
    t_ref[f]) / dt, in samples; slows[f] is frame f's slowness profile over
    depth."""
    B, F, R = len(src_ijk), len(slows), len(rec_ijk)
    out = np.empty((B, F, R))
    for b in range(B):
        for f in range(F):
            for r in range(R):
                out[b, f, r] = (ray_time(src_ijk[b], rec_ijk[r], slows[f], h) - t_ref[f]) / dt
    return out
