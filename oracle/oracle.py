"""ctypes wrapper of the FP64 CPU oracle (test infrastructure only).

The C code lives next to this file (offt.c, opstd.c, ocombine.c); it is built
into liboracle.so by oracle/build.py (or on first use if nothing is built).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

ORC_OK, ORC_EINVAL, ORC_ENOMEM, ORC_EUNSTABLE = 0, -1, -2, -4


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed with code {code}")
        self.code = code


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        fp = C.POINTER(C.c_float)
        L.offt_1d.argtypes = [C.c_void_p, C.c_int, C.c_int]
        L.offt_3d.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int]
        L.opstd_create.restype = C.c_void_p
        L.opstd_create.argtypes = [C.c_int, C.c_int, C.c_int, dp, dp, dp, C.c_double, C.c_double,
                                   C.c_double, C.c_double, C.c_int, C.c_double, C.c_double, C.c_int,
                                   C.c_double, C.c_int, ip, ip]
        L.opstd_set_sources.argtypes = [C.c_void_p, C.c_int, ip, dp, dp, C.c_int]
        L.opstd_run.argtypes = [C.c_void_p, C.c_int, dp]
        L.opstd_set_source_smoothing.argtypes = [C.c_void_p, C.c_int]
        L.opstd_set_viscosity.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.opstd_n_state.argtypes = [C.c_void_p]
        L.opstd_smoothed_source.argtypes = [C.c_void_p, C.c_int, C.c_int, ip, dp]
        L.opstd_get_state.argtypes = [C.c_void_p, dp]
        L.opstd_set_state.argtypes = [C.c_void_p, dp]
        L.opstd_step_index.argtypes = [C.c_void_p]
        L.opstd_step_index.restype = C.c_long
        L.opstd_set_step.argtypes = [C.c_void_p, C.c_long]
        L.opstd_destroy.argtypes = [C.c_void_p]
        L.oracle_threads.restype = C.c_int
        L.opstd_deriv.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double,
                                  dp, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, dp]
        L.ocombine.argtypes = [fp, C.c_int, C.c_int, C.c_int, C.c_double, dp, C.c_int, ip, dp, dp,
                               C.c_int, C.c_double, dp]
        _LIB = L
    return _LIB


def threads():
    """OpenMP threads the oracle's loops use."""
    return int(lib().oracle_threads())


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


# ----------------------------------------------------------------------------
def fft(x, inverse=False):
    """1-D FFT (forward e^{-2 pi i jk/n}; inverse includes 1/n)."""
    a = np.ascontiguousarray(x, dtype=np.complex128).copy()
    lib().offt_1d(a.ctypes.data, a.size, +1 if inverse else -1)
    return a


def fft3(x, inverse=False):
    """3-D FFT of an array [nz][ny][nx]."""
    a = np.ascontiguousarray(x, dtype=np.complex128).copy()
    nz, ny, nx = a.shape
    lib().offt_3d(a.ctypes.data, nx, ny, nz, +1 if inverse else -1)
    return a


def deriv(f, axis, sign, h=(1.0, 1.0, 1.0), kspace=0, c_ref=0.0, dt=0.0):
    """Staggered spectral derivative D_axis^{sign} of a real field [nz][ny][nx].

    axis: 0 = x, 1 = y, 2 = z; sign +1 moves integer -> half nodes, -1 half -> integer.
    """
    f = _f64(f)
    nz, ny, nx = f.shape
    out = np.empty_like(f)
    lib().opstd_deriv(nx, ny, nz, h[0], h[1], h[2], _dp(f), axis, sign, kspace, c_ref, dt, _dp(out))
    return out


class Solver:
    """FP64 oracle solver for one shot (the point sources of one simulation)."""

    N_STATE = 24

    def __init__(self, vp, vs, rho, d, dt, pml=0, pml_A=2.0, kspace=1, c_ref=0.0, rec=None, pml_p=0.1):
        self.vp, self.vs, self.rho = _f64(vp), _f64(vs), _f64(rho)
        self.shape = self.vp.shape
        nz, ny, nx = self.shape
        self.rec = _i32(np.zeros((0, 3)) if rec is None else rec).reshape(-1, 3)
        err = C.c_int(0)
        self._h = lib().opstd_create(nx, ny, nz, _dp(self.vp), _dp(self.vs), _dp(self.rho),
                                     float(d[0]), float(d[1]), float(d[2]), float(dt), int(pml),
                                     float(pml_A), float(pml_p), int(kspace), float(c_ref), self.rec.shape[0],
                                     _ip(self.rec), C.byref(err))
        if not self._h:
            raise OracleError(err.value, "create")
        self.n_rec = self.rec.shape[0]

    @classmethod
    def from_workload(cls, w, **over):
        kw = dict(d=w.d, dt=w.dt, pml=w.pml, pml_A=w.pml_A, pml_p=w.pml_p, kspace=w.kspace, c_ref=w.c_ref,
                  rec=w.rec)
        kw.update(over)
        s = cls(w.model.vp, w.model.vs, w.model.rho, **kw)
        if getattr(w, "smooth", 0):
            s.set_source_smoothing(w.smooth)
        if getattr(w, "chi", None) is not None:
            s.set_viscosity(w.chi, w.eta)
        return s

    def set_viscosity(self, chi, eta):
        """Kelvin-Voigt viscosities per cell [nz][ny][nx] (None, None: lossless); clears the state."""
        if chi is None and eta is None:
            rc = lib().opstd_set_viscosity(self._h, None, None)
        else:
            self._chi, self._eta = _f64(chi), _f64(eta)
            rc = lib().opstd_set_viscosity(self._h, self._chi.ctypes.data, self._eta.ctypes.data)
        if rc:
            raise OracleError(rc, "set_viscosity")

    @property
    def n_state(self):
        return int(lib().opstd_n_state(self._h))

    def set_source_smoothing(self, window):
        """0: point sources; 1: Blackman window in k-space (next set_sources)."""
        rc = lib().opstd_set_source_smoothing(self._h, int(window))
        if rc:
            raise OracleError(rc, "set_source_smoothing")

    def smoothed_source(self, q, max_cells=4096):
        """(ijk [n][3], weights [n]) of source q's smoothed delta."""
        ijk = np.zeros((max_cells, 3), np.int32)
        w = np.zeros(max_cells)
        n = lib().opstd_smoothed_source(self._h, int(q), max_cells, _ip(ijk), _dp(w))
        if n < 0:
            raise OracleError(n, "smoothed_source")
        return ijk[:n], w[:n]

    def set_sources(self, src_ijk, m6, wavelet):
        src = _i32(src_ijk).reshape(-1, 3)
        m = _f64(m6).reshape(-1, 6)
        wav = _f64(wavelet)
        wav = wav.reshape(src.shape[0], -1) if src.shape[0] else np.zeros((0, 1))
        rc = lib().opstd_set_sources(self._h, src.shape[0], _ip(src), _dp(m), _dp(wav), wav.shape[1])
        if rc:
            raise OracleError(rc, "set_sources")

    def run(self, nt):
        out = np.zeros((4, self.n_rec, nt))
        rc = lib().opstd_run(self._h, int(nt), _dp(out))
        if rc:
            raise OracleError(rc, "run")
        return out

    def get_state(self):
        out = np.empty((self.n_state,) + self.shape)
        lib().opstd_get_state(self._h, _dp(out))
        return out

    def set_state(self, fields):
        f = _f64(fields).reshape((self.n_state,) + self.shape)
        lib().opstd_set_state(self._h, _dp(f))

    @property
    def step(self):
        return lib().opstd_step_index(self._h)

    @step.setter
    def step(self, n):
        lib().opstd_set_step(self._h, int(n))

    def close(self):
        if self._h:
            lib().opstd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_shot(w, shot=0, nt=None, **over):
    """Oracle traces [4][n_rec][nt] for one shot of a workload."""
    s = Solver.from_workload(w, **over)
    a, b = int(w.shot_ofs[shot]), int(w.shot_ofs[shot + 1])
    s.set_sources(w.src_ijk[a:b], w.src_m[a:b], w.wavelet[a:b])
    out = s.run(w.nt if nt is None else nt)
    s.close()
    return out


def combine(tr, t0, src_idx, amp, t_origin, nt_out, dt_in, dt_out):
    """Superposition of single-event traces: returns float64 [4][n_rec][nt_out]."""
    tr = np.ascontiguousarray(tr, dtype=np.float32)
    n_src, four, n_rec, nt_in = tr.shape
    assert four == 4
    t0 = _f64(t0)
    si = _i32(src_idx)
    amp = _f64(amp)
    to = _f64(t_origin)
    out = np.empty((4, n_rec, nt_out))
    rc = lib().ocombine(tr.ctypes.data_as(C.POINTER(C.c_float)), n_src, n_rec, nt_in, float(dt_in),
                        _dp(t0), si.size, _ip(si), _dp(amp), _dp(to), int(nt_out), float(dt_out),
                        _dp(out))
    if rc:
        raise OracleError(rc, "combine")
    return out


# state-field order used by get_state / set_state
STATE_NAMES = (["vx_x", "vx_y", "vx_z", "vy_x", "vy_y", "vy_z", "vz_x", "vz_y", "vz_z"] +
               ["sxx_x", "sxx_y", "sxx_z", "syy_x", "syy_y", "syy_z", "szz_x", "szz_y", "szz_z"] +
               ["sxy_x", "sxy_y", "sxz_x", "sxz_z", "syz_y", "syz_z"])
