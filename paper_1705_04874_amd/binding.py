"""ctypes binding of libpstd3d.so (the C ABI declared in include/pstd3d.h).

Argument marshalling only: every step of the solver and of the superposition
runs in the HIP kernels of the library. torch supplies device memory for the
trace buffers and the HIP stream. If the library has not been built this
module raises at import time; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpstd3d.so")

PSTD_OK, PSTD_EINVAL, PSTD_ENOMEM, PSTD_EDEVICE, PSTD_EUNSTABLE, PSTD_EUNSUPPORTED = 0, -1, -2, -3, -4, -5

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
                      "(hipcc, gfx950); there is no fallback path")

_L = C.CDLL(LIB_PATH)


class PstdModel(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("vp", C.POINTER(C.c_double)), ("vs", C.POINTER(C.c_double)), ("rho", C.POINTER(C.c_double)),
                ("n_rec", C.c_int), ("rec_ijk", C.POINTER(C.c_int32)),
                ("kspace", C.c_int), ("c_ref", C.c_double)]


class PstdPml(C.Structure):
    _fields_ = [("thickness", C.c_int), ("A", C.c_double), ("mratio", C.c_double)]


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_fp = C.POINTER(C.c_float)
_L.pstd3d_create.argtypes = [C.POINTER(PstdModel), _dp, C.c_double, C.POINTER(PstdPml), C.POINTER(C.c_void_p)]
_L.pstd3d_set_sources.argtypes = [C.c_void_p, C.c_int, _ip, _ip, _dp, _dp, C.c_int]
_L.pstd3d_run.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]
_L.pstd3d_run_many.argtypes = [C.POINTER(C.c_void_p), C.c_int, C.c_int, C.POINTER(C.c_void_p), C.c_void_p]
_L.pstd3d_get_state.argtypes = [C.c_void_p, C.c_int, _fp]
_L.pstd3d_set_state.argtypes = [C.c_void_p, C.c_int, _fp, C.c_long]
_L.pstd3d_step.argtypes = [C.c_void_p]
_L.pstd3d_step.restype = C.c_long
_L.pstd3d_undamped_range.argtypes = [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int)]
_L.pstd3d_undamped_range.restype = C.c_int
_L.pstd3d_derivs.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]
_L.pstd3d_reset.argtypes = [C.c_void_p, C.c_void_p]
_L.pstd3d_profile.argtypes = [C.c_void_p, C.c_int]
_L.pstd3d_profile_read.argtypes = [C.c_void_p, C.c_int, _dp, C.POINTER(C.c_long)]
_L.pstd3d_set_source_smoothing.argtypes = [C.c_void_p, C.c_int]
_L.pstd3d_set_viscosity.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
_L.pstd3d_state_fields.argtypes = [C.c_void_p]
_L.pstd3d_set_tuning.argtypes = [C.c_void_p, C.POINTER(C.c_int)]
_L.pstd3d_get_tuning.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), _fp, C.c_int]
TUNE_KNOBS = ("y_tile", "z_tile", "vel_threads", "str_threads", "z_threads", "z_fields")
_L.pstd3d_device_bytes.argtypes = [C.c_void_p]
_L.pstd3d_n_rec.argtypes = [C.c_void_p]
_L.pstd3d_device_bytes.restype = C.c_long
_L.pstd3d_workspace_size.argtypes = [C.c_void_p, C.c_int]
_L.pstd3d_workspace_size.restype = C.c_long
_L.pstd3d_set_workspace.argtypes = [C.c_void_p, C.c_void_p, C.c_long]
_L.pstd3d_destroy.argtypes = [C.c_void_p]
_L.pstd3d_last_error.restype = C.c_char_p
_L.seis_combine.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_double, _dp, C.c_int, _ip, _dp, _dp,
                            C.c_int, C.c_double, C.c_void_p, C.c_void_p]
_L.seis_combine_last_error.restype = C.c_char_p
_L.seis_combine_noalloc.argtypes = _L.seis_combine.argtypes
_L.seis_combine_noalloc_max_bytes.restype = C.c_long


class PstdError(RuntimeError):
    def __init__(self, code, what, last_error=None):
        msg = (last_error or _L.pstd3d_last_error)().decode(errors="replace")
        super().__init__(f"{what} failed with code {code}: {msg}")
        self.code = code


def _check(rc, what, last_error=None):
    if rc != PSTD_OK:
        raise PstdError(rc, what, last_error)


def _stream_handle(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


class Solver:
    """One velocity model on the current GPU; shots are batched inside."""

    def __init__(self, vp, vs, rho, d, dt, pml=16, pml_A=2.0, kspace=1, c_ref=0.0, rec=None, pml_p=0.1):
        self.vp, self.vs, self.rho = _f64(vp), _f64(vs), _f64(rho)
        nz, ny, nx = self.vp.shape
        self.shape = (nz, ny, nx)
        self.rec = _i32(np.zeros((0, 3)) if rec is None else rec).reshape(-1, 3)
        m = PstdModel(nx, ny, nz, self.vp.ctypes.data_as(_dp), self.vs.ctypes.data_as(_dp),
                      self.rho.ctypes.data_as(_dp), self.rec.shape[0], self.rec.ctypes.data_as(_ip),
                      int(kspace), float(c_ref))
        dd = (C.c_double * 3)(*[float(x) for x in d])
        p = PstdPml(int(pml), float(pml_A), float(pml_p))
        h = C.c_void_p()
        _check(_L.pstd3d_create(C.byref(m), dd, float(dt), C.byref(p), C.byref(h)), "pstd3d_create")
        self._h = h
        self.n_rec = self.rec.shape[0]
        self.n_shots = 0

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
        """Kelvin-Voigt viscosities (Pa s) per cell [nz][ny][nx]; None, None: lossless.
        Clears the shots (call set_sources again)."""
        if chi is None and eta is None:
            rc = _L.pstd3d_set_viscosity(self._h, None, None)
        else:
            c, e = _f64(chi), _f64(eta)
            assert c.shape == self.shape and e.shape == self.shape
            rc = _L.pstd3d_set_viscosity(self._h, c.ctypes.data, e.ctypes.data)
        _check(rc, "pstd3d_set_viscosity")
        self.n_shots = 0

    @property
    def n_state(self):
        """State fields per shot: 24, or 33 with viscosity."""
        return int(_L.pstd3d_state_fields(self._h))

    def set_source_smoothing(self, window):
        """0: point sources; 1: Blackman window in k-space (for later set_sources)."""
        _check(_L.pstd3d_set_source_smoothing(self._h, int(window)), "pstd3d_set_source_smoothing")

    def set_tuning(self, y_tile=0, z_tile=0, vel_threads=0, str_threads=0, z_threads=0, z_fields=0):
        """Force launch-shape knobs (0: autotuned at the next set_sources)."""
        v = (C.c_int * len(TUNE_KNOBS))(int(y_tile), int(z_tile), int(vel_threads), int(str_threads),
                                        int(z_threads), int(z_fields))
        _check(_L.pstd3d_set_tuning(self._h, v), "pstd3d_set_tuning")

    def tuning_values(self):
        """The chosen value of every knob, as keyword arguments of set_tuning."""
        t = self.tuning()
        return {k: t[k] for k in TUNE_KNOBS}

    def tuning(self):
        """{knob: chosen value} and {knob + '_candidates': {value: measured us per launch}}."""
        out = {}
        for k, name in enumerate(TUNE_KNOBS):
            ch = C.c_int()
            vals = (C.c_int * 8)()
            us = (C.c_float * 8)()
            n = _L.pstd3d_get_tuning(self._h, k, C.byref(ch), vals, us, 8)
            if n < 0:
                _check(n, "pstd3d_get_tuning")
            out[name] = ch.value
            out[name + "_candidates"] = {int(vals[i]): round(float(us[i]), 2) for i in range(n)}
        return out

    def set_sources(self, shot_ofs, src_ijk, m6, wavelet):
        so = _i32(shot_ofs)
        src = _i32(src_ijk).reshape(-1, 3)
        m = _f64(m6).reshape(-1, 6)
        w = _f64(wavelet)
        nt_w = w.shape[-1] if w.size else 0
        w = w.reshape(-1)
        _check(_L.pstd3d_set_sources(self._h, so.size - 1, so.ctypes.data_as(_ip), src.ctypes.data_as(_ip),
                                     m.ctypes.data_as(_dp), w.ctypes.data_as(_dp), nt_w), "pstd3d_set_sources")
        self.n_shots = so.size - 1

    def set_workload_sources(self, w):
        self.set_sources(w.shot_ofs, w.src_ijk, w.src_m, w.wavelet)

    def run(self, nt, out=None, stream=None):
        """Advance nt steps; returns float32 device tensor [n_shots][4][n_rec][nt]."""
        import torch
        if out is None:
            out = torch.empty((self.n_shots, 4, self.n_rec, nt), dtype=torch.float32, device="cuda")
        assert out.is_cuda and out.dtype == torch.float32 and out.is_contiguous()
        assert out.numel() == self.n_shots * 4 * self.n_rec * nt
        _check(_L.pstd3d_run(self._h, int(nt), C.c_void_p(out.data_ptr()), _stream_handle(stream)), "pstd3d_run")
        return out

    def reset(self, stream=None):
        _check(_L.pstd3d_reset(self._h, _stream_handle(stream)), "pstd3d_reset")

    KERNEL_KINDS = ["y_fwd_stress", "z_op_V", "y_inv_V", "vel_update", "y_fwd_vel", "z_op_S", "y_inv_S",
                    "stress_update"]

    def profile(self, enable=True):
        _check(_L.pstd3d_profile(self._h, int(bool(enable))), "pstd3d_profile")

    def profile_read(self):
        out = {}
        for k, name in enumerate(self.KERNEL_KINDS):
            ms = C.c_double()
            n = C.c_long()
            _check(_L.pstd3d_profile_read(self._h, k, C.byref(ms), C.byref(n)), "pstd3d_profile_read")
            out[name] = (ms.value, n.value)
        return out

    def get_state(self, shot=0):
        out = np.empty((self.n_state,) + self.shape, np.float32)
        _check(_L.pstd3d_get_state(self._h, shot, out.ctypes.data_as(_fp)), "pstd3d_get_state")
        return out

    def set_state(self, fields, step, shot=0):
        f = np.ascontiguousarray(fields, dtype=np.float32)
        assert f.size == self.n_state * int(np.prod(self.shape))
        _check(_L.pstd3d_set_state(self._h, shot, f.ctypes.data_as(_fp), int(step)), "pstd3d_set_state")

    @property
    def step(self):
        return _L.pstd3d_step(self._h)

    def undamped_range(self):
        """(lo, hi): per axis (x, y, z) the index range of the undamped cells,
        where each field's value sits in its first split part."""
        lo, hi = (C.c_int * 3)(), (C.c_int * 3)()
        _check(_L.pstd3d_undamped_range(self._h, lo, hi), "pstd3d_undamped_range")
        return tuple(lo), tuple(hi)

    def derivs(self, phase, fields, stream=None):
        """Nine staggered spectral derivatives of one phase (see include/pstd3d.h)."""
        import torch
        nin = 6 if phase == 0 else 3
        x = fields.contiguous()
        assert x.is_cuda and x.dtype == torch.float32 and x.shape == (nin,) + self.shape
        out = torch.empty((9,) + self.shape, dtype=torch.float32, device=x.device)
        _check(_L.pstd3d_derivs(self._h, int(phase), C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()),
                                _stream_handle(stream)), "pstd3d_derivs")
        return out

    def workspace_size(self, n_shots):
        """Device bytes the state of n_shots shots needs in a caller workspace."""
        n = _L.pstd3d_workspace_size(self._h, int(n_shots))
        if n < 0:
            _check(int(n), "pstd3d_workspace_size")
        return int(n)

    def set_workspace(self, buf):
        """Keep the shots' state in `buf` (a contiguous CUDA tensor, kept referenced
        here) from the next set_sources on; None returns to the library's own
        memory.  Clears the shots."""
        if buf is None:
            _check(_L.pstd3d_set_workspace(self._h, None, 0), "pstd3d_set_workspace")
        else:
            assert buf.is_cuda and buf.is_contiguous()
            nbytes = buf.numel() * buf.element_size()
            _check(_L.pstd3d_set_workspace(self._h, C.c_void_p(buf.data_ptr()), nbytes), "pstd3d_set_workspace")
        self._ws = buf
        self.n_shots = 0

    @property
    def device_bytes(self):
        return _L.pstd3d_device_bytes(self._h)

    def close(self):
        if self._h:
            _L.pstd3d_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_many(solvers, nt, outs=None, stream=None):
    """Advance several solvers (uneven grids) together; returns their trace tensors."""
    import torch
    if outs is None:
        outs = [torch.empty((s.n_shots, 4, s.n_rec, nt), dtype=torch.float32, device="cuda") for s in solvers]
    hs = (C.c_void_p * len(solvers))(*[s._h for s in solvers])
    ts = (C.c_void_p * len(solvers))(*[o.data_ptr() for o in outs])
    _check(_L.pstd3d_run_many(hs, len(solvers), int(nt), ts, _stream_handle(stream)), "pstd3d_run_many")
    return outs


def seis_combine(traces, t0, src_idx, amp, t_origin, nt_out, dt_in, dt_out, out=None, stream=None,
                 noalloc=False):
    """Superposition of single-event traces on the GPU.

    traces: float32 device tensor [n_src][4][n_rec][nt_in]; returns [4][n_rec][nt_out].
    noalloc: call seis_combine_noalloc (event lists in the library's static device
    memory; `out` must then be given, so that nothing is allocated)."""
    import torch
    if noalloc and out is None:
        raise ValueError("noalloc needs a preallocated out tensor")
    assert traces.is_cuda and traces.dtype == torch.float32 and traces.is_contiguous()
    n_src, four, n_rec, nt_in = traces.shape
    assert four == 4
    if out is None:
        out = torch.empty((4, n_rec, nt_out), dtype=torch.float32, device=traces.device)
    t0 = (C.c_double * 4)(*[float(v) for v in t0])
    si = _i32(src_idx)
    am = _f64(amp)
    to = _f64(t_origin)
    fn = _L.seis_combine_noalloc if noalloc else _L.seis_combine
    _check(fn(C.c_void_p(traces.data_ptr()), n_src, n_rec, nt_in, float(dt_in), t0, si.size,
                           si.ctypes.data_as(_ip), am.ctypes.data_as(_dp), to.ctypes.data_as(_dp), int(nt_out),
                           float(dt_out), C.c_void_p(out.data_ptr()), _stream_handle(stream)), "seis_combine",
           _L.seis_combine_last_error)
    return out


# ---------------------------------------------------------------------------
# spectral neural operator surrogate (include/sno.h)
class SnoCfg(C.Structure):
    _fields_ = [("n_rec", C.c_int), ("T", C.c_int), ("C", C.c_int), ("K", C.c_int), ("L", C.c_int), ("H", C.c_int),
                ("feat_off", C.c_double * 9), ("feat_scale", C.c_double * 9),
                ("n_four", C.c_int), ("four_cycles", C.c_double * 64), ("pos_mod", C.c_int),
                ("frames", C.c_int), ("rec_ijk", C.POINTER(C.c_int32)), ("nz_slow", C.c_int),
                ("slow_p", C.POINTER(C.c_double)), ("slow_s", C.POINTER(C.c_double)), ("h", C.c_double * 3),
                ("dt", C.c_double), ("t_ref", C.c_double * 2)]


_EPOCH_CB = C.CFUNCTYPE(None, C.c_int, C.c_float, C.c_void_p)


class SnoTrainCfg(C.Structure):
    _fields_ = [("epochs", C.c_int), ("batch", C.c_int), ("lr", C.c_double), ("seed", C.c_uint64),
                ("n_calib", C.c_int), ("on_epoch", _EPOCH_CB), ("user", C.c_void_p), ("rel_loss", C.c_int)]


_L.sno_n_params.argtypes = [C.POINTER(SnoCfg)]
_L.sno_n_params.restype = C.c_long
_L.sno_create.argtypes = [C.POINTER(SnoCfg), _fp, C.POINTER(C.c_void_p)]
_L.sno_destroy.argtypes = [C.c_void_p]
_L.sno_train.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.POINTER(SnoTrainCfg), _fp, C.c_void_p]
_L.sno_predict.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]
_L.sno_predict_or_solve.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, _ip, _dp, _dp, C.c_int, C.c_int, C.c_int,
                                    C.c_double, C.c_int, C.c_void_p, C.c_void_p, C.POINTER(C.c_int), C.c_void_p]
_L.sno_forward.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]
_L.sno_gradient.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, _fp, C.c_void_p]
_L.sno_gradient_weighted.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, _fp,
                                     C.c_void_p]
_L.sno_get_params.argtypes = [C.c_void_p, _fp]
_L.sno_adam_step.argtypes = [C.c_void_p, C.c_void_p, C.c_long, C.c_double, C.c_void_p]
_L.sno_get_moments.argtypes = [C.c_void_p, _fp, _fp]
_L.sno_get_scale.argtypes = [C.c_void_p, _fp]
_L.sno_decimate.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p]
_L.sno_last_error.restype = C.c_char_p


def _scheck(rc, what):
    if rc != PSTD_OK:
        msg = _L.sno_last_error().decode(errors="replace")
        err = PstdError.__new__(PstdError)
        RuntimeError.__init__(err, f"{what} failed with code {rc}: {msg}")
        err.code = rc
        raise err


def _dev(t):
    import torch
    assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
    return C.c_void_p(t.data_ptr())


class Surrogate:
    """Spectral neural operator surrogate on the current GPU (see include/sno.h)."""

    def __init__(self, n_rec, T, C_, K, L, H, feat_off, feat_scale, params, four_cycles=(), pos_mod=False,
                 frames=None):
        """frames: None for the plain time axis, or a dict with the travel-time
        alignment of include/sno.h: rec_ijk [n_rec][3], slow_p and slow_s
        (slowness per depth cell, s/m), h (3 cell sizes, m), dt (s) and t_ref
        (the P and S reference times, s)."""
        four = [float(v) for v in four_cycles]
        if len(four) > 64:
            raise ValueError("at most 64 Fourier feature frequencies")
        self.cfg = SnoCfg(int(n_rec), int(T), int(C_), int(K), int(L), int(H),
                          (C.c_double * 9)(*[float(v) for v in feat_off]),
                          (C.c_double * 9)(*[float(v) for v in feat_scale]),
                          len(four), (C.c_double * 64)(*(four + [0.0] * (64 - len(four)))), int(bool(pos_mod)))
        self.cfg.frames = 1
        if frames is not None:
            # kept alive until sno_create has copied them
            self._rec = _i32(frames["rec_ijk"]).reshape(-1, 3)
            self._sp = _f64(frames["slow_p"])
            self._ss = _f64(frames["slow_s"])
            assert self._rec.shape[0] == n_rec and self._sp.size == self._ss.size
            self.cfg.frames = 2
            self.cfg.rec_ijk = self._rec.ctypes.data_as(_ip)
            self.cfg.nz_slow = self._sp.size
            self.cfg.slow_p = self._sp.ctypes.data_as(_dp)
            self.cfg.slow_s = self._ss.ctypes.data_as(_dp)
            self.cfg.h = (C.c_double * 3)(*[float(v) for v in frames["h"]])
            self.cfg.dt = float(frames["dt"])
            self.cfg.t_ref = (C.c_double * 2)(*[float(v) for v in frames["t_ref"]])
        self.n_lift = 4 + 2 * len(four) + (6 * len(four) if pos_mod else 0)
        self.n_params = _L.sno_n_params(C.byref(self.cfg))
        if self.n_params < 0:
            raise ValueError("bad surrogate configuration")
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == self.n_params
        h = C.c_void_p()
        _scheck(_L.sno_create(C.byref(self.cfg), p.ctypes.data_as(_fp), C.byref(h)), "sno_create")
        self._h = h
        self.O = 4 * int(n_rec)

    def _out(self, n):
        import torch
        return torch.empty((n, 4, self.cfg.n_rec, self.cfg.T), dtype=torch.float32, device="cuda")

    def train(self, X, Y, epochs, batch, lr, seed=0, n_calib=0, stream=None, on_epoch=None, rel_loss=False):
        """Train; on_epoch(epoch, mean_loss), if given, is called after every
        epoch; rel_loss: the mean squared relative error per sample and
        component instead of the mean squared error (include/sno.h)."""
        cb = _EPOCH_CB(lambda ep, loss, _u: on_epoch(int(ep), float(loss))) if on_epoch else _EPOCH_CB()
        tc = SnoTrainCfg(int(epochs), int(batch), float(lr), int(seed), int(n_calib), cb, None, int(bool(rel_loss)))
        curve = np.zeros(max(1, int(epochs)), np.float32)
        _scheck(_L.sno_train(self._h, _dev(X), _dev(Y), X.shape[0], C.byref(tc), curve.ctypes.data_as(_fp),
                             _stream_handle(stream)), "sno_train")
        return curve[:epochs]

    def predict(self, X, stream=None):
        import torch
        n = X.shape[0]
        Y = self._out(n)
        est = torch.empty(n, dtype=torch.float32, device="cuda")
        _scheck(_L.sno_predict(self._h, _dev(X), n, _dev(Y), _dev(est), _stream_handle(stream)), "sno_predict")
        return Y, est

    def predict_or_solve(self, solver, X, src_ijk, m6, wavelet, decim, tol, max_batch=64, stream=None):
        import torch
        if _L.pstd3d_n_rec(solver._h) != self.cfg.n_rec:
            raise ValueError(f"the solver has {_L.pstd3d_n_rec(solver._h)} receivers, the surrogate "
                             f"{self.cfg.n_rec}")
        n = X.shape[0]
        Y = self._out(n)
        est = torch.empty(n, dtype=torch.float32, device="cuda")
        ijk = _i32(src_ijk).reshape(-1, 3)
        mm = _f64(m6).reshape(-1, 6)
        wv = _f64(wavelet).reshape(-1)
        used = (C.c_int * max(1, n))()
        _scheck(_L.sno_predict_or_solve(self._h, solver._h, _dev(X), ijk.ctypes.data_as(_ip), mm.ctypes.data_as(_dp),
                                        wv.ctypes.data_as(_dp), wv.size, int(decim), n, float(tol), int(max_batch),
                                        _dev(Y), _dev(est), used, _stream_handle(stream)), "sno_predict_or_solve")
        return Y, est, np.array(used[:n], dtype=bool)

    def adam_step(self, grad, step, lr, stream=None):
        """One Adam step of the weights with a device gradient (test entry)."""
        _scheck(_L.sno_adam_step(self._h, _dev(grad), int(step), float(lr), _stream_handle(stream)), "sno_adam_step")

    def moments(self):
        m = np.empty(self.n_params, np.float32)
        v = np.empty(self.n_params, np.float32)
        _scheck(_L.sno_get_moments(self._h, m.ctypes.data_as(_fp), v.ctypes.data_as(_fp)), "sno_get_moments")
        return m, v

    def forward(self, X, stream=None):
        Y = self._out(X.shape[0])
        _scheck(_L.sno_forward(self._h, _dev(X), X.shape[0], _dev(Y), _stream_handle(stream)), "sno_forward")
        return Y

    def gradient(self, X, Yt, stream=None, w=None):
        """Gradient (and loss) of the mean squared error against normalised
        targets Yt; w: optional device weights [n][4] per sample and component."""
        import torch
        g = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        loss = C.c_float()
        if w is None:
            _scheck(_L.sno_gradient(self._h, _dev(X), _dev(Yt), X.shape[0], _dev(g), C.byref(loss),
                                    _stream_handle(stream)), "sno_gradient")
        else:
            assert tuple(w.shape) == (X.shape[0], 4)
            _scheck(_L.sno_gradient_weighted(self._h, _dev(X), _dev(Yt), _dev(w), X.shape[0], _dev(g), C.byref(loss),
                                             _stream_handle(stream)), "sno_gradient_weighted")
        return g, loss.value

    def params(self):
        out = np.empty(self.n_params, np.float32)
        _scheck(_L.sno_get_params(self._h, out.ctypes.data_as(_fp)), "sno_get_params")
        return out

    def scale(self):
        out = np.empty(4, np.float32)
        _scheck(_L.sno_get_scale(self._h, out.ctypes.data_as(_fp)), "sno_get_scale")
        return out

    def close(self):
        if self._h:
            _L.sno_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def decimate(traces, decim, stream=None):
    """Keep every decim-th sample of float32 device traces [n][4][n_rec][nt]."""
    import torch
    n, four, n_rec, nt = traces.shape
    out = torch.empty((n, 4, n_rec, nt // decim), dtype=torch.float32, device=traces.device)
    _scheck(_L.sno_decimate(_dev(traces), n, n_rec, nt, int(decim), _dev(out), _stream_handle(stream)), "sno_decimate")
    return out


# ---------------------------------------------------------------------------
# clustered event catalogue (include/seis_catalog.h)
_L.seis_laplacian.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p]
_L.seis_pick_interfaces.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, _ip, C.c_int, C.c_float, _ip, C.c_void_p]
_L.seis_kmeans.argtypes = [_dp, C.c_int, C.c_int, C.c_int, _ip, C.c_int, _ip, _dp, _dp]
_L.seis_cluster_catalogue.argtypes = [_ip, _dp, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, _dp,
                                      C.c_double, C.c_double, _dp, _dp, _dp, _ip]
_L.seis_catalog_last_error.restype = C.c_char_p


def _ccheck(rc, what):
    if rc < 0:
        msg = _L.seis_catalog_last_error().decode(errors="replace")
        err = PstdError.__new__(PstdError)
        RuntimeError.__init__(err, f"{what} failed with code {rc}: {msg}")
        err.code = rc
        raise err
    return rc


def laplacian(rho, stream=None):
    """Laplacian of the density (eq. 8) of a float32 device tensor [nz][ny][nx]."""
    import torch
    nz, ny, nx = rho.shape
    out = torch.empty_like(rho)
    _ccheck(_L.seis_laplacian(_dev(rho), nx, ny, nz, _dev(out), _stream_handle(stream)), "seis_laplacian")
    return out


def pick_interfaces(lap, cand_ijk, threshold, stream=None):
    """Host int32 mask of the candidates (i, j, k) where |L| > threshold."""
    nz, ny, nx = lap.shape
    c = _i32(cand_ijk).reshape(-1, 3)
    keep = np.zeros(c.shape[0], np.int32)
    _ccheck(_L.seis_pick_interfaces(_dev(lap), nx, ny, nz, c.ctypes.data_as(_ip), c.shape[0], float(threshold),
                                    keep.ctypes.data_as(_ip), _stream_handle(stream)), "seis_pick_interfaces")
    return keep


def kmeans(pts, k, init_idx, max_iter=100):
    """(labels, centroids, sse) of the library's best-of-runs k-means."""
    p = _f64(pts).reshape(-1, 3)
    init = _i32(init_idx).reshape(-1, k)
    lab = np.zeros(p.shape[0], np.int32)
    cen = np.zeros((k, 3))
    sse = C.c_double()
    _ccheck(_L.seis_kmeans(p.ctypes.data_as(_dp), p.shape[0], int(k), init.shape[0], init.ctypes.data_as(_ip),
                           int(max_iter), lab.ctypes.data_as(_ip), cen.ctypes.data_as(_dp), C.byref(sse)),
            "seis_kmeans")
    return lab, cen, sse.value


def cluster_catalogue(labels, depth, k, t_first, dt_between, sigma, gauss, lo, hi, unif):
    """(t_origin, amp, rank) of the cluster timing rules of Sec. VI-A."""
    lab = _i32(labels)
    dep = _f64(depth)
    g = _f64(gauss)
    u = _f64(unif)
    n = lab.size
    t = np.zeros(n)
    a = np.zeros(n)
    r = np.zeros(n, np.int32)
    _ccheck(_L.seis_cluster_catalogue(lab.ctypes.data_as(_ip), dep.ctypes.data_as(_dp), n, int(k), float(t_first),
                                      float(dt_between), float(sigma), g.ctypes.data_as(_dp), float(lo), float(hi),
                                      u.ctypes.data_as(_dp), t.ctypes.data_as(_dp), a.ctypes.data_as(_dp),
                                      r.ctypes.data_as(_ip)), "seis_cluster_catalogue")
    return t, a, r
