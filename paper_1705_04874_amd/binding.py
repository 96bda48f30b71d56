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
_L.pstd3d_derivs.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]
_L.pstd3d_reset.argtypes = [C.c_void_p, C.c_void_p]
_L.pstd3d_profile.argtypes = [C.c_void_p, C.c_int]
_L.pstd3d_profile_read.argtypes = [C.c_void_p, C.c_int, _dp, C.POINTER(C.c_long)]
_L.pstd3d_device_bytes.argtypes = [C.c_void_p]
_L.pstd3d_device_bytes.restype = C.c_long
_L.pstd3d_destroy.argtypes = [C.c_void_p]
_L.pstd3d_last_error.restype = C.c_char_p
_L.seis_combine.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_double, _dp, C.c_int, _ip, _dp, _dp,
                            C.c_int, C.c_double, C.c_void_p, C.c_void_p]


class PstdError(RuntimeError):
    def __init__(self, code, what):
        msg = _L.pstd3d_last_error().decode(errors="replace")
        super().__init__(f"{what} failed with code {code}: {msg}")
        self.code = code


def _check(rc, what):
    if rc != PSTD_OK:
        raise PstdError(rc, what)


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
        return cls(w.model.vp, w.model.vs, w.model.rho, **kw)

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
        out = np.empty((24,) + self.shape, np.float32)
        _check(_L.pstd3d_get_state(self._h, shot, out.ctypes.data_as(_fp)), "pstd3d_get_state")
        return out

    def set_state(self, fields, step, shot=0):
        f = np.ascontiguousarray(fields, dtype=np.float32)
        assert f.size == 24 * int(np.prod(self.shape))
        _check(_L.pstd3d_set_state(self._h, shot, f.ctypes.data_as(_fp), int(step)), "pstd3d_set_state")

    @property
    def step(self):
        return _L.pstd3d_step(self._h)

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


def seis_combine(traces, t0, src_idx, amp, t_origin, nt_out, dt_in, dt_out, out=None, stream=None):
    """Superposition of single-event traces on the GPU.

    traces: float32 device tensor [n_src][4][n_rec][nt_in]; returns [4][n_rec][nt_out]."""
    import torch
    assert traces.is_cuda and traces.dtype == torch.float32 and traces.is_contiguous()
    n_src, four, n_rec, nt_in = traces.shape
    assert four == 4
    if out is None:
        out = torch.empty((4, n_rec, nt_out), dtype=torch.float32, device=traces.device)
    t0 = (C.c_double * 4)(*[float(v) for v in t0])
    si = _i32(src_idx)
    am = _f64(amp)
    to = _f64(t_origin)
    _check(_L.seis_combine(C.c_void_p(traces.data_ptr()), n_src, n_rec, nt_in, float(dt_in), t0, si.size,
                           si.ctypes.data_as(_ip), am.ctypes.data_as(_dp), to.ctypes.data_as(_dp), int(nt_out),
                           float(dt_out), C.c_void_p(out.data_ptr()), _stream_handle(stream)), "seis_combine")
    return out
