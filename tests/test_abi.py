"""The C ABI library loads and exports every symbol its header declares, and its
argument validation (which runs before any device call) rejects bad input.
No compute call here needs a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1705_04874_amd", "libpstd3d.so")
INCLUDE = os.path.join(ROOT, "include")


def declared_functions():
    """Every function declared in include/*.h (comments stripped)."""
    names = set()
    for h in sorted(os.listdir(INCLUDE)):
        if not h.endswith(".h"):
            continue
        text = re.sub(r"/\*.*?\*/", "", open(os.path.join(INCLUDE, h)).read(), flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        names |= set(re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([a-z]\w*)\s*\(", text, flags=re.M))
    return sorted(n for n in names if n not in ("defined",))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libpstd3d.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n


def test_validation_without_device(lib):
    from paper_1705_04874_amd import binding as B
    shape = (16, 16, 16)
    vp, vs, rho = [np.full(shape, v) for v in (3000.0, 1700.0, 2300.0)]
    # CFL violation with the plain operator
    with pytest.raises(B.PstdError) as e:
        B.Solver(vp, vs, rho, (10, 10, 10), 2e-3, kspace=0, pml=2)
    assert e.value.code == B.PSTD_EUNSTABLE
    # a length with a factor 17 is not supported
    shp = (16, 16, 17)
    with pytest.raises(B.PstdError) as e:
        B.Solver(np.full(shp, 3000.0), np.full(shp, 1700.0), np.full(shp, 2300.0), (10, 10, 10), 1e-3, pml=2)
    assert e.value.code == B.PSTD_EUNSUPPORTED
    bad = vp.copy()
    bad[3, 3, 3] = np.nan
    with pytest.raises(B.PstdError) as e:
        B.Solver(bad, vs, rho, (10, 10, 10), 1e-3, pml=2)
    assert e.value.code == B.PSTD_EINVAL
    with pytest.raises(B.PstdError) as e:
        B.Solver(vp, vs, rho, (10, 10, 10), 1e-3, pml=2, rec=np.array([[0, 16, 0]]))
    assert e.value.code == B.PSTD_EINVAL
    with pytest.raises(B.PstdError) as e:
        B.Solver(vp, vs, rho, (10, 10, 10), 1e-3, pml=9)
    assert e.value.code == B.PSTD_EINVAL


def test_combine_validation_without_device(lib):
    """seis_combine checks its host arguments before any device call (the
    pointers below are never dereferenced)."""
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    lib.seis_combine.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, dp,
                                 ctypes.c_int, ip, dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_void_p,
                                 ctypes.c_void_p]
    lib.seis_combine_last_error.restype = ctypes.c_char_p
    t0 = (ctypes.c_double * 4)(0, 0, 0, 0)
    fake = ctypes.c_void_p(0x1000)

    def call(src, amp, to, n_src=2, nt_in=10, dt_in=1e-3, n_rec=3, nt_out=20):
        s = np.ascontiguousarray(src, np.int32)
        a = np.ascontiguousarray(amp, np.float64)
        t = np.ascontiguousarray(to, np.float64)
        return lib.seis_combine(fake, n_src, n_rec, nt_in, dt_in, t0, s.size, s.ctypes.data_as(ip),
                                a.ctypes.data_as(dp), t.ctypes.data_as(dp), nt_out, 1e-3, fake, None)

    assert call([2], [1.0], [0.0]) == -1
    assert b"source index" in lib.seis_combine_last_error()
    assert call([-1], [1.0], [0.0]) == -1
    assert call([0], [np.inf], [0.0]) == -1
    assert call([0], [1.0], [np.nan]) == -1
    assert call([0], [1.0], [0.0], nt_in=0) == -1
    assert call([0], [1.0], [0.0], dt_in=0.0) == -1
    assert call([0], [1.0], [0.0], n_src=0) == -1
    assert call([0], [1.0], [0.0], nt_in=(1 << 30) + 1) == -1
    assert b"nt_in" in lib.seis_combine_last_error()
    # 2^22 output rows in 2 segments of 512-thread blocks: 2^32 work-items
    assert call([0], [1.0], [0.0], n_rec=1 << 20, nt_out=12000) == -1
    assert b"too large" in lib.seis_combine_last_error()
