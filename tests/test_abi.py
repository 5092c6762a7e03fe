"""CPU-side checks of the C ABI: the library loads, exports every symbol the
header declares, and validates descriptors on the host (no kernel runs)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "hofks.h")).read()
    return sorted(set(re.findall(r"\b(hofks_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    from paper_1212_0204_amd import _lib
    assert declared_symbols() == sorted(_lib.SYMBOLS)


def test_library_exports_every_declared_symbol():
    from paper_1212_0204_amd import _lib
    L = _lib.lib()
    for name in declared_symbols():
        assert hasattr(L, name), name


def desc(dim=2, n=(256, 256, 1), dx=1 / 256, nv=32, dv=0.5, bc=(0, 0, 0), precision=0, scheme=0):
    from paper_1212_0204_amd import _lib
    return _lib.GridDesc(dim, (ctypes.c_int * 3)(*n), dx, nv, dv, (ctypes.c_int * 3)(*bc),
                         precision, scheme)


def ws(d):
    from paper_1212_0204_amd import _lib
    sz = ctypes.c_size_t(0)
    st = _lib.lib().hofks_workspace_size(ctypes.byref(d), ctypes.byref(sz))
    return st, sz.value


def test_workspace_sizes_of_the_workloads():
    # pieces (two buffers) dominate: 2 * Nv * Nc * bytes per piece
    st, b = ws(desc())
    assert st == 0 and 2 * 1024 * 65536 * 8 <= b < 1.2 * 2 * 1024 * 65536 * 8
    st, b = ws(desc(3, (64, 64, 64), 1 / 64, 24, 0.5, precision=1))
    assert st == 0 and 2 * 13824 * 262144 * 4 <= b < 1.1 * 2 * 13824 * 262144 * 4
    st, b = ws(desc(1, (200, 1, 1), 1 / 200, 64, 0.25, bc=(1, 0, 0)))
    assert st == 0 and b >= 2 * 64 * 200 * 8


@pytest.mark.parametrize("kw", [dict(dim=0), dict(dim=4), dict(nv=1), dict(dv=0.0),
                                dict(dx=-1.0), dict(precision=2), dict(scheme=4),
                                dict(bc=(2, 0, 0)), dict(n=(0, 4, 1)),
                                dict(n=(8, 8, 1), nv=32)])  # periodic x shorter than the shift
def test_bad_descriptors_are_rejected(kw):
    st, _ = ws(desc(**kw))
    assert st == -1


def test_create_rejects_small_workspace():
    from paper_1212_0204_amd import _lib
    h = ctypes.c_void_p(0)
    d = desc()
    st = _lib.lib().hofks_create(ctypes.byref(d), ctypes.c_void_p(256), 1024, None, ctypes.byref(h))
    assert st == -2 and not h.value


@pytest.mark.parametrize("dt", [-1e-3, 0.5])
def test_offlattice_step_outside_range_rejected(dt):
    """a free time step must lie in (0, dx/dv]"""
    d = desc(dx=0.1, dv=0.5)
    d.dt = dt
    st, _ = ws(d)
    assert st == -1


def test_offlattice_needs_nvel_multiple_of_4_in_2d():
    d = desc(dim=2, n=(16, 16, 1), nv=10, dx=1 / 16, dv=0.5)
    d.dt = 0.5 * (1 / 16) / 0.5
    st, _ = ws(d)
    assert st == -1
    d = desc(dim=2, n=(16, 16, 1), nv=12, dx=1 / 16, dv=0.5)
    d.dt = 0.5 * (1 / 16) / 0.5
    st, _ = ws(d)
    assert st == 0


def batch_ws(descs):
    from paper_1212_0204_amd import _lib
    arr = (_lib.GridDesc * max(1, len(descs)))(*descs)
    sz = ctypes.c_size_t(0)
    st = _lib.lib().hofks_batch_workspace_size(arr, len(descs), ctypes.byref(sz))
    return st, sz.value


def tube_desc(nx=100, nv=32, dv=0.25, **kw):
    d = dict(dim=1, n=(nx, 1, 1), dx=1.0 / nx, nv=nv, dv=dv, bc=(1, 0, 0), precision=1, scheme=0)
    d.update(kw)
    return desc(**d)


def test_batch_workspace_of_the_512_tubes():
    """two FP32 piece buffers of every tube, plus moments, records and lists"""
    import workloads as W
    tubes = W.batched_tubes()
    st, b = batch_ws([tube_desc(t.nx, t.nv, t.dv) for t in tubes])
    ncv = sum(t.nx * t.nv for t in tubes)
    assert st == 0 and 2 * ncv * 4 <= b < 1.5 * 2 * ncv * 4


@pytest.mark.parametrize("kw", [dict(dim=2, n=(16, 16, 1)), dict(precision=0), dict(bc=(0, 0, 0)),
                                dict(scheme=1), dict(nv=12), dict(nv=4)])
def test_bad_batch_tubes_are_rejected(kw):
    """batches hold 1D outflow FP32 HOFKS tubes with n_vel a multiple of 8;
    one bad tube rejects the batch"""
    st, _ = batch_ws([tube_desc(), tube_desc(**kw)])
    assert st == -1
    st, _ = batch_ws([])
    assert st == -1
