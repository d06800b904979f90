"""The C ABI without a GPU: the library loads, exports every entry point that
include/mtvd.h declares, and rejects bad parameters before any device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mtvd.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mtvd_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    import paper_2411_10372_amd as mtvd
    if not os.path.exists(mtvd.LIB_PATH):
        pytest.fail("libmtvd.so is not built (run __graft_entry__.build())")
    return mtvd.lib()


def test_every_declared_symbol_is_exported(L):
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n


def test_default_params_and_sizes(L):
    import paper_2411_10372_amd as mtvd
    p = mtvd._Params()
    L.mtvd_default_params(ctypes.byref(p))
    assert (p.ndim, p.nx, p.ny, p.nz) == (2, 256, 1, 64)
    assert (p.gamma, p.Pr, p.Ra, p.eps, p.D, p.cfl) == (1.4, 1.0, 1e6, 0.1, 0.4, 0.5)
    assert p.bulk_coef == -2.0 / 3.0 and p.wall_order == 2 and p.limiter_form == 0
    sb, wb = mtvd.state_bytes(mtvd.Params())
    assert sb == 4 * 64 * 256 * 8
    assert wb % 256 == 0 and wb > 0
    sb3, _ = mtvd.state_bytes(mtvd.Params(ndim=3, nx=16, ny=8, nz=9))
    assert sb3 == 5 * 9 * 8 * 16 * 8


@pytest.mark.parametrize("bad,code", [
    (dict(ndim=4), -1), (dict(nz=4), -1), (dict(nx=0), -1), (dict(gamma=1.0), -1),
    (dict(Ra=-1.0), -1), (dict(eps=0.6, D=0.5), -1), (dict(limiter_form=2), -1),
    (dict(wall_order=3), -1), (dict(cfl=1.5), -3), (dict(cfl=0.0), -3),
    (dict(Ra=1.0, nx=4096, nz=1024), -3), (dict(ny=2), -1),
])
def test_create_rejects_bad_parameters(L, bad, code):
    import paper_2411_10372_amd as mtvd
    p = mtvd.Params(**bad)._c()
    ctx = ctypes.c_void_p()
    rc = L.mtvd_create(ctypes.byref(p), None, ctypes.byref(ctx))
    assert rc == code
    assert not ctx.value


def test_strerror_covers_every_code(L):
    for code in range(0, -7, -1):
        s = L.mtvd_strerror(code).decode()
        assert s and s != "unknown status"


def test_adjoint_sizes_and_restrictions(L):
    # workspace: checkpoints (ceil(N/E) states), two intervals' operator
    # inputs (2 x 4E states), two work and two cotangent states, the
    # forward values of two operators (2 x 13 doubles per node) and the mu
    # and K accumulators; 2D and the printed limiter only
    import paper_2411_10372_amd as mtvd
    wb = ctypes.c_size_t()
    p = mtvd.Params(nx=512, nz=128, Ra=1e7)._c()
    assert L.mtvd_adj_bytes(ctypes.byref(p), 500, 50, ctypes.byref(wb)) == 0
    one = 512 * 128 * 8
    least = (10 + 2 * 200 + 2 + 2) * 4 * one + 2 * 13 * one + 2 * one
    assert wb.value >= least
    assert wb.value <= least + (1 << 20)
    small = wb.value
    assert L.mtvd_adj_bytes(ctypes.byref(p), 500, 10, ctypes.byref(wb)) == 0
    assert wb.value < small                      # fewer recomputed states
    assert L.mtvd_adj_bytes(ctypes.byref(p), 0, 50, ctypes.byref(wb)) == -1
    assert L.mtvd_adj_bytes(ctypes.byref(p), 10, 0, ctypes.byref(wb)) == -1
    for bad in (dict(limiter_form=1), dict(ndim=3, ny=8, nx=16, nz=9)):
        q = mtvd.Params(**bad)._c()
        assert L.mtvd_adj_bytes(ctypes.byref(q), 10, 5, ctypes.byref(wb)) == -1
    ctx = ctypes.c_void_p()
    q = mtvd.Params(limiter_form=1)._c()
    assert L.mtvd_adj_create(ctypes.byref(q), 10, 5, None, ctypes.byref(ctx)) == -1
    assert not ctx.value


@pytest.mark.parametrize("kw,code", [
    (dict(stretch=1.0), -1),              # uniform z grids only
    (dict(nz=8193, nx=16384), -2),        # beyond the static scratch
    (dict(ndim=4), -1),
    (dict(cfl=1.5), -3),
])
def test_noalloc_step_rejects_before_device_work(L, kw, code):
    # the checks come before any device call, so no GPU is needed; the
    # buffer pointers are never touched on these paths
    import paper_2411_10372_amd as mtvd
    p = mtvd.Params(**kw)._c()
    which = ctypes.c_int32(-7)
    dummy = ctypes.c_void_p(256)
    rc = L.mtvd_step_noalloc(ctypes.byref(p), dummy, ctypes.c_void_p(512), 1, None,
                             ctypes.byref(which))
    assert rc == code
    assert which.value == -7
    assert L.mtvd_step_noalloc(ctypes.byref(p), dummy, dummy, -1, None,
                               ctypes.byref(which)) == -1
