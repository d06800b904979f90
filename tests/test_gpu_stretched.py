"""The tanh-stretched z grid (Sec. 3.1: non-uniform tangent-hyperbolic grid
in z), GPU (HIP, through the C ABI) against the oracle.

Bars as for the uniform grid (tests/test_gpu_parity.py): parity error
<= 1e-13 after one operator, 3e-13 after three steps, 1e-10 after 200
steps of 256x64, 1e-12 after two steps at 4096x1024.  The metric table the
kernels read holds reciprocals (the oracle divides), which moves each
difference by at most an ulp; the heights themselves are the same libm
tanh on both sides.  Grids span several 60-column strips with a ragged
last strip and several row chunks; nz = 5 is the minimum grid.

3D: every operator (x, y, z) on grids with ragged strips, several wave
blocks and chunks that do and do not touch a plate, and three steps with
reading knobs, to the same bars.

Host-side rejections (batches, the adjoint, bad parameters) run on the CPU.
"""
import ctypes

import numpy as np
import pytest

import oracle
from helpers import both, gpu_or_skip, parity_error
from inputs import perturb

SWEEP_TOL = 1e-13


def _say(*a):
    print("[case]", *a, flush=True)


def _solver(pg, tiling=None):
    gpu_or_skip()
    import paper_2411_10372_amd as mtvd
    s = mtvd.Solver(pg)
    if tiling is not None:
        s.set_tiling(*tiling)
    return s


@pytest.mark.gpu
@pytest.mark.parametrize("nx,nz,s", [(150, 37, 1.2), (64, 5, 2.0), (4096, 1024, 1.2)])
def test_stretched_init_matches_oracle(nx, nz, s):
    _say("init stretched", nx, nz, s)
    po, pg = both(nx=nx, nz=nz, seed=1, Ra=1e10 if nx == 4096 else 1e6, stretch=s)
    sv = _solver(pg)
    sv.init_state()
    Xg = sv.get_state()
    d = sv.diagnostics()
    sv.close()
    Xo = oracle.init(po)
    assert np.array_equal(Xg[1], Xo[1]) and np.array_equal(Xg[2], Xo[2])
    assert np.max(np.abs(Xg[0] - Xo[0]) / Xo[0]) <= 4e-16
    assert np.max(np.abs(Xg[3] - Xo[3]) / Xo[3]) <= 8e-16
    assert abs(d["dt"] - oracle.dt(po, Xo)) <= 1e-14 * d["dt"]


GRIDS = [(150, 37), (8, 5), (61, 11), (121, 16), (64, 64)]


@pytest.mark.gpu
@pytest.mark.parametrize("axis", [0, 2])
@pytest.mark.parametrize("nx,nz", GRIDS)
@pytest.mark.parametrize("s", [0.8, 2.0])
@pytest.mark.parametrize("rows", [0, 3])
def test_stretched_single_operator_parity(axis, nx, nz, s, rows):
    _say("sweep stretched", axis, nx, nz, s, rows)
    po, pg = both(nx=nx, nz=nz, Ra=1e6, seed=5, stretch=s)
    X0 = perturb(oracle.init(po), seed=nx * 31 + nz, amp=0.03)
    sv = _solver(pg, (rows, rows))
    sv.set_state(X0)
    sv.sweep(axis)
    Xg = sv.get_state()
    sv.close()
    Xo = oracle.sweep(po, axis, 0.5 * oracle.dt(po, X0), X0)
    e = parity_error(Xg, Xo, po)
    assert e <= SWEEP_TOL, e


KNOBS = [{}, {"limiter_form": 1}, {"sweep_order": 1}, {"tvd_on": 0}, {"wall_order": 1},
         {"dt_mode": 1}, {"bulk_coef": 2.0 / 3.0}, {"gravity_scale": 0.0}]


@pytest.mark.gpu
@pytest.mark.parametrize("knobs", KNOBS,
                         ids=lambda k: ",".join(f"{a}={b:g}" for a, b in k.items()) or "default")
def test_stretched_steps_parity_with_reading_knobs(knobs):
    _say("stretched knobs", knobs)
    po, pg = both(nx=150, nz=37, Ra=1e5, seed=8, stretch=1.5, **knobs)
    X0 = perturb(oracle.init(po), seed=17, amp=0.02)
    sv = _solver(pg, (5, 6))
    sv.set_state(X0)
    sv.step(3)
    Xg = sv.get_state()
    d = sv.diagnostics()
    sv.close()
    Xo, t, _ = oracle.step(po, X0, 3)
    e = parity_error(Xg, Xo, po)
    assert e <= 3 * SWEEP_TOL, e
    assert abs(d["time"] - t) <= 1e-14 * t
    do = oracle.diag(po, Xo)
    for k in ("mass", "total_energy"):
        assert abs(d[k] - do[k]) <= 1e-12 * abs(do[k]), (k, d[k], do[k])
    for k in ("nu_bottom", "nu_top", "nu_mean"):
        assert abs(d[k] - do[k]) <= 1e-10 * max(1.0, abs(do[k])), (k, d[k], do[k])


@pytest.mark.gpu
def test_stretched_256x64_200_steps():
    kw = dict(nx=256, nz=64, Ra=1e6, Pr=1.0, seed=0, stretch=1.2)
    po, pg = both(**kw)
    sv = _solver(pg)
    sv.init_state()
    _say("stretched 256x64 200 steps")
    sv.step(200)
    Xg = sv.get_state()
    dg = sv.diagnostics()
    sv.close()
    Xo, t, _ = oracle.step(po, oracle.init(po), 200)
    e = parity_error(Xg, Xo, po)
    print("stretched 256x64 parity after 200 steps", e, flush=True)
    assert e <= 1e-10, e
    do = oracle.diag(po, Xo)
    assert dg["step"] == 200
    assert abs(dg["time"] - t) <= 1e-13 * t
    for k in ("mass", "total_energy", "nu_mean"):
        assert abs(dg[k] - do[k]) <= 1e-12 * abs(do[k]), (k, dg[k], do[k])


@pytest.mark.gpu
def test_stretched_4096x1024_two_steps():
    kw = dict(nx=4096, nz=1024, Ra=1e10, Pr=1.0, seed=1, stretch=1.2)
    po, pg = both(**kw)
    sv = _solver(pg)
    sv.init_state()
    _say("stretched 4096x1024 two steps")
    sv.step(2)
    Xg = sv.get_state()
    sv.close()
    Xo, _, _ = oracle.step(po, oracle.init(po), 2)
    e = parity_error(Xg, Xo, po)
    print("stretched 4096x1024 parity after 2 steps", e, flush=True)
    # the same conditioning argument as the uniform 4096x1024 case
    assert e <= 1e-12, e


@pytest.mark.gpu
def test_stretched_mass_conserved_on_gpu():
    _, pg = both(nx=256, nz=64, Ra=1e6, seed=3, noise_amp=1e-2, stretch=2.0)
    sv = _solver(pg)
    sv.init_state()
    m0 = sv.diagnostics()["mass"]
    sv.step(300)
    X = sv.get_state()
    m1 = sv.diagnostics()["mass"]
    sv.close()
    assert abs(m1 - m0) / m0 < 1e-13
    assert np.max(np.abs(X[2])) > 1e-6


@pytest.mark.gpu
def test_stretched_conduction_with_uniform_pressure_is_steady_on_gpu():
    po, pg = both(nx=96, nz=33, noise_amp=0.0, gravity_scale=0.0, Ra=1e5, stretch=2.0)
    z = oracle.heights(po)
    a = (po.gamma - 1.0) / (po.gamma * po.eps * po.D)
    cv = 1.0 / (po.gamma * po.eps * po.D)
    T = 1.0 - (po.eps + po.D) * z
    rho = 1.0 / (a * T)
    X = np.zeros(po.shape)
    X[0] = rho[:, None]
    X[3] = (rho * cv * T)[:, None]
    sv = _solver(pg)
    sv.set_state(X)
    sv.step(10)
    Y = sv.get_state()
    d = sv.diagnostics()
    sv.close()
    scale = np.array([max(np.max(np.abs(X[f])), 1.0) for f in range(4)])
    assert np.max(np.abs(Y - X) / scale[:, None, None]) < 1e-13
    for k in ("nu_bottom", "nu_top", "nu_mean"):
        assert abs(d[k] - 1.0) < 1e-11, (k, d[k])


# ---- 3D ----------------------------------------------------------------------

GRIDS3 = [(70, 11, 9), (16, 6, 7), (61, 9, 12), (8, 4, 5), (24, 20, 40)]


@pytest.mark.gpu
@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("nx,ny,nz", GRIDS3)
@pytest.mark.parametrize("rows", [0, 3])
def test_stretched_3d_single_operator_parity(axis, nx, ny, nz, rows):
    _say("sweep3d stretched", axis, nx, ny, nz, rows)
    po, pg = both(ndim=3, nx=nx, ny=ny, nz=nz, Ra=1e6, seed=5, stretch=1.3)
    X0 = perturb(oracle.init(po), seed=nx * 31 + nz, amp=0.03)
    sv = _solver(pg, (rows, rows))
    sv.set_state(X0)
    sv.sweep(axis)
    Xg = sv.get_state()
    sv.close()
    Xo = oracle.sweep(po, axis, 0.5 * oracle.dt(po, X0), X0)
    e = parity_error(Xg, Xo, po)
    assert e <= SWEEP_TOL, e


@pytest.mark.gpu
@pytest.mark.parametrize("knobs", [{}, {"sweep_order": 1}, {"limiter_form": 1}, {"dt_mode": 1},
                                   {"wall_order": 1}],
                         ids=lambda k: ",".join(f"{a}={b:g}" for a, b in k.items()) or "default")
def test_stretched_3d_steps_parity(knobs):
    _say("stretched 3d knobs", knobs)
    po, pg = both(ndim=3, nx=40, ny=24, nz=33, Ra=1e6, seed=6, stretch=1.5, **knobs)
    X0 = perturb(oracle.init(po), seed=23, amp=0.02)
    sv = _solver(pg, (4, 4))
    sv.set_state(X0)
    sv.step(3)
    Xg = sv.get_state()
    d = sv.diagnostics()
    sv.close()
    Xo, t, _ = oracle.step(po, X0, 3)
    e = parity_error(Xg, Xo, po)
    assert e <= 3 * SWEEP_TOL, e
    assert abs(d["time"] - t) <= 1e-14 * t
    do = oracle.diag(po, Xo)
    assert abs(d["mass"] - do["mass"]) <= 1e-12 * do["mass"]


@pytest.mark.gpu
def test_stretched_3d_y_uniform_equals_2d():
    # a y-uniform 3D state on the stretched grid evolves as the 2D one
    _, p2 = both(ndim=2, nx=64, nz=33, Ra=1e6, seed=2, noise_amp=1e-2, stretch=1.2)
    _, p3 = both(ndim=3, nx=64, ny=6, nz=33, Ra=1e6, seed=2, noise_amp=0.0, stretch=1.2)
    s2 = _solver(p2)
    s2.init_state()
    X2 = s2.get_state()
    X3 = np.zeros(p3.shape)
    for f2, f3 in ((0, 0), (1, 1), (2, 3), (3, 4)):
        X3[f3] = X2[f2][:, None, :]
    s3 = _solver(p3)
    s3.set_state(X3)
    s2.step(5)
    s3.step(5)
    Y2, Y3 = s2.get_state(), s3.get_state()
    s2.close()
    s3.close()
    assert np.max(np.abs(Y3[2])) == 0.0
    for f2, f3 in ((0, 0), (1, 1), (2, 3), (3, 4)):
        scale = max(1.0, np.max(np.abs(Y2[f2])))
        assert np.max(np.abs(Y3[f3] - Y2[f2][:, None, :])) <= 1e-13 * scale, (f2, f3)


# ---- host-side rules (CPU) ---------------------------------------------------

def _lib():
    import os
    import paper_2411_10372_amd as mtvd
    if not os.path.exists(mtvd.LIB_PATH):
        pytest.fail("libmtvd.so is not built")
    return mtvd, mtvd.lib()


def test_stretched_grid_rules_on_the_host():
    mtvd, L = _lib()
    ctx = ctypes.c_void_p()
    for bad in (dict(stretch=-0.5), dict(stretch=10.5), dict(stretch=float("nan")),
                dict(ndim=3, nx=8, ny=8, nz=2049, Ra=1e12, stretch=0.5)):
        p = mtvd.Params(**bad)._c()
        assert L.mtvd_create(ctypes.byref(p), None, ctypes.byref(ctx)) == -1, bad
    # sizes are still reported for a stretched 2D grid; the metric table adds
    # nz * 8 doubles to the workspace
    sb0, wb0 = mtvd.state_bytes(mtvd.Params(nx=64, nz=33))
    sb1, wb1 = mtvd.state_bytes(mtvd.Params(nx=64, nz=33, stretch=1.0))
    assert sb0 == sb1 and wb1 >= wb0 + 33 * 8 * 8
    # batches and the adjoint keep the uniform grid
    boxes = (mtvd._Params * 2)(mtvd.Params(nx=64, nz=17)._c(),
                               mtvd.Params(nx=64, nz=17, stretch=1.0)._c())
    sb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    assert L.mtvd_batch_bytes(boxes, 2, ctypes.byref(sb), ctypes.byref(wb)) == -1
    p = mtvd.Params(nx=64, nz=17, stretch=1.0)._c()
    assert L.mtvd_adj_bytes(ctypes.byref(p), 10, 5, ctypes.byref(wb)) == -1
    # the grid form of the boundary-layer thickness wants increasing heights
    with pytest.raises(mtvd.MtvdError):
        mtvd.bl_thickness(np.ones(9), 0.4, 0.1, z=np.zeros(9))


def test_library_and_oracle_grids_are_the_same_bits():
    # the heights the kernels use (made on the host, copied at bind) and the
    # oracle's: the same definition evaluated with the same libm tanh
    mtvd, _ = _lib()
    for nz, s in ((5, 2.0), (37, 0.8), (1024, 1.2), (64, 0.0)):
        po = oracle.Params(nz=nz, stretch=s)
        zg = mtvd.grid_heights(mtvd.Params(nz=nz, stretch=s))
        assert np.array_equal(zg, oracle.heights(po)), (nz, s)
    with pytest.raises(mtvd.MtvdError):
        mtvd.grid_heights(mtvd.Params(nz=9, stretch=-1.0))
