"""3D GPU kernels against the CPU oracle.

Small grids span several 60-column strips, several 4-wide wave blocks along
the exchanged axis and several row chunks, all with ragged ends.  The full
1024 x 1024 x 256 case is checked on sampled columns: the oracle builds the
initial state of a 32 x 32 column box around each sample (the initial state
is pointwise), takes dt from the whole initial state, and applies the six
operators of one step to the box; after them the inner 8 x 8 columns are
exact.
"""
import numpy as np
import pytest

import oracle
from helpers import both, gpu_or_skip, parity_error
from inputs import perturb

pytestmark = pytest.mark.gpu

TOL = 1e-13


def _solver(pg, tiling=None):
    gpu_or_skip()
    import paper_2411_10372_amd as mtvd
    s = mtvd.Solver(pg)
    if tiling is not None:
        s.set_tiling(*tiling)
    return s


def _say(*a):
    print("[case]", *a, flush=True)


GRIDS3 = [(70, 11, 9), (16, 6, 7), (61, 9, 12), (8, 4, 5)]


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("nx,ny,nz", GRIDS3)
@pytest.mark.parametrize("rows", [0, 3])
def test_3d_single_operator_parity(axis, nx, ny, nz, rows):
    _say("sweep3d", axis, nx, ny, nz, rows)
    po, pg = both(ndim=3, nx=nx, ny=ny, nz=nz, Ra=1e5, seed=5)
    X0 = perturb(oracle.init(po), seed=nx + 7 * ny + 31 * nz, amp=0.03)
    s = _solver(pg, (rows, rows))
    s.set_state(X0)
    s.sweep(axis)
    Xg = s.get_state()
    Xo = oracle.sweep(po, axis, 0.5 * oracle.dt(po, X0), X0)
    e = parity_error(Xg, Xo, po)
    assert e <= TOL, e


@pytest.mark.parametrize("knobs", [{}, {"sweep_order": 1}, {"limiter_form": 1},
                                   {"dt_mode": 1}, {"wall_order": 1}],
                         ids=lambda k: ",".join(f"{a}={b:g}" for a, b in k.items()) or "default")
def test_3d_steps_parity(knobs):
    _say("steps3d", knobs)
    po, pg = both(ndim=3, nx=70, ny=11, nz=9, Ra=1e5, seed=8, **knobs)
    X0 = perturb(oracle.init(po), seed=17, amp=0.02)
    s = _solver(pg)
    s.set_state(X0)
    s.step(2)
    Xg = s.get_state()
    Xo, t, _ = oracle.step(po, X0, 2)
    e = parity_error(Xg, Xo, po)
    assert e <= 2 * TOL, e
    d = s.diagnostics()
    do = oracle.diag(po, Xo)
    assert abs(d["time"] - t) <= 1e-14 * t
    assert abs(d["mass"] - do["mass"]) <= 1e-13 * do["mass"]


def test_2d_equals_y_uniform_3d_on_gpu():
    """A y-uniform 3D box evolves like the 2D box (L_y is the identity)."""
    p2o, p2 = both(nx=100, nz=17, Ra=1e5, seed=9, noise_amp=1e-2)
    p3o, p3 = both(ndim=3, nx=100, ny=4, nz=17, Ra=1e5, seed=9, noise_amp=1e-2)
    X2 = oracle.init(p2o)
    X3 = np.zeros(p3o.shape)
    for f2, f3 in ((0, 0), (1, 1), (2, 3), (3, 4)):
        X3[f3] = X2[f2][:, None, :]
    a, b = _solver(p2), _solver(p3)
    a.set_state(X2)
    b.set_state(X3)
    a.step(5)
    b.step(5)
    Y2, Y3 = a.get_state(), b.get_state()
    assert np.all(Y3[2] == 0)
    for f2, f3 in ((0, 0), (1, 1), (2, 3), (3, 4)):
        ref = np.repeat(Y2[f2][:, None, :], 4, axis=1)
        scale = max(np.max(np.abs(ref)), 1.0)
        assert np.max(np.abs(Y3[f3] - ref)) <= 1e-14 * scale
    assert a.diagnostics()["time"] == b.diagnostics()["time"]


def test_3d_mass_conserved_and_deterministic():
    _, pg = both(ndim=3, nx=64, ny=16, nz=17, Ra=1e5, seed=3, noise_amp=1e-2)
    a, b = _solver(pg), _solver(pg)
    a.init_state()
    b.init_state()
    m0 = a.diagnostics()["mass"]
    a.step(20)
    b.step(20)
    assert np.array_equal(a.get_state(), b.get_state())
    m1 = a.diagnostics()["mass"]
    assert abs(m1 - m0) / m0 <= 1e-13


@pytest.mark.parametrize("workload", ["3d_1024x1024x256_ra1e9", "3d_1024x1024x256_ra1e9_tanh1.2"])
def test_3d_full_size_one_step_sampled(workload):
    """1024 x 1024 x 256, Ra 1e9 (uniform and tanh z grid): one GPU step from
    the GPU's own initial state against the oracle on sampled 8 x 8 column
    patches (one of them across the periodic corner), in the launch
    configuration the benchmark times."""
    from paper_2411_10372_amd.workloads import params_dict
    kw = params_dict(workload)
    po, pg = both(**kw)
    _say("3d full size: oracle dt of the initial state", workload)
    X0 = oracle.init(po)
    dt = oracle.dt(po, X0)
    del X0
    s = _solver(pg)
    s.init_state()
    d0 = s.diagnostics()
    assert abs(d0["dt"] - dt) <= 1e-14 * dt
    _say("3d full size: one GPU step")
    s.step(1)
    Xg = s.state_tensor()
    H = 12                      # 6 operators x 2 columns of halo each
    for (i0, j0) in [(0, 0), (1020, 1018), (517, 260)]:
        _say("patch", i0, j0)
        B = oracle.init_box(po, i0 - H, j0 - H, 8 + 2 * H, 8 + 2 * H)
        for axis in (2, 1, 0, 2, 1, 0):
            B = oracle.sweep_box(po, axis, 0.5 * dt, B)
        ref = B[:, :, H:H + 8, H:H + 8]
        ii = [(i0 + a) % po.nx for a in range(8)]
        jj = [(j0 + a) % po.ny for a in range(8)]
        got = Xg[:, :, jj][:, :, :, ii].cpu().numpy()
        e = parity_error(got, ref, po)
        assert e <= TOL, (i0, j0, e)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_3d_results_do_not_depend_on_the_tiling(axis):
    # rows per wave only change which wave computes a node: one operator
    # with 4-row chunks and with 32-row chunks (every chunk touches a plate)
    # agree bit for bit.  L_z runs the chunks clear of the plates in a
    # separately compiled copy of the same arithmetic, which rounds as
    # written (no fused multiply-adds) like the plate copy
    po, pg = both(ndim=3, nx=70, ny=24, nz=33, Ra=1e6, seed=4)
    X0 = perturb(oracle.init(po), seed=77, amp=0.03)
    out = []
    for rows in (4, 32):
        _say("tiling3d", axis, rows)
        s = _solver(pg, (rows, rows))
        s.set_state(X0)
        s.sweep(axis)
        out.append(s.get_state())
        s.close()
    assert np.array_equal(out[0], out[1]), float(np.max(np.abs(out[0] - out[1])))
