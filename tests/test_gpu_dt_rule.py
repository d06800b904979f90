"""dt_rule = 1 (dt also within the explicit diffusion limit, the reading of
the silent time-step rule that lets low-Ra boxes run at any grid) on the
GPU against the oracle: dt of a state, whole steps, and that boxes where the
acoustic limit is the smaller one give the same bits as dt_rule = 0.

Bars: dt of one state equal to the oracle's on the same state (the
diffusion part is a minimum of rho h^2 over nodes divided by one constant,
exact on both sides; the acoustic part agrees to an ulp); steps at the
parity bar of one step, 1e-13, times the steps taken."""
import numpy as np
import pytest

import oracle
from helpers import both, gpu_or_skip, parity_error
from inputs import perturb

pytestmark = pytest.mark.gpu

# diffusion-bound cases (the oracle's dt with dt_rule = 1 is below the
# acoustic one for each: 2D uniform and tanh grid, 3D uniform and tanh grid)
CASES = [
    ("2D 96x48 Ra 2e3", dict(ndim=2, nx=96, ny=1, nz=48, Ra=2e3, seed=1)),
    ("2D 64x33 tanh 1.5 Ra 5e3", dict(ndim=2, nx=64, ny=1, nz=33, Ra=5e3, seed=2, stretch=1.5)),
    ("3D 24x20x17 Ra 2e3", dict(ndim=3, nx=24, ny=20, nz=17, Ra=2e3, seed=3)),
    ("3D 20x16x17 tanh 1.0 Ra 2e3", dict(ndim=3, nx=20, ny=16, nz=17, Ra=2e3, seed=4,
                                         stretch=1.0)),
]


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.mark.parametrize("name,kw", CASES, ids=[c[0] for c in CASES])
def test_dt_of_a_state_matches_oracle(name, kw):
    gpu_or_skip()
    import paper_2411_10372_amd as mtvd
    _say("dt_rule dt", name)
    po, pg = both(**kw, dt_rule=1)
    po0, _ = both(**kw)
    s = mtvd.Solver(pg)
    s.init_state()
    Xg = s.get_state()
    d = s.diagnostics()
    s.close()
    dto = oracle.dt(po, Xg)
    assert dto < oracle.dt(po0, Xg)          # the diffusion limit binds
    assert d["dt"] == dto, (d["dt"], dto)


@pytest.mark.parametrize("name,kw", CASES, ids=[c[0] for c in CASES])
def test_steps_match_oracle(name, kw):
    gpu_or_skip()
    import paper_2411_10372_amd as mtvd
    n = 6
    _say("dt_rule steps", name, n)
    po, pg = both(**kw, dt_rule=1)
    X0 = perturb(oracle.init(po), seed=11, amp=1e-4)
    Xo, t, _ = oracle.step(po, X0, n)
    s = mtvd.Solver(pg)
    s.set_state(X0)
    s.step(n)
    Xg = s.get_state()
    d = s.diagnostics()
    s.close()
    e = parity_error(Xg, Xo, po)
    _say("e", e)
    assert e <= 1e-13 * n, e
    assert abs(d["time"] - t) <= 1e-14 * t


def test_rule_0_rejects_what_rule_1_runs():
    gpu_or_skip()
    import paper_2411_10372_amd as mtvd
    _, pg0 = both(**CASES[0][1])
    with pytest.raises(mtvd.MtvdError) as e:
        mtvd.Solver(pg0)
    assert e.value.code == mtvd.MTVD_ESTABILITY
    _, pg1 = both(**CASES[0][1], dt_rule=1)
    mtvd.Solver(pg1).close()


@pytest.mark.parametrize("ndim", [2, 3])
def test_acoustic_bound_boxes_are_unchanged(ndim):
    # where the acoustic limit is the smaller, dt_rule = 1 changes no bit
    gpu_or_skip()
    import paper_2411_10372_amd as mtvd
    kw = (dict(ndim=2, nx=256, ny=1, nz=64, Ra=1e6, seed=0) if ndim == 2 else
          dict(ndim=3, nx=40, ny=24, nz=17, Ra=1e6, seed=3))
    _say("acoustic-bound", ndim)
    out = []
    for rule in (0, 1):
        _, pg = both(**kw, dt_rule=rule)
        s = mtvd.Solver(pg)
        s.init_state()
        s.step(5)
        out.append((s.get_state(), s.diagnostics()["time"]))
        s.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert out[0][1] == out[1][1]
