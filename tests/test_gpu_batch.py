"""Batches of independent 2D boxes (one launch per operator for all boxes,
graph-replayed step pairs) against single-box runs and the oracle."""
import numpy as np
import pytest

import oracle
from helpers import both, gpu_or_skip, parity_error

pytestmark = pytest.mark.gpu

SMALL = [dict(nx=64, nz=9, Ra=1e5, seed=11), dict(nx=128, nz=32, Ra=3e6, seed=12),
         dict(nx=70, nz=17, Ra=2e5, seed=13), dict(nx=128, nz=32, Ra=8e7, seed=14),
         dict(nx=200, nz=33, Ra=5e6, seed=15), dict(nx=61, nz=12, Ra=1e5, seed=16)]


def _say(*a):
    print("[case]", *a, flush=True)


def _batch(kws, **common):
    gpu_or_skip()
    import paper_2411_10372_amd as mtvd
    ps = [both(**{**k, **common})[1] for k in kws]
    return mtvd.Batch(ps), ps


def test_batch_equals_single_boxes_and_oracle():
    _say("batch vs single vs oracle")
    import paper_2411_10372_amd as mtvd
    b, ps = _batch(SMALL, noise_amp=1e-2)
    b.init_state()
    b.step(5)                       # a graph pair, a graph pair, one direct step
    for i, kw in enumerate(SMALL):
        po, pg = both(**kw, noise_amp=1e-2)
        s = mtvd.Solver(pg)
        s.init_state()
        s.step(5)
        Xs = s.get_state()
        Xb = b.get_state(i)
        assert np.array_equal(Xb, Xs), i
        Xo, t, _ = oracle.step(po, oracle.init(po), 5)
        assert parity_error(Xb, Xo, po) <= 5e-13, i
        d = b.diagnostics(i)
        assert d["step"] == 5 and abs(d["time"] - t) <= 1e-14 * t


def test_graph_pairs_equal_direct_steps():
    _say("graph vs direct")
    a, _ = _batch(SMALL)
    c, _ = _batch(SMALL)
    a.init_state()
    c.init_state()
    a.step(4)                       # two graph replays
    for _ in range(4):
        c.step(1)                   # four direct steps
    for i in range(len(SMALL)):
        assert np.array_equal(a.get_state(i), c.get_state(i)), i


def test_autotune_keeps_results():
    _say("autotune")
    a, _ = _batch(SMALL)
    c, _ = _batch(SMALL)
    a.init_state()
    c.init_state()
    default = [a.tiling(i) for i in range(len(SMALL))]
    a.autotune(trial_steps=2)
    for i in range(len(SMALL)):
        rx, rz = a.tiling(i)
        assert rx in (4, 8, 16, 32, 64, default[i][0]) and rz in (4, 8, 16, 32, 64, default[i][1])
        assert a.diagnostics(i)["step"] == 0
    a.step(3)
    c.step(3)
    for i in range(len(SMALL)):
        assert np.array_equal(a.get_state(i), c.get_state(i)), i


def test_64_box_layout_runs_and_matches_single_box():
    from paper_2411_10372_amd.workloads import batch_boxes
    import paper_2411_10372_amd as mtvd
    kws = batch_boxes()
    _say("64 boxes", len(kws))
    ps = [mtvd.Params(**{k: v for k, v in kw.items() if k in mtvd.Params.__dataclass_fields__})
          for kw in kws]
    gpu_or_skip()
    b = mtvd.Batch(ps)
    b.init_state()
    b.step(4)
    masses = [b.diagnostics(i)["mass"] for i in range(len(ps))]
    assert all(np.isfinite(masses))
    for i in (0, 17, 63):
        s = mtvd.Solver(ps[i])
        s.init_state()
        s.step(4)
        assert np.array_equal(b.get_state(i), s.get_state()), i
