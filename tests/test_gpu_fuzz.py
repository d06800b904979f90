"""Seeded random parameter sets, GPU against the oracle (tiny grids).

Each case draws a grid (down to one column in x and y and the minimum nz;
uniform or tanh-stretched in z), all parameters of Sec. 2, every switch of
the scheme, the rows per wave and a perturbation of the oracle's initial
state (tests/inputs.random_case), then takes 1-4 full steps (Sec. 3.1) on
both sides.  The cases are a fixed
list: the same draws on every run, each printed before it runs.

Bar: parity error (tests/helpers.parity_error) <= max(3e-13, 16 s), where s
is the oracle's own sensitivity for that case -- the parity error between
the oracle's result and its result from the input moved by one ulp in every
value.  The GPU's arithmetic differs from the oracle's by a few roundings
per operation (contractions, reduction order of dt), which moves the result
like a perturbation of a few ulps; where the TVD ratios sit near a switch
of the limiter, s exceeds the fixed 1e-13-per-step bar of the hand-picked
cases.  A case whose s is above 1e-11 is too ill-conditioned to compare
element by element and fails the test rather than hide a mistake: the
draws are fixed, so this is settled once.  A parameter set the library
rejects (diffusion number above 1/2) must be rejected with
MTVD_ESTABILITY and nothing else, and then runs with dt_rule = 1 (dt also
within the diffusion limit) on both sides, so every case runs.
"""
import ctypes
import os

import numpy as np
import pytest

import oracle
from helpers import both, gpu_or_skip, parity_error
from inputs import perturb, random_case

CASES = [(2, s) for s in range(40)] + [(3, 1000 + s) for s in range(20)]
SENS_MAX = 1e-11


def _case(ndim, seed):
    kw = random_case(seed, ndim)
    extra = {k: kw.pop(k) for k in ("amp", "pseed", "tiling", "steps")}
    return kw, extra


def _one_ulp_up(X):
    return np.nextafter(X, np.inf)


@pytest.mark.gpu
@pytest.mark.parametrize("ndim,seed", CASES, ids=[f"{d}d-{s}" for d, s in CASES])
def test_random_parameters_match_oracle(ndim, seed):
    gpu_or_skip()
    import paper_2411_10372_amd as mtvd
    kw, ex = _case(ndim, seed)
    print(f"[case] fuzz {ndim}d seed {seed}: {kw} {ex}", flush=True)
    po, pg = both(**kw)
    try:
        s = mtvd.Solver(pg)
    except mtvd.MtvdError as err:
        # the acoustic rule alone would break the explicit diffusion limit:
        # rejected as documented, and run with dt_rule = 1 on both sides
        assert err.code == -3, err
        kw["dt_rule"] = 1
        print("[case] diffusion-bound: dt_rule = 1", flush=True)
        po, pg = both(**kw)
        s = mtvd.Solver(pg)
    try:
        s.set_tiling(*ex["tiling"])
        X0 = perturb(oracle.init(po), seed=ex["pseed"], amp=ex["amp"])
        Xo, t, _ = oracle.step(po, X0, ex["steps"])
        assert np.all(np.isfinite(Xo)), "oracle result not finite"
        Xs, _, _ = oracle.step(po, _one_ulp_up(X0), ex["steps"])
        sens = parity_error(Xs, Xo, po)
        assert sens <= SENS_MAX, f"ill-conditioned case: oracle sensitivity {sens:.3g}"
        s.set_state(X0)
        s.step(ex["steps"])
        Xg = s.get_state()
        d = s.diagnostics()
    finally:
        s.close()
    e = parity_error(Xg, Xo, po)
    bar = max(3e-13, 16.0 * sens)
    print(f"[case] e {e:.3g} sensitivity {sens:.3g} bar {bar:.3g}", flush=True)
    assert e <= bar, (e, sens)
    assert abs(d["time"] - t) <= 1e-14 * t
    assert d["step"] == ex["steps"]


def test_most_cases_are_accepted():
    # The draws are meant to exercise the scheme, not the rejection path.
    # mtvd_create validates before its first HIP call, so this runs on the
    # CPU: a rejected set returns MTVD_ESTABILITY (-3) here as on the GPU.
    import paper_2411_10372_amd as mtvd
    if not os.path.exists(mtvd.LIB_PATH):
        pytest.fail("libmtvd.so is not built")
    L = mtvd.lib()
    rejected = 0
    for ndim, seed in CASES:
        kw, _ = _case(ndim, seed)
        _, pg = both(**kw)
        p = pg._c()
        ctx = ctypes.c_void_p()
        rc = L.mtvd_create(ctypes.byref(p), None, ctypes.byref(ctx))
        if rc == 0:
            L.mtvd_destroy(ctx)
        assert rc in (0, -3, -6), (ndim, seed, rc)   # -6: no GPU here
        rejected += rc == -3
    assert rejected <= len(CASES) // 4, rejected
