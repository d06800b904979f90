"""Hand-written adjoint of the time-averaged mean Nusselt number (2D, frozen
dt) against the oracle: the objective itself, directional derivatives and
d/dRa against the oracle's complex-step mode (exact on the branches taken)
and against central differences; checkpoint interval, repeated backward
passes and the autograd wrapper."""
import hashlib
import os

import numpy as np
import pytest

import oracle
from helpers import both, gpu_or_skip
from inputs import theta_field, unit_directions

pytestmark = pytest.mark.gpu

# small case: 48 columns (one column strip), 13 rows; 12 steps in
# checkpoint intervals of 5, 5 and 2
SMALL = dict(nx=48, nz=13, Ra=2e5, noise_amp=0.0, dt_mode=1)
N_SMALL, EVERY_SMALL = 12, 5
# narrower than one tile of the fused reverse (the periodic x direction
# wraps inside a tile's region), and so short that both plates' Nusselt
# numbers read the middle row
NARROW = dict(nx=8, nz=5, Ra=2e5, noise_amp=0.0, dt_mode=1)
# the adjoint workload: 512 x 128, Ra 1e7, gamma 1.4, aspect 4, 500 steps,
# checkpoints every 50, theta seed 4, directions seed 5
C4 = dict(nx=512, nz=128, Ra=1e7, gamma=1.4, aspect=4.0, noise_amp=0.0, dt_mode=1)
N_C4, EVERY_C4 = 500, 50
H = 1e-6
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "adjoint_c4.txt")


def _say(*a):
    print("[case]", *a, flush=True)


def _digest(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.float64).tobytes()).hexdigest()[:16]


def _setup(kw, theta_amp, theta_seed=4):
    po, pg = both(**kw)
    th = theta_field(po.nz, po.nx, seed=theta_seed, amp=theta_amp)
    X0 = oracle.init_theta(po, th)
    return po, pg, th, X0, oracle.dt(po, X0)


def _j_bar(po):
    # Nu_mean reads the row means of T through one-sided differences over
    # 2 dz, weights summing in magnitude to 8 per plate pair, divided by
    # 2 eps; a per-step state parity of 1e-13 (relative; T ~ 1) bounds the
    # objective's difference by 1e-13 * 8 * (M / 2) / (2 eps) * 4 (margin)
    M = po.nz - 1
    return 1e-13 * 8 * (M / 2) / (2 * po.eps) * 4


def test_objective_and_dt_match_oracle():
    gpu_or_skip()
    import paper_2411_10372_amd as mtvd
    _say("objective small")
    po, pg, th, X0, dt = _setup(SMALL, 0.05)
    a = mtvd.Adjoint(pg, N_SMALL, EVERY_SMALL)
    J, dt_used = a.forward(th, 0.0)              # dt of X_0 on the device
    assert abs(dt_used - dt) <= 4e-16 * dt
    J, _ = a.forward(th, dt)
    Jo = oracle.time_avg_nu(po, X0, N_SMALL, dt)
    assert abs(J - Jo) <= _j_bar(po), (J, Jo)


def _cs_bar(gn):
    # the library and the oracle follow trajectories equal to ~1e-13 per
    # step (the per-step parity bar); their derivatives along them differ by
    # that times the conditioning of the N-step map, bounded here by 1e4
    return 1e-9 * gn


@pytest.mark.parametrize("grid", ["small", "narrow"])
def test_gradient_matches_oracle_complex_step(grid):
    gpu_or_skip()
    import paper_2411_10372_amd as mtvd
    _say("gradient", grid, "4 directions, complex step")
    po, pg, th, X0, dt = _setup(SMALL if grid == "small" else NARROW, 0.05)
    a = mtvd.Adjoint(pg, N_SMALL, EVERY_SMALL)
    a.forward(th, dt)
    g, _, _ = a.backward(1.0)
    g = g.cpu().numpy()
    assert not g[0].any() and not g[-1].any()    # plates carry no perturbation
    gn = float(np.sqrt(np.sum(g * g)))
    for v in unit_directions(po.nz, po.nx, 4, seed=5):
        _, d = oracle.time_avg_nu_cs(po, X0, oracle.theta_direction(po, X0, v), N_SMALL, dt)
        ad = float(np.sum(g * v))
        _say("complex step", d, "adjoint", ad, "err/|g|", abs(d - ad) / gn)
        assert abs(d - ad) <= _cs_bar(gn), (d, ad, gn)
        # central differences agree up to their truncation, rounding and the
        # limiter kinks they cross
        jp = oracle.time_avg_nu(po, oracle.init_theta(po, th + H * v), N_SMALL, dt)
        jm = oracle.time_avg_nu(po, oracle.init_theta(po, th - H * v), N_SMALL, dt)
        assert abs((jp - jm) / (2 * H) - ad) <= 1e-6 * gn


@pytest.mark.parametrize("knob", [dict(sweep_order=1), dict(wall_order=1), dict(tvd_on=0)])
def test_gradient_with_reading_knobs_matches_oracle_complex_step(knob):
    """The reading knobs the adjoint accepts: the symmetric split order
    (whose reverse pairs operators of the same axis), first-order plate
    derivatives, the step without its TVD term."""
    gpu_or_skip()
    import paper_2411_10372_amd as mtvd
    _say("gradient with", knob)
    po, pg, th, X0, dt = _setup({**SMALL, **knob}, 0.05)
    a = mtvd.Adjoint(pg, N_SMALL, EVERY_SMALL)
    a.forward(th, dt)
    g, _, _ = a.backward(1.0)
    g = g.cpu().numpy()
    gn = float(np.sqrt(np.sum(g * g)))
    for v in unit_directions(po.nz, po.nx, 2, seed=6):
        _, d = oracle.time_avg_nu_cs(po, X0, oracle.theta_direction(po, X0, v), N_SMALL, dt)
        ad = float(np.sum(g * v))
        _say("complex step", d, "adjoint", ad, "err/|g|", abs(d - ad) / gn)
        assert abs(d - ad) <= _cs_bar(gn), (d, ad, gn)


def _coef_bar(po, dmu, dK):
    # d/dRa = dJ/dmu* dmu*/dRa + dJ/dK* dK*/dRa can cancel; its error is
    # bounded by the same relative error on the scale of the two parts
    _, _, mr, kr = oracle.mu_K(po)
    return 1e-8 * (abs(dmu * mr) + abs(dK * kr))


def test_coefficient_and_ra_gradients_match_oracle_complex_step():
    gpu_or_skip()
    import paper_2411_10372_amd as mtvd
    _say("d/dmu*, d/dK*, d/dRa small")
    po, pg, th, X0, dt = _setup(SMALL, 0.05)
    a = mtvd.Adjoint(pg, N_SMALL, EVERY_SMALL)
    a.forward(th, dt)
    _, _, gr = a.backward(1.0)
    gm, gk = a.coef_grads()
    _, dmu = oracle.time_avg_nu_cs(po, X0, None, N_SMALL, dt, dmu=1.0)
    _, dK = oracle.time_avg_nu_cs(po, X0, None, N_SMALL, dt, dK=1.0)
    _, d = oracle.time_avg_nu_cs(po, X0, None, N_SMALL, dt, dRa=1.0)
    _say("mu", dmu, gm, "K", dK, gk, "Ra", d, gr)
    assert abs(gm - dmu) <= 1e-8 * abs(dmu) and abs(gk - dK) <= 1e-8 * abs(dK)
    assert abs(d - gr) <= _coef_bar(po, dmu, dK), (d, gr)
    hr = 1e-4
    pp = oracle.Params(**{**po.__dict__, "Ra": po.Ra * (1 + hr)})
    pm = oracle.Params(**{**po.__dict__, "Ra": po.Ra * (1 - hr)})
    fd = (oracle.time_avg_nu(pp, X0, N_SMALL, dt) - oracle.time_avg_nu(pm, X0, N_SMALL, dt)) / (
        2 * hr * po.Ra)
    assert abs(fd - gr) <= 1e-5 * abs(fd), (fd, gr)


def test_checkpoint_interval_and_repeats_do_not_change_results():
    torch = gpu_or_skip()
    import paper_2411_10372_amd as mtvd
    _say("checkpoint intervals")
    po, pg, th, X0, dt = _setup(SMALL, 0.05)
    ref = None
    for every in (1, EVERY_SMALL, N_SMALL, 100):
        a = mtvd.Adjoint(pg, N_SMALL, every)
        J, _ = a.forward(th, dt)
        g, gx, gr = a.backward(1.0, want_x0=True)
        g2, gx2, gr2 = a.backward(2.0, want_x0=True)   # again, cotangent x 2
        assert torch.equal(g2, 2 * g) and torch.equal(gx2, 2 * gx) and gr2 == 2 * gr
        out = (J, g.cpu().numpy(), gx.cpu().numpy(), gr)
        if ref is None:
            ref = out
        else:
            assert out[0] == ref[0] and out[3] == ref[3], every
            assert np.array_equal(out[1], ref[1]) and np.array_equal(out[2], ref[2]), every


def test_autograd_wrapper():
    torch = gpu_or_skip()
    import paper_2411_10372_amd as mtvd
    _say("autograd")
    po, pg, th, X0, dt = _setup(SMALL, 0.05)
    a = mtvd.Adjoint(pg, N_SMALL, EVERY_SMALL)
    t = torch.tensor(th, dtype=torch.float64, device="cuda", requires_grad=True)
    ra = torch.tensor(pg.Ra, dtype=torch.float64, requires_grad=True)
    J = mtvd.time_averaged_nu(t, ra, a, dt)
    (3.0 * J).backward()
    b = mtvd.Adjoint(pg, N_SMALL, EVERY_SMALL)
    Jb, _ = b.forward(th, dt)
    g, _, gr = b.backward(3.0)
    assert float(J.detach()) == Jb
    assert torch.equal(t.grad, g)
    assert float(ra.grad) == gr
    with pytest.raises(ValueError):
        mtvd.time_averaged_nu(t, torch.tensor(2 * pg.Ra, dtype=torch.float64), a, dt)


def test_autograd_two_applications_before_backward():
    # J(th1) + J(th2) on one adjoint: the second forward replaces the
    # checkpoints, so the first application's backward recomputes its own;
    # each gradient equals the direct one, and a flat theta gets a flat
    # gradient
    torch = gpu_or_skip()
    import paper_2411_10372_amd as mtvd
    _say("autograd, two applications on one adjoint")
    po, pg, th, X0, dt = _setup(SMALL, 0.05)
    th2 = theta_field(po.nz, po.nx, seed=9, amp=0.05)
    a = mtvd.Adjoint(pg, N_SMALL, EVERY_SMALL)
    t1 = torch.tensor(th, dtype=torch.float64, device="cuda", requires_grad=True)
    t2 = torch.tensor(th2.reshape(-1), dtype=torch.float64, device="cuda", requires_grad=True)
    ra = torch.tensor(pg.Ra, dtype=torch.float64, requires_grad=True)
    J = mtvd.time_averaged_nu(t1, ra, a, dt) + mtvd.time_averaged_nu(t2, ra, a, dt)
    J.backward()
    b = mtvd.Adjoint(pg, N_SMALL, EVERY_SMALL)
    b.forward(th, dt)
    g1, _, r1 = b.backward(1.0)
    b.forward(th2, dt)
    g2, _, r2 = b.backward(1.0)
    assert t2.grad.shape == t2.shape
    assert torch.equal(t1.grad, g1)
    assert torch.equal(t2.grad, g2.reshape(-1))
    assert float(ra.grad) == r1 + r2


def test_autograd_default_dt_is_frozen_at_the_first_application():
    # dt = 0: the first application takes the CFL dt of its X_0, later ones
    # on the same adjoint reuse it, so J(theta) is one function of theta
    torch = gpu_or_skip()
    import paper_2411_10372_amd as mtvd
    _say("autograd, default dt")
    po, pg, th, X0, dt = _setup(SMALL, 0.05)
    th2 = theta_field(po.nz, po.nx, seed=9, amp=0.05)
    a = mtvd.Adjoint(pg, N_SMALL, EVERY_SMALL)
    ra = torch.tensor(pg.Ra, dtype=torch.float64)
    t1 = torch.tensor(th, dtype=torch.float64, device="cuda", requires_grad=True)
    J1 = mtvd.time_averaged_nu(t1, ra, a)
    assert abs(a.frozen_dt - dt) <= 4e-16 * dt
    t2 = torch.tensor(th2, dtype=torch.float64, device="cuda", requires_grad=True)
    J2 = mtvd.time_averaged_nu(t2, ra, a)
    J2.backward()
    b = mtvd.Adjoint(pg, N_SMALL, EVERY_SMALL)
    Jb, _ = b.forward(th2, a.frozen_dt)
    g, _, _ = b.backward(1.0)
    assert float(J2.detach()) == Jb
    assert torch.equal(t2.grad, g)
    assert float(J1.detach()) == b.forward(th, a.frozen_dt)[0]


def test_rejects_what_it_does_not_reverse():
    gpu_or_skip()
    import paper_2411_10372_amd as mtvd
    _, pg = both(**{**SMALL, "limiter_form": 1})
    with pytest.raises(mtvd.MtvdError):
        mtvd.Adjoint(pg, 4, 2)
    _, pg = both(**SMALL)
    with pytest.raises(mtvd.MtvdError):
        mtvd.Adjoint(pg, 0, 2)


def _golden():
    vals = {"dir": {}}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            if "sha" in line:
                vals["header"] = line
            continue
        w = line.split()
        if w[0] == "dir":
            vals["dir"][int(w[1])] = float(w[2])
        else:
            vals[w[0]] = float(w[1])
    return vals


def test_c4_gradient_against_complex_step_golden():
    # the adjoint workload: 16 directional derivatives, d/dmu*, d/dK* and
    # d/dRa stored by
    # tests/golden/make_adjoint_c4.py from the oracle's complex-step mode
    gpu_or_skip()
    import paper_2411_10372_amd as mtvd
    _say("C4 gradient, 16 directions + Ra, complex-step golden")
    gold = _golden()
    po, pg, th, X0, dt = _setup(C4, 1e-3)
    V = unit_directions(po.nz, po.nx, 16, seed=5)
    assert f"sha {_digest(th)}" in gold["header"] and f"sha {_digest(V)}" in gold["header"]
    assert dt == gold["dt"]
    a = mtvd.Adjoint(pg, N_C4, EVERY_C4)
    J, _ = a.forward(th, dt)
    assert abs(J - gold["J"]) <= _j_bar(po), (J, gold["J"])
    g, _, gr = a.backward(1.0)
    g = g.cpu().numpy()
    gn = float(np.sqrt(np.sum(g * g)))
    errs = [abs(float(np.sum(g * v)) - gold["dir"][i]) / gn for i, v in enumerate(V)]
    _say("C4 max |adjoint - complex step| / |g|", max(errs))
    assert max(errs) <= _cs_bar(gn) / gn, errs
    gm, gk = a.coef_grads()
    _say("C4 mu", gm, gold["mu"], "K", gk, gold["K"], "Ra", gr, gold["ra"])
    # dJ/dmu* and dJ/dK* integrate over the whole 500-step trajectory: the
    # oracle's own values move by 1.03e-8 and 3.5e-9 (relative) when its
    # input moves by one ulp, and two FP64 codes differ by rounding at every
    # step, so the bar is N times that one-ulp sensitivity (linear growth,
    # no cancellation assumed)
    rm, rk = N_C4 * 1.03e-8, N_C4 * 3.5e-9
    assert abs(gm - gold["mu"]) <= rm * abs(gold["mu"]), (gm, gold["mu"])
    assert abs(gk - gold["K"]) <= rk * abs(gold["K"]), (gk, gold["K"])
    _, _, mr, kr = oracle.mu_K(po)
    assert abs(gr - gold["ra"]) <= rm * abs(gold["mu"] * mr) + rk * abs(gold["K"] * kr), (
        gr, gold["ra"])


def test_c4_central_differences_within_the_kink_bound():
    # central differences (h = 1e-6) of the library's forward objective along
    # the same 16 directions: over 500 steps of 65536 nodes they cross limiter
    # kinks (phi, the max of the two Courant numbers), so they agree with the
    # exact derivative only to ~1e-5 |g|; the bound checks the size of that
    # disagreement, not the adjoint
    gpu_or_skip()
    import paper_2411_10372_amd as mtvd
    _say("C4 central differences, 16 directions")
    po, pg, th, X0, dt = _setup(C4, 1e-3)
    a = mtvd.Adjoint(pg, N_C4, EVERY_C4)
    a.forward(th, dt)
    g, _, _ = a.backward(1.0)
    g = g.cpu().numpy()
    gn = float(np.sqrt(np.sum(g * g)))
    errs, rels = [], []
    for v in unit_directions(po.nz, po.nx, 16, seed=5):
        jp, _ = a.forward(th + H * v, dt)
        jm, _ = a.forward(th - H * v, dt)
        gv = float(np.sum(g * v))
        d = abs((jp - jm) / (2 * H) - gv)
        errs.append(d / gn)
        rels.append(d / abs(gv))
    _say("C4 max |fd - adjoint| / |g|", max(errs))
    _say("C4 per-direction |fd - adjoint| / |adjoint|", " ".join(f"{r:.2e}" for r in rels))
    assert max(errs) <= 1e-4, errs
    # per direction, relative to the directional derivative itself: over
    # these 16 seeded directions the kink crossings move the difference
    # quotients by 3e-4 to 4.6e-2 of g.v (measured on MI355X); the bar is
    # three times the largest, so a wrong sign or a dropped term in any
    # direction fails while the kink spread does not
    assert max(rels) <= 0.15, rels
