"""Pins of the oracle's objective pieces used by the adjoint tests: the
initial state from a temperature perturbation (Sec. 2 conduction state) and
the time-averaged mean Nusselt number (Sec. 2, mean_Nu, over steps of
Sec. 3.1)."""
import numpy as np

import oracle
from inputs import theta_field


def _p(**kw):
    base = dict(nx=32, nz=13, Ra=1e5, dt_mode=1, noise_amp=0.0)
    base.update(kw)
    return oracle.Params(**base)


def test_init_theta_zero_is_the_noise_free_initial_state():
    p = _p()
    X = oracle.init_theta(p, np.zeros((p.nz, p.nx)))
    assert np.array_equal(X, oracle.init(p))


def test_init_theta_row_means_are_T0_plus_theta():
    # the diagnostics compute T from (rho, m, E) on their own; rows 1, 2,
    # M-2, M-1 carry the perturbation, the plates do not
    p = _p()
    th = theta_field(p.nz, p.nx, seed=3, amp=1e-2)
    X = oracle.init_theta(p, th)
    tm = oracle.diag(p, X)["tmean"]
    M = p.nz - 1
    rows = [0, 1, 2, M - 2, M - 1, M]
    for r, k in enumerate(rows):
        T0 = 1.0 - (p.eps + p.D) * k / M
        want = T0 + (th[k].mean() if 0 < k < M else 0.0)
        assert abs(tm[r] - want) <= 1e-14, (k, tm[r], want)
    # momenta stay zero and density is the conduction one
    assert not X[1:3].any()
    assert np.array_equal(X[0], oracle.init(p)[0])


def test_time_avg_nu_is_the_mean_over_the_step_states():
    p = _p()
    X0 = oracle.init_theta(p, theta_field(p.nz, p.nx, seed=4))
    dt = oracle.dt(p, X0)
    X1, _, _ = oracle.step(p, X0, 1, dt_frozen=dt)
    X2, _, _ = oracle.step(p, X1, 1, dt_frozen=dt)
    n1, n2 = oracle.diag(p, X1)["nu_mean"], oracle.diag(p, X2)["nu_mean"]
    assert oracle.time_avg_nu(p, X0, 1, dt) == n1
    assert abs(oracle.time_avg_nu(p, X0, 2, dt) - 0.5 * (n1 + n2)) <= 1e-15
    # the conduction state has Nu = 1 exactly at t = 0 (linear T) and stays
    # near it for a few steps
    Xc = oracle.init_theta(p, np.zeros((p.nz, p.nx)))
    assert abs(oracle.diag(p, Xc)["nu_mean"] - 1.0) <= 1e-12
    assert abs(oracle.time_avg_nu(p, Xc, 3, dt) - 1.0) <= 0.05


def test_time_avg_nu_uses_the_given_dt():
    # a frozen dt is used as given, not recomputed from the state
    p = _p()
    X0 = oracle.init_theta(p, theta_field(p.nz, p.nx, seed=5))
    dt = oracle.dt(p, X0)
    a = oracle.time_avg_nu(p, X0, 3, dt)
    b = oracle.time_avg_nu(p, X0, 3, 0.5 * dt)
    assert a != b
    Xa, _, d = oracle.step(p, X0, 3, dt_frozen=0.5 * dt)
    assert d == 0.5 * dt


def _cs_case(tvd, nsteps=6):
    from inputs import unit_directions
    p = _p(tvd_on=tvd, Ra=1e5)
    th = theta_field(p.nz, p.nx, seed=6, amp=2e-2)
    X0 = oracle.init_theta(p, th)
    dt = oracle.dt(p, X0)
    v = unit_directions(p.nz, p.nx, 1, seed=7)[0]
    return p, th, X0, dt, v, nsteps


def test_complex_step_real_part_is_the_objective():
    p, th, X0, dt, v, N = _cs_case(1)
    J, _ = oracle.time_avg_nu_cs(p, X0, oracle.theta_direction(p, X0, v), N, dt)
    # complex division rounds its real part differently from real division
    assert abs(J - oracle.time_avg_nu(p, X0, N, dt)) <= 1e-13


def test_complex_step_matches_central_differences_where_smooth():
    # without the limiter the map is smooth: central differences converge to
    # the complex-step value as h^2 until rounding (~1e-16/h) takes over
    p, th, X0, dt, v, N = _cs_case(0)
    _, d = oracle.time_avg_nu_cs(p, X0, oracle.theta_direction(p, X0, v), N, dt)
    errs = []
    for h in (1e-3, 1e-4, 1e-5):
        jp = oracle.time_avg_nu(p, oracle.init_theta(p, th + h * v), N, dt)
        jm = oracle.time_avg_nu(p, oracle.init_theta(p, th - h * v), N, dt)
        errs.append(abs((jp - jm) / (2 * h) - d))
    assert errs[1] <= 1e-8 * abs(d) and errs[2] <= 1e-8 * abs(d)
    assert errs[1] < errs[0]
    # d/dRa the same way
    _, dr = oracle.time_avg_nu_cs(p, X0, None, N, dt, dRa=1.0)
    hr = 1e-3
    jp = oracle.time_avg_nu(oracle.Params(**{**p.__dict__, "Ra": p.Ra * (1 + hr)}), X0, N, dt)
    jm = oracle.time_avg_nu(oracle.Params(**{**p.__dict__, "Ra": p.Ra * (1 - hr)}), X0, N, dt)
    assert abs((jp - jm) / (2 * hr * p.Ra) - dr) <= 1e-6 * abs(dr)


def test_complex_step_with_the_limiter_matches_small_differences():
    # with the limiter, a few steps of a strongly perturbed state: central
    # differences with a small h cross few kinks
    p, th, X0, dt, v, N = _cs_case(1, nsteps=3)
    _, d = oracle.time_avg_nu_cs(p, X0, oracle.theta_direction(p, X0, v), N, dt)
    h = 1e-6
    jp = oracle.time_avg_nu(p, oracle.init_theta(p, th + h * v), N, dt)
    jm = oracle.time_avg_nu(p, oracle.init_theta(p, th - h * v), N, dt)
    assert abs((jp - jm) / (2 * h) - d) <= 1e-6 * abs(d)


def test_complex_step_is_linear_in_the_direction():
    # scaling the direction by 2 scales every imaginary part exactly
    p, th, X0, dt, v, N = _cs_case(1)
    V = oracle.theta_direction(p, X0, v)
    _, d1 = oracle.time_avg_nu_cs(p, X0, V, N, dt)
    _, d2 = oracle.time_avg_nu_cs(p, X0, 2.0 * V, N, dt)
    assert d2 == 2.0 * d1
    _, da = oracle.time_avg_nu_cs(p, X0, V, N, dt, dRa=1.0)
    _, dr = oracle.time_avg_nu_cs(p, X0, None, N, dt, dRa=1.0)
    assert abs(da - (d1 + dr)) <= 1e-12 * abs(d1)
