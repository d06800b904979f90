"""Pins of the oracle on the tanh-stretched z grid (Sec. 3.1: a non-uniform
tangent-hyperbolic grid in z, uniform in x and y).

The paper names the grid family but not its formula or parameter; the
oracle takes z_k = (1 + tanh(s (2k/M - 1)) / tanh s) / 2 and divides every z
difference by the same difference of the heights (the reading is written
out in oracle/mtvd_oracle.h).  The pins fix that reading from outside the
oracle:

* the grid: plates at exactly 0 and 1, monotone and symmetric, and the
  plate spacing of the tanh map's derivative, 2 s / (M sinh 2 s), with the
  centre spacing s / (M tanh s);
* the uniform limit: as s -> 0 every result tends to the uniform scheme
  (pinned elsewhere) at the rate s^2;
* exact invariants that hold only when each difference uses the right
  spacing: mass conserved with the dual-cell (trapezoid) weights of the
  stretched grid; the conduction state with uniform pressure (gravity off,
  T linear in z, rho = p0 / (a T)) is steady to roundoff, with Nu = 1;
* consistency: the discrete error of the hydrostatic-conductive state falls
  as dz^2 on a fixed stretched map;
* dt uses the narrowest z face.
"""
import numpy as np
import pytest

from oracle import Params


def _heights_ok(z):
    return z[0] == 0.0 and z[-1] == 1.0 and np.all(np.diff(z) > 0)


@pytest.mark.parametrize("s", [0.5, 1.2, 2.5])
def test_grid_ends_symmetry_and_spacing(ora, s):
    for nz in (9, 64, 1025):
        p = Params(nz=nz, stretch=s)
        z = ora.heights(p)
        M = nz - 1
        assert _heights_ok(z)
        assert np.max(np.abs(z + z[::-1] - 1.0)) <= 2.3e-16
        if nz == 1025:
            # derivative of the map: dz/dxi = s (1 - tanh^2(s (2 xi - 1))) / tanh s
            # times 2 / 2, i.e. 2 s / sinh(2 s) at the plates, s / tanh s at the centre
            h0 = (z[1] - z[0]) * M
            hc = (z[M // 2 + 1] - z[M // 2 - 1]) * M / 2
            assert abs(h0 / (2 * s / np.sinh(2 * s)) - 1.0) < 5e-3, h0
            assert abs(hc / (s / np.tanh(s)) - 1.0) < 1e-5, hc
    # s = 0 is the uniform grid, exactly
    z0 = ora.heights(Params(nz=17, stretch=0.0))
    assert np.array_equal(z0, np.arange(17) / 16.0)


def _scale(X):
    return np.array([max(np.max(np.abs(X[f])), 1.0) for f in range(X.shape[0])])


@pytest.mark.parametrize("ndim", [2, 3])
def test_uniform_limit(ora, ndim):
    """s -> 0: z_k = k/M (1 + O(s^2)), so every stage tends to the uniform
    scheme; the difference falls 100x per 10x in s until roundoff."""
    kw = dict(ndim=ndim, nx=12, ny=6 if ndim == 3 else 1, nz=11, Ra=1e5, noise_amp=1e-2, seed=4)
    pu = Params(**kw)
    Xu0 = ora.init(pu)
    Yu, _, _ = ora.step(pu, Xu0, 2)
    du = ora.diag(pu, Yu)
    errs = []
    for s in (1e-2, 1e-3):
        ps = Params(**kw, stretch=s)
        Ys, _, _ = ora.step(ps, ora.init(ps), 2)
        errs.append(np.max(np.abs(Ys - Yu) / _scale(Yu)[:, None, None] if ndim == 2 else
                           np.abs(Ys - Yu) / _scale(Yu)[:, None, None, None]))
        ds = ora.diag(ps, Ys)
        assert abs(ds["mass"] - du["mass"]) < 10 * s * s * du["mass"]
        assert abs(ds["nu_mean"] - du["nu_mean"]) < 100 * s * s
    assert 50 < errs[0] / errs[1] < 200, errs


@pytest.mark.parametrize("s", [1.0, 2.5])
def test_mass_conserved_with_dual_cell_weights(ora, s):
    """No mass crosses the plates, so sum_k w_k rho_k (w_k the dual cell,
    half a face at a plate) is constant: it telescopes only if the predictor,
    corrector, plate updates and TVD fluxes all use the right spacing."""
    p = Params(nx=32, nz=17, noise_amp=1e-2, seed=3, Ra=1e5, stretch=s)
    X = ora.init(p)
    m0 = ora.diag(p, X)["mass"]
    Y, t, dt = ora.step(p, X, 150)
    m1 = ora.diag(p, Y)["mass"]
    assert abs(m1 - m0) / m0 < 1e-13, (m0, m1)
    assert np.max(np.abs(Y[2])) > 1e-6
    # the weights themselves: heights -> trapezoid weights sum to the height 1
    z = ora.heights(p)
    w = np.empty_like(z)
    w[1:-1] = 0.5 * (z[2:] - z[:-2])
    w[0], w[-1] = 0.5 * (z[1] - z[0]), 0.5 * (z[-1] - z[-2])
    assert abs(w.sum() - 1.0) < 1e-15
    rho_lin = 1.0 + 0.3 * z                      # linear: trapezoid is exact
    Xl = np.zeros(p.shape)
    Xl[0] = rho_lin[:, None]
    Xl[3] = 1.0
    assert abs(ora.diag(p, Xl)["mass"] - 1.15 * p.aspect) < 1e-13


@pytest.mark.parametrize("s", [0.8, 2.0])
@pytest.mark.parametrize("wall_order,lf", [(2, 0), (1, 0), (2, 1)])
def test_conduction_with_uniform_pressure_is_steady(ora, s, wall_order, lf):
    """Gravity off, u = 0, T = 1 - (eps + D) z linear between the plate
    temperatures, rho = p0 / (a T): the pressure is uniform and the heat flux
    K dT/dz is the same at every node and plate, so every flux difference is
    zero; E = rho cv T = p0 cv / a is uniform, only rho varies and the TVD
    ratios stay near 1 (no limiter action).  A face-spacing mistake anywhere
    in the z operator shows up as a drift."""
    p = Params(nx=8, nz=21, noise_amp=0.0, gravity_scale=0.0, Ra=1e5, stretch=s,
               wall_order=wall_order, limiter_form=lf)
    z = ora.heights(p)
    a = (p.gamma - 1.0) / (p.gamma * p.eps * p.D)
    cv = 1.0 / (p.gamma * p.eps * p.D)
    T = 1.0 - (p.eps + p.D) * z
    rho = 1.0 / (a * T)
    X = np.zeros(p.shape)
    X[0] = rho[:, None]
    X[3] = (rho * cv * T)[:, None]
    Y, _, _ = ora.step(p, X, 3)
    rel = np.abs(Y - X) / _scale(X)[:, None, None]
    assert np.max(rel) < 2e-14, np.max(rel)
    d = ora.diag(p, X)
    for k in ("nu_bottom", "nu_top", "nu_mean"):
        assert abs(d[k] - 1.0) < 1e-12, (k, d[k])


def test_hydrostatic_error_is_second_order_on_a_stretched_map(ora):
    """The conductive-hydrostatic profile solves the equations exactly but
    not the scheme: on a fixed tanh map (s = 1.5) the spurious velocity at a
    fixed time falls about 4x per doubling of nz, as on the uniform grid.
    A first-order slip (a one-sided spacing where a central one belongs)
    would halve it instead."""
    umax = []
    for nz in (33, 65, 129):
        p = Params(nx=4, nz=nz, noise_amp=0.0, Ra=1e5, stretch=1.5)
        X = ora.init(p)
        n = int(round(0.1 / ora.dt(p, X)))
        Y, t, _ = ora.step(p, X, n)
        umax.append(np.max(np.abs(Y[2] / Y[0])))
    assert umax[0] / umax[1] > 3.3 and umax[1] / umax[2] > 3.3, umax
    # the centre cells are s / tanh s = 1.66x the uniform ones: about 2.8x
    # the uniform grid's 1e-4 bound at nz = 129
    assert umax[2] < 3e-4


def test_dt_uses_the_narrowest_face(ora):
    """Uniform state at rest, gravity off: c is the same everywhere, so
    dt = cfl min(dx, z_1 - z_0) / c with the plate face the narrowest."""
    p = Params(nx=4, nz=33, noise_amp=0.0, gravity_scale=0.0, stretch=2.0, aspect=4.0)
    T0 = 0.7
    X = np.zeros(p.shape)
    X[0] = 1.0
    X[3] = 1.0 / (p.gamma * p.eps * p.D) * T0
    c = np.sqrt((p.gamma - 1.0) / (p.eps * p.D) * T0)
    z = ora.heights(p)
    want = p.cfl * min(p.aspect / p.nx, z[1] - z[0]) / c
    assert abs(ora.dt(p, X) - want) <= 1e-15 * want


def test_2d_equals_y_uniform_3d_on_the_stretched_grid(ora):
    p2 = Params(ndim=2, nx=10, nz=9, Ra=1e5, noise_amp=1e-2, seed=2, stretch=1.3)
    p3 = Params(ndim=3, nx=10, ny=4, nz=9, Ra=1e5, noise_amp=0.0, stretch=1.3)
    X2 = ora.init(p2)
    X3 = np.zeros(p3.shape)
    X3[0] = X2[0][:, None, :]
    X3[1] = X2[1][:, None, :]
    X3[3] = X2[2][:, None, :]
    X3[4] = X2[3][:, None, :]
    Y2, _, _ = ora.step(p2, X2, 2)
    Y3, _, _ = ora.step(p3, X3, 2)
    assert np.max(np.abs(Y3[2])) == 0.0
    for f2, f3 in ((0, 0), (1, 1), (2, 3), (3, 4)):
        assert np.max(np.abs(Y3[f3] - Y2[f2][:, None, :])) <= 1e-14 * max(1.0, np.max(np.abs(Y2[f2])))


def test_stretched_grid_parameter_is_checked(ora):
    for bad in (-0.1, float("nan"), 11.0):
        with pytest.raises(Exception):
            ora.init(Params(nz=9, stretch=bad))


def test_tvd_term_at_an_isolated_spike_in_z(ora):
    """z operator on a stretched grid, uniform state at rest (gravity and
    diffusion off) plus a spike s in E on row k: both faces of the spike get
    phi = 0, G = C/2 with C = Co (1 - Co) and Co = tau c / h_face (the face's
    own spacing); the term is the difference of the face fluxes h G dE over
    the dual cell w of each row.  On the uniform grid this is the printed
    term (the x version is pinned in test_oracle_pins)."""
    p = Params(nx=4, nz=17, gravity_scale=0.0, diffusion_scale=0.0, noise_amp=0.0,
               stretch=1.8)
    z = ora.heights(p)
    cv = 1.0 / (p.gamma * p.eps * p.D)
    X = np.zeros(p.shape)
    X[0] = 1.0
    X[3] = cv * 0.75
    k, s = 5, 0.2
    X[3, k] += s
    tau = 0.5 * ora.dt(p, X)
    Y1 = ora.sweep(p, 2, tau, X)
    Y0 = ora.sweep(Params(**{**p.__dict__, "tvd_on": 0}), 2, tau, X)
    d = (Y1 - Y0)[3, :, 0]
    a = (p.gamma - 1) / (p.gamma * p.eps * p.D)
    c = np.sqrt(p.gamma * a * X[3, :, 0] / (cv * X[0, :, 0]))
    hl, hr = z[k] - z[k - 1], z[k + 1] - z[k]
    w = lambda j: 0.5 * (z[j + 1] - z[j - 1])
    Col = tau / hl * max(c[k - 1], c[k])
    Cor = tau / hr * max(c[k], c[k + 1])
    Gl, Gr = 0.5 * Col * (1 - Col), 0.5 * Cor * (1 - Cor)
    assert abs(d[k - 1] - hl * Gl * s / w(k - 1)) < 1e-14
    assert abs(d[k] + (hl * Gl + hr * Gr) * s / w(k)) < 1e-14
    assert abs(d[k + 1] - hr * Gr * s / w(k + 1)) < 1e-14
    assert np.all(d[:k - 1] == 0) and np.all(d[k + 2:] == 0)
    assert np.all((Y1 - Y0)[:3] == 0)


def test_cross_derivative_in_z_of_the_x_operator(ora):
    """The x operator reads z derivatives only through the centred cross
    terms (d_z u_x in tau_xz).  Gravity off, uniform rho and T, u_z = 0 and
    a tiny shear u_x = U sin(kx) (a + b z) that is linear in z: to first
    order in U every predicted field stays linear in z, so the centred
    differences are exact on any grid, d_z u_x = b U sin(kx) on every row,
    and the m_z the operator creates (from -mu d_z u_x) is the same on
    every row whose stencils stay off the plates.  A centred difference over the wrong span (twice a
    face instead of z_k+1 - z_k-1) makes it vary from row to row by the
    face-to-face growth of the tanh grid."""
    p = Params(nx=16, nz=13, gravity_scale=0.0, noise_amp=0.0, Ra=1e3, aspect=1.0,
               stretch=2.0)
    z = ora.heights(p)
    x = np.arange(p.nx) * p.aspect / p.nx
    cv = 1.0 / (p.gamma * p.eps * p.D)
    U = 1e-7
    ux = U * np.sin(2 * np.pi * x)[None, :] * (0.3 + 0.8 * z)[:, None]
    X = np.zeros(p.shape)
    X[0] = 1.0
    X[1] = ux
    X[3] = cv * 0.8 + 0.5 * ux * ux
    Y = ora.sweep(p, 0, 1e-3, X)
    # rows 2..M-2: the corrector's centred differences of rows 1 and M-1
    # read the plate rows, which the x operator copies through unpredicted
    mz = Y[2, 2:-2]
    spread = np.max(np.abs(mz - mz[0][None, :]))
    assert np.max(np.abs(mz)) > 1e-12
    assert spread <= 1e-5 * np.max(np.abs(mz)), spread / np.max(np.abs(mz))
