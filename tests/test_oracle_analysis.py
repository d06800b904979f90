"""Pins of the analysis oracle (oracle/analysis.py) against what the paper and
the mathematics fix: the conduction state in closed form, manufactured
fields with known derivatives (second-order convergence), the limits of a
correlation coefficient, the Reynolds number of a uniform flow and a
boundary-layer profile whose crossing height is known in closed form.

Paper: arXiv:2411.10372, Sec. 2 (Re, adiabatic profiles), Secs. 4-5
(profiles, boundary layers), Sec. 6.1 (momentum balance), Sec. 6.2
(correlation C).
"""
import numpy as np
import pytest

import oracle
from oracle import analysis as an


def _params(ndim=2, nx=64, nz=17, ny=8, **kw):
    d = dict(ndim=ndim, nx=nx, nz=nz, ny=ny if ndim == 3 else 1, noise_amp=0.0)
    d.update(kw)
    return oracle.Params(**d)


def _state(p, rho, ux, uy, uz, T):
    """conserved fields from primitive node arrays (Sec. 2: E = rho (u^2/2 +
    c_v T + g z))"""
    cv = 1.0 / (p.gamma * p.eps * p.D)
    g = p.gravity_scale / p.eps
    z = (np.arange(p.nz) / (p.nz - 1)).reshape((-1,) + (1,) * (rho.ndim - 1))
    E = rho * (0.5 * (ux * ux + uy * uy + uz * uz) + cv * T + g * z)
    if p.ndim == 3:
        return np.stack([rho, rho * ux, rho * uy, rho * uz, E])
    return np.stack([rho, rho * ux, rho * uz, E])


def _grid(p):
    x = np.arange(p.nx) * (p.aspect / p.nx)
    z = np.arange(p.nz) / (p.nz - 1)
    if p.ndim == 3:
        y = np.arange(p.ny) * (p.aspect / p.ny)
        Z, Y, Xg = np.meshgrid(z, y, x, indexing="ij")
        return Xg, Y, Z
    Z, Xg = np.meshgrid(z, x, indexing="ij")
    return Xg, np.zeros_like(Xg), Z


def test_conduction_state_closed_forms():
    # u = 0, T = 1 - (eps + D) z, rho = T^(m-1): T_sa = -eps z, rho - rho_A in
    # closed form, every velocity quantity zero
    p = _params(nz=33, nx=128)
    X = oracle.init(p)
    prof, _ = an.profiles(p, X)
    A = an.analysis(p, prof)
    z = np.arange(p.nz) / (p.nz - 1)
    Dl = p.eps + p.D
    m = p.gamma * p.D / ((p.gamma - 1.0) * Dl)
    assert np.max(np.abs(A["Tsa_z"] + p.eps * z)) < 1e-14
    rhoA = (1.0 - p.D * z) ** (1.0 / (p.gamma - 1.0))
    assert np.max(np.abs(A["drho_z"] - ((1.0 - Dl * z) ** (m - 1.0) - rhoA))) < 1e-14
    for n in ("u2", "rho_uz_Tsa", "rho_uz2", "Fn", "Fv"):
        assert np.all(prof[an.NAMES.index(n)] == 0.0), n
    assert A["Re"] == 0.0 and A["C"] == 0.0
    assert np.all(A["U_z"] == 0.0)


def test_hydrostatic_balance_converges_at_second_order():
    # the conduction state solves dp/dz = -rho/eps exactly, so the discrete
    # F_p - F_b is the truncation error of the z difference
    errs = []
    for nz in (17, 33, 65, 129):
        p = _params(nz=nz, nx=8)
        prof, _ = an.profiles(p, oracle.init(p))
        errs.append(np.max(np.abs(prof[an.NAMES.index("Fp")] - prof[an.NAMES.index("Fb")])))
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert all(1.9 < o < 2.2 for o in orders), (errs, orders)


def _manufactured(p):
    Xg, Y, Z = _grid(p)
    k = 2.0 * np.pi / p.aspect
    rho = 1.0 + 0.2 * np.cos(k * Xg) * np.cos(np.pi * Z) + 0.1 * np.sin(k * Y)
    ux = 0.3 * np.sin(k * Xg) * np.sin(np.pi * Z) + 0.05 * np.cos(k * Y)
    uy = 0.2 * np.cos(k * Y) * np.cos(np.pi * Z) if p.ndim == 3 else np.zeros_like(Xg)
    uz = 0.4 * np.cos(k * Xg) * np.sin(2.0 * np.pi * Z) + 0.1 * np.sin(k * Y) * Z
    T = 1.0 - 0.5 * Z + 0.01 * np.sin(k * Xg) * np.cos(2.0 * np.pi * Z)
    # exact derivatives
    d = dict(
        uz_x=-0.4 * k * np.sin(k * Xg) * np.sin(2.0 * np.pi * Z),
        uz_y=0.1 * k * np.cos(k * Y) * Z,
        uz_z=0.8 * np.pi * np.cos(k * Xg) * np.cos(2.0 * np.pi * Z) + 0.1 * np.sin(k * Y),
        uz_xx=-0.4 * k * k * np.cos(k * Xg) * np.sin(2.0 * np.pi * Z),
        uz_yy=-0.1 * k * k * np.sin(k * Y) * Z,
        uz_zz=-1.6 * np.pi ** 2 * np.cos(k * Xg) * np.sin(2.0 * np.pi * Z),
        ux_xz=0.3 * k * np.pi * np.cos(k * Xg) * np.cos(np.pi * Z),
        uy_yz=(0.2 * k * np.pi * np.sin(k * Y) * np.sin(np.pi * Z)) if p.ndim == 3 else 0.0,
    )
    return rho, ux, uy, uz, T, d


@pytest.mark.parametrize("ndim", [2, 3])
def test_momentum_terms_converge_to_manufactured_values(ndim):
    errs = {"Fn": [], "Fv": [], "Fp": []}
    for nz in (17, 33, 65):
        n = 4 * (nz - 1)
        p = _params(ndim=ndim, nz=nz, nx=n, ny=n, Ra=1e2, Pr=1.0)
        rho, ux, uy, uz, T, d = _manufactured(p)
        f = an.node_fields(p, _state(p, rho, ux, uy, uz, T))
        c = an._coefs(p)
        Fn = rho * (ux * d["uz_x"] + uy * d["uz_y"] + uz * d["uz_z"]) if ndim == 3 else \
            rho * (ux * d["uz_x"] + uz * d["uz_z"])
        lap = d["uz_xx"] + d["uz_zz"] + (d["uz_yy"] if ndim == 3 else 0.0)
        dzdiv = d["ux_xz"] + d["uz_zz"] + (d["uy_yz"] if ndim == 3 else 0.0)
        Fv = c["mu"] * (lap + (1.0 + c["lam"]) * dzdiv)
        # p = a rho T: its z derivative from the product rule
        Xg, Y, Z = _grid(p)
        k = 2.0 * np.pi / p.aspect
        rho_z = -0.2 * np.pi * np.cos(k * Xg) * np.sin(np.pi * Z)
        T_z = -0.5 - 0.02 * np.pi * np.sin(k * Xg) * np.sin(2.0 * np.pi * Z)
        Fp = -c["a"] * (rho_z * T + rho * T_z)
        errs["Fn"].append(np.max(np.abs(f["Fn"] - Fn)))
        errs["Fv"].append(np.max(np.abs(f["Fv"] - Fv)))
        errs["Fp"].append(np.max(np.abs(f["Fp"] - Fp)))
    for key, e in errs.items():
        orders = [np.log2(e[i] / e[i + 1]) for i in range(len(e) - 1)]
        assert all(o > 1.8 for o in orders), (key, e, orders)


def test_correlation_limits_and_reynolds_of_a_uniform_flow():
    p = _params(nz=17, nx=64)
    Xg, Y, Z = _grid(p)
    k = 2.0 * np.pi / p.aspect
    rho = 1.0 + 0.1 * Z
    uz = 0.2 * np.sin(k * Xg) * np.sin(np.pi * Z)
    TA = 1.0 - p.D * Z
    ux = np.zeros_like(Xg)
    # T_sa = alpha rho u_z: C = sign(alpha)
    for alpha, want in ((0.7, 1.0), (-0.3, -1.0)):
        X = _state(p, rho, ux, ux, uz, TA + alpha * rho * uz)
        A = an.analysis(p, an.profiles(p, X)[0])
        assert abs(A["C"] - want) < 1e-12, (alpha, A["C"])
    # orthogonal in x: every row mean of rho u_z T_sa vanishes
    X = _state(p, rho, ux, ux, uz, TA + 0.01 * np.cos(k * Xg) * np.sin(np.pi * Z))
    A = an.analysis(p, an.profiles(p, X)[0])
    assert abs(A["C"]) < 1e-12
    # uniform flow: Re = sqrt(Ra/Pr) U0 and U(z) = U0
    U0 = 0.037
    X = _state(p, rho, ux + U0, ux, ux, TA)
    A = an.analysis(p, an.profiles(p, X)[0])
    assert abs(A["Re"] - np.sqrt(p.Ra / p.Pr) * U0) < 1e-12 * A["Re"]
    assert np.max(np.abs(A["U_z"] - U0)) < 1e-15


def test_volume_mean_is_the_trapezoid_rule():
    # exact for linear profiles; the mean of z over [0, 1] is 1/2
    z = np.arange(33) / 32.0
    assert an.volume_mean(3.0 + 2.0 * z) == pytest.approx(4.0, abs=1e-15)
    assert an.volume_mean(z * z) == pytest.approx(1.0 / 3.0 + 1.0 / (6.0 * 32 ** 2), abs=1e-15)


def test_boundary_layer_thickness_of_an_exponential_profile():
    # <T>(z) = 1 - D z - Ab db (1 - e^(-z/db)) + At dt (1 - e^(-(1-z)/dt)):
    # slope -D - Ab e^(-z/db) near the bottom, -D - At e^(-(1-z)/dt) near the
    # top, so the slope reaches -(1 + r) D at z = db ln(Ab/(r D)) and at
    # 1 - z = dt ln(At/(r D))
    D, r = 0.4, 0.1
    Ab, db, At, dt = 6.0, 0.02, 3.0, 0.05
    want_b = db * np.log(Ab / (r * D))
    want_t = dt * np.log(At / (r * D))
    for nz in (257, 513, 1025):
        h = 1.0 / (nz - 1)
        z = np.arange(nz) * h
        t = 1.0 - D * z - Ab * db * (1.0 - np.exp(-z / db)) + At * dt * (1.0 - np.exp(-(1.0 - z) / dt))
        lb, lt = an.bl_thickness(t, D, r)
        # second order with a fixed constant (the crossing's position within
        # its cell varies with nz, so the error is not monotone); a half-cell
        # slip would be ~h/2, far above this bound
        assert abs(lb - want_b) < 8.0 * h * h and abs(lt - want_t) < 8.0 * h * h, (nz, lb, lt)
    # slope -D everywhere: within the threshold at the first midpoint, so
    # half a cell; slope -2 D everywhere: never within it, so -1
    z = np.arange(65) / 64.0
    assert an.bl_thickness(1.0 - D * z, D, r) == (0.5 / 64, 0.5 / 64)
    assert an.bl_thickness(1.0 - 2.0 * D * z, D, r) == (-1.0, -1.0)


# ---- the tanh-stretched grid -------------------------------------------------

@pytest.mark.parametrize("s", [0.7, 1.8])
def test_stretched_stencils_are_exact_on_polynomials(s):
    # first derivatives exact for linear data, the interior second derivative
    # for quadratics, the plate second derivative for cubics (its stencil is
    # the Lagrange cubic through the plate and three rows)
    p = _params(nz=13, stretch=s)
    z = oracle.heights(p)
    f1 = (0.3 + 1.7 * z)[:, None] * np.ones((1, 4))
    assert np.max(np.abs(an.d_z_grid(f1, z) - 1.7)) < 1e-12
    f2 = (0.3 + 1.7 * z - 2.2 * z * z)[:, None] * np.ones((1, 4))
    assert np.max(np.abs(an.d_zz_grid(f2, z) + 4.4)) < 1e-9
    f3 = (z ** 3)[:, None] * np.ones((1, 4))
    d2 = an.d_zz_grid(f3, z)
    assert abs(d2[0, 0] - 6.0 * z[0]) < 1e-8 and abs(d2[-1, 0] - 6.0 * z[-1]) < 1e-8
    # and on the uniform grid they are the uniform stencils
    zu = np.arange(13) / 12.0
    g = np.sin(3.0 * zu)[:, None] * np.ones((1, 2))
    assert np.max(np.abs(an.d_z_grid(g, zu) - an.d_z(g, 1.0 / 12))) < 1e-13
    assert np.max(np.abs(an.d_zz_grid(g, zu) - an.d_zz(g, 1.0 / 12))) < 1e-10


def test_stretched_conduction_closed_forms_and_volume_weights():
    p = _params(nz=33, nx=32, stretch=1.5)
    X = oracle.init(p)
    prof, _ = an.profiles(p, X)
    A = an.analysis(p, prof)
    z = oracle.heights(p)
    assert np.max(np.abs(A["Tsa_z"] + p.eps * z)) < 1e-14
    for n in ("u2", "rho_uz_Tsa", "rho_uz2", "Fn", "Fv"):
        assert np.all(prof[an.NAMES.index(n)] == 0.0), n
    # dual-cell weights integrate linear profiles exactly over the height 1
    assert abs(an.volume_mean(0.4 + 2.0 * z, z) - 1.4) < 1e-15


def test_stretched_hydrostatic_balance_converges_at_second_order():
    errs = []
    for nz in (17, 33, 65, 129):
        p = _params(nz=nz, nx=8, stretch=1.2)
        prof, _ = an.profiles(p, oracle.init(p))
        errs.append(np.max(np.abs(prof[an.NAMES.index("Fp")] - prof[an.NAMES.index("Fb")])))
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert all(1.8 < o < 2.3 for o in orders), (errs, orders)


def test_stretched_grid_tends_to_the_uniform_analysis():
    kw = dict(nx=32, nz=17, noise_amp=0.0)
    pu = _params(**kw)
    Xu = oracle.init(pu)
    rng = np.random.default_rng(5)
    Xu[1, 1:-1] += 1e-2 * rng.uniform(-1, 1, Xu[1, 1:-1].shape)
    Xu[2, 1:-1] += 1e-2 * rng.uniform(-1, 1, Xu[2, 1:-1].shape)
    pu_prof, scale = an.profiles(pu, Xu)
    errs = []
    for s in (1e-2, 1e-3):
        ps = _params(stretch=s, **kw)
        prof, _ = an.profiles(ps, Xu)
        errs.append(np.max(np.abs(prof - pu_prof) / np.maximum(scale, 1e-300)))
    assert errs[1] < 1e-4 and errs[0] / errs[1] > 30, errs


def test_stretched_boundary_layer_thickness():
    # the exponential layer of the uniform test, sampled on a tanh grid:
    # the crossing height of the slope -(1 + r) D is known in closed form
    D, A, d, r = 0.4, 6.0, 0.02, 0.1
    p = _params(nz=129, stretch=1.5)
    z = oracle.heights(p)
    t = 1.0 - D * z - A * d * (1.0 - np.exp(-z / d)) + A * d * (1.0 - np.exp(-(1.0 - z) / d))
    lb, lt = an.bl_thickness(t, D, r, z=z)
    exact = -d * np.log(r * D / A)     # slope -D - A e^{-z/d} meets -(1+r)D
    assert abs(lb - exact) < 0.05 * exact and abs(lt - exact) < 0.05 * exact, (lb, lt, exact)
