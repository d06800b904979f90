"""Plain CPU FP64 oracle of the analysis quantities of the paper's Secs. 4-6.

TEST INFRASTRUCTURE ONLY (as the rest of ``oracle/``): only ``tests/`` may
import it.  Plain numpy, one formula per quantity, no blocking or fusion.

Paper: Tiwari, Sharma & Verma, arXiv:2411.10372.
  Sec. 2, Eq. (Re): Re = sqrt(Ra/Pr) U, U the rms velocity of a snapshot;
      the adiabatic profiles T_A(z) = 1 - D z, rho_A(z) = (1 - D z)^beta with
      beta = 1/(gamma - 1); T_sa = T - T_A.
  Secs. 4-5 (adiabatic profile, boundary layers): horizontally averaged
      profiles <T>_A(z), T_sa(z), rho - rho_A(z) and the rms velocity U(z);
      the boundary-layer thicknesses lambda_b, lambda_t where the slope of
      <T>_A meets the adiabatic gradient -D.
  Sec. 6.1 (Re scaling, momentum balance): z components F_n = rho (u . grad) u_z,
      F_p = -dp/dz, F_b = rho g (g = 1/eps in these units: the momentum
      equation's source is -rho/eps), F_v = d_i tau_iz, volume averaged.
  Sec. 6.2 (Nu scaling): the correlation
      C = <rho u_z T_sa> / sqrt(<(rho u_z)^2> <T_sa^2>).

Readings where the paper is silent (listed with the others in the design
notes):
  * <.>_A: the mean over the nx (x ny) nodes of a row; <.>_V: the
    trapezoid rule over the rows (weight 1/2 on the two plates) times
    dz, over a box of height 1 -- the weights of the solver's diagnostics.
  * First derivatives: central second order along x, y (periodic) and at
    interior rows; second-order one-sided on the plates, (-3, 4, -1)/(2 dz)
    at z = 0 and (3, -4, 1)/(2 dz) at z = 1.  Second derivatives: (1, -2,
    1)/h^2; on the plates (2, -5, 4, -1)/dz^2 over the plate and the three
    rows next to it.  Mixed derivatives: the z operator applied to the
    central x (or y) difference of each row it reads.
  * F_v = mu (lap u_z + (1 + lambda) d_z div u), which equals d_i tau_iz for
    the constant mu of these units, tau_ij = mu (d_j u_i + d_i u_j +
    lambda div u delta_ij), lambda the solver's bulk coefficient.
  * |u|^2 = u_x^2 (+ u_y^2) + u_z^2.
  * On the tanh-stretched grid every z derivative is the stencil on the
    node heights z_k: first derivatives (f_k+1 - f_k-1)/(z_k+1 - z_k-1)
    inside and the one-sided plate stencil over the same stencil of z
    (exact for linear f); second derivatives 2[(f_k+1 - f_k)/h+ - (f_k -
    f_k-1)/h-]/(h+ + h-) inside (exact for quadratics) and the four-point
    one-sided Lagrange stencil on the plate and the three rows next to it
    (exact for cubics); both reduce to the uniform stencils above when the
    spacing is uniform.  <.>_V weighs rows by their dual cells.
  * Boundary layers: slopes of the profile at the midpoints between rows;
    lambda_b is the height where, going up from z = 0, the slope first rises
    to -(1 + rtol) D (linear interpolation between midpoints); lambda_t the
    same from z = 1 going down, measured from the top plate.  rtol
    (default 0.1) states how close "approximates" has to be.

Parity status (stretched grid): the stencils pinned by exactness on
polynomials of the stated degrees and the uniform limit; the conduction
state and the second-order hydrostatic balance on a fixed map as below.

Parity status: profiles and volume means pinned (conduction state in
closed form: u = 0, T_sa = -eps z, rho and rho_A closed forms, F_p - F_b
-> 0 at second order; manufactured velocity fields for F_n and F_v at
second order; C = +-1 and 0 for (anti)aligned and orthogonal fields; Re of
a uniform flow); boundary-layer thickness pinned by an exponential profile
whose crossing height is known in closed form.
"""
from __future__ import annotations

import numpy as np

# rows of the profile array (the same order as the library's output)
NAMES = ("T", "rho", "u2", "rho_uz_Tsa", "rho_uz2", "Tsa2", "Fn", "Fp", "Fb", "Fv")


def heights(p):
    """Node heights of the grid (uniform k/M, or the tanh grid)."""
    if getattr(p, "stretch", 0.0) > 0.0:
        from . import heights as _h
        return _h(p)
    return np.arange(p.nz, dtype=np.float64) / (p.nz - 1)


def _coefs(p):
    """The nondimensional constants of Sec. 2 the analysis needs."""
    cv = 1.0 / (p.gamma * p.eps * p.D)
    return dict(
        z=heights(p),
        stretched=getattr(p, "stretch", 0.0) > 0.0,
        cv=cv,
        a=(p.gamma - 1.0) / (p.gamma * p.eps * p.D),
        g=p.gravity_scale / p.eps,
        mu=np.sqrt(p.Pr / p.Ra) * p.diffusion_scale,
        lam=p.bulk_coef,
        hx=p.aspect / p.nx,
        hy=p.aspect / p.ny if p.ndim == 3 else 1.0,
        hz=1.0 / (p.nz - 1),
    )


def primitives(p, X):
    """rho, velocity components, T and p of every node (arrays shaped like
    one field of X: (nz, nx) in 2D, (nz, ny, nx) in 3D)."""
    c = _coefs(p)
    X = np.asarray(X, dtype=np.float64)
    rho = X[0]
    ux = X[1] / rho
    uy = X[2] / rho if p.ndim == 3 else np.zeros_like(rho)
    uz = X[p.ndim] / rho
    E = X[p.ndim + 1]
    zz = c["z"].reshape((-1,) + (1,) * (rho.ndim - 1))
    u2 = ux * ux + uy * uy + uz * uz
    T = (E / rho - 0.5 * u2 - c["g"] * zz) / c["cv"]
    pr = c["a"] * rho * T
    return rho, ux, uy, uz, T, pr, zz


def d_x(f, h):
    return (np.roll(f, -1, axis=-1) - np.roll(f, 1, axis=-1)) / (2.0 * h)


def d_xx(f, h):
    return (np.roll(f, -1, axis=-1) - 2.0 * f + np.roll(f, 1, axis=-1)) / (h * h)


def d_y(f, h):
    return (np.roll(f, -1, axis=-2) - np.roll(f, 1, axis=-2)) / (2.0 * h)


def d_yy(f, h):
    return (np.roll(f, -1, axis=-2) - 2.0 * f + np.roll(f, 1, axis=-2)) / (h * h)


def d_z(f, h):
    """first z derivative along axis 0: central inside, one-sided second
    order on the plates"""
    out = np.empty_like(f)
    out[1:-1] = (f[2:] - f[:-2]) / (2.0 * h)
    out[0] = (-3.0 * f[0] + 4.0 * f[1] - f[2]) / (2.0 * h)
    out[-1] = (3.0 * f[-1] - 4.0 * f[-2] + f[-3]) / (2.0 * h)
    return out


def d_zz(f, h):
    out = np.empty_like(f)
    out[1:-1] = (f[2:] - 2.0 * f[1:-1] + f[:-2]) / (h * h)
    out[0] = (2.0 * f[0] - 5.0 * f[1] + 4.0 * f[2] - f[3]) / (h * h)
    out[-1] = (2.0 * f[-1] - 5.0 * f[-2] + 4.0 * f[-3] - f[-4]) / (h * h)
    return out


def _col(v, f):
    """a per-row array shaped to broadcast against f (rows on axis 0)"""
    return np.asarray(v).reshape((-1,) + (1,) * (f.ndim - 1))


def d_z_grid(f, z):
    """first z derivative on node heights z: central inside, the one-sided
    second-order stencil on the plates, each over the same stencil of z"""
    out = np.empty_like(f)
    out[1:-1] = (f[2:] - f[:-2]) / _col(z[2:] - z[:-2], f)
    out[0] = (-3.0 * f[0] + 4.0 * f[1] - f[2]) / ((-3.0 * z[0] + 4.0 * z[1]) - z[2])
    out[-1] = (3.0 * f[-1] - 4.0 * f[-2] + f[-3]) / ((3.0 * z[-1] - 4.0 * z[-2]) + z[-3])
    return out


def lagrange_d2(zs, x0):
    """weights of the second derivative at x0 of the cubic through the four
    nodes zs: L_j''(x0) = 2 sum_{l != j} (x0 - z_l) / prod_{l != j} (z_j - z_l)"""
    w = np.empty(4)
    for j in range(4):
        o = [zs[l] for l in range(4) if l != j]
        w[j] = 2.0 * sum(x0 - zl for zl in o) / np.prod([zs[j] - zl for zl in o])
    return w


def d_zz_grid(f, z):
    """second z derivative on node heights z: the three-point formula inside,
    the four-point one-sided Lagrange stencil on the plates"""
    out = np.empty_like(f)
    hm = z[1:-1] - z[:-2]
    hp = z[2:] - z[1:-1]
    out[1:-1] = 2.0 * ((f[2:] - f[1:-1]) / _col(hp, f) - (f[1:-1] - f[:-2]) / _col(hm, f)) / \
        _col(hp + hm, f)
    wb = lagrange_d2(z[:4], z[0])
    wt = lagrange_d2(z[-1:-5:-1], z[-1])
    out[0] = ((wb[0] * f[0] + wb[1] * f[1]) + wb[2] * f[2]) + wb[3] * f[3]
    out[-1] = ((wt[0] * f[-1] + wt[1] * f[-2]) + wt[2] * f[-3]) + wt[3] * f[-4]
    return out


def node_fields(p, X):
    """The ten per-node quantities whose row means make the profiles."""
    c = _coefs(p)
    rho, ux, uy, uz, T, pr, zz = primitives(p, X)
    if c["stretched"]:
        z = c["z"]
        dz1 = lambda f, h: d_z_grid(f, z)      # noqa: E731
        dz2 = lambda f, h: d_zz_grid(f, z)     # noqa: E731
    else:
        dz1, dz2 = d_z, d_zz
    TA = 1.0 - p.D * zz
    Tsa = T - TA
    u2 = ux * ux + uy * uy + uz * uz
    hx, hy, hz = c["hx"], c["hy"], c["hz"]
    dzuz = dz1(uz, hz)
    if p.ndim == 3:
        adv = ux * d_x(uz, hx) + uy * d_y(uz, hy) + uz * dzuz
        lap = d_xx(uz, hx) + d_yy(uz, hy) + dz2(uz, hz)
        dz_div = dz1(d_x(ux, hx) + d_y(uy, hy), hz) + dz2(uz, hz)
    else:
        adv = ux * d_x(uz, hx) + uz * dzuz
        lap = d_xx(uz, hx) + dz2(uz, hz)
        dz_div = dz1(d_x(ux, hx), hz) + dz2(uz, hz)
    Fn = rho * adv
    Fp = -dz1(pr, hz)
    Fb = rho * c["g"]
    Fv = c["mu"] * (lap + (1.0 + c["lam"]) * dz_div)
    ruz = rho * uz
    return dict(T=T, rho=rho, u2=u2, rho_uz_Tsa=ruz * Tsa, rho_uz2=ruz * ruz,
                Tsa2=Tsa * Tsa, Fn=Fn, Fp=Fp, Fb=Fb, Fv=Fv)


def profiles(p, X):
    """(10, nz) row means <.>_A of the node quantities, in NAMES order, and
    (10, nz) row means of their absolute values (the scale of each mean,
    for tolerances)."""
    f = node_fields(p, X)
    axes = tuple(range(1, f["T"].ndim))
    mean = np.stack([f[n].mean(axis=axes) for n in NAMES])
    mabs = np.stack([np.abs(f[n]).mean(axis=axes) for n in NAMES])
    return mean, mabs


def volume_mean(prof_row, z=None):
    """<f>_V from row means: trapezoid in z over a height of 1 (on the node
    heights z when given: the dual cells as weights)."""
    v = np.asarray(prof_row, dtype=np.float64)
    if z is not None:
        w = np.empty_like(z)
        w[1:-1] = 0.5 * (z[2:] - z[:-2])
        w[0], w[-1] = 0.5 * (z[1] - z[0]), 0.5 * (z[-1] - z[-2])
        return float(np.sum(w * v))
    M = v.shape[-1] - 1
    w = np.ones(M + 1)
    w[0] = w[-1] = 0.5
    return float(np.sum(w * v) / M)


def analysis(p, prof):
    """Snapshot scalars of Secs. 2 and 4-6 from the (10, nz) profile array: Re, the
    correlation C, the volume means of F_n, F_p, F_b, F_v and of the
    correlation's three inputs, and the derived profiles T_sa(z),
    rho - rho_A(z), U(z)."""
    zg = heights(p) if getattr(p, "stretch", 0.0) > 0.0 else None
    V = {n: volume_mean(prof[i], zg) for i, n in enumerate(NAMES)}
    den = np.sqrt(V["rho_uz2"] * V["Tsa2"])
    z = heights(p)
    beta = 1.0 / (p.gamma - 1.0)
    return dict(
        Re=float(np.sqrt(p.Ra / p.Pr) * np.sqrt(V["u2"])),
        C=float(V["rho_uz_Tsa"] / den) if den > 0.0 else 0.0,
        Fn=V["Fn"], Fp=V["Fp"], Fb=V["Fb"], Fv=V["Fv"],
        rho_uz_Tsa=V["rho_uz_Tsa"], rho_uz2=V["rho_uz2"], Tsa2=V["Tsa2"], u2=V["u2"],
        Tsa_z=prof[0] - (1.0 - p.D * z),
        drho_z=prof[1] - (1.0 - p.D * z) ** beta,
        U_z=np.sqrt(prof[2]),
    )


def bl_thickness(tmean, D, rtol=0.1, z=None):
    """(lambda_b, lambda_t) of a profile <T>_A on nz node-counted rows
    (uniform, or on the node heights z); -1.0 where the slope never reaches
    -(1 + rtol) D."""
    t = np.asarray(tmean, dtype=np.float64)
    M = t.size - 1
    if z is None:
        hz = 1.0 / M
        s = (t[1:] - t[:-1]) / hz              # slope at midpoint z_(k+1/2)
        zm = (np.arange(M) + 0.5) * hz
    else:
        z = np.asarray(z, dtype=np.float64)
        s = (t[1:] - t[:-1]) / (z[1:] - z[:-1])
        zm = 0.5 * (z[1:] + z[:-1])
    thr = -(1.0 + rtol) * D

    def crossing(order):
        prev = None
        for k in order:
            if s[k] >= thr:
                if prev is None:
                    return zm[k]
                # linear interpolation of the slope between the midpoints
                f = (thr - s[prev]) / (s[k] - s[prev])
                return zm[prev] + f * (zm[k] - zm[prev])
            prev = k
        return None

    zb = crossing(range(M))
    zt = crossing(range(M - 1, -1, -1))
    return (zb if zb is not None else -1.0, (1.0 - zt) if zt is not None else -1.0)
