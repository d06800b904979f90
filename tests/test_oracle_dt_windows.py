"""Pins of the oracle's time step rule and of its sub-box (window) entry
points.

Time step (reading A8 of the silent passage of Sec. 3.1: the acoustic CFL
rule dt = cfl * min over nodes and directions a of h_a / (|u_a| + c), with
c = sqrt(gamma p / rho) of Sec. 2).  The pins build states whose every node
has a known velocity and sound speed and compare with that closed form
written out here, so that each plausible slip fails one of them: dropping
the velocity term, using |u| instead of |u_a|, a signed u_a, a direction
left out of the minimum, the wrong spacing of a direction, the gravity term
missing from T, or on the tanh grid a face other than the narrowest one of
the node that decides.

Windows: the 3D full-size parity tests evaluate the oracle on sampled
column patches with ``init_box`` and ``sweep_box``.  Here both are pinned to
the whole-domain routines (``init``, pinned by closed forms and published
SplitMix64 outputs; ``sweep``, pinned by the amplification matrices,
conservation and symmetries): a window anywhere on the periodic domain,
also across the periodic seams, holds exactly the matching slice.
"""
import math

import numpy as np
import pytest

from oracle import Params
from inputs import perturb


def _tanh_heights(s, nz):
    """z_k = (1 + tanh(s (2k/M - 1)) / tanh s) / 2, the tanh grid (A30)."""
    M = nz - 1
    k = np.arange(nz)
    return 0.5 * (1.0 + np.tanh(s * (2.0 * k / M - 1.0)) / np.tanh(s))


def _state(p, rho, u, T, z):
    """A state with the given rho, velocity components u (one array per
    direction present, broadcastable to the grid) and T on node heights z,
    E = rho (c_v T + |u|^2 / 2 + g z) (Sec. 2)."""
    X = np.zeros(p.shape)
    cv = 1.0 / (p.gamma * p.eps * p.D)
    g = p.gravity_scale / p.eps
    zz = z.reshape((p.nz,) + (1,) * (len(p.shape) - 2))
    rho = np.broadcast_to(rho, p.shape[1:])
    uu = np.zeros(p.shape[1:])
    for f, ua in enumerate(u, start=1):
        ua = np.broadcast_to(ua, p.shape[1:])
        X[f] = rho * ua
        uu = uu + ua * ua
    X[0] = rho
    X[-1] = rho * (cv * T + 0.5 * uu + g * zz)
    return X


def _sound(p, T):
    # c = sqrt(gamma p / rho) with p = (gamma-1) rho T / (gamma eps D)
    return math.sqrt((p.gamma - 1.0) * T / (p.eps * p.D))


@pytest.mark.parametrize("nx,ux,uz,wins", [
    (8, -1.9, -0.45, "z"),     # coarse x: the z direction decides
    (64, -1.9, 0.45, "x"),     # fine x and a fast, negative u_x: x decides
    (64, 0.4, -4.5, "z"),      # fine x but u_z dominates
])
def test_dt_of_a_uniform_moving_state_2d(ora, nx, ux, uz, wins):
    p = Params(ndim=2, nx=nx, nz=9, aspect=4.0, noise_amp=0.0)
    T, rho = 0.8, 1.3
    z = np.arange(p.nz) / (p.nz - 1)
    X = _state(p, rho, (ux, uz), T, z)
    c = _sound(p, T)
    hx, hz = p.aspect / p.nx, 1.0 / (p.nz - 1)
    cand = {"x": hx / (abs(ux) + c), "z": hz / (abs(uz) + c)}
    want = p.cfl * min(cand.values())
    assert min(cand, key=cand.get) == wins
    got = ora.dt(p, X)
    assert abs(got - want) <= 1e-14 * want, (got, want)
    # the slips this pins (the deciding u_a is negative in every case): |u|
    # in place of |u_a|, no velocity term, signed u_a
    speed = math.hypot(ux, uz)
    for wrong in (p.cfl * min(hx / (speed + c), hz / (speed + c)),
                  p.cfl * min(hx, hz) / c,
                  p.cfl * min(hx / (ux + c), hz / (uz + c))):
        assert abs(wrong - want) > 1e-3 * want


@pytest.mark.parametrize("u,wins", [
    ((3.0, 0.1, 0.2), "x"),
    ((0.1, -3.5, 0.2), "y"),
    ((0.1, 0.3, -2.2), "z"),
])
def test_dt_of_a_uniform_moving_state_3d(ora, u, wins):
    # three different spacings: hx = 4/40, hy = 4/24, hz = 1/12
    p = Params(ndim=3, nx=40, ny=24, nz=13, aspect=4.0, noise_amp=0.0)
    T, rho = 0.65, 0.9
    z = np.arange(p.nz) / (p.nz - 1)
    X = _state(p, rho, u, T, z)
    c = _sound(p, T)
    h = (p.aspect / p.nx, p.aspect / p.ny, 1.0 / (p.nz - 1))
    cand = {a: h[i] / (abs(u[i]) + c) for i, a in enumerate("xyz")}
    assert min(cand, key=cand.get) == wins
    want = p.cfl * min(cand.values())
    got = ora.dt(p, X)
    assert abs(got - want) <= 1e-14 * want, (got, want)


@pytest.mark.parametrize("ndim", [2, 3])
def test_dt_at_a_single_fast_node_on_the_tanh_grid(ora, ndim):
    """At rest except one node; that node's velocity and its row's narrowest
    face decide.  Its row sits off the centre so that its two faces differ."""
    s, nz = 2.0, 33
    if ndim == 2:
        p = Params(ndim=2, nx=16, nz=nz, aspect=4.0, noise_amp=0.0, stretch=s)
    else:
        p = Params(ndim=3, nx=12, ny=10, nz=nz, aspect=4.0, noise_amp=0.0, stretch=s)
    z = _tanh_heights(s, nz)
    T, rho = 0.7, 1.1
    c = _sound(p, T)
    k = 11
    shape = p.shape[1:]
    uz = np.zeros(shape)
    ux = np.zeros(shape)
    at = (k, 3) if ndim == 2 else (k, 4, 3)
    uz[at] = -40.0 * c
    ux[at] = 2.0 * c     # the x direction of the fast node does not decide
    u = (ux, uz) if ndim == 2 else (ux, np.zeros(shape), uz)
    X = _state(p, rho, u, T, z)
    faces = np.diff(z)
    hk = min(faces[k - 1], faces[k])
    assert faces[k - 1] != faces[k]
    hx = p.aspect / p.nx
    want_node = hk / (40.0 * c + c)
    rest = min(hx, faces[0]) / c      # at rest: the plate face is the narrowest
    want = p.cfl * min(want_node, rest, hx / (2.0 * c + c))
    assert want == p.cfl * want_node
    got = ora.dt(p, X)
    assert abs(got - want) <= 1e-14 * want, (got, want)
    # the other face of that row, or the uniform spacing, would not do
    for wrong in (max(faces[k - 1], faces[k]), 1.0 / (nz - 1)):
        assert abs(p.cfl * wrong / (41.0 * c) - want) > 1e-3 * want


def test_dt_includes_gravity_in_the_temperature(ora):
    """T = (E/rho - |u|^2/2 - g z)/c_v: with gravity on and a state built
    with the g z term, c is uniform; a rule that forgets g z would see T
    grow with z and the sound speed change from row to row."""
    p = Params(ndim=2, nx=8, nz=9, aspect=1.0, noise_amp=0.0, gravity_scale=1.0)
    z = np.arange(p.nz) / (p.nz - 1)
    X = _state(p, 1.0, (0.0, 0.0), 0.5, z)
    c = _sound(p, 0.5)
    want = p.cfl * min(p.aspect / p.nx, 1.0 / (p.nz - 1)) / c
    assert abs(ora.dt(p, X) - want) <= 1e-14 * want
    # without the g z term T at the top row would read 0.5 + g / c_v, and
    # its faster sound would set dt
    cv = 1.0 / (p.gamma * p.eps * p.D)
    c_wrong = _sound(p, 0.5 + (p.gravity_scale / p.eps) / cv)
    wrong = p.cfl * min(p.aspect / p.nx, 1.0 / (p.nz - 1)) / c_wrong
    assert abs(wrong - want) > 0.1 * want


# ---------------------------------------------------------------------------
# windows


def _window(X, p, i0, j0, bx, by):
    """Columns i0..i0+bx-1 (and rows j0..j0+by-1 in y) of X, wrapped."""
    ii = np.arange(i0, i0 + bx) % p.nx
    if p.ndim == 2:
        return X[:, :, ii]
    jj = np.arange(j0, j0 + by) % p.ny
    return X[:, :, jj][:, :, :, ii]


@pytest.mark.parametrize("ndim,i0,j0,bx,by", [
    (2, 0, 0, 9, 1), (2, 27, 0, 9, 1), (2, -3, 0, 7, 1), (2, 5, 0, 40, 1),
    (3, 0, 0, 9, 7), (3, 28, 17, 9, 7), (3, -2, -4, 8, 9), (3, 31, 0, 6, 22),
])
def test_init_box_is_the_slice_of_init(ora, ndim, i0, j0, bx, by):
    """A window of the initial state, also one that wraps around x, y or
    both (or is wider than the domain), holds the same bits as the slice."""
    if ndim == 2:
        p = Params(ndim=2, nx=32, nz=11, seed=7, noise_amp=1e-2)
    else:
        p = Params(ndim=3, nx=32, ny=20, nz=9, seed=8, noise_amp=1e-2)
    X = ora.init(p)
    B = ora.init_box(p, i0, j0, bx, by)
    assert np.array_equal(B, _window(X, p, i0, j0, bx, by))


@pytest.mark.parametrize("ndim,axis", [(2, 0), (2, 2), (3, 0), (3, 1), (3, 2)])
@pytest.mark.parametrize("wrap", [False, True])
def test_sweep_box_inner_columns_are_those_of_sweep(ora, ndim, axis, wrap):
    """The box operator on a window with a two-column halo gives, on the
    inner columns, exactly what the whole-domain operator gives there."""
    if ndim == 2:
        p = Params(ndim=2, nx=30, nz=10, seed=3, Ra=1e5, noise_amp=1e-2)
        i0, j0, bx, by = ((-4, 0, 11, 1) if wrap else (6, 0, 12, 1))
    else:
        p = Params(ndim=3, nx=18, ny=14, nz=8, seed=5, Ra=1e5, noise_amp=1e-2)
        i0, j0, bx, by = ((15, -3, 9, 8) if wrap else (4, 3, 9, 8))
    X = perturb(ora.init(p), seed=11, amp=0.02)
    tau = 0.5 * ora.dt(p, X)
    full = ora.sweep(p, axis, tau, X)
    B = _window(X, p, i0, j0, bx, by)
    out = ora.sweep_box(p, axis, tau, B)
    want = _window(full, p, i0, j0, bx, by)
    if ndim == 2:
        assert np.array_equal(out[:, :, 2:bx - 2], want[:, :, 2:bx - 2])
    else:
        assert np.array_equal(out[:, :, 2:by - 2, 2:bx - 2], want[:, :, 2:by - 2, 2:bx - 2])


# ---------------------------------------------------------------------------
# the explicit diffusion limit (dt_rule = 1)


def _kappa(p):
    """The largest diffusivity times rho of Sec. 2: viscous mu* (2 + |lambda|)
    (the normal stress with the bulk term), thermal K* / c_v*."""
    mu = math.sqrt(p.Pr / p.Ra)
    K = 1.0 / (p.eps * p.D * math.sqrt(p.Ra * p.Pr))
    cv = 1.0 / (p.gamma * p.eps * p.D)
    return max(mu * (2.0 + abs(p.bulk_coef)), K / cv)


@pytest.mark.parametrize("ndim,Pr,lam,stretch", [
    (2, 1.0, -2.0 / 3.0, 0.0),   # viscous diffusivity the larger
    (2, 0.3, -2.0 / 3.0, 0.0),   # thermal the larger
    (2, 1.0, 0.0, 0.0),          # no bulk term: mu* 2
    (3, 1.0, 2.0 / 3.0, 0.0),
    (2, 1.0, -2.0 / 3.0, 1.5),   # tanh grid: the narrowest face of the row
    (3, 0.5, -2.0 / 3.0, 1.5),
])
def test_dt_rule_diffusion_limit_closed_form(ora, ndim, Pr, lam, stretch):
    """At rest, uniform T, density falling with height: at low Ra the
    diffusion limit cfl rho_min h^2 / kappa decides, at the least dense
    node (the top row) with the smallest spacing there."""
    if ndim == 2:
        p = Params(ndim=2, nx=40, nz=17, aspect=1.0, Ra=50.0, Pr=Pr, bulk_coef=lam,
                   noise_amp=0.0, stretch=stretch, dt_rule=1)
    else:
        p = Params(ndim=3, nx=24, ny=20, nz=13, aspect=1.0, Ra=50.0, Pr=Pr, bulk_coef=lam,
                   noise_amp=0.0, stretch=stretch, dt_rule=1)
    z = _tanh_heights(stretch, p.nz) if stretch else np.arange(p.nz) / (p.nz - 1)
    T = 0.6
    rho = (1.3 - 0.8 * z).reshape((p.nz,) + (1,) * (len(p.shape) - 2))
    zeros = [np.zeros(p.shape[1:]) for _ in range(ndim)]
    X = _state(p, rho, zeros, T, z)
    c = _sound(p, T)
    faces = np.diff(z)
    hz_top = faces[-1]
    hs = [p.aspect / p.nx] + ([p.aspect / p.ny] if ndim == 3 else [])
    h_top = min(hs + [hz_top])
    acoustic = min(hs + [faces.min()]) / c
    diffusive = (1.3 - 0.8) * h_top ** 2 / _kappa(p)
    assert diffusive < acoustic
    want = p.cfl * diffusive
    got = ora.dt(p, X)
    # on the tanh grid the top face is a difference of two heights near 1,
    # each from a tanh (numpy's here, libm's in the oracle) that may differ
    # by an ulp: about 1e-14 relative in the face, twice that in h^2
    tol = 1e-12 if stretch else 1e-14
    assert abs(got - want) <= tol * want, (got, want)
    # the acoustic rule alone ignores it
    q = Params(**{**p.__dict__, "dt_rule": 0})
    assert abs(ora.dt(q, X) - p.cfl * acoustic) <= tol * p.cfl * acoustic


def test_dt_rule_keeps_a_diffusion_dominated_box_stable(ora):
    """Ra = 100 on a 32 x 17 box: with the acoustic step alone the diffusion
    number of each operator is about 2, and the seeded +-1e-2 noise drives
    grid-scale motion over a hundred times that of the diffusion-limited
    run (the limiter and the nonlinearity keep it bounded, not small); with
    the diffusion limit the number is cfl/2 = 1/4 and the sub-critical box
    relaxes (kinetic energy falls after the initial adjustment)."""
    kw = dict(ndim=2, nx=32, nz=17, aspect=1.0, Ra=100.0, noise_amp=1e-2, seed=4)
    bad = Params(**kw, dt_rule=0)
    good = Params(**kw, dt_rule=1)
    X0 = ora.init(bad)
    Xb, Xg = X0, X0
    mb = mg = 0.0
    for i in range(6):
        Xb = ora.step(bad, Xb, 5)[0]
        Xg = ora.step(good, Xg, 5)[0]
        mb = max(mb, float(np.max(np.abs(Xb[1]))))
        mg = max(mg, float(np.max(np.abs(Xg[1]))))
        if i == 2:
            k15 = ora.diag(good, Xg)["kinetic"]
    assert np.all(np.isfinite(Xg))
    assert mb > 100.0 * mg, (mb, mg)
    assert ora.diag(good, Xg)["kinetic"] < 0.9 * k15
