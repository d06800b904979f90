"""Seeded inputs shared by the oracle and the GPU tests.

Only random numbers and array plumbing live here; none of the method's
arithmetic.  A perturbed state is an oracle-made state with seeded,
relative noise added to the interior rows of every conserved field (plate
rows untouched), so the limiter, the viscous terms and the cross
derivatives all see non-trivial data.
"""
from __future__ import annotations

import numpy as np


def perturb(X: np.ndarray, seed: int, amp: float = 0.02, mom_scale: float = 1.0) -> np.ndarray:
    """X[f][k]... with rho and E scaled by (1 + amp*U) and momenta shifted
    by amp*mom_scale*rho*U, U uniform in [-1, 1), rows 1..nz-2 only."""
    rng = np.random.default_rng(seed)
    Y = np.array(X, dtype=np.float64, copy=True)
    nf = Y.shape[0]
    inner = (slice(None), slice(1, Y.shape[1] - 1))
    U = rng.uniform(-1.0, 1.0, size=Y[inner].shape)
    rho = Y[0][1:-1].copy()
    Y[0][1:-1] = rho * (1.0 + amp * U[0])
    for f in range(1, nf - 1):
        Y[f][1:-1] = Y[f][1:-1] + amp * mom_scale * rho * U[f]
    Y[nf - 1][1:-1] = Y[nf - 1][1:-1] * (1.0 + amp * U[nf - 1])
    return Y


def roll_x(X: np.ndarray, s: int) -> np.ndarray:
    """Periodic shift by s columns along x (the last axis)."""
    return np.roll(X, s, axis=-1)


def theta_field(nz: int, nx: int, seed: int, amp: float = 1e-3) -> np.ndarray:
    """(nz, nx) temperature perturbation, amp*U with U uniform in [-1, 1)."""
    rng = np.random.default_rng(seed)
    return amp * rng.uniform(-1.0, 1.0, size=(nz, nx))


def unit_directions(nz: int, nx: int, count: int, seed: int) -> np.ndarray:
    """(count, nz, nx) Gaussian directions on the interior rows (plate rows
    zero), each scaled to unit Euclidean norm."""
    rng = np.random.default_rng(seed)
    V = np.zeros((count, nz, nx))
    V[:, 1:nz - 1, :] = rng.standard_normal((count, nz - 2, nx))
    V /= np.sqrt(np.sum(V * V, axis=(1, 2)))[:, None, None]
    return V


def random_case(seed: int, ndim: int) -> dict:
    """One seeded random problem for the parameter fuzz: a small grid (down
    to one column in x and y and the minimum nz = 5), every parameter of
    Sec. 2 drawn over a wide range and every switch of the scheme drawn,
    plus the perturbation, the rows per wave and the z grid (uniform or
    tanh-stretched).  Keys: the parameter names, and 'amp', 'pseed',
    'tiling', 'steps'."""
    rng = np.random.default_rng(seed)
    if ndim == 2:
        nx, ny, nz = int(rng.integers(1, 131)), 1, int(rng.integers(5, 41))
    else:
        nx, ny, nz = int(rng.integers(1, 41)), int(rng.integers(1, 25)), int(rng.integers(5, 21))
    eps = float(rng.uniform(0.02, 0.3))
    kw = dict(
        ndim=ndim, nx=nx, ny=ny, nz=nz,
        aspect=float(rng.uniform(0.5, 8.0)),
        gamma=float(rng.uniform(1.1, 1.8)),
        Pr=float(10.0 ** rng.uniform(-0.5, 1.0)),
        Ra=float(10.0 ** rng.uniform(4.0, 9.0)),
        eps=eps,
        D=float(rng.uniform(0.05, 0.9 - eps)),
        cfl=float(rng.uniform(0.2, 0.9)),
        seed=int(rng.integers(0, 2**31)),
        noise_amp=float(rng.choice([0.0, 1e-3, 1e-2])),
        dt_mode=int(rng.integers(0, 2)),
        bulk_coef=float(rng.choice([-2.0 / 3.0, 2.0 / 3.0, 0.0])),
        limiter_form=int(rng.integers(0, 2)),
        sweep_order=int(rng.integers(0, 2)),
        tvd_on=int(rng.random() >= 0.2),
        gravity_scale=float(rng.choice([1.0, 1.0, 0.5, 0.0])),
        wall_order=int(rng.integers(1, 3)),
    )
    tiling = (0, 0) if rng.random() < 0.3 else (int(rng.integers(1, 9)), int(rng.integers(1, 9)))
    kw.update(amp=float(rng.uniform(0.0, 0.03)), pseed=int(rng.integers(0, 2**31)),
              tiling=tiling, steps=int(rng.integers(1, 5)))
    # the z grid: uniform for half of the draws, else the tanh grid with s
    # in [0.3, 2] (drawn last, so the draws above do not depend on it)
    u, sv = rng.random(), float(rng.uniform(0.3, 2.0))
    kw["stretch"] = 0.0 if u < 0.5 else sv
    return kw
