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
