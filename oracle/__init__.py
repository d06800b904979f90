"""Plain CPU FP64 oracle of the MacCormack-TVD compressible-convection step.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package; the product path
never does.  It shares no code with the GPU library: the C source here
(``mtvd_oracle.c``) is compiled with gcc, ``-O2 -ffp-contract=off``, no
fast-math, and loaded through ctypes.

Paper: Tiwari, Sharma & Verma, arXiv:2411.10372, Sec. 2 (nondimensional
equations, Nusselt numbers) and Sec. 3.1 (MacCormack-TVD scheme).

Parity status of each function (what pins it is in ``tests/test_oracle_*``):
  init, splitmix64  -- pinned (closed forms, published SplitMix64 outputs)
  init_box          -- pinned (equal bit for bit to the matching slice of
                       init, also for windows across the periodic seams)
  dt                -- pinned (closed form cfl min h_a/(|u_a| + c) on moving
                       uniform states in 2D and 3D, each direction deciding
                       in turn; one fast node on the tanh grid, whose row's
                       narrowest face decides; gravity inside T)
  sweep_box         -- pinned (its inner columns equal those of sweep, also
                       for windows across the periodic seams)
  sweep x/y/z, step -- pinned (linear acoustics/viscous/thermal amplification
                       in closed form, conservation, symmetries, hydrostatic
                       convergence, second-order self-convergence)
  TVD term          -- pinned for both limiter forms (closed forms at an
                       isolated spike, phi = 0, and inside the limiter's ramp,
                       0 < phi < 1, with the face Co from the larger |u|+c;
                       zero on linear data; conservative; no new extrema at
                       a contact for the Davis form).  Which form the paper
                       means is a reading (A4), not a pin.
  diag              -- pinned (conduction Nu = 1, closed-form sums)
  init_theta        -- pinned (equals init without noise at theta = 0; T of
                       interior nodes recovered as T0 + theta)
  time_avg_nu       -- pinned through step and diag, plus the conduction
                       value 1 and the one-step identity
  stretched z grid  -- pinned (tests/test_oracle_stretched.py: grid ends,
                       symmetry and the map's derivative; the s -> 0 limit;
                       dual-cell mass conservation; the uniform-pressure
                       conduction state steady with Nu = 1; second-order
                       decay of the hydrostatic error; the TVD term at a
                       spike in z; the z cross derivative of the x operator;
                       dt from the narrowest face).  The face spacing that
                       multiplies the TVD flux is a reading (the Harten-Yee
                       flux form); the spike pin fixes it.
  time_avg_nu_cs    -- complex-step derivative of time_avg_nu: pinned by its
                       real part (equal to time_avg_nu), by central
                       differences where the method is smooth (TVD off) and
                       by linearity in the direction
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field, fields

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mtvd_oracle.c")
_LIB = os.path.join(_HERE, "libmtvd_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP on, contraction off)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unused-function",
               "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True, cwd=_HERE)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("nz", ctypes.c_int32), ("aspect", ctypes.c_double),
        ("gamma", ctypes.c_double), ("Pr", ctypes.c_double), ("Ra", ctypes.c_double),
        ("eps", ctypes.c_double), ("D", ctypes.c_double), ("cfl", ctypes.c_double),
        ("seed", ctypes.c_uint64), ("noise_amp", ctypes.c_double),
        ("dt_mode", ctypes.c_int32), ("bulk_coef", ctypes.c_double),
        ("limiter_form", ctypes.c_int32), ("sweep_order", ctypes.c_int32),
        ("tvd_on", ctypes.c_int32), ("gravity_scale", ctypes.c_double),
        ("wall_order", ctypes.c_int32), ("pred_dir", ctypes.c_int32), ("diffusion_scale", ctypes.c_double),
        ("nthreads", ctypes.c_int32), ("stretch", ctypes.c_double),
        ("dt_rule", ctypes.c_int32),
    ]


class _Diag(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in (
        "mass", "kinetic", "total_energy", "nu_bottom", "nu_top", "nu_mean",
        "nu_bulk", "nu_conv", "nu_kin")] + [("tmean", ctypes.c_double * 6)]


@dataclass
class Params:
    """Problem parameters (defaults: the 256x64 2D case)."""
    ndim: int = 2
    nx: int = 256
    ny: int = 1
    nz: int = 64
    aspect: float = 4.0
    gamma: float = 1.4
    Pr: float = 1.0
    Ra: float = 1e6
    eps: float = 0.1
    D: float = 0.4
    cfl: float = 0.5
    seed: int = 0
    noise_amp: float = 1e-3
    dt_mode: int = 0
    bulk_coef: float = -2.0 / 3.0
    limiter_form: int = 0
    sweep_order: int = 0
    tvd_on: int = 1
    gravity_scale: float = 1.0
    wall_order: int = 2
    pred_dir: int = 0
    diffusion_scale: float = 1.0
    nthreads: int = 0
    stretch: float = 0.0
    dt_rule: int = 0

    def _c(self) -> _Params:
        return _Params(**{f.name: getattr(self, f.name) for f in fields(self)})

    @property
    def nf(self) -> int:
        return self.ndim + 2

    @property
    def shape(self):
        ny = self.ny if self.ndim == 3 else 1
        if self.ndim == 3:
            return (self.nf, self.nz, ny, self.nx)
        return (self.nf, self.nz, self.nx)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(_Params)
        dp = ctypes.POINTER(ctypes.c_double)
        L.ora_threads.argtypes = []
        L.ora_threads.restype = ctypes.c_int
        L.ora_state_len.argtypes = [P]
        L.ora_state_len.restype = ctypes.c_size_t
        L.ora_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.ora_splitmix64.restype = ctypes.c_uint64
        L.ora_init.argtypes = [P, dp]
        L.ora_heights.argtypes = [P, dp]
        L.ora_init_box.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int, dp]
        L.ora_dt.argtypes = [P, dp]
        L.ora_dt.restype = ctypes.c_double
        L.ora_sweep.argtypes = [P, ctypes.c_int, ctypes.c_double, dp, dp]
        L.ora_sweep_box.argtypes = [P, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                    ctypes.c_int, dp, dp]
        L.ora_step.argtypes = [P, dp, ctypes.c_int, dp, dp]
        L.ora_diag.argtypes = [P, dp, ctypes.POINTER(_Diag)]
        L.ora_time_avg_nu_cs.argtypes = [P, dp, dp, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_int, ctypes.c_double, dp, dp]
        for fn in ("ora_init", "ora_init_box", "ora_sweep", "ora_sweep_box",
                   "ora_step", "ora_diag", "ora_time_avg_nu_cs"):
            getattr(L, fn).restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ok(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} rejected its arguments (rc={rc})")


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().ora_threads())


def splitmix64(seed: int, n: int) -> int:
    return int(lib().ora_splitmix64(seed, n))


def heights(p: Params) -> np.ndarray:
    """The nz node heights z_k (uniform, or the tanh grid when stretch > 0)."""
    z = np.empty(p.nz, dtype=np.float64)
    pc = p._c()
    _ok(lib().ora_heights(ctypes.byref(pc), _ptr(z)), "heights")
    return z


def init(p: Params) -> np.ndarray:
    X = np.empty(p.shape, dtype=np.float64)
    pc = p._c()
    _ok(lib().ora_init(ctypes.byref(pc), _ptr(X)), "init")
    return X


def init_box(p: Params, i0: int, j0: int, bx: int, by: int = 1) -> np.ndarray:
    if p.ndim == 2:
        by = 1
        B = np.empty((p.nf, p.nz, bx), dtype=np.float64)
    else:
        B = np.empty((p.nf, p.nz, by, bx), dtype=np.float64)
    pc = p._c()
    _ok(lib().ora_init_box(ctypes.byref(pc), i0, j0, bx, by, _ptr(B)), "init_box")
    return B


def dt(p: Params, X: np.ndarray) -> float:
    X = np.ascontiguousarray(X, dtype=np.float64)
    pc = p._c()
    return float(lib().ora_dt(ctypes.byref(pc), _ptr(X)))


def sweep(p: Params, axis: int, tau: float, X: np.ndarray) -> np.ndarray:
    """One directional operator L_axis(tau); axis 0 = x, 1 = y, 2 = z."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    Y = np.empty_like(X)
    pc = p._c()
    _ok(lib().ora_sweep(ctypes.byref(pc), axis, tau, _ptr(X), _ptr(Y)), "sweep")
    return Y


def sweep_box(p: Params, axis: int, tau: float, B: np.ndarray) -> np.ndarray:
    """L_axis(tau) on a box with a two-column halo in x (and y in 3D).
    Only the non-halo columns of the result are meaningful."""
    B = np.ascontiguousarray(B, dtype=np.float64)
    out = np.zeros_like(B)
    bx = B.shape[-1]
    by = B.shape[-2] if p.ndim == 3 else 1
    pc = p._c()
    _ok(lib().ora_sweep_box(ctypes.byref(pc), axis, tau, bx, by, _ptr(B), _ptr(out)),
        "sweep_box")
    return out


def step(p: Params, X: np.ndarray, nsteps: int, time: float = 0.0,
         dt_frozen: float = 0.0):
    """Advance X by nsteps full steps.  Returns (X, time, last_dt)."""
    X = np.array(X, dtype=np.float64, order="C", copy=True)
    t = ctypes.c_double(time)
    d = ctypes.c_double(dt_frozen)
    pc = p._c()
    _ok(lib().ora_step(ctypes.byref(pc), _ptr(X), nsteps, ctypes.byref(t),
                       ctypes.byref(d)), "step")
    return X, t.value, d.value


def diag(p: Params, X: np.ndarray) -> dict:
    X = np.ascontiguousarray(X, dtype=np.float64)
    d = _Diag()
    pc = p._c()
    _ok(lib().ora_diag(ctypes.byref(pc), _ptr(X), ctypes.byref(d)), "diag")
    out = {n: getattr(d, n) for n, _ in _Diag._fields_ if n != "tmean"}
    out["tmean"] = list(d.tmean)
    return out


def init_theta(p: Params, theta: np.ndarray) -> np.ndarray:
    """Sec. 2 initial state (conduction T0 = 1 - (eps+D) z, hydrostatic rho,
    u = 0) with T = T0 + theta on interior rows instead of random noise.
    theta: (nz, nx) in 2D; plate rows are ignored."""
    if p.ndim != 2:
        raise ValueError("2D only")
    q = Params(**{**p.__dict__, "noise_amp": 0.0})
    X = init(q)
    M = p.nz - 1
    z = heights(p)[:, None]     # k/M on the uniform grid
    T0 = 1.0 - (p.eps + p.D) * z
    cv = 1.0 / (p.gamma * p.eps * p.D)
    g = p.gravity_scale / p.eps
    rho = X[0]
    T = T0 + np.asarray(theta, dtype=np.float64).reshape(p.nz, p.nx)
    X[3, 1:M] = rho[1:M] * (cv * T[1:M] + g * z[1:M])
    return X


def time_avg_nu(p: Params, X0: np.ndarray, nsteps: int, dt: float) -> float:
    """(1/N) sum_{n=1..N} Nu_mean(X_n) over N steps of Sec. 3.1 with the
    fixed step dt (Nu_mean of Sec. 2: plate Nusselt numbers averaged)."""
    q = Params(**{**p.__dict__, "dt_mode": 1})
    X = np.array(X0, dtype=np.float64, copy=True)
    acc = 0.0
    for _ in range(nsteps):
        X, _, _ = step(q, X, 1, dt_frozen=dt)
        acc += diag(q, X)["nu_mean"]
    return acc / nsteps


def mu_K(p: Params):
    """The viscosity and conductivity coefficients of Sec. 2 (mu* = sqrt(Pr/Ra),
    K* = 1/(eps D sqrt(Ra Pr))) and their derivatives with respect to Ra."""
    mu = np.sqrt(p.Pr / p.Ra)
    K = 1.0 / (p.eps * p.D * np.sqrt(p.Ra * p.Pr))
    return mu, K, -mu / (2.0 * p.Ra), -K / (2.0 * p.Ra)


def time_avg_nu_cs(p: Params, X0: np.ndarray, V, nsteps: int, dt: float,
                   dRa: float = 0.0, h: float = 1e-20, dmu: float = 0.0, dK: float = 0.0):
    """Complex-step mode of :func:`time_avg_nu`: (J, dJ) with dJ the
    derivative of J along the state direction V (None: no state direction),
    plus dmu times d/dmu* and dK times d/dK*, plus dRa times d/dRa (through
    mu* and K*), on the branches the run takes."""
    if dRa:
        _, _, dmu_dRa, dK_dRa = mu_K(p)
        dmu = dmu + dRa * dmu_dRa
        dK = dK + dRa * dK_dRa
    X0 = np.ascontiguousarray(X0, dtype=np.float64)
    Vp = None
    if V is not None:
        V = np.ascontiguousarray(V, dtype=np.float64)
        if V.shape != X0.shape:
            raise ValueError("V must have the state's shape")
        Vp = _ptr(V)
    J, dJ = ctypes.c_double(), ctypes.c_double()
    pc = p._c()
    _ok(lib().ora_time_avg_nu_cs(ctypes.byref(pc), _ptr(X0), Vp, h, dmu, dK, nsteps, dt,
                                 ctypes.byref(J), ctypes.byref(dJ)), "time_avg_nu_cs")
    return J.value, dJ.value


def theta_direction(p: Params, X0: np.ndarray, v: np.ndarray) -> np.ndarray:
    """The state direction of a temperature direction v at X0: the derivative
    of init_theta, E = rho (cv T + g z) on interior rows, is rho cv v."""
    V = np.zeros_like(X0)
    M = p.nz - 1
    cv = 1.0 / (p.gamma * p.eps * p.D)
    V[3, 1:M] = X0[0, 1:M] * cv * np.asarray(v, dtype=np.float64).reshape(p.nz, p.nx)[1:M]
    return V
