"""Named workloads: the parameter sets the tests and the benchmark run.

Plain data (grid, physical parameters, seed, step counts); no arithmetic of
the method.  eps = 0.1 and D = 0.4 give plate temperatures 1 and 0.5
(bottom/top ratio 2) with the paper's eps (Sec. 3.4 fixes eps = 0.1).
"""
from __future__ import annotations

COMMON = dict(aspect=4.0, gamma=1.4, Pr=1.0, eps=0.1, D=0.4, cfl=0.5, noise_amp=1e-3)

WORKLOADS = {
    # 2D 256 x 64, Ra 1e6, 200 steps: the small parity case
    "2d_256x64_ra1e6": dict(COMMON, ndim=2, nx=256, ny=1, nz=64, Ra=1e6, seed=0, steps=200),
    # 2D 4096 x 1024, Ra 1e10, 1000 steps, diagnostics every 100: the benchmark case
    "2d_4096x1024_ra1e10": dict(COMMON, ndim=2, nx=4096, ny=1, nz=1024, Ra=1e10, seed=1,
                                steps=1000, diag_every=100),
    # 3D 1024 x 1024 x 256, Ra 1e9, 200 steps
    "3d_1024x1024x256_ra1e9": dict(COMMON, ndim=3, nx=1024, ny=1024, nz=256, Ra=1e9, seed=2,
                                   steps=200),
    # 2D 512 x 128, Ra 1e7, 500 steps, dt frozen: the adjoint case
    "2d_512x128_ra1e7": dict(COMMON, ndim=2, nx=512, ny=1, nz=128, Ra=1e7, seed=4, steps=500,
                             dt_mode=1),
}

PARAM_KEYS = ("ndim", "nx", "ny", "nz", "aspect", "gamma", "Pr", "Ra", "eps", "D", "cfl",
              "seed", "noise_amp", "dt_mode")


def params_dict(name: str, **overrides) -> dict:
    """Parameter fields of a workload (plus overrides), without step counts."""
    w = dict(WORKLOADS[name])
    w.update(overrides)
    return {k: w[k] for k in PARAM_KEYS if k in w}
