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
    # one GPU's share of it on eight: a 512-column slab plus the 6 halo
    # columns on each side that one exchange per step needs (z, x, z, x read
    # 1 + 2 + 1 + 2), run as a periodic box of that shape
    "2d_slab524x1024_ra1e10": dict(COMMON, ndim=2, nx=524, ny=1, nz=1024, Ra=1e10, seed=1,
                                   steps=1000, diag_every=100),
    # the same on the tanh-stretched z grid, s = 1.2 (the plate cells are
    # 2s/sinh(2s) = 0.44 of the uniform spacing)
    "2d_4096x1024_ra1e10_tanh1.2": dict(COMMON, ndim=2, nx=4096, ny=1, nz=1024, Ra=1e10,
                                        seed=1, steps=1000, diag_every=100, stretch=1.2),
    # 3D 1024 x 1024 x 256, Ra 1e9, 200 steps
    "3d_1024x1024x256_ra1e9": dict(COMMON, ndim=3, nx=1024, ny=1024, nz=256, Ra=1e9, seed=2,
                                   steps=200),
    # the same on the tanh-stretched z grid, s = 1.2
    "3d_1024x1024x256_ra1e9_tanh1.2": dict(COMMON, ndim=3, nx=1024, ny=1024, nz=256, Ra=1e9,
                                           seed=2, steps=200, stretch=1.2),
    # one GPU's share of the 1024 x 1024 x 256 box on eight: an x slab of 128
    # columns plus the 2 halo columns on each side that its sweeps read, run
    # as a periodic box of that shape (its cells are wider in x than the full
    # box's; a step's cost does not depend on the cell sizes)
    "3d_slab132x1024x256_ra1e9": dict(COMMON, ndim=3, nx=132, ny=1024, nz=256, Ra=1e9,
                                      seed=2, steps=200),
    # 2D 512 x 128, Ra 1e7, 500 steps, dt frozen: the adjoint case
    "2d_512x128_ra1e7": dict(COMMON, ndim=2, nx=512, ny=1, nz=128, Ra=1e7, seed=4, steps=500,
                             dt_mode=1),
    # its gradient: time-averaged Nu-bar over 500 steps, checkpoints every 50,
    # theta uniform +-1e-3 (seed 4) on interior T of the noise-free state
    "adjoint_512x128_ra1e7": dict(COMMON, ndim=2, nx=512, ny=1, nz=128, Ra=1e7, seed=4,
                                  steps=500, dt_mode=1, noise_amp=0.0, adjoint_every=50,
                                  theta_seed=4, theta_amp=1e-3),
}

PARAM_KEYS = ("ndim", "nx", "ny", "nz", "aspect", "gamma", "Pr", "Ra", "eps", "D", "cfl",
              "seed", "noise_amp", "dt_mode", "stretch", "dt_rule")


def params_dict(name: str, **overrides) -> dict:
    """Parameter fields of a workload (plus overrides), without step counts."""
    w = dict(WORKLOADS[name])
    w.update(overrides)
    return {k: w[k] for k in PARAM_KEYS if k in w}


# ---------------------------------------------------------------------------
# 64 independent 2D boxes advanced together

BATCH_SIZES = ((128, 32), (256, 64), (512, 128), (1024, 256))


def _splitmix64(seed: int, n: int) -> int:
    """n-th output of SplitMix64 from `seed` (Steele, Lea & Flood 2014);
    used here only to draw the batch layout."""
    m = (1 << 64) - 1
    z = (seed + n * 0x9E3779B97F4A7C15) & m
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
    return z ^ (z >> 31)


def _u01(seed: int, n: int) -> float:
    return (_splitmix64(seed, n) >> 11) * 2.0 ** -53


def batch_boxes(nbox: int = 64, seed: int = 3):
    """Parameter sets of the batch: box b takes size option floor(4 U) of
    BATCH_SIZES with U the draw 2b+1 of stream `seed`, Ra = 10^(5 + 4 U')
    with U' the draw 2b+2, noise seed 1000 + b.  Every box takes dt_rule 1
    (dt also within the explicit diffusion limit), so each box runs at the
    size and Ra drawn for it: where the acoustic limit is the smaller one,
    dt and the results are those of the acoustic rule alone."""
    out = []
    for b in range(nbox):
        k = min(3, int(4 * _u01(seed, 2 * b + 1)))
        Ra = 10.0 ** (5.0 + 4.0 * _u01(seed, 2 * b + 2))
        nx, nz = BATCH_SIZES[k]
        out.append(dict(COMMON, ndim=2, nx=nx, ny=1, nz=nz, Ra=Ra, seed=1000 + b, dt_rule=1))
    return out


WORKLOADS["batch_64_mixed_2d"] = dict(COMMON, ndim=2, boxes=64, layout_seed=3, steps=500)
