"""Write tests/golden/adjoint_c4.txt: directional derivatives of the
time-averaged mean Nusselt number of the adjoint workload (512 x 128, Ra 1e7,
gamma 1.4, aspect 4, 500 steps with the dt of X_0 frozen; theta = seeded
uniform +-1e-3, seed 4; 16 unit Gaussian directions, seed 5; d/dmu*, d/dK*
and d/dRa),
from the oracle's complex-step mode.  Calls only oracle/ and the seeded
input generators.  Run from the repository root:

    python tests/golden/make_adjoint_c4.py
"""
import hashlib
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, os.path.dirname(HERE))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from inputs import theta_field, unit_directions  # noqa: E402

KW = dict(nx=512, nz=128, Ra=1e7, gamma=1.4, aspect=4.0, noise_amp=0.0, dt_mode=1)
NSTEPS, THETA_SEED, THETA_AMP, DIR_SEED, NDIR = 500, 4, 1e-3, 5, 16


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.float64).tobytes()).hexdigest()[:16]


def main(out=os.path.join(HERE, "adjoint_c4.txt")):
    p = oracle.Params(**KW)
    th = theta_field(p.nz, p.nx, seed=THETA_SEED, amp=THETA_AMP)
    X0 = oracle.init_theta(p, th)
    dt = oracle.dt(p, X0)
    V = unit_directions(p.nz, p.nx, NDIR, seed=DIR_SEED)
    J = oracle.time_avg_nu(p, X0, NSTEPS, dt)
    lines = ["# complex-step directional derivatives of J = (1/N) sum_n Nu_mean(X_n)",
             f"# params {KW} nsteps {NSTEPS}",
             f"# theta seed {THETA_SEED} amp {THETA_AMP} sha {digest(th)}; "
             f"directions seed {DIR_SEED} count {NDIR} sha {digest(V)}",
             f"dt {dt!r}", f"J {J!r}"]
    t0 = time.time()
    for i, v in enumerate(V):
        _, d = oracle.time_avg_nu_cs(p, X0, oracle.theta_direction(p, X0, v), NSTEPS, dt)
        lines.append(f"dir {i} {d!r}")
        print(f"direction {i}: {d!r} ({time.time() - t0:.0f} s)", flush=True)
    # the diffusion coefficients mu* and K*, each alone, and Ra through both
    _, dmu = oracle.time_avg_nu_cs(p, X0, None, NSTEPS, dt, dmu=1.0)
    lines.append(f"mu {dmu!r}")
    _, dK = oracle.time_avg_nu_cs(p, X0, None, NSTEPS, dt, dK=1.0)
    lines.append(f"K {dK!r}")
    _, dra = oracle.time_avg_nu_cs(p, X0, None, NSTEPS, dt, dRa=1.0)
    lines.append(f"ra {dra!r}")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("wrote", out)


if __name__ == "__main__":
    main()
