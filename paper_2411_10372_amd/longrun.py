"""Long runs to a statistically steady state and their time averages.

The quantities are those the paper reports for its runs (Sec. 2: Nu-bar,
the bulk Nu with Nu_conv and Nu_K, Re; Secs. 4-6: the profiles T_sa(z),
rho - rho_A(z), U(z), the boundary-layer thicknesses, the z-momentum
balance and the correlation C).  Every number comes from the library's
diagnostics and analysis entry points; this module only steps the solver,
samples snapshots and averages them over time.  The mean of each scalar
comes with the standard error of five consecutive block means.

Command line (one JSON line on stdout, progress on stderr):

    python -m paper_2411_10372_amd.longrun --ndim 3 --nx 128 --nz 65 \\
        --aspect 2 --gamma 5/3 --D 0.49 --Ra 1e6 --t0 50 --t1 150

Paper: Tiwari, Sharma & Verma, arXiv:2411.10372, Sec. 2 (Nu, Re), Sec. 3.3
(validation runs, Tables 1 and 2), Secs. 4-5 (profiles, boundary layers),
Sec. 6 (momentum balance, C(Ra)).
"""
from __future__ import annotations

import argparse
import json
import sys
import time
from fractions import Fraction

import numpy as np

from . import Params, Solver, analysis, bl_thickness, grid_heights

SCALARS = ("nu_mean", "nu_bottom", "nu_top", "nu_bulk", "nu_conv", "nu_kin", "Re", "C",
           "Fn", "Fp", "Fb", "Fv")


def _mean_err(x: np.ndarray):
    blocks = np.array_split(np.asarray(x, dtype=np.float64), 5)
    m = np.array([b.mean() for b in blocks if b.size])
    err = float(m.std(ddof=1) / np.sqrt(m.size)) if m.size > 1 else float("nan")
    return float(np.mean(x)), err


def time_averages(p: Params, t0: float, t1: float, sample_steps: int = 100,
                  wall_limit: float | None = None, rtol: float = 0.1, progress=None) -> dict:
    """Run from the initial state until the simulated time reaches t1 (or
    the wall-clock limit), sampling every `sample_steps` steps; average the
    samples with time >= t0."""
    z = grid_heights(p) if p.stretch > 0.0 else None
    s = Solver(p)
    try:
        s.init_state()
        start = time.time()
        last = start
        samples, prof_sum, n_prof = [], None, 0
        d = None
        while True:
            s.step(sample_steps)
            d = s.diagnostics()
            row = {k: d[k] for k in SCALARS if k in d}
            prof = s.profiles()
            a = analysis(p, prof)
            row.update({k: a[k] for k in ("Re", "C", "Fn", "Fp", "Fb", "Fv")})
            if d["time"] >= t0:
                prof_sum = prof.copy() if prof_sum is None else prof_sum + prof
                n_prof += 1
            row["time"] = d["time"]
            samples.append(row)
            now = time.time()
            if progress and now - last > 20.0:
                progress({"step": d["step"], "time": round(d["time"], 3), "dt": d["dt"],
                          "nu_mean": round(d["nu_mean"], 4), "Re": round(a["Re"], 3),
                          "wall_s": round(now - start, 1)})
                last = now
            if d["time"] >= t1 or (wall_limit is not None and now - start > wall_limit):
                break
        sel = [r for r in samples if r["time"] >= t0]
        out = {"steps": int(d["step"]), "t_end": float(d["time"]), "samples": len(sel),
               "wall_s": round(time.time() - start, 1)}
        if len(sel) >= 5:
            for k in SCALARS:
                if k in sel[0]:
                    out[k] = _mean_err(np.array([r[k] for r in sel]))
        if len(sel) >= 5 and n_prof:
            mean_prof = prof_sum / n_prof
            a = analysis(p, mean_prof)
            out["lambda_b"], out["lambda_t"] = bl_thickness(mean_prof[0], p.D, rtol, z)
            out["profiles"] = {"Tsa_z": a["Tsa_z"].tolist(), "drho_z": a["drho_z"].tolist(),
                               "U_z": a["U_z"].tolist()}
        return out
    finally:
        s.close()


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--ndim", type=int, default=3)
    ap.add_argument("--nx", type=int, required=True)
    ap.add_argument("--ny", type=int, default=0, help="default: nx")
    ap.add_argument("--nz", type=int, required=True)
    ap.add_argument("--aspect", type=float, default=4.0)
    ap.add_argument("--gamma", type=str, default="1.4", help="a number or a fraction, e.g. 5/3")
    ap.add_argument("--Pr", type=float, default=0.7)
    ap.add_argument("--Ra", type=float, required=True)
    ap.add_argument("--eps", type=float, default=0.1)
    ap.add_argument("--D", type=float, default=0.5)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--noise", type=float, default=1e-3)
    ap.add_argument("--limiter-form", type=int, default=0)
    ap.add_argument("--wall-order", type=int, default=2,
                    help="z-derivatives in the plate fluxes: 2 one-sided second order, 1 first")
    ap.add_argument("--stretch", type=float, default=0.0,
                    help="tanh z-grid parameter s (0: uniform; 3D: nz <= 2048)")
    ap.add_argument("--t0", type=float, required=True, help="start of the averaging window")
    ap.add_argument("--t1", type=float, required=True, help="simulated end time")
    ap.add_argument("--sample-steps", type=int, default=100)
    ap.add_argument("--wall", type=float, default=None, help="wall-clock limit in seconds")
    ap.add_argument("--rtol", type=float, default=0.1, help="boundary-layer slope tolerance")
    ap.add_argument("--profiles", action="store_true", help="include the averaged profiles")
    a = ap.parse_args(argv)
    p = Params(ndim=a.ndim, nx=a.nx, ny=(a.ny or a.nx) if a.ndim == 3 else 1, nz=a.nz,
               aspect=a.aspect, gamma=float(Fraction(a.gamma)), Pr=a.Pr, Ra=a.Ra, eps=a.eps,
               D=a.D, seed=a.seed, noise_amp=a.noise, limiter_form=a.limiter_form,
               stretch=a.stretch, wall_order=a.wall_order)
    out = time_averages(p, a.t0, a.t1, a.sample_steps, a.wall, a.rtol,
                        progress=lambda d: print(json.dumps(d), file=sys.stderr, flush=True))
    if not a.profiles:
        out.pop("profiles", None)
    out["params"] = {k: getattr(p, k) for k in ("ndim", "nx", "ny", "nz", "aspect", "gamma", "Pr",
                                                 "Ra", "eps", "D", "seed", "noise_amp",
                                                 "limiter_form", "stretch", "wall_order")}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
