"""The long-run driver (paper_2411_10372_amd/longrun.py) on small boxes.

Below the onset of convection (Ra = 500, under the critical value of a box
heated from below) the seeded perturbation decays to a steady state: the
conduction state plus the steady residual velocity of the discrete
hydrostatic balance, a discretisation error.  So the time averages do not
fluctuate, Nu-bar and the bulk Nu are 1 up to that error, the pressure
gradient balances gravity (F_p = F_b), and the residual Re falls at about
second order when the grid is refined (9 -> 17 rows: at least 3x).

Paper: arXiv:2411.10372, Sec. 2 (Nu, Re), Sec. 6.1 (momentum balance).
"""
import math

import pytest

from helpers import gpu_or_skip


@pytest.mark.gpu
def test_below_onset_the_run_settles_to_conduction():
    gpu_or_skip()
    import paper_2411_10372_amd as mtvd
    from paper_2411_10372_amd.longrun import time_averages
    res = []
    for nx, nz in ((32, 9), (64, 17)):
        p = mtvd.Params(ndim=2, nx=nx, nz=nz, Ra=500.0, Pr=0.7, seed=3, noise_amp=1e-3)
        print(f"[case] longrun {nx}x{nz} Ra 500", flush=True)
        out = time_averages(p, t0=20.0, t1=30.0, sample_steps=20)
        print(out["nu_mean"], out["nu_bulk"], out["Re"], out["Fp"], out["Fb"], flush=True)
        assert out["samples"] >= 5
        for k in ("nu_mean", "nu_bulk", "Re"):
            assert out[k][1] < 1e-9 * max(1.0, out[k][0]), (k, out[k])     # steady
        assert abs(out["nu_mean"][0] - 1.0) < 2e-2
        assert abs(out["nu_bulk"][0] - 1.0) < 3e-2
        assert abs(out["Fp"][0] - out["Fb"][0]) < 1e-3 * out["Fb"][0]
        for k in ("lambda_b", "lambda_t"):
            assert math.isfinite(out[k])
        res.append(out)
    assert res[0]["Re"][0] < 0.2
    assert res[0]["Re"][0] / res[1]["Re"][0] > 3.0, (res[0]["Re"], res[1]["Re"])


@pytest.mark.gpu
def test_below_onset_on_the_stretched_grid():
    # the same settling on the tanh grid (the analysis on the node heights):
    # steady, Nu-bar and bulk Nu near 1, F_p = F_b, and the residual Re of
    # the same size and decay as above (s = 0.3: at
    # Ra = 500 a stronger stretch narrows the plate cells past the explicit
    # diffusion limit of these grids)
    gpu_or_skip()
    import paper_2411_10372_amd as mtvd
    from paper_2411_10372_amd.longrun import time_averages
    res = []
    for nx, nz in ((32, 9), (64, 17)):
        p = mtvd.Params(ndim=2, nx=nx, nz=nz, Ra=500.0, Pr=0.7, seed=3, noise_amp=1e-3,
                        stretch=0.3)
        print(f"[case] longrun stretched {nx}x{nz} Ra 500", flush=True)
        out = time_averages(p, t0=20.0, t1=30.0, sample_steps=20)
        print(out["nu_mean"], out["nu_bulk"], out["Re"], flush=True)
        assert out["samples"] >= 5 and "C" in out
        # F_p - F_b is the truncation error of the discrete hydrostatic
        # balance: 2e-3 of F_b on 9 rows here, falling at second order
        assert abs(out["Fp"][0] - out["Fb"][0]) < 5e-3 * out["Fb"][0]
        for k in ("nu_mean", "nu_bulk", "Re"):
            assert out[k][1] < 1e-9 * max(1.0, out[k][0]), (k, out[k])
        assert abs(out["nu_mean"][0] - 1.0) < 2e-2
        assert abs(out["nu_bulk"][0] - 1.0) < 3e-2
        res.append(out)
    assert res[0]["Re"][0] < 0.2
    assert res[0]["Re"][0] / res[1]["Re"][0] > 3.0, (res[0]["Re"], res[1]["Re"])
    fb = [abs(r["Fp"][0] - r["Fb"][0]) for r in res]
    assert fb[0] / fb[1] > 3.0, fb
