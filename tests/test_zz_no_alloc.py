"""mtvd_step_noalloc (the step with its scratch in a static device array, for
callers that cannot allocate) against mtvd_set_state + mtvd_step on the same
state: bit for bit, on two calls in a row (the second on a smaller grid, so
the scratch keeps the first call's contents when the second starts), and on
a 3D grid and a frozen-dt box after them."""
import numpy as np
import pytest

from helpers import gpu_or_skip

pytestmark = pytest.mark.gpu

CASES = [
    ("2D 256x64, 12 steps", dict(ndim=2, nx=256, ny=1, nz=64, Ra=1e6, seed=0), 12),
    ("2D 64x16, 5 steps (smaller, second call)", dict(ndim=2, nx=64, ny=1, nz=16, Ra=1e5,
                                                      seed=7), 5),
    ("3D 40x24x9, 3 steps", dict(ndim=3, nx=40, ny=24, nz=9, Ra=1e5, seed=3), 3),
    ("2D 48x13 frozen dt, 4 steps", dict(ndim=2, nx=48, ny=1, nz=13, Ra=2e5, seed=5,
                                         dt_mode=1), 4),
]


def _say(*a):
    print("[case]", *a, flush=True)


def _reference(mtvd, p, X0, nsteps):
    s = mtvd.Solver(p, device="cuda:0")
    s.set_state(X0, time=0.0, step=0)
    s.step(nsteps)
    X = s.get_state()
    s.close()
    return X


def test_noalloc_matches_the_context_step_bit_for_bit():
    torch = gpu_or_skip()
    import paper_2411_10372_amd as mtvd
    for name, kw, n in CASES:
        _say("noalloc", name)
        p = mtvd.Params(**kw)
        s = mtvd.Solver(p, device="cuda:0")
        s.init_state()
        s.step(2)                    # a state with flow in it
        X0 = s.get_state()
        s.close()
        ref = _reference(mtvd, p, X0, n)
        a = torch.tensor(X0.reshape(-1), dtype=torch.float64, device="cuda:0")
        b = torch.full_like(a, float("nan"))
        which = mtvd.step_noalloc(p, a, b, n)
        torch.cuda.synchronize()
        out = (a, b)[which].cpu().numpy().reshape(p.shape)
        assert which == (n * (6 if p.ndim == 3 else 4)) % 2
        assert np.array_equal(out, ref), (name, float(np.max(np.abs(out - ref))))


def test_noalloc_zero_steps_and_limits():
    torch = gpu_or_skip()
    import paper_2411_10372_amd as mtvd
    p = mtvd.Params(ndim=2, nx=64, ny=1, nz=16, Ra=1e5)
    a = torch.zeros(4 * 64 * 16, dtype=torch.float64, device="cuda:0")
    b = torch.zeros_like(a)
    s = mtvd.Solver(p, device="cuda:0")
    s.init_state()
    a.copy_(s.state_tensor().reshape(-1))
    torch.cuda.synchronize()
    s.close()
    keep = a.clone()
    assert mtvd.step_noalloc(p, a, b, 0) == 0
    torch.cuda.synchronize()
    assert torch.equal(a, keep)
    with pytest.raises(mtvd.MtvdError) as e:
        mtvd.step_noalloc(mtvd.Params(ndim=2, nx=64, ny=1, nz=16, Ra=1e5, stretch=1.0), a, b, 1)
    assert e.value.code == mtvd.MTVD_EINVAL
