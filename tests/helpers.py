"""Helpers shared by the GPU tests: building both sides from one parameter
set and the parity error measure."""
from __future__ import annotations

import math
import os

import numpy as np
import pytest

import oracle
import paper_2411_10372_amd as mtvd

GPU_KEYS = [f.name for f in mtvd.Params.__dataclass_fields__.values()]


def both(**kw):
    """(oracle Params, GPU Params) from one set of keyword values."""
    po = oracle.Params(**kw)
    pg = mtvd.Params(**{k: v for k, v in kw.items() if k in GPU_KEYS})
    return po, pg


def parity_error(Xg: np.ndarray, Xo: np.ndarray, p) -> float:
    """max over fields of ||X_gpu - X_ora||_inf / s_f with s_f = ||X_ora,f||_inf
    for rho and E and max(||X_ora,f||_inf, rho_b c_b) for momenta (momenta
    start at exactly zero); rho_b = 1, c_b = sqrt((gamma-1)/(eps D))."""
    cb = math.sqrt((p.gamma - 1.0) / (p.eps * p.D))
    e = 0.0
    nf = Xo.shape[0]
    for f in range(nf):
        s = float(np.max(np.abs(Xo[f])))
        if 0 < f < nf - 1:
            s = max(s, cb)
        d = float(np.max(np.abs(Xg[f] - Xo[f])))
        e = max(e, d / s)
    return e


def gpu_or_skip():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(mtvd.LIB_PATH):
        pytest.fail("libmtvd.so not built: the GPU tests need the HIP library")
    return torch
