"""MI355X (gfx950) MacCormack-TVD step of compressible convection.

A thin ctypes binding of ``libmtvd.so`` (C ABI in ``include/mtvd.h``): every
step of the method runs in the library's HIP kernels; this module only
marshals arguments.  PyTorch supplies device memory (the two state buffers
and the workspace) and the stream.  There is no CPU fallback: importing works
without a GPU, but creating a :class:`Solver` needs the built library and a
GPU, and raises otherwise.

Paper: Tiwari, Sharma & Verma, arXiv:2411.10372 (Sec. 2 equations and
Nusselt numbers, Sec. 3.1 MacCormack-TVD scheme).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, fields

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmtvd.so")

MTVD_OK = 0
MTVD_EINVAL = -1
MTVD_ESIZE = -2
MTVD_ESTABILITY = -3
MTVD_ESTATE = -4
MTVD_ENONFINITE = -5
MTVD_EHIP = -6


class MtvdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mtvd error {code}: {msg}")
        self.code = code


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
        ("wall_order", ctypes.c_int32), ("stretch", ctypes.c_double),
        ("dt_rule", ctypes.c_int32),
    ]


class _Diag(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("time", ctypes.c_double), ("dt", ctypes.c_double)] + \
        [(n, ctypes.c_double) for n in ("mass", "kinetic", "total_energy", "nu_bottom",
                                        "nu_top", "nu_mean", "nu_bulk", "nu_conv", "nu_kin")] + \
        [("tmean", ctypes.c_double * 6), ("flags", ctypes.c_int32)]


@dataclass
class Params:
    """Problem parameters; field names and meaning as in ``mtvd_params``."""
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
    stretch: float = 0.0
    dt_rule: int = 0

    def _c(self) -> _Params:
        return _Params(**{f.name: getattr(self, f.name) for f in fields(self)})

    @property
    def nf(self) -> int:
        return self.ndim + 2

    @property
    def shape(self):
        if self.ndim == 3:
            return (self.nf, self.nz, self.ny, self.nx)
        return (self.nf, self.nz, self.nx)

    @property
    def nodes(self) -> int:
        return self.nx * (self.ny if self.ndim == 3 else 1) * self.nz


class _Analysis(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in (
        "Re", "C", "Fn", "Fp", "Fb", "Fv", "u2", "rho_uz_Tsa", "rho_uz2", "Tsa2")]


# rows of Solver.profiles(), in order (the library's MTVD_NUM_PROFILES rows)
PROFILE_NAMES = ("T", "rho", "u2", "rho_uz_Tsa", "rho_uz2", "Tsa2", "Fn", "Fp", "Fb", "Fv")

_lib = None


def lib() -> ctypes.CDLL:
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise MtvdError(MTVD_EHIP, f"{LIB_PATH} is missing: run __graft_entry__.build() "
                                       "(or python paper_2411_10372_amd/build.py)")
        # torch first: its HIP runtime and the one the library was linked
        # against share the soname libamdhip64.so.7, and the process keeps
        # whichever is loaded first for both.  Loading the library first
        # would hand torch a runtime it was not built with (the GPU calls of
        # both then fail).
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER(_Params)
        vp = ctypes.c_void_p
        dp = ctypes.POINTER(ctypes.c_double)
        L.mtvd_default_params.argtypes = [P]
        L.mtvd_default_params.restype = None
        L.mtvd_state_bytes.argtypes = [P, ctypes.POINTER(ctypes.c_size_t),
                                       ctypes.POINTER(ctypes.c_size_t)]
        L.mtvd_grid_heights.argtypes = [P, dp, ctypes.c_size_t]
        L.mtvd_create.argtypes = [P, vp, ctypes.POINTER(vp)]
        L.mtvd_bind.argtypes = [vp, vp, vp, vp]
        L.mtvd_init_state.argtypes = [vp]
        L.mtvd_step.argtypes = [vp, ctypes.c_int32]
        L.mtvd_sweep.argtypes = [vp, ctypes.c_int32]
        L.mtvd_diagnostics.argtypes = [vp, ctypes.POINTER(_Diag)]
        L.mtvd_get_state.argtypes = [vp, dp, ctypes.c_size_t]
        L.mtvd_set_state.argtypes = [vp, dp, ctypes.c_size_t, ctypes.c_double, ctypes.c_int64]
        L.mtvd_current.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
        L.mtvd_sync.argtypes = [vp]
        L.mtvd_set_tiling.argtypes = [vp, ctypes.c_int32, ctypes.c_int32]
        L.mtvd_set_timing.argtypes = [vp, ctypes.c_int32]
        L.mtvd_kernel_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_int64)]
        L.mtvd_destroy.argtypes = [vp]
        L.mtvd_strerror.argtypes = [ctypes.c_int]
        L.mtvd_strerror.restype = ctypes.c_char_p
        L.mtvd_last_error.argtypes = [vp]
        L.mtvd_last_error.restype = ctypes.c_char_p
        PA = ctypes.POINTER(_Params)
        L.mtvd_batch_bytes.argtypes = [PA, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t),
                                       ctypes.POINTER(ctypes.c_size_t)]
        L.mtvd_batch_create.argtypes = [PA, ctypes.c_int32, vp, ctypes.POINTER(vp)]
        L.mtvd_batch_bind.argtypes = [vp, vp, vp, vp]
        L.mtvd_batch_offset.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]
        L.mtvd_batch_init_state.argtypes = [vp]
        L.mtvd_batch_step.argtypes = [vp, ctypes.c_int32]
        L.mtvd_batch_diagnostics.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(_Diag)]
        L.mtvd_batch_get_state.argtypes = [vp, ctypes.c_int32, dp, ctypes.c_size_t]
        L.mtvd_batch_set_state.argtypes = [vp, ctypes.c_int32, dp, ctypes.c_size_t,
                                           ctypes.c_double, ctypes.c_int64]
        L.mtvd_batch_current.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
        L.mtvd_batch_set_tiling.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        L.mtvd_batch_get_tiling.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                            ctypes.POINTER(ctypes.c_int32)]
        L.mtvd_batch_autotune.argtypes = [vp, vp, ctypes.c_int32]
        L.mtvd_batch_destroy.argtypes = [vp]
        L.mtvd_batch_last_error.argtypes = [vp]
        L.mtvd_batch_last_error.restype = ctypes.c_char_p
        L.mtvd_adj_bytes.argtypes = [P, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_size_t)]
        L.mtvd_adj_create.argtypes = [P, ctypes.c_int32, ctypes.c_int32, vp, ctypes.POINTER(vp)]
        L.mtvd_adj_bind.argtypes = [vp, vp]
        L.mtvd_adj_forward.argtypes = [vp, vp, ctypes.c_double, dp, dp]
        L.mtvd_adj_backward.argtypes = [vp, ctypes.c_double, vp, vp, dp]
        L.mtvd_adj_coef_grads.argtypes = [vp, dp, dp]
        L.mtvd_adj_destroy.argtypes = [vp]
        L.mtvd_adj_last_error.argtypes = [vp]
        L.mtvd_adj_last_error.restype = ctypes.c_char_p
        L.mtvd_profiles.argtypes = [vp, dp, ctypes.c_size_t]
        L.mtvd_analysis_from_profiles.argtypes = [P, dp, ctypes.c_size_t,
                                                  ctypes.POINTER(_Analysis), dp, dp, dp]
        L.mtvd_bl_thickness.argtypes = [dp, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                        dp, dp]
        L.mtvd_bl_thickness_grid.argtypes = [dp, dp, ctypes.c_int32, ctypes.c_double,
                                             ctypes.c_double, dp, dp]
        L.mtvd_step_noalloc.argtypes = [P, vp, vp, ctypes.c_int32, vp,
                                        ctypes.POINTER(ctypes.c_int32)]
        for fn in ("mtvd_profiles", "mtvd_analysis_from_profiles", "mtvd_bl_thickness",
                   "mtvd_bl_thickness_grid", "mtvd_step_noalloc"):
            getattr(L, fn).restype = ctypes.c_int
        for fn in ("mtvd_adj_bytes", "mtvd_adj_create", "mtvd_adj_bind", "mtvd_adj_forward",
                   "mtvd_adj_backward", "mtvd_adj_coef_grads", "mtvd_adj_destroy"):
            getattr(L, fn).restype = ctypes.c_int
        for fn in ("mtvd_batch_bytes", "mtvd_batch_create", "mtvd_batch_bind",
                   "mtvd_batch_offset", "mtvd_batch_init_state", "mtvd_batch_step",
                   "mtvd_batch_diagnostics", "mtvd_batch_get_state", "mtvd_batch_set_state",
                   "mtvd_batch_current", "mtvd_batch_set_tiling", "mtvd_batch_get_tiling",
                   "mtvd_batch_autotune", "mtvd_batch_destroy"):
            getattr(L, fn).restype = ctypes.c_int
        for fn in ("mtvd_state_bytes", "mtvd_create", "mtvd_bind", "mtvd_init_state",
                   "mtvd_step", "mtvd_sweep", "mtvd_diagnostics", "mtvd_get_state",
                   "mtvd_set_state", "mtvd_current", "mtvd_sync", "mtvd_set_tiling",
                   "mtvd_set_timing", "mtvd_kernel_times", "mtvd_destroy"):
            getattr(L, fn).restype = ctypes.c_int
        _lib = L
    return _lib


def analysis(p: Params, prof: np.ndarray) -> dict:
    """Snapshot scalars (Re, C, volume means) and the derived profiles
    T_sa(z), rho - rho_A(z), U(z) of a (10, nz) profile array."""
    prof = np.ascontiguousarray(prof, dtype=np.float64)
    a = _Analysis()
    tsa, drho, U = (np.empty(p.nz, dtype=np.float64) for _ in range(3))
    dp = ctypes.POINTER(ctypes.c_double)
    pc = p._c()
    rc = lib().mtvd_analysis_from_profiles(ctypes.byref(pc), prof.ctypes.data_as(dp), prof.size,
                                           ctypes.byref(a), tsa.ctypes.data_as(dp),
                                           drho.ctypes.data_as(dp), U.ctypes.data_as(dp))
    if rc != MTVD_OK:
        raise MtvdError(rc, lib().mtvd_strerror(rc).decode())
    out = {n: getattr(a, n) for n, _ in _Analysis._fields_}
    out.update(Tsa_z=tsa, drho_z=drho, U_z=U)
    return out


def bl_thickness(tmean, D: float, rtol: float = 0.1, z=None):
    """(lambda_b, lambda_t) of a <T>_A profile (on uniform rows, or at the
    node heights z); -1 where not found."""
    t = np.ascontiguousarray(tmean, dtype=np.float64)
    lb, lt = ctypes.c_double(), ctypes.c_double()
    dp = ctypes.POINTER(ctypes.c_double)
    if z is None:
        rc = lib().mtvd_bl_thickness(t.ctypes.data_as(dp), t.size, D, rtol, ctypes.byref(lb),
                                     ctypes.byref(lt))
    else:
        zz = np.ascontiguousarray(z, dtype=np.float64)
        if zz.size != t.size:
            raise ValueError("z and tmean differ in length")
        rc = lib().mtvd_bl_thickness_grid(t.ctypes.data_as(dp), zz.ctypes.data_as(dp), t.size, D,
                                          rtol, ctypes.byref(lb), ctypes.byref(lt))
    if rc != MTVD_OK:
        raise MtvdError(rc, lib().mtvd_strerror(rc).decode())
    return lb.value, lt.value


def grid_heights(p: Params) -> np.ndarray:
    """The nz node heights of the grid (uniform, or the tanh grid of
    p.stretch)."""
    z = np.empty(p.nz, dtype=np.float64)
    pc = p._c()
    rc = lib().mtvd_grid_heights(ctypes.byref(pc), z.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                 z.size)
    if rc != MTVD_OK:
        raise MtvdError(rc, lib().mtvd_strerror(rc).decode())
    return z


def state_bytes(p: Params):
    """(state_bytes, workspace_bytes) for these parameters."""
    sb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    pc = p._c()
    rc = lib().mtvd_state_bytes(ctypes.byref(pc), ctypes.byref(sb), ctypes.byref(wb))
    if rc != MTVD_OK:
        raise MtvdError(rc, lib().mtvd_strerror(rc).decode())
    return sb.value, wb.value


def step_noalloc(p: Params, buf_a, buf_b, nsteps: int, stream=None) -> int:
    """``mtvd_step_noalloc``: nsteps steps of the state in ``buf_a`` (a
    float64 CUDA tensor of the state's size; ``buf_b`` the same, the second
    buffer) with no allocation; returns which buffer (0 = a, 1 = b) holds
    the result.  Asynchronous on ``stream`` (default: torch's current
    stream)."""
    import torch
    for b in (buf_a, buf_b):
        if not (torch.is_tensor(b) and b.is_cuda and b.dtype == torch.float64
                and b.is_contiguous() and b.numel() * 8 >= state_bytes(p)[0]):
            raise ValueError("buffers must be contiguous float64 CUDA tensors of the state's size")
    st = stream if stream is not None else torch.cuda.current_stream(buf_a.device)
    which = ctypes.c_int32()
    pc = p._c()
    rc = lib().mtvd_step_noalloc(ctypes.byref(pc), ctypes.c_void_p(buf_a.data_ptr()),
                                 ctypes.c_void_p(buf_b.data_ptr()), int(nsteps),
                                 ctypes.c_void_p(st.cuda_stream), ctypes.byref(which))
    if rc != MTVD_OK:
        raise MtvdError(rc, lib().mtvd_strerror(rc).decode())
    return which.value


class Solver:
    """One box on one GPU.  Buffers are torch tensors on ``device``; calls are
    stream-ordered on ``stream`` (default: the current torch stream)."""

    def __init__(self, p: Params, device=None, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise MtvdError(MTVD_EHIP, "no GPU visible: the HIP library needs one")
        self.p = p
        self.device = torch.device(device if device is not None else "cuda")
        L = lib()
        sb, wb = state_bytes(p)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            n = sb // 8
            # 256-byte aligned by the caching allocator; checked by mtvd_bind
            self.bufs = [torch.empty(n, dtype=torch.float64, device=self.device) for _ in range(2)]
            self.ws = torch.empty((wb + 7) // 8, dtype=torch.float64, device=self.device)
            ctx = ctypes.c_void_p()
            pc = p._c()
            self._check(L.mtvd_create(ctypes.byref(pc), ctypes.c_void_p(self.stream.cuda_stream),
                                      ctypes.byref(ctx)), None)
            self.ctx = ctx
            self._check(L.mtvd_bind(self.ctx, ctypes.c_void_p(self.bufs[0].data_ptr()),
                                    ctypes.c_void_p(self.bufs[1].data_ptr()),
                                    ctypes.c_void_p(self.ws.data_ptr())))

    def _check(self, rc: int, ctx="self"):
        if rc != MTVD_OK:
            L = lib()
            msg = L.mtvd_strerror(rc).decode()
            c = self.ctx if ctx == "self" else ctx
            if c:
                extra = L.mtvd_last_error(c).decode()
                if extra:
                    msg += f" ({extra})"
            raise MtvdError(rc, msg)

    # -- the C ABI, one method per entry point --------------------------------
    def init_state(self):
        self._check(lib().mtvd_init_state(self.ctx))

    def step(self, n: int = 1):
        self._check(lib().mtvd_step(self.ctx, int(n)))

    def sweep(self, axis: int):
        self._check(lib().mtvd_sweep(self.ctx, int(axis)))

    def diagnostics(self, check: bool = True) -> dict:
        d = _Diag()
        rc = lib().mtvd_diagnostics(self.ctx, ctypes.byref(d))
        if check:
            self._check(rc)
        out = {n: getattr(d, n) for n, _ in _Diag._fields_ if n != "tmean"}
        out["tmean"] = list(d.tmean)
        return out

    def profiles(self) -> np.ndarray:
        """(10, nz) row means of the analysis quantities (PROFILE_NAMES)."""
        out = np.empty((len(PROFILE_NAMES), self.p.nz), dtype=np.float64)
        self._check(lib().mtvd_profiles(self.ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        out.size))
        return out

    def get_state(self) -> np.ndarray:
        X = np.empty(self.p.shape, dtype=np.float64)
        self._check(lib().mtvd_get_state(self.ctx, X.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                         X.size))
        return X

    def set_state(self, X: np.ndarray, time: float = 0.0, step: int = 0):
        X = np.ascontiguousarray(X, dtype=np.float64)
        if X.shape != self.p.shape:
            raise ValueError(f"state shape {X.shape} != {self.p.shape}")
        self._check(lib().mtvd_set_state(self.ctx, X.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                         X.size, float(time), int(step)))

    def current(self) -> int:
        w = ctypes.c_int32()
        self._check(lib().mtvd_current(self.ctx, ctypes.byref(w)))
        return w.value

    def state_tensor(self):
        """The device buffer holding the current state (a view, canonical
        layout).  Valid until the next step."""
        return self.bufs[self.current()].view(self.p.shape)

    def sync(self):
        self._check(lib().mtvd_sync(self.ctx))

    def set_tiling(self, rows_x: int = 0, rows_z: int = 0):
        self._check(lib().mtvd_set_tiling(self.ctx, int(rows_x), int(rows_z)))

    def set_timing(self, enable: bool):
        self._check(lib().mtvd_set_timing(self.ctx, 1 if enable else 0))

    def kernel_times(self):
        """(ms[3], counts[3]) of the launches recorded since the last call,
        indexed by axis (0 = x, 1 = y, 2 = z)."""
        ms = (ctypes.c_double * 3)()
        cnt = (ctypes.c_int64 * 3)()
        self._check(lib().mtvd_kernel_times(self.ctx, ms, cnt))
        return list(ms), list(cnt)

    def close(self):
        if getattr(self, "ctx", None):
            lib().mtvd_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent 2D boxes advanced together (one launch per
    directional operator for all boxes; pairs of steps replay a captured
    HIP graph).  ``params`` is a list of :class:`Params`."""

    def __init__(self, params, device=None, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise MtvdError(MTVD_EHIP, "no GPU visible: the HIP library needs one")
        self.params = list(params)
        self.n = len(self.params)
        self.device = torch.device(device if device is not None else "cuda")
        L = lib()
        arr = (_Params * self.n)(*[p._c() for p in self.params])
        self._arr = arr
        sb, wb = ctypes.c_size_t(), ctypes.c_size_t()
        rc = L.mtvd_batch_bytes(arr, self.n, ctypes.byref(sb), ctypes.byref(wb))
        if rc != MTVD_OK:
            raise MtvdError(rc, L.mtvd_strerror(rc).decode())
        self.state_bytes = sb.value
        self.ctx = None
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.bufs = [torch.empty(sb.value // 8, dtype=torch.float64, device=self.device)
                         for _ in range(2)]
            self.ws = torch.empty((wb.value + 7) // 8, dtype=torch.float64, device=self.device)
            ctx = ctypes.c_void_p()
            rc = L.mtvd_batch_create(arr, self.n, ctypes.c_void_p(self.stream.cuda_stream),
                                     ctypes.byref(ctx))
            if rc != MTVD_OK:
                raise MtvdError(rc, L.mtvd_strerror(rc).decode())
            self.ctx = ctx
            self._check(L.mtvd_batch_bind(self.ctx, ctypes.c_void_p(self.bufs[0].data_ptr()),
                                          ctypes.c_void_p(self.bufs[1].data_ptr()),
                                          ctypes.c_void_p(self.ws.data_ptr())))

    def _check(self, rc: int):
        if rc != MTVD_OK:
            L = lib()
            msg = L.mtvd_strerror(rc).decode()
            if self.ctx:
                extra = L.mtvd_batch_last_error(self.ctx).decode()
                if extra:
                    msg += f" ({extra})"
            raise MtvdError(rc, msg)

    def init_state(self):
        self._check(lib().mtvd_batch_init_state(self.ctx))

    def step(self, n: int = 1):
        self._check(lib().mtvd_batch_step(self.ctx, int(n)))

    def diagnostics(self, box: int, check: bool = True) -> dict:
        d = _Diag()
        rc = lib().mtvd_batch_diagnostics(self.ctx, int(box), ctypes.byref(d))
        if check:
            self._check(rc)
        out = {n: getattr(d, n) for n, _ in _Diag._fields_ if n != "tmean"}
        out["tmean"] = list(d.tmean)
        return out

    def get_state(self, box: int) -> np.ndarray:
        p = self.params[box]
        X = np.empty(p.shape, dtype=np.float64)
        self._check(lib().mtvd_batch_get_state(self.ctx, int(box),
                                               X.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                               X.size))
        return X

    def set_state(self, box: int, X: np.ndarray, time: float = 0.0, step: int = 0):
        X = np.ascontiguousarray(X, dtype=np.float64)
        if X.shape != self.params[box].shape:
            raise ValueError("state shape mismatch")
        self._check(lib().mtvd_batch_set_state(self.ctx, int(box),
                                               X.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                               X.size, float(time), int(step)))

    def set_tiling(self, box: int, rows_x: int = 0, rows_z: int = 0):
        self._check(lib().mtvd_batch_set_tiling(self.ctx, int(box), int(rows_x), int(rows_z)))

    def tiling(self, box: int):
        a, b = ctypes.c_int32(), ctypes.c_int32()
        self._check(lib().mtvd_batch_get_tiling(self.ctx, int(box), ctypes.byref(a),
                                                ctypes.byref(b)))
        return a.value, b.value

    def autotune(self, trial_steps: int = 4):
        """Pick rows per wave per box size by timing (state restored)."""
        import torch
        scratch = torch.empty((self.state_bytes + 2048 * self.n + 7) // 8 + 32,
                              dtype=torch.float64, device=self.device)
        self._check(lib().mtvd_batch_autotune(self.ctx, ctypes.c_void_p(scratch.data_ptr()),
                                              int(trial_steps)))

    def close(self):
        if getattr(self, "ctx", None):
            lib().mtvd_batch_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Adjoint:
    """Reverse mode of the time-averaged mean Nusselt number of a 2D box
    with a frozen dt (``mtvd_adj_*`` in ``include/mtvd.h``):
    J(theta, Ra) = (1/N) sum_{n=1..N} Nu_mean(X_n), X_0 = conduction state
    with T0 + theta on interior rows.  Checkpoints every ``every`` steps live
    in the workspace between :meth:`forward` and :meth:`backward`."""

    def __init__(self, p: Params, nsteps: int, every: int = 50, device=None, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise MtvdError(MTVD_EHIP, "no GPU visible: the HIP library needs one")
        self.p, self.nsteps, self.every = p, int(nsteps), int(every)
        self.device = torch.device(device if device is not None else "cuda")
        self.ctx = None
        L = lib()
        pc = p._c()
        wb = ctypes.c_size_t()
        rc = L.mtvd_adj_bytes(ctypes.byref(pc), self.nsteps, self.every, ctypes.byref(wb))
        if rc != MTVD_OK:
            raise MtvdError(rc, L.mtvd_strerror(rc).decode())
        self.workspace_bytes = wb.value
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.ws = torch.empty((wb.value + 7) // 8, dtype=torch.float64, device=self.device)
            ctx = ctypes.c_void_p()
            rc = L.mtvd_adj_create(ctypes.byref(pc), self.nsteps, self.every,
                                   ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx))
            if rc != MTVD_OK:
                raise MtvdError(rc, L.mtvd_strerror(rc).decode())
            self.ctx = ctx
            self._check(L.mtvd_adj_bind(self.ctx, ctypes.c_void_p(self.ws.data_ptr())))

    def _check(self, rc: int):
        if rc != MTVD_OK:
            L = lib()
            msg = L.mtvd_strerror(rc).decode()
            if self.ctx:
                extra = L.mtvd_adj_last_error(self.ctx).decode()
                if extra:
                    msg += f" ({extra})"
            raise MtvdError(rc, msg)

    def _theta(self, theta):
        import torch
        if theta is None:
            return None
        t = torch.as_tensor(theta, dtype=torch.float64, device=self.device).contiguous()
        if t.numel() != self.p.nx * self.p.nz:
            raise ValueError(f"theta must hold nz*nx = {self.p.nx * self.p.nz} values")
        return t

    def forward(self, theta=None, dt: float = 0.0):
        """J and the dt used (dt = 0: the CFL dt of X_0).  Every call replaces
        the checkpoints that :meth:`backward` reverses and advances
        :attr:`generation`."""
        t = self._theta(theta)
        self._theta_keep = t
        J, d = ctypes.c_double(), ctypes.c_double()
        self._check(lib().mtvd_adj_forward(self.ctx, ctypes.c_void_p(t.data_ptr() if t is not None else 0),
                                           float(dt), ctypes.byref(J), ctypes.byref(d)))
        self.generation = getattr(self, "generation", 0) + 1
        return J.value, d.value

    def backward(self, Jbar: float = 1.0, want_x0: bool = False):
        """(dJ/dtheta as an (nz, nx) tensor, dJ/dX_0 or None, dJ/dRa), each
        times Jbar."""
        import torch
        gt = torch.empty((self.p.nz, self.p.nx), dtype=torch.float64, device=self.device)
        gx = torch.empty(self.p.shape, dtype=torch.float64, device=self.device) if want_x0 else None
        gr = ctypes.c_double()
        self._check(lib().mtvd_adj_backward(self.ctx, float(Jbar), ctypes.c_void_p(gx.data_ptr() if gx is not None else 0),
                                            ctypes.c_void_p(gt.data_ptr()), ctypes.byref(gr)))
        return gt, gx, gr.value

    def coef_grads(self):
        """(dJ/dmu*, dJ/dK*) of the latest backward pass, times its Jbar."""
        gm, gk = ctypes.c_double(), ctypes.c_double()
        self._check(lib().mtvd_adj_coef_grads(self.ctx, ctypes.byref(gm), ctypes.byref(gk)))
        return gm.value, gk.value

    def close(self):
        if getattr(self, "ctx", None):
            lib().mtvd_adj_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _nu_function():
    import torch

    class TimeAveragedNu(torch.autograd.Function):
        """J(theta, Ra) as a differentiable torch op; the backward pass is the
        library's hand-written adjoint (recomputation from checkpoints).

        dt is held fixed in the derivative.  With dt = 0 the first
        application takes the CFL dt of its X_0 and the adjoint keeps it
        (``frozen_dt``) for every later application, so that J is one smooth
        function of theta whose gradient the backward pass returns.  The
        adjoint's checkpoints belong to its latest forward pass: if another
        forward ran on the same adjoint since this application's, the
        backward pass first recomputes this one's from its saved theta."""

        @staticmethod
        def forward(ctx, theta, ra, adjoint, dt):
            if abs(float(ra) - adjoint.p.Ra) > 1e-12 * adjoint.p.Ra:
                raise ValueError("Ra differs from the one the adjoint was created for")
            dt = float(dt)
            if dt <= 0.0:
                dt = getattr(adjoint, "frozen_dt", 0.0)
            th = theta.detach().clone()
            J, dt_used = adjoint.forward(th, dt)
            if dt <= 0.0:
                adjoint.frozen_dt = dt_used
            ctx.adjoint = adjoint
            ctx.generation = adjoint.generation
            ctx.theta = th
            ctx.dt = dt_used
            ctx.theta_shape = theta.shape
            ctx.ra_device = ra.device if torch.is_tensor(ra) else None
            return torch.tensor(J, dtype=torch.float64, device=theta.device)

        @staticmethod
        def backward(ctx, gJ):
            a = ctx.adjoint
            if a.generation != ctx.generation:
                a.forward(ctx.theta, ctx.dt)
            gt, _, gr = a.backward(float(gJ))
            gra = None
            if ctx.ra_device is not None:
                gra = torch.tensor(gr, dtype=torch.float64, device=ctx.ra_device)
            return gt.reshape(ctx.theta_shape).to(gJ.device), gra, None, None

    return TimeAveragedNu


_TAN = None


def time_averaged_nu(theta, ra, adjoint: Adjoint, dt: float = 0.0):
    """Differentiable J(theta, Ra) (see :class:`Adjoint`).  ``theta`` is a
    float64 tensor of nz*nx values on the GPU (any shape; its gradient has
    the same shape), ``ra`` a 0-d float64 tensor equal to the adjoint's Ra;
    gradients flow to both.  ``dt`` > 0 fixes the time step; dt = 0 takes
    the CFL dt of the first application's initial state and keeps it for
    every later one on the same adjoint (the derivative holds dt fixed)."""
    global _TAN
    if _TAN is None:
        _TAN = _nu_function()
    return _TAN.apply(theta, ra, adjoint, dt)
