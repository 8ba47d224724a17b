"""Thin Python binding of libslepian's C ABI (include/slepian.h).

Argument marshalling only: every step runs in the HIP library.  Functions
carry the C names.  Signals are torch tensors on the plan's GPU, a batch of b
length-N signals being a (b, N) tensor whose rows are contiguous (the C
layout N x b column-major with leading dimension = row stride).  Work is
enqueued on torch's current stream of that device.

The library must be built (paper_1611_04950_amd/build.py); importing this
module without it raises, there is no fallback.
"""

from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libslepian.so")

SLEPIAN_OK = 0
SLEPIAN_EINVAL = -1
SLEPIAN_EGAP = -2
SLEPIAN_ENOMEM = -3
SLEPIAN_EHIP = -4
SLEPIAN_ENOCONV = -5
SLEPIAN_ENOTSUP = -6
SLEPIAN_ENONFINITE = -7
SLEPIAN_EIO = -8
SLEPIAN_ESCRATCH = -9
SLEPIAN_EINTERNAL = -10

SLEPIAN_FP32, SLEPIAN_MIXED, SLEPIAN_BF16_RAW = 0, 1, 2
SLEPIAN_PINV, SLEPIAN_TIKHONOV = 0, 1
SLEPIAN_OP_PROJECT, SLEPIAN_OP_COEFFS, SLEPIAN_OP_LSQ, SLEPIAN_OP_MULTIBAND = 0, 1, 2, 3
SLEPIAN_FACTOR_THEOREM1, SLEPIAN_FACTOR_EIG = 0, 1

EXPORTED = [
    "slepian_plan", "slepian_plan_ex", "slepian_plan_batch", "slepian_plan_info_get", "slepian_plan_eigenpairs",
    "slepian_plan_save", "slepian_plan_load", "slepian_plan_destroy", "slepian_workspace_size",
    "slepian_project", "slepian_project_ex", "slepian_project_noalloc", "slepian_project_multiband", "slepian_bands_create",
    "slepian_bands_destroy", "slepian_bands_workspace_size", "slepian_project_bands",
    "slepian_bands_span_workspace_size", "slepian_project_bands_span", "slepian_coeffs", "slepian_lsq",
    "slepian_factor_create", "slepian_factor_create_ex", "slepian_factor_destroy", "slepian_factor_info", "slepian_factor_mu",
    "slepian_factor_workspace_size", "slepian_factor_compress", "slepian_factor_recover",
    "slepian_apply_b64",
    "slepian_group_create", "slepian_group_project", "slepian_group_destroy", "slepian_group_info",
    "slepian_status_string",
    "slepian_trace_enable", "slepian_trace_read",
]


class PlanOpts(C.Structure):
    _fields_ = [("alpha", C.c_double), ("K", C.c_int64), ("precision", C.c_int), ("device", C.c_int),
                ("tune", C.c_int), ("tune_batch", C.c_int64), ("tune_cache", C.c_char_p)]


class FactorInfo(C.Structure):
    _fields_ = [("kf", C.c_int64), ("r1", C.c_int64), ("r", C.c_int64), ("kprime", C.c_int64),
                ("subspace", C.c_int64), ("mu_dropped", C.c_double), ("ritz_residual", C.c_double),
                ("method", C.c_int32), ("r_h", C.c_int32), ("r_a", C.c_int32), ("r_b", C.c_int32),
                ("deflated_norm", C.c_double)]


class PlanInfo(C.Structure):
    _fields_ = [
        ("N", C.c_int64), ("W", C.c_double), ("eps", C.c_double), ("alpha", C.c_double),
        ("K", C.c_int64), ("L", C.c_int64), ("r", C.c_int64), ("l_first", C.c_int64),
        ("r_tik", C.c_int64), ("l_first_tik", C.c_int64), ("window_lo", C.c_int64),
        ("window_hi", C.c_int64), ("lam_Km1", C.c_double), ("lam_K", C.c_double),
        ("eps_achieved", C.c_double), ("precision", C.c_int), ("device", C.c_int),
        ("row_log2", C.c_int32), ("col_log2", C.c_int32), ("cic_shape", C.c_int32), ("cic_maxlog1", C.c_int32),
        ("tuned", C.c_int32), ("tune_batch", C.c_int64), ("tune_us", C.c_double),
    ]


class KernelStat(C.Structure):
    _fields_ = [("name", C.c_char * 48), ("launches", C.c_int64), ("total_ms", C.c_double),
                ("min_ms", C.c_double), ("max_ms", C.c_double)]


class GroupInfo(C.Structure):
    _fields_ = [("plans", C.c_int32), ("grouped", C.c_int32), ("other", C.c_int32), ("tuned", C.c_int32),
                ("partial_variant", C.c_int32), ("cic_variant", C.c_int32 * 5)]


class LsqReport(C.Structure):
    _fields_ = [("iterations", C.c_int), ("rel_residual", C.c_double),
                ("rel_residual_first", C.c_double), ("converged", C.c_int)]


def load_library(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise RuntimeError(f"libslepian is not built ({path} missing); run paper_1611_04950_amd/build.py")
    lib = C.CDLL(path)
    vp, i64, dbl, i32, sz = C.c_void_p, C.c_int64, C.c_double, C.c_int, C.c_size_t
    sig = {
        "slepian_plan": [i64, dbl, dbl, C.POINTER(vp)],
        "slepian_plan_ex": [i64, dbl, dbl, C.POINTER(PlanOpts), C.POINTER(vp)],
        "slepian_plan_batch": [i32, C.POINTER(i64), C.POINTER(dbl), C.POINTER(dbl), C.POINTER(PlanOpts),
                               C.POINTER(vp)],
        "slepian_plan_info_get": [vp, C.POINTER(PlanInfo)],
        "slepian_plan_eigenpairs": [vp, C.POINTER(i64), C.POINTER(i64), vp, vp, i64, i64],
        "slepian_plan_save": [vp, C.c_char_p],
        "slepian_plan_load": [C.c_char_p, i32, C.POINTER(vp)],
        "slepian_plan_destroy": [vp],
        "slepian_workspace_size": [vp, i32, i64, C.POINTER(sz)],
        "slepian_project": [vp, vp, i64, vp, i64, i64, vp, sz, vp],
        "slepian_project_ex": [vp, i32, vp, i64, vp, i64, i64, vp, sz, vp],
        "slepian_project_noalloc": [vp, vp, i64, vp, i64, i64, vp],
        "slepian_project_multiband": [vp, i32, C.POINTER(dbl), vp, i64, vp, i64, i64, vp, sz, vp],
        "slepian_bands_create": [vp, i32, C.POINTER(dbl), C.POINTER(vp)],
        "slepian_bands_destroy": [vp],
        "slepian_bands_workspace_size": [vp, i64, C.POINTER(sz)],
        "slepian_project_bands": [vp, vp, i64, vp, i64, i64, vp, sz, vp],
        "slepian_bands_span_workspace_size": [vp, i64, C.POINTER(sz)],
        "slepian_project_bands_span": [vp, vp, i64, vp, i64, i64, dbl, i32, vp, sz, vp, C.POINTER(i32)],
        "slepian_coeffs": [vp, vp, i64, vp, i64, i64, vp, sz, vp],
        "slepian_factor_create": [vp, C.POINTER(vp)],
        "slepian_factor_create_ex": [vp, i32, C.POINTER(vp)],
        "slepian_factor_destroy": [vp],
        "slepian_factor_info": [vp, C.POINTER(FactorInfo)],
        "slepian_factor_mu": [vp, C.POINTER(dbl), i64],
        "slepian_factor_workspace_size": [vp, i64, C.POINTER(sz)],
        "slepian_factor_compress": [vp, vp, i64, vp, i64, i64, vp, sz, vp],
        "slepian_factor_recover": [vp, vp, i64, vp, i64, i64, vp, sz, vp],
        "slepian_lsq": [vp, i32, dbl, vp, i64, vp, i64, i64, dbl, i32, vp, sz, vp, C.POINTER(LsqReport)],
        "slepian_apply_b64": [vp, vp, i64, vp, i64, i64, vp, sz, vp],
        "slepian_group_create": [C.POINTER(vp), i32, C.POINTER(i64), C.POINTER(vp)],
        "slepian_group_project": [vp, C.POINTER(vp), C.POINTER(vp), vp],
        "slepian_group_destroy": [vp],
        "slepian_group_info": [vp, C.POINTER(GroupInfo)],
        "slepian_status_string": [i32],
        "slepian_trace_enable": [i32],
        "slepian_trace_read": [C.POINTER(KernelStat), i32, C.POINTER(i32), i32],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_char_p if name == "slepian_status_string" else C.c_int
    return lib


_lib = load_library()


class SlepianError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {_lib.slepian_status_string(status).decode()} ({status})")


def _check(status: int, where: str) -> None:
    if status != SLEPIAN_OK:
        raise SlepianError(status, where)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(t: torch.Tensor):
    return C.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _signals(t: torch.Tensor, N: int, dtype, name: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if t.dim() == 1:
        t = t.view(1, -1)
    if t.dim() != 2 or t.shape[1] != N or t.stride(1) != 1:
        raise ValueError(f"{name} must have shape (batch, {N}) with contiguous rows")
    ld = t.stride(0) if t.shape[0] > 1 else N
    return t, ld


class Plan:
    """Owns a slepian_plan_t."""

    def __init__(self, handle: int):
        self.handle = C.c_void_p(handle)
        self.info = slepian_plan_info_get(self)

    def __del__(self):
        h = getattr(self, "handle", None)
        # at interpreter exit the module globals may already be gone
        if h is not None and h.value and _lib is not None:
            _lib.slepian_plan_destroy(h)
            self.handle = C.c_void_p(0)

    @property
    def N(self):
        return self.info["N"]

    @property
    def K(self):
        return self.info["K"]


def slepian_plan(N: int, W: float, eps: float, alpha: float = 0.0, K: int = 0,
                 precision: int = SLEPIAN_FP32, device: int = -1, tune: bool = False, tune_batch: int = 0,
                 tune_cache: str | None = None) -> Plan:
    h = C.c_void_p()
    opts = PlanOpts(alpha, K, precision, device, int(tune), tune_batch,
                    None if tune_cache is None else tune_cache.encode())
    _check(_lib.slepian_plan_ex(N, W, eps, C.byref(opts), C.byref(h)), "slepian_plan")
    return Plan(h.value)


def slepian_plan_batch(specs, alpha: float = 0.0, K: int = 0, precision: int = SLEPIAN_FP32,
                       device: int = -1, tune: bool = False, tune_batch: int = 0,
                       tune_cache: str | None = None) -> list:
    """Plans for (N, W, eps) triples in one call (the eigensolves run
    together); the options apply to every plan (tune_batch may also be a
    list, one batch size per plan)."""
    n = len(specs)
    if n == 0:
        return []
    Ns = (C.c_int64 * n)(*[int(sp[0]) for sp in specs])
    Ws = (C.c_double * n)(*[float(sp[1]) for sp in specs])
    Es = (C.c_double * n)(*[float(sp[2]) for sp in specs])
    cache = None if tune_cache is None else tune_cache.encode()
    tb = list(tune_batch) if isinstance(tune_batch, (list, tuple)) else [tune_batch] * n
    opts = (PlanOpts * n)(*[PlanOpts(alpha, K, precision, device, int(tune), int(tb[i]), cache) for i in range(n)])
    hs = (C.c_void_p * n)()
    _check(_lib.slepian_plan_batch(n, Ns, Ws, Es, opts, hs), "slepian_plan_batch")
    return [Plan(h) for h in hs]


def slepian_plan_info_get(plan: Plan) -> dict:
    info = PlanInfo()
    _check(_lib.slepian_plan_info_get(plan.handle, C.byref(info)), "slepian_plan_info_get")
    return {f: getattr(info, f) for f, _ in PlanInfo._fields_}


def slepian_plan_eigenpairs(plan: Plan, vectors: bool = True):
    """(l_first, lam (float64 CPU tensor), vecs (count, N) float64 CUDA tensor or None)."""
    l0, cnt = C.c_int64(), C.c_int64()
    _check(_lib.slepian_plan_eigenpairs(plan.handle, C.byref(l0), C.byref(cnt), None, None, 0, 0),
           "slepian_plan_eigenpairs")
    n = cnt.value
    lam = torch.empty(max(n, 1), dtype=torch.float64)
    vecs = None
    if vectors:
        vecs = torch.empty((max(n, 1), plan.N), dtype=torch.float64, device=f"cuda:{plan.info['device']}")
    _check(_lib.slepian_plan_eigenpairs(plan.handle, C.byref(l0), C.byref(cnt), _ptr(lam), _ptr(vecs),
                                        plan.N, max(n, 1)), "slepian_plan_eigenpairs")
    return l0.value, lam[:n], (vecs[:n] if vecs is not None else None)


def slepian_plan_save(plan: Plan, path: str) -> None:
    _check(_lib.slepian_plan_save(plan.handle, path.encode()), "slepian_plan_save")


def slepian_plan_load(path: str, device: int = -1) -> Plan:
    h = C.c_void_p()
    _check(_lib.slepian_plan_load(path.encode(), device, C.byref(h)), "slepian_plan_load")
    return Plan(h.value)


def slepian_workspace_size(plan: Plan, op: int, batch: int) -> int:
    n = C.c_size_t()
    _check(_lib.slepian_workspace_size(plan.handle, op, batch, C.byref(n)), "slepian_workspace_size")
    return n.value


def slepian_project(plan: Plan, x: torch.Tensor, y: torch.Tensor | None = None,
                    work: torch.Tensor | None = None, precision: int | None = None) -> torch.Tensor:
    x, ldx = _signals(x, plan.N, torch.float32, "x")
    if y is None:
        y = torch.empty_like(x)
    y, ldy = _signals(y, plan.N, torch.float32, "y")
    wb = 0 if work is None else work.numel() * work.element_size()
    prec = plan.info["precision"] if precision is None else precision
    _check(_lib.slepian_project_ex(plan.handle, prec, _ptr(x), ldx, _ptr(y), ldy, x.shape[0], _ptr(work), wb,
                                   _stream(x)), "slepian_project")
    return y


def slepian_project_noalloc(plan: Plan, x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    """slepian_project through the entry point that allocates nothing (its
    workspace is the library's fixed device array); y must be given."""
    x, ldx = _signals(x, plan.N, torch.float32, "x")
    y, ldy = _signals(y, plan.N, torch.float32, "y")
    _check(_lib.slepian_project_noalloc(plan.handle, _ptr(x), ldx, _ptr(y), ldy, x.shape[0], _stream(x)),
           "slepian_project_noalloc")
    return y


def slepian_project_multiband(plan: Plan, freqs, x: torch.Tensor, y: torch.Tensor | None = None,
                              work: torch.Tensor | None = None) -> torch.Tensor:
    """Band sum of the Slepian projections modulated to the band centres
    `freqs`, band by band (see include/slepian.h; the projection onto the
    dictionary's span is slepian_project_bands_span)."""
    x, ldx = _signals(x, plan.N, torch.float32, "x")
    if y is None:
        y = torch.empty_like(x)
    y, ldy = _signals(y, plan.N, torch.float32, "y")
    f = (C.c_double * len(freqs))(*[float(v) for v in freqs])
    wb = 0 if work is None else work.numel() * work.element_size()
    _check(_lib.slepian_project_multiband(plan.handle, len(freqs), f, _ptr(x), ldx, _ptr(y), ldy, x.shape[0],
                                          _ptr(work), wb, _stream(x)), "slepian_project_multiband")
    return y


class Bands:
    """Owns a slepian_bands_t; keeps its plan alive."""

    def __init__(self, handle: int, plan: Plan, freqs):
        self.handle = C.c_void_p(handle)
        self.plan = plan
        self.freqs = list(freqs)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.slepian_bands_destroy(h)
            self.handle = C.c_void_p(0)


def slepian_bands_create(plan: Plan, freqs) -> Bands:
    """Prepared band set for slepian_project_bands (see include/slepian.h)."""
    f = (C.c_double * len(freqs))(*[float(v) for v in freqs])
    h = C.c_void_p()
    _check(_lib.slepian_bands_create(plan.handle, len(freqs), f, C.byref(h)), "slepian_bands_create")
    return Bands(h.value, plan, freqs)


def slepian_bands_workspace_size(bands: Bands, batch: int) -> int:
    n = C.c_size_t()
    _check(_lib.slepian_bands_workspace_size(bands.handle, batch, C.byref(n)), "slepian_bands_workspace_size")
    return n.value


class Factor:
    """Owns a slepian_factor_t (fast factorization T1 T2^T); keeps its plan alive."""

    def __init__(self, handle: int, plan: Plan):
        self.handle = C.c_void_p(handle)
        self.plan = plan
        inf = FactorInfo()
        _check(_lib.slepian_factor_info(self.handle, C.byref(inf)), "slepian_factor_info")
        self.info = {f: getattr(inf, f) for f, _ in FactorInfo._fields_}
        self.mu = None
        if self.info["method"] == SLEPIAN_FACTOR_EIG:
            n = max(self.info["r1"], 1)
            mu = (C.c_double * n)()
            _check(_lib.slepian_factor_mu(self.handle, mu, n), "slepian_factor_mu")
            self.mu = [mu[i] for i in range(self.info["r1"])]

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.slepian_factor_destroy(h)
            self.handle = C.c_void_p(0)


def slepian_factor_create(plan: Plan, method: int = SLEPIAN_FACTOR_THEOREM1) -> Factor:
    """Fast factorization S_K S_K^T ~= T1 T2^T of the plan, with L1, L2 from
    Theorem 1's construction (default) or from the eigenpairs of B - F F^*
    (SLEPIAN_FACTOR_EIG); see include/slepian.h."""
    h = C.c_void_p()
    _check(_lib.slepian_factor_create_ex(plan.handle, method, C.byref(h)), "slepian_factor_create_ex")
    return Factor(h.value, plan)


def slepian_factor_workspace_size(f: Factor, batch: int) -> int:
    n = C.c_size_t()
    _check(_lib.slepian_factor_workspace_size(f.handle, batch, C.byref(n)), "slepian_factor_workspace_size")
    return n.value


def slepian_factor_compress(f: Factor, x: torch.Tensor, c: torch.Tensor | None = None,
                            work: torch.Tensor | None = None) -> torch.Tensor:
    """c = T2^T x: (batch, N) -> (batch, kprime) FP32."""
    x, ldx = _signals(x, f.plan.N, torch.float32, "x")
    kp = f.info["kprime"]
    if c is None:
        c = torch.empty((x.shape[0], kp), dtype=torch.float32, device=x.device)
    c, ldc = _signals(c, kp, torch.float32, "c")
    wb = 0 if work is None else work.numel() * work.element_size()
    _check(_lib.slepian_factor_compress(f.handle, _ptr(x), ldx, _ptr(c), ldc, x.shape[0], _ptr(work), wb,
                                        _stream(x)), "slepian_factor_compress")
    return c


def slepian_factor_recover(f: Factor, c: torch.Tensor, y: torch.Tensor | None = None,
                           work: torch.Tensor | None = None) -> torch.Tensor:
    """y = T1 c: (batch, kprime) -> (batch, N) FP32."""
    c, ldc = _signals(c, f.info["kprime"], torch.float32, "c")
    N = f.plan.N
    if y is None:
        y = torch.empty((c.shape[0], N), dtype=torch.float32, device=c.device)
    y, ldy = _signals(y, N, torch.float32, "y")
    wb = 0 if work is None else work.numel() * work.element_size()
    _check(_lib.slepian_factor_recover(f.handle, _ptr(c), ldc, _ptr(y), ldy, c.shape[0], _ptr(work), wb,
                                       _stream(c)), "slepian_factor_recover")
    return y


def slepian_project_bands(bands: Bands, x: torch.Tensor, y: torch.Tensor | None = None,
                          work: torch.Tensor | None = None) -> torch.Tensor:
    N = bands.plan.N
    x, ldx = _signals(x, N, torch.float32, "x")
    if y is None:
        y = torch.empty_like(x)
    y, ldy = _signals(y, N, torch.float32, "y")
    wb = 0 if work is None else work.numel() * work.element_size()
    _check(_lib.slepian_project_bands(bands.handle, _ptr(x), ldx, _ptr(y), ldy, x.shape[0], _ptr(work), wb,
                                      _stream(x)), "slepian_project_bands")
    return y


def slepian_bands_span_workspace_size(bands: Bands, batch: int) -> int:
    n = C.c_size_t()
    _check(_lib.slepian_bands_span_workspace_size(bands.handle, batch, C.byref(n)),
           "slepian_bands_span_workspace_size")
    return n.value


def slepian_project_bands_span(bands: Bands, x: torch.Tensor, y: torch.Tensor | None = None, tol: float = 0.0,
                               max_iter: int = 100, work: torch.Tensor | None = None, check: bool = True):
    """Orthogonal projection onto the span of the band set's modulated
    Slepian dictionary (conjugate gradients on the band sum); returns
    (y, iterations per signal).  With check=False a non-convergence
    (SLEPIAN_ENOCONV) is returned in place of raising."""
    N = bands.plan.N
    x, ldx = _signals(x, N, torch.float32, "x")
    if y is None:
        y = torch.empty_like(x)
    y, ldy = _signals(y, N, torch.float32, "y")
    wb = 0 if work is None else work.numel() * work.element_size()
    b = x.shape[0]
    it = (C.c_int32 * max(b, 1))()
    st = _lib.slepian_project_bands_span(bands.handle, _ptr(x), ldx, _ptr(y), ldy, b, float(tol), int(max_iter),
                                         _ptr(work), wb, _stream(x), it)
    if check:
        _check(st, "slepian_project_bands_span")
    iters = [it[i] for i in range(b)]
    return (y, iters) if check else (y, iters, st)


def slepian_coeffs(plan: Plan, x: torch.Tensor, c: torch.Tensor | None = None,
                   work: torch.Tensor | None = None) -> torch.Tensor:
    """c = S_K^T x as a (batch, K) tensor (row s holds signal s's K coefficients)."""
    x, ldx = _signals(x, plan.N, torch.float32, "x")
    if c is None:
        c = torch.empty((x.shape[0], plan.K), dtype=torch.float32, device=x.device)
    wb = 0 if work is None else work.numel() * work.element_size()
    ldc = c.stride(0) if c.shape[0] > 1 else plan.K
    _check(_lib.slepian_coeffs(plan.handle, _ptr(x), ldx, _ptr(c), ldc, x.shape[0], _ptr(work), wb, _stream(x)),
           "slepian_coeffs")
    return c


def slepian_lsq(plan: Plan, y: torch.Tensor, mode: int = SLEPIAN_TIKHONOV, alpha: float | None = None,
                tol: float = 1e-10, max_iter: int = 10, x: torch.Tensor | None = None,
                work: torch.Tensor | None = None):
    """Returns (x float64 (batch, N), report dict)."""
    y, ldy = _signals(y, plan.N, torch.float32, "y")
    if x is None:
        x = torch.empty(y.shape, dtype=torch.float64, device=y.device)
    x, ldx = _signals(x, plan.N, torch.float64, "x")
    if alpha is None:
        alpha = plan.info["alpha"]
    rep = LsqReport()
    wb = 0 if work is None else work.numel() * work.element_size()
    st = _lib.slepian_lsq(plan.handle, mode, alpha, _ptr(y), ldy, _ptr(x), ldx, y.shape[0], tol, max_iter,
                          _ptr(work), wb, _stream(y), C.byref(rep))
    report = {f: getattr(rep, f) for f, _ in LsqReport._fields_}
    _check(st, "slepian_lsq")
    return x, report


def slepian_apply_b64(plan: Plan, x: torch.Tensor, y: torch.Tensor | None = None) -> torch.Tensor:
    x, ldx = _signals(x, plan.N, torch.float64, "x")
    if y is None:
        y = torch.empty_like(x)
    y, ldy = _signals(y, plan.N, torch.float64, "y")
    _check(_lib.slepian_apply_b64(plan.handle, _ptr(x), ldx, _ptr(y), ldy, x.shape[0], None, 0, _stream(x)),
           "slepian_apply_b64")
    return y


class Group:
    def __init__(self, handle: int, plans):
        self.handle = C.c_void_p(handle)
        self.plans = list(plans)   # the plans must outlive the group

    @property
    def info(self) -> dict:
        gi = GroupInfo()
        _check(_lib.slepian_group_info(self.handle, C.byref(gi)), "slepian_group_info")
        return {"plans": gi.plans, "grouped": gi.grouped, "other": gi.other, "tuned": gi.tuned,
                "partial_variant": gi.partial_variant, "cic_variant": list(gi.cic_variant)}

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.slepian_group_destroy(h)
            self.handle = C.c_void_p(0)


def slepian_group_create(plans, batch) -> Group:
    n = len(plans)
    arr = (C.c_void_p * n)(*[p.handle.value for p in plans])
    b = (C.c_int64 * n)(*batch)
    h = C.c_void_p()
    _check(_lib.slepian_group_create(arr, n, b, C.byref(h)), "slepian_group_create")
    return Group(h.value, plans)


def slepian_group_project(group: Group, xs, ys) -> None:
    n = len(group.plans)
    for p, x, y in zip(group.plans, xs, ys):
        for t in (x, y):
            if t.dtype != torch.float32 or not t.is_contiguous() or t.shape[-1] != p.N:
                raise ValueError("group signals must be contiguous float32 (batch, N) tensors")
    xa = (C.c_void_p * n)(*[x.data_ptr() for x in xs])
    ya = (C.c_void_p * n)(*[y.data_ptr() for y in ys])
    _check(_lib.slepian_group_project(group.handle, xa, ya, _stream(xs[0])), "slepian_group_project")


def slepian_status_string(status: int) -> str:
    return _lib.slepian_status_string(status).decode()


def slepian_trace_enable(on: bool = True) -> None:
    _check(_lib.slepian_trace_enable(1 if on else 0), "slepian_trace_enable")


def slepian_trace_read(reset: bool = True) -> dict:
    """{kernel name: {launches, total_ms, min_ms, max_ms}} over the traced launches."""
    cap = 64
    arr = (KernelStat * cap)()
    n = C.c_int()
    _check(_lib.slepian_trace_read(arr, cap, C.byref(n), 1 if reset else 0), "slepian_trace_read")
    return {arr[i].name.decode(): {"launches": arr[i].launches, "total_ms": arr[i].total_ms,
                                   "min_ms": arr[i].min_ms, "max_ms": arr[i].max_ms}
            for i in range(min(n.value, cap))}
