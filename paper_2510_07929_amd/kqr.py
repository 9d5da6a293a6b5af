"""ctypes binding of libkqr (the C ABI declared in include/kqr.h).

Argument marshalling only: every function takes torch tensors that already
live on the GPU (or host arrays where the C ABI wants host memory), checks
dtype / device / layout, and passes raw pointers and the current HIP stream
to the library.  All arithmetic happens in the library's HIP kernels.  If
the library has not been built, every call raises.
"""
from __future__ import annotations

import ctypes as C
import json
import math
import os
import threading

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libkqr.so")
_lib_handle = None
_lib_lock = threading.Lock()

KQR_OK, KQR_NOT_CONVERGED = 0, 1
KQR_EINVAL, KQR_ENOMEM, KQR_ENODEVICE, KQR_EHIP, KQR_ENUMERIC = -1, -2, -3, -4, -5
KQR_RBF, KQR_LAPLACIAN, KQR_LINEAR = 0, 1, 2
KQR_FP32, KQR_BF16 = 0, 1
KQR_KMODE_AUTO, KQR_KMODE_MATERIALIZE, KQR_KMODE_ON_THE_FLY = 0, 1, 2
KQR_APPLY_FAST, KQR_APPLY_EXACT, KQR_APPLY_KV = 0, 1, 2

KERNELS = {"rbf": KQR_RBF, "laplacian": KQR_LAPLACIAN, "linear": KQR_LINEAR}
KDTYPES = {"fp32": KQR_FP32, "bf16": KQR_BF16}


class KqrOptions(C.Structure):
    _fields_ = [
        ("tol", C.c_double), ("admm_tol", C.c_double),
        ("admm_max_iter", C.c_int), ("alm_max_iter", C.c_int),
        ("admm_sigma", C.c_double), ("admm_step", C.c_double), ("admm_eps0", C.c_double),
        ("etabar", C.c_double), ("iota", C.c_double), ("armijo", C.c_double),
        ("ls_shrink", C.c_double), ("ls_max", C.c_int),
        ("tau1", C.c_double), ("tau2", C.c_double), ("eps_floor", C.c_double),
        ("ssn_max_iter", C.c_int), ("ssn_rel", C.c_double),
        ("sigma_factor", C.c_double), ("sigma_stall", C.c_double), ("sigma_max", C.c_double),
        ("rank", C.c_int), ("xi", C.c_double), ("pcg_max_iter", C.c_int),
        ("k_dtype", C.c_int), ("kmode", C.c_int), ("refine", C.c_int),
        ("pivot_uniforms", C.POINTER(C.c_double)), ("seed", C.c_uint64), ("verbose", C.c_int),
        ("profile", C.c_int), ("exact_k", C.c_int), ("ssn_adapt", C.c_double),
        ("trace", C.POINTER(C.c_double)), ("trace_cap", C.c_int), ("k_layout", C.c_int),
        ("z_out", C.c_void_p), ("v_out", C.c_void_p),
        ("warm_alpha", C.c_void_p), ("warm_v", C.c_void_p), ("warm_z", C.c_void_p),
        ("warm_beta", C.c_double), ("warm_sigma", C.c_double),
    ]


class KqrInfo(C.Structure):
    _fields_ = [
        ("eta_p", C.c_double), ("eta_d", C.c_double), ("eta_c", C.c_double),
        ("eta_kkt", C.c_double), ("eta_gap", C.c_double),
        ("obj_p", C.c_double), ("obj_d", C.c_double), ("sigma", C.c_double),
        ("admm_iters", C.c_int), ("alm_iters", C.c_int), ("newton_iters", C.c_int),
        ("line_search_steps", C.c_int), ("admm_pcg_iters", C.c_int), ("pcg_iters", C.c_int),
        ("rank_used", C.c_int), ("refinements", C.c_int),
        ("kapply_calls", C.c_int64), ("n_interior", C.c_int64),
        ("t_kbuild", C.c_double), ("t_precond", C.c_double), ("t_admm", C.c_double),
        ("t_alm", C.c_double), ("t_total", C.c_double),
        ("kapply_fast_calls", C.c_int64), ("kapply_exact_calls", C.c_int64),
        ("t_kapply_fast", C.c_double), ("t_kapply_exact", C.c_double),
        ("trace_len", C.c_int), ("core_retries", C.c_int),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_P = C.c_void_p
_I64 = C.c_int64
_SIGS = {
    "kqr_default_options": (C.c_int, [C.POINTER(KqrOptions)]),
    "kqr_status_string": (C.c_char_p, [C.c_int]),
    "kqr_last_error": (C.c_char_p, []),
    "kqr_device_count": (C.c_int, []),
    "kqr_test_core_breakdowns": (C.c_int, [C.c_int, C.c_int]),
    "kqr_test_batch_steps": (C.c_int, [C.c_int]),
    "kqr_set_batch_threads": (C.c_int, [C.c_int]),
    "kqr_kernel_build": (C.c_int, [_P, _I64, _I64, C.c_int, C.c_double, C.c_int, _P, _I64, _P]),
    "kqr_kernel_apply": (C.c_int, [_P, _I64, _I64, C.c_int, C.c_double, _P, C.c_int, _I64, _P, _I64, _I64,
                                   _P, _I64, C.c_int, _P]),
    "kqr_predict": (C.c_int, [_P, _I64, _I64, _P, C.c_double, C.c_double, C.c_int, C.c_double, _P, _I64, _P, _P]),
    "kqr_rpcholesky": (C.c_int, [_P, _I64, _I64, C.c_int, C.c_double, _P, C.c_int, _I64, _I64, _P, _P, _I64,
                                 _P, _P, _P]),
    "kqr_woodbury_apply": (C.c_int, [_P, _I64, _I64, _I64, C.c_double, _P, _P, _P, _P]),
    "kqr_adaptive_rank": (C.c_int, [_P, _I64, _I64, _I64, C.c_double, _P, _P, _P]),
    "kqr_autotune_apply": (C.c_int, [_P, C.c_int, _I64, _I64, C.c_int, C.c_int, C.c_char_p, _I64, _P]),
    "kqr_set_apply_shape": (C.c_int, [C.c_int, C.c_int, _I64, C.c_int, C.c_int, C.c_int]),
    "kqr_set_kv_shape": (C.c_int, [C.c_int, _I64, C.c_int, C.c_int, C.c_int]),
    "kqr_pcg_solve": (C.c_int, [_P, _I64, _I64, C.c_int, C.c_double, _P, C.c_int, _I64, _P, _I64, _I64,
                                C.c_double, _P, _P, C.c_double, C.c_int, _P, _P, _P, _P]),
    "kqr_ssn_gradient": (C.c_int, [_I64, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double,
                                   C.c_double, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "kqr_kkt_residuals": (C.c_int, [_I64, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double, C.c_int,
                                    _P, _P, _P, _P, _P, _P, _P]),
    "kqr_fit": (C.c_int, [_P, _P, _I64, _I64, C.c_double, C.c_double, C.c_int, C.c_double,
                          C.POINTER(KqrOptions), _P, _P, C.POINTER(KqrInfo), _P]),
    "kqr_fit_multi_tau": (C.c_int, [_P, _P, _I64, _I64, _P, C.c_int, C.c_double, C.c_int, C.c_double,
                                    C.POINTER(KqrOptions), _P, _P, _P, _P, _P]),
    "kqr_fit_path": (C.c_int, [_P, _P, _I64, _I64, C.c_double, _P, C.c_int, C.c_int, C.c_double,
                               C.POINTER(KqrOptions), _P, _P, _P, _P, _P]),
    "kqr_packed_bytes": (C.c_int64, [_I64, C.c_int]),
    "kqr_kernel_build_packed": (C.c_int, [_P, _I64, _I64, C.c_int, C.c_double, C.c_int, _P, _P]),
    "kqr_kernel_apply_packed": (C.c_int, [_P, C.c_int, _I64, _P, _P, C.c_int, _P]),
    "kqr_autotune_packed": (C.c_int, [_P, C.c_int, _I64, C.c_int, C.c_int, C.c_char_p, _I64, _P]),
    "kqr_set_packed_shape": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int]),
    "kqr_set_otf_symmetric_limit": (C.c_int, [C.c_int64]),
    "kqr_set_otf_shape": (C.c_int, [C.c_int, C.c_int64]),
    "kqr_kernel_apply_static": (C.c_int, [_P, C.c_int, _I64, _I64, _P, _I64, _P, _I64, C.c_int, _P]),
    "kqr_autotune_otf": (C.c_int, [_P, _I64, _I64, C.c_int, C.c_double, C.c_int, C.c_int, C.c_char_p, _I64, _P]),
    "kqr_tune_save": (C.c_int, [C.c_char_p, C.POINTER(C.c_int)]),
    "kqr_tune_load": (C.c_int, [C.c_char_p, C.POINTER(C.c_int)]),
    "kqr_fit_batch": (C.c_int, [C.c_int, _P, _P, _P, _I64, _P, _P, C.c_int, _P, C.POINTER(KqrOptions), _P, _P, _P,
                                _P, _P]),
    "kqr_fit_grad": (C.c_int, [_P, _P, _I64, _I64, C.c_double, C.c_double, C.c_int, C.c_double, _P, _P, _I64,
                               C.POINTER(KqrOptions), _P, _P, _P, _P, _P, _P, C.POINTER(KqrInfo), _P]),
}


class KqrError(RuntimeError):
    def __init__(self, status: int, func: str, msg: str):
        super().__init__(f"{func}: status {status} ({status_string(status)}): {msg}")
        self.status = status


def lib_path() -> str:
    return _LIB_PATH


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib_handle
    with _lib_lock:
        if _lib_handle is None:
            # torch ships its own HIP runtime (same soname); loading torch first
            # makes libkqr bind to that runtime, so one runtime owns the device
            # memory and streams that are passed across.
            import torch  # noqa: F401
            if not os.path.exists(_LIB_PATH):
                raise RuntimeError(
                    f"libkqr.so not found at {_LIB_PATH}; build it with "
                    "`python -m paper_2510_07929_amd.build` (no CPU fallback exists)")
            h = C.CDLL(_LIB_PATH)
            for name, (res, args) in _SIGS.items():
                fn = getattr(h, name)
                fn.restype = res
                fn.argtypes = args
            _lib_handle = h
    return _lib_handle


def status_string(s: int) -> str:
    return lib().kqr_status_string(int(s)).decode()


def last_error() -> str:
    return lib().kqr_last_error().decode()


def _check(status: int, func: str, allow=(KQR_OK,)):
    if status not in allow:
        raise KqrError(status, func, last_error())
    return status


# ----------------------------------------------------------------------- marshalling helpers
def _torch():
    import torch

    return torch


def _stream(stream=None):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dev(t, dtype, name, ndim=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if ndim is not None and t.dim() != ndim:
        raise ValueError(f"{name} must have {ndim} dims")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return C.c_void_p(t.data_ptr())


def _kernel_id(kernel):
    return KERNELS[kernel] if isinstance(kernel, str) else int(kernel)


def _kdtype_id(kd):
    return KDTYPES[kd] if isinstance(kd, str) else int(kd)


def padded_ld(n: int) -> int:
    """Leading dimension used for materialised K (multiple of 64 elements)."""
    return (int(n) + 63) // 64 * 64


# ----------------------------------------------------------------------- entry points
def kqr_default_options(**overrides) -> KqrOptions:
    o = KqrOptions()
    _check(lib().kqr_default_options(C.byref(o)), "kqr_default_options")
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise AttributeError(f"kqr_options has no field {k!r}")
        setattr(o, k, v)
    return o


def kqr_device_count() -> int:
    return int(lib().kqr_device_count())


def kqr_set_batch_threads(threads: int) -> None:
    """Host threads of the batched fits (1..16; 0 = default)."""
    _check(lib().kqr_set_batch_threads(int(threads)), "kqr_set_batch_threads")


def kqr_test_core_breakdowns(skip: int, count: int) -> None:
    """Test hook: after `skip` more Woodbury core factorisations, the next
    `count` report a breakdown (kqr_info.core_retries counts the retries)."""
    _check(lib().kqr_test_core_breakdowns(int(skip), int(count)), "kqr_test_core_breakdowns")


def kqr_test_batch_steps(on: bool) -> None:
    """Test hook: whether kqr_fit_batch runs its problems' PCG iterations
    (vector and preconditioner kernels) in batched launches (default True)."""
    _check(lib().kqr_test_batch_steps(1 if on else 0), "kqr_test_batch_steps")


def kqr_kernel_build(X, kernel, gamma, k_dtype="fp32", K=None, stream=None):
    """Materialise K (n x ld, ld = padded_ld(n)) on the GPU; returns K."""
    torch = _torch()
    n, p = X.shape
    ld = padded_ld(n) if K is None else K.shape[1]
    kd = _kdtype_id(k_dtype)
    tdt = torch.float32 if kd == KQR_FP32 else torch.bfloat16
    if K is None:
        K = torch.empty((n, ld), dtype=tdt, device=X.device)
    _check(lib().kqr_kernel_build(_dev(X, torch.float32, "X", 2), n, p, _kernel_id(kernel), float(gamma), kd,
                                  _dev(K, tdt, "K", 2), ld, _stream(stream)), "kqr_kernel_build")
    return K


def kqr_packed_bytes(n, k_dtype="fp32"):
    return int(lib().kqr_packed_bytes(int(n), _kdtype_id(k_dtype)))


def kqr_kernel_build_packed(X, kernel, gamma, k_dtype="fp32", stream=None):
    """Materialise K in the symmetric packed layout (upper-triangle tiles); returns a flat GPU tensor."""
    torch = _torch()
    n, p = X.shape
    kd = _kdtype_id(k_dtype)
    tdt = torch.float32 if kd == KQR_FP32 else torch.bfloat16
    nb = kqr_packed_bytes(n, kd)
    K = torch.empty(nb // (4 if kd == KQR_FP32 else 2), dtype=tdt, device=X.device)
    _check(lib().kqr_kernel_build_packed(_dev(X, torch.float32, "X", 2), n, p, _kernel_id(kernel), float(gamma), kd,
                                         _dev(K, tdt, "K", 1), _stream(stream)), "kqr_kernel_build_packed")
    return K


def kqr_kernel_apply_packed(v, K, n, mode=KQR_APPLY_FAST, u=None, stream=None):
    """u = K v for K from kqr_kernel_build_packed and v (n,) float64 on the GPU."""
    torch = _torch()
    kd = KQR_FP32 if K.dtype == torch.float32 else KQR_BF16
    if u is None:
        u = torch.empty(n, dtype=torch.float64, device=v.device)
    _check(lib().kqr_kernel_apply_packed(_dev(K, K.dtype, "K", 1), kd, int(n), _dev(v, torch.float64, "v", 1),
                                         _dev(u, torch.float64, "u", 1), int(mode), _stream(stream)),
           "kqr_kernel_apply_packed")
    return u


def kqr_autotune_packed(K, n, mode=KQR_APPLY_FAST, reps=5, stream=None):
    """Sweep the packed K-apply shapes on K and install the fastest; returns the report dict."""
    torch = _torch()
    kd = KQR_FP32 if K.dtype == torch.float32 else KQR_BF16
    buf = C.create_string_buffer(8192)
    _check(lib().kqr_autotune_packed(_dev(K, K.dtype, "K", 1), kd, int(n), int(mode), int(reps), buf, 8192,
                                     _stream(stream)), "kqr_autotune_packed")
    return json.loads(buf.value.decode())


def kqr_set_packed_shape(k_dtype, mode, map, strip):
    _check(lib().kqr_set_packed_shape(_kdtype_id(k_dtype), int(mode), int(map), int(strip)), "kqr_set_packed_shape")


def kqr_set_otf_symmetric_limit(nbytes):
    """Bound the partial-sum buffer of the symmetric on-the-fly applies (bytes); larger n stream all pairs."""
    _check(lib().kqr_set_otf_symmetric_limit(int(nbytes)), "kqr_set_otf_symmetric_limit")


def kqr_set_otf_shape(strip=0, wgs=0):
    """Launch shape of the on-the-fly applies (strip: tiles per workgroup of the symmetric
    square applies, 0 = by size; wgs: target workgroups of sliced launches, 0 = 8192)."""
    _check(lib().kqr_set_otf_shape(int(strip), int(wgs)), "kqr_set_otf_shape")


def kqr_kernel_apply(V, X=None, kernel="rbf", gamma=1.0, K=None, mode=KQR_APPLY_FAST, U=None, stream=None):
    """U = K V for V (n,) or (n, m) float64 on the GPU; K materialised or None (on the fly)."""
    torch = _torch()
    vec = V.dim() == 1
    V2 = V.reshape(-1, 1) if vec else V
    n, m = V2.shape
    if U is None:
        U = torch.empty((n, m), dtype=torch.float64, device=V.device)
    U2 = U.reshape(n, m)
    if K is not None:
        kd = KQR_FP32 if K.dtype == torch.float32 else KQR_BF16
        kptr, ld = _dev(K, K.dtype, "K", 2), K.shape[1]
    else:
        kd, kptr, ld = KQR_FP32, None, 0
    xptr = _dev(X, torch.float32, "X", 2) if X is not None else None
    p = X.shape[1] if X is not None else 0
    _check(lib().kqr_kernel_apply(xptr, n, p, _kernel_id(kernel), float(gamma), kptr, kd, ld,
                                  _dev(V2, torch.float64, "V"), m, m, _dev(U2, torch.float64, "U"), m,
                                  int(mode), _stream(stream)), "kqr_kernel_apply")
    return U2.reshape(-1) if vec else U2


def kqr_kernel_apply_static(v, K, mode=KQR_APPLY_FAST, u=None, stream=None):
    """u = K v for a materialised K (from kqr_kernel_build) without any allocation in the
    library: v and u are (n,) float64 GPU tensors, any stride."""
    torch = _torch()
    n = v.shape[0]
    if u is None:
        u = torch.empty(n, dtype=torch.float64, device=v.device)
    if v.dtype != torch.float64 or u.dtype != torch.float64 or not (v.is_cuda and u.is_cuda) or v.dim() != 1:
        raise TypeError("v and u must be 1-D float64 GPU tensors")
    kd = KQR_FP32 if K.dtype == torch.float32 else KQR_BF16
    _check(lib().kqr_kernel_apply_static(_dev(K, K.dtype, "K", 2), kd, n, K.shape[1], C.c_void_p(v.data_ptr()),
                                         v.stride(0), C.c_void_p(u.data_ptr()), u.stride(0), int(mode),
                                         _stream(stream)), "kqr_kernel_apply_static")
    return u


def kqr_predict(Xtrain, alpha, beta, lam, kernel, gamma, Xnew, stream=None):
    torch = _torch()
    n, p = Xtrain.shape
    m = Xnew.shape[0]
    f = torch.empty(m, dtype=torch.float64, device=Xnew.device)
    _check(lib().kqr_predict(_dev(Xtrain, torch.float32, "Xtrain", 2), n, p, _dev(alpha, torch.float64, "alpha", 1),
                             float(beta), float(lam), _kernel_id(kernel), float(gamma),
                             _dev(Xnew, torch.float32, "Xnew", 2), m, _dev(f, torch.float64, "f", 1),
                             _stream(stream)), "kqr_predict")
    return f


def kqr_rpcholesky(rank, uniforms, X=None, kernel="rbf", gamma=1.0, K=None, n=None, stream=None):
    """Returns (F (n x ldf float32 GPU tensor, first rank_out columns valid), pivots (np.int64), rank_out)."""
    torch = _torch()
    if n is None:
        n = X.shape[0] if X is not None else K.shape[0]
    rank = int(rank)
    ldf = (min(rank, n) + 3) // 4 * 4
    dev = X.device if X is not None else K.device
    F = torch.empty((n, ldf), dtype=torch.float32, device=dev)
    u = np.ascontiguousarray(np.asarray(uniforms, dtype=np.float64))
    if u.size < min(rank, n):
        raise ValueError("need at least rank uniforms")
    piv = np.zeros(rank, dtype=np.int64)
    rout = C.c_int64(0)
    if K is not None:
        kd = KQR_FP32 if K.dtype == torch.float32 else KQR_BF16
        kptr, ld = _dev(K, K.dtype, "K", 2), K.shape[1]
    else:
        kd, kptr, ld = KQR_FP32, None, 0
    xptr = _dev(X, torch.float32, "X", 2) if X is not None else None
    p = X.shape[1] if X is not None else 0
    _check(lib().kqr_rpcholesky(xptr, n, p, _kernel_id(kernel), float(gamma), kptr, kd, ld, rank,
                                u.ctypes.data_as(C.c_void_p), _dev(F, torch.float32, "F", 2), ldf,
                                piv.ctypes.data_as(C.c_void_p), C.byref(rout), _stream(stream)), "kqr_rpcholesky")
    r = int(rout.value)
    return F, piv[:r].copy(), r


def kqr_adaptive_rank(F0, r0, xi=1e-3, stream=None):
    """Section 3 rank rule on the first r0 columns of F0 (GPU float32 n x ldf); returns (r, lambda_1)."""
    torch = _torch()
    n, ldf = F0.shape
    r = C.c_int64(0)
    l1 = C.c_double(0.0)
    _check(lib().kqr_adaptive_rank(_dev(F0, torch.float32, "F0", 2), n, int(r0), ldf, float(xi), C.byref(r),
                                   C.byref(l1), _stream(stream)), "kqr_adaptive_rank")
    return int(r.value), float(l1.value)


def kqr_autotune_apply(K, mode=KQR_APPLY_FAST, reps=5, stream=None):
    """Sweep the K-apply tile shapes on K (GPU, from kqr_kernel_build); returns the JSON report (dict)."""
    torch = _torch()
    kd = KQR_FP32 if K.dtype == torch.float32 else KQR_BF16
    buf = C.create_string_buffer(1 << 16)
    _check(lib().kqr_autotune_apply(_dev(K, K.dtype, "K", 2), kd, K.shape[0], K.shape[1], int(mode), int(reps), buf,
                                    len(buf), _stream(stream)), "kqr_autotune_apply")
    return json.loads(buf.value.decode())


def kqr_autotune_otf(X, kernel, gamma, mode=KQR_APPLY_FAST, reps=3, stream=None):
    """Sweep the on-the-fly apply's strip (square, symmetric form) and slice target (rectangle) on X;
    installs the fastest; returns the JSON report (dict)."""
    torch = _torch()
    n, p = X.shape
    buf = C.create_string_buffer(1 << 14)
    _check(lib().kqr_autotune_otf(_dev(X, torch.float32, "X", 2), n, p, _kernel_id(kernel), float(gamma), int(mode),
                                  int(reps), buf, len(buf), _stream(stream)), "kqr_autotune_otf")
    return json.loads(buf.value.decode())


def kqr_tune_save(path) -> int:
    """Write every launch shape installed in this process to a JSON file keyed by the GPU architecture."""
    c = C.c_int(0)
    _check(lib().kqr_tune_save(os.fsencode(path), C.byref(c)), "kqr_tune_save")
    return int(c.value)


def kqr_tune_load(path) -> int:
    """Install the launch shapes a file records for this GPU's architecture; returns how many."""
    c = C.c_int(0)
    _check(lib().kqr_tune_load(os.fsencode(path), C.byref(c)), "kqr_tune_load")
    return int(c.value)


def kqr_set_apply_shape(k_dtype, mode, n, rows, unroll, segs):
    _check(lib().kqr_set_apply_shape(_kdtype_id(k_dtype), int(mode), int(n), int(rows), int(unroll), int(segs)),
           "kqr_set_apply_shape")


def kqr_set_kv_shape(k_dtype, n, nld, prefetch, segs):
    _check(lib().kqr_set_kv_shape(_kdtype_id(k_dtype), int(n), int(nld), int(prefetch), int(segs)),
           "kqr_set_kv_shape")


def kqr_woodbury_apply(F, r, c, Ldiag, w, stream=None):
    torch = _torch()
    n = Ldiag.shape[0]
    out = torch.empty_like(w)
    fptr = _dev(F, torch.float32, "F", 2) if r > 0 else None
    ldf = F.shape[1] if r > 0 else 0
    _check(lib().kqr_woodbury_apply(fptr, n, int(r), ldf, float(c), _dev(Ldiag, torch.float64, "Ldiag", 1),
                                    _dev(w, torch.float64, "w", 1), _dev(out, torch.float64, "out", 1),
                                    _stream(stream)), "kqr_woodbury_apply")
    return out


def kqr_pcg_solve(X, kernel, gamma, c, Ldiag, b, tol, maxit, K=None, F=None, r=0, x0=None, stream=None):
    torch = _torch()
    n, p = X.shape
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    it = C.c_int(0)
    res = C.c_double(0.0)
    if K is not None:
        kd = KQR_FP32 if K.dtype == torch.float32 else KQR_BF16
        kptr, ld = _dev(K, K.dtype, "K", 2), K.shape[1]
    else:
        kd, kptr, ld = KQR_FP32, None, 0
    fptr = _dev(F, torch.float32, "F", 2) if r > 0 else None
    ldf = F.shape[1] if r > 0 else 0
    _check(lib().kqr_pcg_solve(_dev(X, torch.float32, "X", 2), n, p, _kernel_id(kernel), float(gamma), kptr, kd, ld,
                               fptr, int(r), ldf, float(c), _dev(Ldiag, torch.float64, "Ldiag", 1),
                               _dev(b, torch.float64, "b", 1), float(tol), int(maxit), _dev(x, torch.float64, "x", 1),
                               C.byref(it), C.byref(res), _stream(stream)), "kqr_pcg_solve")
    return x, int(it.value), float(res.value)


def kqr_ssn_gradient(tau, lam, beta, sigma, alpha, Kalpha, y, z, tau1=0.1, tau2=0.1, eps_floor=1e-12, stream=None):
    torch = _torch()
    n = alpha.shape[0]
    grad = torch.empty_like(alpha)
    L = torch.empty_like(alpha)
    rhs = torch.empty_like(alpha)
    S = torch.empty(n, dtype=torch.uint8, device=alpha.device)
    gn, et = C.c_double(0.0), C.c_double(0.0)
    f64 = torch.float64
    _check(lib().kqr_ssn_gradient(n, float(tau), float(lam), float(beta), float(sigma), float(tau1), float(tau2),
                                  float(eps_floor), _dev(alpha, f64, "alpha", 1), _dev(Kalpha, f64, "Kalpha", 1),
                                  _dev(y, f64, "y", 1), _dev(z, f64, "z", 1), _dev(grad, f64, "grad", 1),
                                  _dev(S, torch.uint8, "S", 1), _dev(L, f64, "Ldiag", 1), _dev(rhs, f64, "rhs", 1),
                                  C.byref(gn), C.byref(et), _stream(stream)), "kqr_ssn_gradient")
    return dict(grad=grad, S=S, Ldiag=L, rhs=rhs, gnorm=float(gn.value), eps_t=float(et.value))


def kqr_kkt_residuals(tau, lam, beta, alpha, Kalpha, y, z, v, sigma=1.0, step=1.0, update=False, stream=None):
    """Section 4 measures at (alpha, v, beta, z) with the supplied K alpha (update: the multiplier
    step first, z and v overwritten).  Returns a dict of eta_p, eta_d, eta_c, eta_kkt, eta_gap, obj_p, obj_d."""
    torch = _torch()
    n = alpha.shape[0]
    out = (C.c_double * 7)()
    f64 = torch.float64
    _check(lib().kqr_kkt_residuals(n, float(tau), float(lam), float(beta), float(sigma), float(step), int(bool(update)),
                                   _dev(alpha, f64, "alpha", 1), _dev(Kalpha, f64, "Kalpha", 1), _dev(y, f64, "y", 1),
                                   _dev(z, f64, "z", 1), _dev(v, f64, "v", 1), out, _stream(stream)),
           "kqr_kkt_residuals")
    keys = ("eta_p", "eta_d", "eta_c", "eta_kkt", "eta_gap", "obj_p", "obj_d")
    return {k: float(out[i]) for i, k in enumerate(keys)}


def kqr_fit(X, y, tau, lam, kernel="rbf", gamma=1.0, options: KqrOptions | None = None, uniforms=None,
            stream=None, trace: int = 0, out_vz: bool = False, warm=None, **overrides):
    """PALM-KQR fit on the GPU.  Returns (alpha (GPU float64), beta, info dict, status).

    ``trace`` > 0 records up to that many outer iterations; info["trace"] is
    then an array of rows (phase, iteration, max(eta_kkt, eta_gap), seconds).
    ``out_vz``: info["v"], info["z"] hold the final v and z (GPU float64), the
    iterate the Section 4 measures in info were taken at.
    ``warm``: (alpha, v, z, beta, sigma) of an earlier fit of the same problem
    (GPU float64 vectors, floats): Phase II resumes from it, Phase I is skipped."""
    torch = _torch()
    n, p = X.shape
    o = options if options is not None else kqr_default_options()
    for k, v in overrides.items():
        setattr(o, k, v)
    warm_keep = None
    if warm is not None:
        wa, wv, wz, wb, ws = warm
        warm_keep = (_dev(wa, torch.float64, "warm alpha", 1), _dev(wv, torch.float64, "warm v", 1),
                     _dev(wz, torch.float64, "warm z", 1))
        if any(t.shape[0] != n for t in (wa, wv, wz)):
            raise ValueError("warm start vectors must have n entries")
        o.warm_alpha, o.warm_v, o.warm_z = (p_.value for p_ in warm_keep)
        o.warm_beta, o.warm_sigma = float(wb), float(ws)
    vz = None
    if out_vz:
        vz = torch.empty((2, n), dtype=torch.float64, device=X.device)
        o.v_out, o.z_out = vz[0].data_ptr(), vz[1].data_ptr()
    keep = None
    if uniforms is not None:
        keep = np.ascontiguousarray(np.asarray(uniforms, dtype=np.float64))
        o.pivot_uniforms = keep.ctypes.data_as(C.POINTER(C.c_double))
    tbuf = None
    if trace > 0:
        tbuf = np.zeros((int(trace), 4))
        o.trace = tbuf.ctypes.data_as(C.POINTER(C.c_double))
        o.trace_cap = int(trace)
    alpha = torch.empty(n, dtype=torch.float64, device=X.device)
    beta = C.c_double(0.0)
    info = KqrInfo()
    st = lib().kqr_fit(_dev(X, torch.float32, "X", 2), _dev(y, torch.float64, "y", 1), n, p, float(tau), float(lam),
                       _kernel_id(kernel), float(gamma), C.byref(o), _dev(alpha, torch.float64, "alpha", 1),
                       C.byref(beta), C.byref(info), _stream(stream))
    _check(st, "kqr_fit", allow=(KQR_OK, KQR_NOT_CONVERGED))
    del keep
    out = info.as_dict()
    if tbuf is not None:
        out["trace"] = tbuf[: info.trace_len].copy()
        o.trace, o.trace_cap = None, 0
    if vz is not None:
        out["v"], out["z"] = vz[0], vz[1]
        o.v_out, o.z_out = None, None
    if warm_keep is not None:
        o.warm_alpha = o.warm_v = o.warm_z = None
    return alpha, float(beta.value), out, st


def _options(options, uniforms, overrides):
    o = options if options is not None else kqr_default_options()
    for k, v in overrides.items():
        setattr(o, k, v)
    keep = None
    if uniforms is not None:
        keep = np.ascontiguousarray(np.asarray(uniforms, dtype=np.float64))
        o.pivot_uniforms = keep.ctypes.data_as(C.POINTER(C.c_double))
    return o, keep


def kqr_fit_multi_tau(X, y, taus, lam, kernel="rbf", gamma=1.0, options: KqrOptions | None = None, uniforms=None,
                      stream=None, **overrides):
    """Joint fit of several quantile levels.  Returns (alpha (ntau x n GPU), betas, infos, statuses)."""
    torch = _torch()
    n, p = X.shape
    taus = np.ascontiguousarray(np.asarray(taus, dtype=np.float64))
    m = int(taus.size)
    o, keep = _options(options, uniforms, overrides)
    alpha = torch.empty((m, n), dtype=torch.float64, device=X.device)
    beta = np.zeros(m)
    info = (KqrInfo * m)()
    status = np.zeros(m, dtype=np.int32)
    _check(lib().kqr_fit_multi_tau(_dev(X, torch.float32, "X", 2), _dev(y, torch.float64, "y", 1), n, p,
                                   taus.ctypes.data_as(C.c_void_p), m, float(lam), _kernel_id(kernel), float(gamma),
                                   C.byref(o), _dev(alpha, torch.float64, "alpha", 2), beta.ctypes.data_as(C.c_void_p),
                                   info, status.ctypes.data_as(C.c_void_p), _stream(stream)), "kqr_fit_multi_tau")
    del keep
    return alpha, beta, [info[i].as_dict() for i in range(m)], status.tolist()


def kqr_fit_path(X, y, tau, lams, kernel="rbf", gamma=1.0, options: KqrOptions | None = None, uniforms=None,
                 stream=None, **overrides):
    """Fits for a sequence of lambda values on one K.  Returns (alpha (nlam x n GPU), betas, infos, statuses)."""
    torch = _torch()
    n, p = X.shape
    lams = np.ascontiguousarray(np.asarray(lams, dtype=np.float64))
    m = int(lams.size)
    o, keep = _options(options, uniforms, overrides)
    alpha = torch.empty((m, n), dtype=torch.float64, device=X.device)
    beta = np.zeros(m)
    info = (KqrInfo * m)()
    status = np.zeros(m, dtype=np.int32)
    _check(lib().kqr_fit_path(_dev(X, torch.float32, "X", 2), _dev(y, torch.float64, "y", 1), n, p, float(tau),
                              lams.ctypes.data_as(C.c_void_p), m, _kernel_id(kernel), float(gamma), C.byref(o),
                              _dev(alpha, torch.float64, "alpha", 2), beta.ctypes.data_as(C.c_void_p), info,
                              status.ctypes.data_as(C.c_void_p), _stream(stream)), "kqr_fit_path")
    del keep
    return alpha, beta, [info[i].as_dict() for i in range(m)], status.tolist()


def kqr_fit_batch(Xs, ys, taus, lams, gammas, kernel="rbf", options: KqrOptions | None = None, uniforms=None,
                  stream=None, **overrides):
    """Independent fits in one batch.  Returns (alphas (list of GPU tensors), betas, infos, statuses)."""
    torch = _torch()
    k = len(Xs)
    p = Xs[0].shape[1]
    ns = np.array([x.shape[0] for x in Xs], dtype=np.int64)
    alphas = [torch.empty(int(ni), dtype=torch.float64, device=Xs[0].device) for ni in ns]
    xp = (C.c_void_p * k)(*[_dev(x, torch.float32, "X", 2).value for x in Xs])
    yp = (C.c_void_p * k)(*[_dev(y, torch.float64, "y", 1).value for y in ys])
    ap = (C.c_void_p * k)(*[_dev(a, torch.float64, "alpha", 1).value for a in alphas])
    taus = np.ascontiguousarray(np.asarray(taus, dtype=np.float64))
    lams = np.ascontiguousarray(np.asarray(lams, dtype=np.float64))
    gammas = np.ascontiguousarray(np.asarray(gammas, dtype=np.float64))
    o, keep = _options(options, uniforms, overrides)
    beta = np.zeros(k)
    info = (KqrInfo * k)()
    status = np.zeros(k, dtype=np.int32)
    _check(lib().kqr_fit_batch(k, xp, yp, ns.ctypes.data_as(C.c_void_p), p, taus.ctypes.data_as(C.c_void_p),
                               lams.ctypes.data_as(C.c_void_p), _kernel_id(kernel), gammas.ctypes.data_as(C.c_void_p),
                               C.byref(o), ap, beta.ctypes.data_as(C.c_void_p), info,
                               status.ctypes.data_as(C.c_void_p), _stream(stream)), "kqr_fit_batch")
    del keep
    return alphas, beta, [info[i].as_dict() for i in range(k)], status.tolist()


def kqr_fit_grad(X, y, tau, lam, kernel, gamma, Xval, yval, options: KqrOptions | None = None, uniforms=None,
                 stream=None, **overrides):
    """Fit, then the implicit gradient of the validation check loss.

    Returns (alpha (GPU float64), beta, J, (dJ/dlog gamma, dJ/dlog lambda), |E|, polished, info, status).
    """
    torch = _torch()
    n, p = X.shape
    nv = Xval.shape[0]
    if Xval.shape[1] != p:
        raise ValueError("Xval must have the columns of X")
    o, keep = _options(options, uniforms, overrides)
    alpha = torch.empty(n, dtype=torch.float64, device=X.device)
    beta = C.c_double(0.0)
    loss = C.c_double(0.0)
    grad = (C.c_double * 2)()
    m = C.c_int64(0)
    pol = C.c_int(0)
    info = KqrInfo()
    st = lib().kqr_fit_grad(_dev(X, torch.float32, "X", 2), _dev(y, torch.float64, "y", 1), n, p, float(tau),
                            float(lam), _kernel_id(kernel), float(gamma), _dev(Xval, torch.float32, "Xval", 2),
                            _dev(yval, torch.float64, "yval", 1), nv, C.byref(o), _dev(alpha, torch.float64, "alpha", 1),
                            C.byref(beta), C.byref(loss), grad, C.byref(m), C.byref(pol), C.byref(info),
                            _stream(stream))
    _check(st, "kqr_fit_grad", allow=(KQR_OK, KQR_NOT_CONVERGED))
    del keep
    return (alpha, float(beta.value), float(loss.value), (float(grad[0]), float(grad[1])), int(m.value),
            bool(pol.value), info.as_dict(), st)


def _make_fit_loss():
    torch = _torch()

    class KQRFitLoss(torch.autograd.Function):
        """(log gamma, log lambda) -> validation check loss of the KQR fit.

        Forward fits on the GPU and computes the implicit gradient in the same
        call; backward scales it by the incoming gradient.
        """

        @staticmethod
        def forward(ctx, log_gamma, log_lambda, X, y, Xval, yval, tau, kernel, fit_kwargs):
            gam = float(torch.exp(log_gamma.detach().double()).item())
            lam = float(torch.exp(log_lambda.detach().double()).item())
            out = kqr_fit_grad(X, y, tau, lam, kernel, gam, Xval, yval, **(fit_kwargs or {}))
            ctx.grads = out[3]
            return torch.tensor(out[2], dtype=torch.float64)

        @staticmethod
        def backward(ctx, gout):
            dg, dl = ctx.grads
            gout = gout.double()
            return gout * dg, gout * dl, None, None, None, None, None, None, None

    return KQRFitLoss


_FIT_LOSS = None


def kqr_validation_loss(log_gamma, log_lambda, X, y, Xval, yval, tau, kernel="rbf", **fit_kwargs):
    """Differentiable validation loss: autograd Function over (log gamma, log lambda)."""
    global _FIT_LOSS
    if _FIT_LOSS is None:
        _FIT_LOSS = _make_fit_loss()
    return _FIT_LOSS.apply(log_gamma, log_lambda, X, y, Xval, yval, tau, kernel, fit_kwargs)


def default_rank(n: int) -> int:
    return min(int(math.ceil(math.sqrt(n))), n, 1023)
