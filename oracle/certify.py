"""FP64 certificate of a returned (alpha, beta) at any n.

TEST INFRASTRUCTURE, NOT PRODUCT CODE.

Two method-independent checks of an approximate KQR solution, each costing
one pass of FP64 kernel products (so they run at sizes whose FP64 K does not
fit in memory):

* the Section 4 measures with the exact FP64 kernel, at the iterate
  (alpha, v, beta, z) an algorithm returned, and at (alpha, Pi_B(alpha), beta,
  y - beta 1 - K alpha / lambda), where eta_p vanishes by the choice of z,
  eta_d measures 1^T alpha and the distance of alpha to B, eta_c the
  complementarity of (v, z), and eta_gap the duality gap;
* a weak-duality sandwich for the optimal value.  alpha~ is alpha projected
  onto {a in B : 1^T a = 0} (clip(alpha - t, tau - 1, tau) with t found by
  bisection), so the dual objective of (1.3) at alpha~ is a lower bound of
  the optimal value, and the primal objective of (1.2) at theta = alpha~ with
  beta~ the sample tau-quantile of y - K alpha~ / lambda (the minimiser of the
  check loss over the intercept) an upper bound.  Any returned point's
  primal objective is at least the optimum, so
      0 <= obj_P(alpha, beta) - OPT <= obj_P(alpha, beta) - obj_D(alpha~),
  which bounds its relative objective error without knowing the optimum.
  The bisection leaves |1^T alpha~| at rounding level; the lower bound then
  holds up to |1^T alpha~| |beta*|, folded in with |beta~| + 1 for |beta*|.

FP64 kernel products come from oracle/kapply.c (direct differences, plain
FP64 sums, rows over OpenMP threads).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import problem

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        from . import build_c

        if not os.path.exists(build_c.LIB) or os.path.getmtime(build_c.LIB) < os.path.getmtime(build_c.SRC):
            build_c.build()
        h = C.CDLL(build_c.LIB)
        h.kqr_oracle_kernel_apply.restype = C.c_int
        h.kqr_oracle_kernel_apply.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_int64, C.c_int,
                                              C.c_double, C.c_void_p, C.c_int64, C.c_void_p]
        _LIB = h
    return _LIB


def kernel_apply(X, V, kind: str, gamma: float, Xrows=None, progress=None) -> np.ndarray:
    """U = K(Xrows, X) V in FP64 (Xrows defaults to X); V (n,) or (n, m), m <= 16.

    ``progress(rows_done, rows)``, when given, is called after each of 16 row
    chunks (every row is an independent sum, so chunking changes nothing)."""
    kid = {"rbf": 0, "laplacian": 1}[kind]
    X = np.ascontiguousarray(X, dtype=np.float64)
    Xr = X if Xrows is None else np.ascontiguousarray(Xrows, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    vec = V.ndim == 1
    V2 = np.ascontiguousarray(V.reshape(V.shape[0], -1))
    n, p = X.shape
    if V2.shape[0] != n or Xr.shape[1] != p or V2.shape[1] > 16:
        raise ValueError("shapes do not match")
    m = Xr.shape[0]
    U = np.empty((m, V2.shape[1]))
    bounds = np.linspace(0, m, 17 if progress else 2).astype(np.int64)
    for r0, r1 in zip(bounds[:-1], bounds[1:]):
        rc = _lib().kqr_oracle_kernel_apply(X.ctypes.data, n, p, Xr[r0:r1].ctypes.data, int(r1 - r0), kid,
                                           float(gamma), V2.ctypes.data, V2.shape[1], U[r0:r1].ctypes.data)
        if rc != 0:
            raise ValueError("kqr_oracle_kernel_apply rejected its arguments")
        if progress:
            progress(int(r1), m)
    return U[:, 0] if vec else U


def project_feasible(alpha, tau: float, iters: int = 200):
    """clip(alpha - t, tau - 1, tau) with 1^T(...) = 0, t by bisection (the sum
    is non-increasing in t; t = min(alpha) - 1 gives n tau > 0, t = max(alpha) + 1
    gives n (tau - 1) < 0)."""
    lo, hi = float(np.min(alpha)) - 1.0, float(np.max(alpha)) + 1.0
    for _ in range(iters):
        t = 0.5 * (lo + hi)
        if np.clip(alpha - t, tau - 1.0, tau).sum() > 0.0:
            lo = t
        else:
            hi = t
    return np.clip(alpha - 0.5 * (lo + hi), tau - 1.0, tau)


def certificate(X, y, tau: float, lam: float, kind: str, gamma: float, alpha, beta: float, v=None, z=None,
                extra=None, progress=None) -> dict:
    """Section 4 measures and the duality sandwich of (alpha, beta), FP64.

    With ``v`` and ``z`` (the iterate an algorithm returned with alpha and
    beta) the measures eta_* are taken at (alpha, v, beta, z); the measures
    res_eta_* are always taken at (alpha, Pi_B(alpha), beta, y - beta 1 -
    K alpha / lambda), where eta_p vanishes by construction.
    ``extra`` (n,) or (n, k), k <= 14: further vectors multiplied by K in the
    same pass (returned as "K_extra")."""
    alpha = np.asarray(alpha, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    at = project_feasible(alpha, tau)
    cols = [alpha, at]
    if extra is not None:
        e = np.asarray(extra, dtype=np.float64)
        cols += [e] if e.ndim == 1 else [e[:, j] for j in range(e.shape[1])]
    KV = kernel_apply(X, np.stack(cols, axis=1), kind, gamma, progress=progress)
    Ka, Kat = KV[:, 0], KV[:, 1]
    zr = y - beta - Ka / lam
    res = problem.kkt(alpha, problem.proj_box(alpha, tau), beta, zr, Ka, y, lam, tau)
    if v is not None and z is not None:
        meas = problem.kkt(alpha, np.asarray(v, dtype=np.float64), beta, np.asarray(z, dtype=np.float64), Ka, y,
                           lam, tau)
    else:
        meas = dict(res)
    obj_gpu = problem.primal_objective(zr, alpha, Ka, lam, tau)
    r = y - Kat / lam
    bt = float(np.quantile(r, tau, method="inverted_cdf"))
    upper = problem.primal_objective(r - bt, at, Kat, lam, tau)
    s = float(at.sum())
    lower = problem.dual_objective(at, Kat, y, lam) - abs(s) * (abs(bt) + 1.0)
    out = dict(meas)
    out.update({"res_" + k: val for k, val in res.items()})
    out.update(
        obj_p_returned=obj_gpu,
        lower=lower,
        upper=upper,
        sum_alpha_tilde=s,
        rel_obj_err_bound=max(obj_gpu - lower, 0.0) / (1.0 + abs(lower)),
        sandwich_rel_width=max(upper - lower, 0.0) / (1.0 + abs(lower)),
        n_interior=int(np.sum((alpha > tau - 1.0) & (alpha < tau))),
    )
    if extra is not None:
        out["K_extra"] = KV[:, 2:]
    return out


def certificate_levels(X, y, taus, lam: float, kind: str, gamma: float, alphas, betas, progress=None) -> list:
    """certificate() for several quantile levels on one (X, y, lambda): the K
    alpha of every level in one pass of FP64 products, the K alpha~ in a
    second (at most 16 levels).  Measures in the residual form only."""
    alphas = [np.asarray(a, dtype=np.float64) for a in alphas]
    if len(alphas) > 16:
        raise ValueError("at most 16 levels")
    y = np.asarray(y, dtype=np.float64)
    ats = [project_feasible(a, t) for a, t in zip(alphas, taus)]
    KA = kernel_apply(X, np.stack(alphas, axis=1), kind, gamma, progress=progress)
    KT = kernel_apply(X, np.stack(ats, axis=1), kind, gamma, progress=progress)
    out = []
    for j, (a, at, t, b) in enumerate(zip(alphas, ats, taus, betas)):
        Ka, Kat = KA[:, j], KT[:, j]
        zr = y - b - Ka / lam
        res = problem.kkt(a, problem.proj_box(a, t), b, zr, Ka, y, lam, t)
        obj = problem.primal_objective(zr, a, Ka, lam, t)
        r = y - Kat / lam
        bt = float(np.quantile(r, t, method="inverted_cdf"))
        upper = problem.primal_objective(r - bt, at, Kat, lam, t)
        s = float(at.sum())
        lower = problem.dual_objective(at, Kat, y, lam) - abs(s) * (abs(bt) + 1.0)
        d = {"res_" + k: val for k, val in res.items()}
        d.update(tau=t, obj_p_returned=obj, lower=lower, upper=upper,
                 rel_obj_err_bound=max(obj - lower, 0.0) / (1.0 + abs(lower)),
                 n_interior=int(np.sum((a > t - 1.0) & (a < t))))
        out.append(d)
    return out

