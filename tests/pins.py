"""Method-independent reference solutions used to pin the oracle.

None of these follows the paper's algorithms:

* ``brute_force``: enumerate every partition of the indices into lower-bound,
  interior and upper-bound sets and keep the one whose KKT system for the
  dual QP (1.3) has a box- and sign-consistent solution (exact, n <= 9).
* ``slsqp_dual``: hand the dual QP (1.3) to SciPy's generic SLSQP solver.
* ``identity_kernel_solution``: closed form when K = I.
* ``linear_primal_qp``: the primal (1.1) with the linear kernel, i.e. linear
  quantile regression with a ridge penalty on the slope, as a generic QP in
  (beta, w, residual parts) for SciPy's SLSQP.
* ``sample_quantile_interval``: the textbook set of tau-quantiles of a sample.
"""
from __future__ import annotations

import itertools

import numpy as np
from scipy.optimize import minimize


def brute_force(K, y, lam, tau):
    """Exact dual optimum by partition enumeration; returns (alpha, beta_lo, beta_hi)."""
    n = y.shape[0]
    for part in itertools.product((0, 1, 2), repeat=n):
        part = np.asarray(part)
        E = np.flatnonzero(part == 1)
        N = np.flatnonzero(part != 1)
        alpha = np.where(part == 2, tau, tau - 1.0).astype(np.float64)
        if E.size:
            m = E.size
            G = np.zeros((m + 1, m + 1))
            G[:m, :m] = K[np.ix_(E, E)] / lam
            G[:m, m] = 1.0
            G[m, :m] = 1.0
            h = np.r_[y[E] - K[np.ix_(E, N)] @ alpha[N] / lam, -alpha[N].sum()]
            try:
                sol = np.linalg.solve(G, h)
            except np.linalg.LinAlgError:
                continue
            aE, beta = sol[:m], sol[m]
            if aE.min() < tau - 1 - 1e-12 or aE.max() > tau + 1e-12:
                continue
            alpha[E] = aE
            z = y - beta - K @ alpha / lam
            if np.all(z[part == 2] >= -1e-10) and np.all(z[part == 0] <= 1e-10):
                return alpha, beta, beta
        else:
            if abs(alpha.sum()) > 1e-12:
                continue
            base = y - K @ alpha / lam
            hi = base[part == 2].min() if np.any(part == 2) else np.inf
            lo = base[part == 0].max() if np.any(part == 0) else -np.inf
            if lo <= hi + 1e-12:
                return alpha, lo, hi
    raise RuntimeError("no KKT-consistent partition")


def slsqp_dual(K, y, lam, tau, x0=None):
    """Generic QP: min alpha^T K alpha/(2 lam) - y^T alpha, alpha in B, 1^T alpha = 0."""
    n = y.shape[0]
    fun = lambda a: a @ K @ a / (2 * lam) - y @ a
    jac = lambda a: K @ a / lam - y
    cons = [dict(type="eq", fun=lambda a: a.sum(), jac=lambda a: np.ones_like(a))]
    bounds = [(tau - 1.0, tau)] * n
    x0 = np.zeros(n) if x0 is None else x0
    res = minimize(fun, x0, jac=jac, bounds=bounds, constraints=cons, method="SLSQP",
                   options=dict(ftol=1e-15, maxiter=2000))
    return res.x, res.fun


def identity_kernel_solution(y, lam, tau):
    """K = I: alpha_i = clip(lam (y_i - beta), tau-1, tau) with sum(alpha) = 0.

    sum_i clip(lam (y_i - b), tau-1, tau) is continuous and non-increasing in
    b; bisection finds the b at which it crosses zero.
    """
    f = lambda b: np.clip(lam * (y - b), tau - 1.0, tau).sum()
    lo, hi = y.min() - 2.0 / lam - 1.0, y.max() + 2.0 / lam + 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(mid) > 0:
            lo = mid
        else:
            hi = mid
    b = 0.5 * (lo + hi)
    return np.clip(lam * (y - b), tau - 1.0, tau), b


def sample_quantile_interval(y, tau):
    """All minimisers of sum_i rho_tau(y_i - b): [y_(k), y_(k+1)] style interval."""
    ys = np.sort(y)
    n = ys.size
    k = tau * n
    if abs(k - round(k)) < 1e-12:
        k = int(round(k))
        return ys[k - 1], ys[k]
    j = int(np.floor(k))
    return ys[j], ys[j]


def linear_primal_qp(X, y, lam, tau):
    """min_{beta, w} sum rho_tau(y_i - beta - x_i^T w) + lam/2 ||w||^2 as a QP:
    y - beta - X w = up - um with up, um >= 0.  Returns (objective, beta, w)."""
    X = np.asarray(X, dtype=np.float64)
    n, p = X.shape
    # variables: [beta, w (p), up (n), um (n)]
    def fun(z):
        w, up, um = z[1:1 + p], z[1 + p:1 + p + n], z[1 + p + n:]
        return tau * up.sum() + (1 - tau) * um.sum() + 0.5 * lam * (w @ w)

    def jac(z):
        g = np.zeros_like(z)
        g[1:1 + p] = lam * z[1:1 + p]
        g[1 + p:1 + p + n] = tau
        g[1 + p + n:] = 1 - tau
        return g

    A = np.zeros((n, 1 + p + 2 * n))
    A[:, 0] = 1.0
    A[:, 1:1 + p] = X
    A[:, 1 + p:1 + p + n] = np.eye(n)
    A[:, 1 + p + n:] = -np.eye(n)
    cons = [dict(type="eq", fun=lambda z: A @ z - y, jac=lambda z: A)]
    r0 = y - np.median(y)
    z0 = np.r_[np.median(y), np.zeros(p), np.maximum(r0, 0), np.maximum(-r0, 0)]
    bounds = [(None, None)] * (1 + p) + [(0, None)] * (2 * n)
    res = minimize(fun, z0, jac=jac, bounds=bounds, constraints=cons, method="SLSQP",
                   options=dict(ftol=1e-15, maxiter=5000))
    return res.fun, res.x[0], res.x[1:1 + p]
