"""Low-rank preconditioner of Section 3 in float64.

* ``rpcholesky``: randomly pivoted Cholesky, F = RPCholesky(K, r) with
  K_hat = F F^T (Section 3, eq. (3.2) and the cited RPCholesky algorithm).
  Each step draws a pivot with probability proportional to the residual
  diagonal; a pivot's residual diagonal is zero afterwards, so pivots are
  drawn without replacement.  The random draws enter as a vector of
  uniforms u_i in [0, 1): step i takes the first index j whose running sum
  of the residual diagonal exceeds u_i times its total.
* ``adaptive_rank``: the rank heuristic of Section 3 (r0 = ceil(sqrt(n)),
  eigenvalues of F0^T F0, r = smallest index with lambda_r <= xi lambda_1).
* ``Woodbury``: P^{-1} for P = F F^T + c 1 1^T + L with L diagonal, by
  Lemma 1 (Sherman-Morrison-Woodbury with U = [F 1]).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla


def sample_pivot(d: np.ndarray, u: float) -> int:
    """First index j with cumsum(d)[j] > u * sum(d)."""
    c = np.cumsum(d)
    t = u * c[-1]
    j = int(np.searchsorted(c, t, side="right"))
    if j >= d.shape[0]:  # u * total rounded up to the total: take the last positive entry
        j = int(np.flatnonzero(d > 0)[-1])
    return j


def rpcholesky(op, rank: int, uniforms, stop_rel: float = 1e-14):
    """Randomly pivoted Cholesky of the PSD operator ``op``.

    ``op`` provides ``n``, ``diag()`` and ``column(j)``.  Returns
    (F, pivots, residual_diagonal).  Stops early once the residual trace is
    below ``stop_rel`` times the trace of K.
    """
    n = op.n
    rank = min(int(rank), n)
    F = np.zeros((n, rank))
    d = np.asarray(op.diag(), dtype=np.float64).copy()
    tr0 = d.sum()
    piv = []
    for i in range(rank):
        if d.sum() <= stop_rel * tr0:
            break
        s = sample_pivot(d, float(uniforms[i]))
        g = op.column(s) - F[:, :i] @ F[s, :i]
        F[:, i] = g / math.sqrt(g[s])
        d = np.maximum(d - F[:, i] ** 2, 0.0)
        d[s] = 0.0
        piv.append(s)
    k = len(piv)
    return F[:, :k].copy(), np.asarray(piv, dtype=np.int64), d


def adaptive_rank(F0: np.ndarray, xi: float) -> int:
    """Smallest r (1-based) with lambda_r(F0^T F0) <= xi lambda_1, else r0."""
    ev = np.linalg.eigvalsh(F0.T @ F0)[::-1]
    hit = np.flatnonzero(ev <= xi * ev[0])
    return int(hit[0] + 1) if hit.size else int(ev.size)


class Woodbury:
    """P^{-1} for P = F F^T + c 1 1^T + diag(L) by Lemma 1.

    C = diag(I_r, 1/c) + U^T L^{-1} U with U = [F 1];
    P^{-1} w = L^{-1} w - L^{-1} U C^{-1} U^T L^{-1} w.
    """

    def __init__(self, F: np.ndarray, c: float, Ldiag: np.ndarray):
        n, r = F.shape
        self.U = np.hstack([F, np.ones((n, 1))])
        self.Ldiag = np.asarray(Ldiag, dtype=np.float64)
        core = np.diag(np.r_[np.ones(r), 1.0 / c])
        self.C = core + self.U.T @ (self.U / self.Ldiag[:, None])
        self.chol = sla.cho_factor(self.C, lower=True)

    def apply(self, w):
        g = w / self.Ldiag
        t = self.U.T @ g
        s = sla.cho_solve(self.chol, t)
        return g - (self.U @ s) / self.Ldiag

    def dense(self, F, c):
        """P itself, for tests."""
        n = F.shape[0]
        return F @ F.T + c * np.ones((n, n)) + np.diag(self.Ldiag)
