"""Problem-level quantities of KQR in float64.

* check loss rho_tau and its conjugate, the indicator of B = [tau-1, tau]^n
  (Section 1, definition of rho_tau and rho_tau^*);
* primal (1.2), dual (1.3) and consensus dual (1.4) objectives;
* the KKT residuals eta_p, eta_d, eta_c and the relative duality gap
  eta_gap used as stopping measures (Section 4);
* the reduced ALM subproblem objective phi_k (2.2) and its gradient (2.3).
"""
from __future__ import annotations

import numpy as np


def check_loss(z, tau: float) -> float:
    """rho_tau(z) = sum_i tau z_i (z_i > 0), -(1-tau) z_i (z_i <= 0)."""
    z = np.asarray(z, dtype=np.float64)
    return float(np.sum(np.where(z > 0, tau * z, -(1.0 - tau) * z)))


def proj_box(w, tau: float):
    """Euclidean projection onto B = [tau-1, tau]^n."""
    return np.clip(w, tau - 1.0, tau)


def dist2_box(w, tau: float) -> float:
    """Squared distance of w to B."""
    r = w - proj_box(w, tau)
    return float(r @ r)


def dual_objective(alpha, Kalpha, y, lam: float) -> float:
    """obj_D = -alpha^T K alpha / (2 lambda) + y^T alpha (dual (1.3))."""
    return float(-(alpha @ Kalpha) / (2.0 * lam) + y @ alpha)


def primal_objective(z, alpha, Kalpha, lam: float, tau: float) -> float:
    """obj_P = rho_tau(z) + alpha^T K alpha / (2 lambda) (primal (1.2) with theta = alpha)."""
    return float(check_loss(z, tau) + (alpha @ Kalpha) / (2.0 * lam))


def kkt(alpha, v, beta, z, Kalpha, y, lam: float, tau: float) -> dict:
    """Relative KKT residuals and duality gap of Section 4.

    eta_p = ||z - y + beta 1 + K alpha / lambda|| / (1 + ||y||)
    eta_d = sqrt((1^T alpha)^2 + ||alpha - v||^2) / (1 + ||alpha||)
    eta_c = ||v - Pi_B(z + v)|| / (1 + ||v||)
    eta_gap = |obj_P - obj_D| / (1 + |obj_P| + |obj_D|)
    """
    rp = z - y + beta + Kalpha / lam
    eta_p = np.linalg.norm(rp) / (1.0 + np.linalg.norm(y))
    s = alpha.sum()
    eta_d = np.sqrt(s * s + np.sum((alpha - v) ** 2)) / (1.0 + np.linalg.norm(alpha))
    eta_c = np.linalg.norm(v - proj_box(z + v, tau)) / (1.0 + np.linalg.norm(v))
    obj_p = primal_objective(z, alpha, Kalpha, lam, tau)
    obj_d = dual_objective(alpha, Kalpha, y, lam)
    eta_gap = abs(obj_p - obj_d) / (1.0 + abs(obj_p) + abs(obj_d))
    eta_kkt = max(eta_p, eta_d, eta_c)
    return dict(
        eta_p=float(eta_p), eta_d=float(eta_d), eta_c=float(eta_c),
        eta_kkt=float(eta_kkt), eta_gap=float(eta_gap),
        obj_p=obj_p, obj_d=obj_d, err=float(max(eta_kkt, eta_gap)),
    )


def phi(alpha, Kalpha, y, lam, tau, beta, z, sigma) -> float:
    """phi_k (2.2): the ALM subproblem after minimising out v.

    The Moreau envelope of the box indicator with parameter sigma is
    (sigma/2) dist^2(., B) (Appendix A, definition of the envelope).
    """
    s = alpha.sum() + beta / sigma
    return float(
        (alpha @ Kalpha) / (2.0 * lam)
        - y @ alpha
        + 0.5 * sigma * s * s
        + 0.5 * sigma * dist2_box(alpha + z / sigma, tau)
    )


def grad_phi(alpha, Kalpha, y, lam, tau, beta, z, sigma):
    """grad phi_k (2.3): K alpha/lambda - y + beta 1 + sigma 1 1^T alpha + sigma (w - Pi_B(w)),
    with w = alpha + z / sigma."""
    w = alpha + z / sigma
    return Kalpha / lam - y + beta + sigma * alpha.sum() + sigma * (w - proj_box(w, tau))


def jacobian_mask(w, tau: float):
    """Diagonal of an element S of the Clarke Jacobian of Pi_B at w (Section 2.2).

    1 strictly inside (tau-1, tau), 0 outside; on the boundary the Jacobian is
    the interval [0, 1] and this oracle takes 0.
    """
    return ((w > tau - 1.0) & (w < tau)).astype(np.float64)
