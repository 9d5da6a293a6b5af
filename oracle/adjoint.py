"""Implicit gradient of a validation check loss w.r.t. log(gamma), log(lambda).

Not in the paper; derived from the KKT conditions of the dual (1.3).  At a
solution with index sets R (alpha = tau), L (alpha = tau - 1) and E (interior),
(alpha_E, beta) solve the bordered system

    G [alpha_E; beta] = [y_E - K_EN alpha_N / lambda; -1^T alpha_N],
    G = [K_EE / lambda, 1; 1^T, 0].

If the partition is locally constant (strict complementarity), alpha_N is
fixed and differentiating the system gives d(alpha_E, beta)/d theta.  The
validation loss J = rho_tau(y' - beta - K(X', X) alpha / lambda) then has

    dJ/dlog(lambda) =  mu_E^T (K alpha)_E / lambda - g^T K' alpha / lambda
    dJ/dlog(gamma)  = -mu_E^T ((K o ln K) alpha)_E / lambda
                      + g^T (K' o ln K') alpha / lambda

with g = -rho_tau'(r') (-tau where r' > 0, 1 - tau where r' < 0), K' = K(X', X)
and G mu = [K'_E^T g / lambda; 1^T g].  d K / d log(gamma) = K o ln K holds for
any kernel of the form exp(-gamma d(x, x')), and K o ln K = -gamma D o K.
"""
from __future__ import annotations

import numpy as np

from .kernel import distance_block
from .problem import check_loss


def validation_loss(Xtr, alpha, beta, Xval, yval, lam, tau, kind, gamma) -> float:
    Kv = np.exp(-gamma * distance_block(Xval, Xtr, kind))
    return check_loss(yval - beta - Kv @ alpha / lam, tau)


def adjoint_gradient(Xtr, alpha, beta, Xval, yval, lam, tau, kind, gamma):
    """Returns (J, dJ/dlog gamma, dJ/dlog lambda, |E|)."""
    Xtr = np.asarray(Xtr, dtype=np.float64)
    Xval = np.asarray(Xval, dtype=np.float64)
    D = distance_block(Xtr, Xtr, kind)
    K = np.exp(-gamma * D)
    KlnK = -gamma * D * K
    Dv = distance_block(Xval, Xtr, kind)
    Kv = np.exp(-gamma * Dv)
    KvlnKv = -gamma * Dv * Kv
    r = yval - beta - Kv @ alpha / lam
    J = check_loss(r, tau)
    g = np.where(r > 0, -tau, 1.0 - tau)
    E = np.flatnonzero((alpha > tau - 1.0) & (alpha < tau))
    m = E.size
    if m == 0:
        raise ValueError("no interior coefficients: beta is not differentiable")
    G = np.zeros((m + 1, m + 1))
    G[:m, :m] = K[np.ix_(E, E)] / lam
    G[:m, m] = 1.0
    G[m, :m] = 1.0
    rhs = np.r_[Kv[:, E].T @ g / lam, g.sum()]
    mu = np.linalg.solve(G, rhs)
    Ka = K @ alpha
    dlam = mu[:m] @ Ka[E] / lam - g @ (Kv @ alpha) / lam
    dgam = -mu[:m] @ (KlnK @ alpha)[E] / lam + g @ (KvlnKv @ alpha) / lam
    return float(J), float(dgam), float(dlam), int(m)
