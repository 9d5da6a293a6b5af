"""PALM-KQR in float64: PCG, Phase I ADMM, Phase II SSN-ALM, polish.

Follows Section 2 (Algorithms 1-3), Section 3 (system (3.1), preconditioner
(3.2), Lemma 1) and the stopping rules of Section 4.  The paper names the
algorithm's constants but not their values; ``OracleOptions`` fixes each one
and says so.  None of those constants changes the converged answer: the dual
optimum is unique because K is positive definite (Section 1, after (1.3)).

Linear solves: for n <= ``direct_max`` the oracle factors the coefficient
matrix densely (an exact solve meets every inexactness rule of the paper);
above that it runs left-preconditioned CG with the Woodbury preconditioner.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict

import numpy as np
import scipy.linalg as sla

from . import problem as pb
from .kernel import DenseKernel, ImplicitKernel
from .precond import Woodbury, rpcholesky, adaptive_rank


@dataclass
class OracleOptions:
    tol: float = 1e-6             # Phase II stop: max(eta_kkt, eta_gap) <= tol (Section 4)
    admm_tol: float = 1e-3        # Phase I stop (Section 4)
    admm_max_iter: int = 100      # Section 4
    alm_max_iter: int = 1000      # Section 4
    admm_sigma: float = 1.0       # Algorithm 1 leaves sigma > 0 open: sigma = 1
    admm_step: float = 1.618      # Algorithm 1: step in (0, (1+sqrt 5)/2)
    admm_eps0: float = 0.1        # eps_k = admm_eps0 ||b_0|| / (k+1)^1.5, a summable sequence
    etabar: float = 0.1           # Algorithm 3 constants
    iota: float = 0.5
    armijo: float = 1e-4          # mu in (0, 1/2)
    ls_shrink: float = 0.5        # r in (0, 1)
    ls_max: int = 40
    tau1: float = 0.1
    tau2: float = 0.1
    eps_floor: float = 1e-12      # keeps L invertible when ||grad|| underflows
    ssn_max_iter: int = 50
    ssn_rel: float = 0.5          # SSN stop: ||grad phi|| <= (1 + ||y||) max(ssn_rel tol, ssn_adapt e_prev)
    ssn_adapt: float = 0.3        # e_prev = max(eta_kkt, eta_gap) of the previous outer iterate
    sigma_factor: float = 5.0     # sigma <- min(sigma_factor sigma, sigma_max) when eta_d stalls
    sigma_stall: float = 0.25
    sigma_max: float = 1e8
    rank: int = 0                 # >0 fixed rank, 0 adaptive (Section 3 heuristic), <0 no preconditioner
    xi: float = 1e-7              # adaptive-rank threshold
    pcg_max_iter: int = 2000
    direct_max: int = 5000        # exact dense solves up to this n
    polish: bool = True


@dataclass
class FitResult:
    alpha: np.ndarray
    v: np.ndarray
    beta: float
    z: np.ndarray
    Kalpha: np.ndarray
    kkt: dict
    info: dict = field(default_factory=dict)
    history: list = field(default_factory=list)


# ---------------------------------------------------------------- linear algebra
def pcg(apply_A, b, x0, tol, apply_Pinv=None, maxit=2000):
    """Left-preconditioned conjugate gradients for an SPD system A x = b.

    Stops when the (unpreconditioned) residual norm ||b - A x|| <= tol.
    Returns (x, iterations, residual_norm).
    """
    x = np.array(x0, dtype=np.float64, copy=True)
    r = b - apply_A(x) if np.any(x) else np.array(b, dtype=np.float64, copy=True)
    rn = float(np.linalg.norm(r))
    if rn <= tol:
        return x, 0, rn
    zv = apply_Pinv(r) if apply_Pinv else r.copy()
    p = zv.copy()
    rz = float(r @ zv)
    it = 0
    while it < maxit:
        it += 1
        q = apply_A(p)
        a = rz / float(p @ q)
        x += a * p
        r -= a * q
        rn = float(np.linalg.norm(r))
        if rn <= tol:
            break
        zv = apply_Pinv(r) if apply_Pinv else r.copy()
        rz_new = float(r @ zv)
        p = zv + (rz_new / rz) * p
        rz = rz_new
    return x, it, rn


class _System:
    """A = K + c 1 1^T + diag(L) with its preconditioner (3.2) or a dense factor."""

    def __init__(self, op, c, Ldiag, F, direct):
        self.op, self.c, self.L = op, float(c), np.asarray(Ldiag, dtype=np.float64)
        self.direct = direct
        if direct:
            A = op.K + self.c
            A[np.diag_indices_from(A)] += self.L
            self.fac = sla.cho_factor(A, lower=True)
            self.P = None
        else:
            self.fac = None
            self.P = Woodbury(F, self.c, self.L).apply if F is not None else None

    def apply(self, x):
        return self.op.apply(x) + self.c * x.sum() + self.L * x

    def solve(self, b, x0, tol, maxit):
        if self.direct:
            return sla.cho_solve(self.fac, b), 0, 0.0
        return pcg(self.apply, b, x0, tol, self.P, maxit)


# ---------------------------------------------------------------- Phase I
def admm(op, y, tau, lam, F, opts: OracleOptions, direct: bool, history=None, start=None):
    """Algorithm 1: inexact ADMM on the consensus dual (1.4).

    M = K + lambda sigma (I + 1 1^T) is fixed, so it is factored (or its
    preconditioner built, with L = lambda sigma I) once.

    ``start`` (alpha, beta, z, Kalpha) replaces the zero initial point; v is
    then the projection of alpha onto the box.  A start that already meets the
    Phase I target is returned as it is (no iteration).
    """
    n = y.shape[0]
    sigma, step = opts.admm_sigma, opts.admm_step
    c = lam * sigma
    res = None
    if start is None:
        alpha, v, z, beta = np.zeros(n), np.zeros(n), np.zeros(n), 0.0
        Ka = np.zeros(n)
    else:
        alpha, beta, z = start["alpha"].copy(), float(start["beta"]), start["z"].copy()
        Ka = start["Kalpha"].copy()
        v = pb.proj_box(alpha, tau)
        res = pb.kkt(alpha, v, beta, z, Ka, y, lam, tau)
        if res["err"] <= opts.admm_tol:
            return dict(alpha=alpha, v=v, beta=beta, z=z, Kalpha=Ka, sigma=sigma, iters=0, pcg=0, kkt=res)
    sysM = _System(op, c, np.full(n, c), F, direct)
    b0 = None
    pcg_total = 0
    k = -1
    for k in range(opts.admm_max_iter):
        b = lam * (y - beta - z + sigma * v)
        if b0 is None:
            b0 = float(np.linalg.norm(b))
        eps_k = opts.admm_eps0 * b0 / (k + 1) ** 1.5
        alpha, its, _ = sysM.solve(b, alpha, eps_k, opts.pcg_max_iter)
        pcg_total += its
        v = pb.proj_box(alpha + z / sigma, tau)
        beta = beta + step * sigma * alpha.sum()
        z = z + step * sigma * (alpha - v)
        Ka = op.apply(alpha)
        res = pb.kkt(alpha, v, beta, z, Ka, y, lam, tau)
        if history is not None:
            history.append(dict(phase="admm", it=k + 1, pcg=its, **res))
        if res["err"] <= opts.admm_tol:
            break
    return dict(alpha=alpha, v=v, beta=beta, z=z, Kalpha=Ka, sigma=sigma,
                iters=k + 1, pcg=pcg_total, kkt=res)


# ---------------------------------------------------------------- Phase II
def _armijo_delta(c, dKa, dKd, yd, ed, s, w, d, lam, sigma, tau):
    """phi(alpha + c d) - phi(alpha), expanded term by term from (2.2)."""
    r0 = w - pb.proj_box(w, tau)
    wc = w + c * d
    r1 = wc - pb.proj_box(wc, tau)
    return (c * dKa / lam + 0.5 * c * c * dKd / lam - c * yd
            + 0.5 * sigma * ((s + c * ed) ** 2 - s * s)
            + 0.5 * sigma * float(r1 @ r1 - r0 @ r0))


def ssn(op, y, tau, lam, beta, z, sigma, alpha, Ka, F, opts: OracleOptions,
        direct: bool, stop: float):
    """Algorithm 3: semismooth Newton on phi_k with Armijo backtracking.

    Newton system (H + eps_t I) d = -grad phi, solved in the lambda-scaled
    form (3.1): (K + lambda sigma 1 1^T + L) d = -lambda grad phi with
    L = lambda sigma (I - S) + lambda eps_t I.
    """
    alpha = alpha.copy()
    Ka = Ka.copy()
    c1 = lam * sigma
    info = dict(newton=0, pcg=0, ls=0)
    for t in range(opts.ssn_max_iter):
        w = alpha + z / sigma
        grad = pb.grad_phi(alpha, Ka, y, lam, tau, beta, z, sigma)
        gn = float(np.linalg.norm(grad))
        if gn <= stop:
            break
        eps_t = max(opts.tau1 * min(opts.tau2, gn), opts.eps_floor)
        S = pb.jacobian_mask(w, tau)
        L = lam * sigma * (1.0 - S) + lam * eps_t
        sysH = _System(op, c1, L, F, direct)
        tol = lam * min(opts.etabar, gn ** (1.0 + opts.iota))
        d, its, _ = sysH.solve(-lam * grad, np.zeros_like(alpha), tol, opts.pcg_max_iter)
        info["pcg"] += its
        Kd = op.apply(d)
        gd = float(grad @ d)
        s = alpha.sum() + beta / sigma
        dKa, dKd, yd, ed = float(d @ Ka), float(d @ Kd), float(y @ d), float(d.sum())
        c = 1.0
        for _ in range(opts.ls_max):
            if _armijo_delta(c, dKa, dKd, yd, ed, s, w, d, lam, sigma, tau) <= opts.armijo * c * gd:
                break
            c *= opts.ls_shrink
            info["ls"] += 1
        alpha += c * d
        Ka += c * Kd
        info["newton"] += 1
    w = alpha + z / sigma
    info["grad_norm"] = float(np.linalg.norm(pb.grad_phi(alpha, Ka, y, lam, tau, beta, z, sigma)))
    return alpha, pb.proj_box(w, tau), Ka, info


def alm(op, y, tau, lam, F, start: dict, opts: OracleOptions, direct: bool, history=None):
    """Algorithm 2: ALM on (1.4) with SSN subproblem solves."""
    alpha, beta, z = start["alpha"].copy(), float(start["beta"]), start["z"].copy()
    sigma = float(start["sigma"])
    Ka = op.apply(alpha)
    eta_d_prev = start["kkt"]["eta_d"] if start.get("kkt") else None
    # Subproblem accuracy: the summable tolerances of criterion (A) are read as
    # a fraction of the previous outer residual, floored at the final target
    # (after the multiplier update ||grad phi_k|| = (1 + ||y||) eta_p).
    scale = 1.0 + float(np.linalg.norm(y))
    e_prev = start["kkt"]["err"] if start.get("kkt") else np.inf
    tot = dict(newton=0, pcg=0, ls=0)
    res, v = None, start.get("v", alpha).copy()
    # a start that already meets the final target (Phase I run alone) is kept
    res = pb.kkt(alpha, v, beta, z, Ka, y, lam, tau)
    if res["err"] <= opts.tol:
        return dict(alpha=alpha, v=v, beta=beta, z=z, Kalpha=Ka, sigma=sigma, iters=0, kkt=res, **tot)
    k = -1
    for k in range(opts.alm_max_iter):
        stop = scale * max(opts.ssn_rel * opts.tol, min(opts.ssn_adapt * e_prev, 1.0))
        alpha, v, Ka, info = ssn(op, y, tau, lam, beta, z, sigma, alpha, Ka, F, opts, direct, stop)
        for key in tot:
            tot[key] += info[key]
        beta = beta + sigma * alpha.sum()
        z = z + sigma * (alpha - v)
        res = pb.kkt(alpha, v, beta, z, Ka, y, lam, tau)
        if history is not None:
            history.append(dict(phase="alm", it=k + 1, sigma=sigma, **info, **res))
        if res["err"] <= opts.tol:
            break
        if eta_d_prev is not None and res["eta_d"] > opts.sigma_stall * eta_d_prev:
            sigma = min(opts.sigma_factor * sigma, opts.sigma_max)
        eta_d_prev = res["eta_d"]
        e_prev = res["err"]
    return dict(alpha=alpha, v=v, beta=beta, z=z, Kalpha=Ka, sigma=sigma,
                iters=k + 1, kkt=res, **tot)


# ---------------------------------------------------------------- polish
def bordered_solve(K, y, lam, tau, E, N, alphaN):
    """Solve [K_EE/lam 1; 1^T 0][alpha_E; beta] = [y_E - K_EN alpha_N/lam; -1^T alpha_N]."""
    m = E.size
    G = np.zeros((m + 1, m + 1))
    G[:m, :m] = K[np.ix_(E, E)] / lam
    G[:m, m] = 1.0
    G[m, :m] = 1.0
    h = np.empty(m + 1)
    h[:m] = y[E] - K[np.ix_(E, N)] @ alphaN / lam
    h[m] = -alphaN.sum()
    sol = np.linalg.solve(G, h)
    return sol[:m], float(sol[m])


def polish(K, y, lam, tau, z, beta, thr=0.0, slack=1e-10):
    """Active-set refinement at a converged ALM iterate.

    After a multiplier update z = sigma (w - Pi_B(w)), z_i == 0 for interior
    w_i; near the solution some weakly active points still carry a tiny z_i,
    so E = {|z_i| <= thr}, R = {z_i > thr} (alpha = tau) and
    L = {z_i < -thr} (alpha = tau - 1).  On that partition the KKT conditions
    of (1.3) reduce to the bordered system above.  Returns None when its
    solution leaves the box or breaks a sign condition (the partition was not
    the optimal one).
    """
    n = y.shape[0]
    inE = np.abs(z) <= thr
    E = np.flatnonzero(inE)
    N = np.flatnonzero(~inE)
    up = (~inE) & (z > 0)
    lo_ = (~inE) & (z < 0)
    alpha = np.where(up, tau, tau - 1.0)
    tol = slack * (1.0 + np.abs(y).max())
    if E.size == 0:
        Ka = K @ alpha
        base = y - Ka / lam
        hi = base[up].min() if np.any(up) else np.inf
        lo = base[lo_].max() if np.any(lo_) else -np.inf
        if lo > hi + tol or abs(alpha.sum()) > 1e-9 * n:
            return None
        b = float(np.clip(beta, lo, hi))
    else:
        aE, b = bordered_solve(K, y, lam, tau, E, N, alpha[N])
        if aE.min() < tau - 1.0 - slack or aE.max() > tau + slack:
            return None
        alpha[E] = np.clip(aE, tau - 1.0, tau)
        Ka = K @ alpha
    znew = y - b - Ka / lam
    if np.any(znew[up] < -tol) or np.any(znew[lo_] > tol):
        return None
    return alpha, b, znew, Ka


def polish_search(K, y, lam, tau, z, beta, err):
    """Try partitions with growing thresholds on |z|; keep the best that passes."""
    scale = err * (1.0 + float(np.linalg.norm(y)))
    best = None
    for thr in [0.0] + [scale * 10.0 ** k for k in range(0, 5)]:
        out = polish(K, y, lam, tau, z, beta, thr)
        if out is None:
            continue
        a, b, zz, Ka = out
        e = pb.kkt(a, a, b, zz, Ka, y, lam, tau)["err"]
        if best is None or e < best[1]:
            best = (out, e)
    return best


# ---------------------------------------------------------------- driver
def build_preconditioner(op, opts: OracleOptions, uniforms):
    """F for (3.2): fixed rank, the adaptive heuristic of Section 3, or none."""
    if opts.rank < 0:
        return None, dict(rank=0)
    if opts.rank > 0:
        F, piv, _ = rpcholesky(op, opts.rank, uniforms)
        return F, dict(rank=F.shape[1], pivots=piv)
    r0 = int(math.ceil(math.sqrt(op.n)))
    F0, piv, _ = rpcholesky(op, r0, uniforms)
    r = adaptive_rank(F0, opts.xi)
    return F0[:, :r].copy(), dict(rank=r, r0=F0.shape[1], pivots=piv[:r])


def fit(X, y, tau, lam, kind, gamma, opts: OracleOptions | None = None,
        uniforms=None, op=None, history: bool = False) -> FitResult:
    """Two-phase PALM-KQR: Algorithm 1 warm start, then Algorithms 2-3."""
    opts = opts or OracleOptions()
    y = np.asarray(y, dtype=np.float64)
    n = y.shape[0]
    direct = n <= opts.direct_max
    if op is None:
        op = DenseKernel(X, kind, gamma) if (direct or n <= 20000) else ImplicitKernel(X, kind, gamma)
    if direct and not isinstance(op, DenseKernel):
        raise ValueError("direct solves need a dense kernel")
    F, pinfo = (None, dict(rank=0)) if direct else build_preconditioner(op, opts, uniforms)
    return _fit_on(op, F, pinfo, y, tau, float(lam), opts, direct, None, history)


def _fit_on(op, F, pinfo, y, tau, lam, opts: OracleOptions, direct: bool, start, history: bool) -> FitResult:
    hist = [] if history else None
    applies0 = op.applies
    ph1 = admm(op, y, tau, lam, F, opts, direct, hist, start)
    ph2 = alm(op, y, tau, lam, F, ph1, opts, direct, hist)
    alpha, v, beta, z, Ka = ph2["alpha"], ph2["v"], ph2["beta"], ph2["z"], ph2["Kalpha"]
    polished = False
    if opts.polish and isinstance(op, DenseKernel):
        best = polish_search(op.K, y, lam, tau, z, beta, ph2["kkt"]["err"])
        if best is not None:
            a2, b2, z2, Ka2 = best[0]
            if best[1] <= ph2["kkt"]["err"]:
                alpha, v, beta, z, Ka, polished = a2, a2.copy(), b2, z2, Ka2, True
    res = pb.kkt(alpha, v, beta, z, Ka, y, lam, tau)
    info = dict(admm_iters=ph1["iters"], admm_pcg=ph1["pcg"], alm_iters=ph2["iters"],
                newton=ph2["newton"], pcg=ph2["pcg"], ls=ph2["ls"], sigma=ph2["sigma"],
                polished=polished, n_interior=int(np.sum((alpha > tau - 1) & (alpha < tau))),
                kapply=op.applies - applies0, direct=direct, **pinfo)
    return FitResult(alpha, v, beta, z, Ka, res, info, hist or [])


def path_start(prev: FitResult, y, lam: float) -> dict:
    """Warm start for the next value of lambda on a regularisation path.

    alpha and beta are kept (the box and the constraint on alpha do not depend
    on lambda) and z is the residual y - beta 1 - K alpha / lambda at the new
    lambda, so that the stationarity condition in alpha holds exactly at the
    start; K alpha is the previous fit's (K does not change along the path).
    """
    z = y - prev.beta - prev.Kalpha / lam
    return dict(alpha=prev.alpha, beta=prev.beta, z=z, Kalpha=prev.Kalpha)


def fit_path(X, y, tau, lams, kind, gamma, opts: OracleOptions | None = None,
             uniforms=None, op=None, warm: bool = True) -> list:
    """KQR over a sequence of lambda values (the regularisation paths of
    Section 4.1): K and the preconditioner factor F are formed once; each fit
    after the first starts from the previous solution (``path_start``) and
    runs Phase I from there (skipped when the start already meets its target),
    then Phase II.  With ``warm`` off every value is a cold start."""
    opts = opts or OracleOptions()
    y = np.asarray(y, dtype=np.float64)
    n = y.shape[0]
    direct = n <= opts.direct_max
    if op is None:
        op = DenseKernel(X, kind, gamma) if (direct or n <= 20000) else ImplicitKernel(X, kind, gamma)
    F, pinfo = (None, dict(rank=0)) if direct else build_preconditioner(op, opts, uniforms)
    out = []
    for lam in lams:
        start = path_start(out[-1], y, float(lam)) if (warm and out) else None
        out.append(_fit_on(op, F, pinfo, y, tau, float(lam), opts, direct, start, False))
    return out


def options_dict(o: OracleOptions) -> dict:
    return asdict(o)
