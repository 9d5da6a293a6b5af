"""GPU parity: every step of the HIP path against the FP64 oracle.

All inputs come from the seeded generators; expected values from ``oracle``.
Tolerances are derived from the arithmetic of each kernel (unit roundoff
u = 2^-24 for FP32, 2^-8 relative rounding for BF16 storage (8-bit significand)) and written next
to each check.
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import kernel as okernel
from oracle import precond as oprecond
from oracle import problem as oproblem
from oracle import solver as osolver
from paper_2510_07929_amd import inputs, kqr

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
# A BF16-stored RBF entry: round-to-nearest (unit roundoff 2^-8) of a value that
# the build's three-product Gram may move by up to 2^-10 relative (the build
# takes three products only within that limit), on top of the FP32 error Kb:
# |K_bf16 - K| <= BF16_REL K + (1 + 2^-8) Kb
BF16_REL = 2.0 ** -8 + 2.0 ** -10 * (1.0 + 2.0 ** -8)


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    kqr.lib()
    return torch.device("cuda:0")


def entry_bound(X, kind, gamma):
    """Per-entry bound |K_fp32 - K| of the norm-expansion FP32 evaluation."""
    Xd = X.astype(np.float64)
    p = X.shape[1]
    D = okernel.distance_block(Xd, Xd, kind)
    K = np.exp(-gamma * D)
    if kind == "rbf":
        q = (Xd * Xd).sum(1)
        dd = 4.0 * (p + 2) * U32 * (q[:, None] + q[None, :]) + 2.0 * U32 * D
    else:
        dd = 2.0 * (p + 2) * U32 * D + 1e-30
    return K, K * (gamma * dd + 8.0 * U32) + 1e-300


# --------------------------------------------------------------------- kernel build
@pytest.mark.parametrize("kind", ["rbf", "laplacian"])
@pytest.mark.parametrize("n,p", [(1337, 10), (700, 20), (129, 3)])
def test_kernel_build_fp32(dev, kind, n, p):
    X, _ = inputs.smooth(n, p, (101, n, p))
    gamma = 1.0 / p
    say("kernel_build fp32", kind, n, p)
    K = kqr.kqr_kernel_build(torch.from_numpy(X).to(dev), kind, gamma, "fp32").cpu().numpy()
    Kref, bound = entry_bound(X, kind, gamma)
    ld = kqr.padded_ld(n)
    assert K.shape == (n, ld)
    assert np.all(K[:, n:] == 0.0)                # padding written as zeros
    assert np.all(np.diag(K[:, :n]) == 1.0)       # d_ii := 0 exactly
    err = np.abs(K[:, :n] - Kref)
    assert np.all(err <= bound), float((err / bound).max())


def three_product_term(X, kind, gamma):
    """Relative change of a BF16-stored RBF entry from the Gram's three leading
    BF16 products (used when gamma max q <= 16/3): 3 2^-15 gamma (q_i + q_j)."""
    q = (X.astype(np.float64) ** 2).sum(1)
    if kind != "rbf" or X.shape[1] > 32 or gamma * q.max() > 16.0 / 3.0:
        return 0.0
    return 3.0 * 2.0 ** -15 * gamma * (q[:, None] + q[None, :])


# (scale, shift) of the inputs: on [-1, 1]^p; stretched so that gamma max q
# sits just under the three-product limit; moved far from the origin, where the
# build takes all six products
@pytest.mark.parametrize("kind,scale,shift", [("rbf", 1.0, 0.0), ("laplacian", 1.0, 0.0),
                                              ("rbf", 2.25, 0.0), ("rbf", 1.0, 20.0)])
def test_kernel_build_bf16(dev, kind, scale, shift):
    n, p = 1000, 10
    X, _ = inputs.smooth(n, p, (102, 0))
    X = (X * np.float32(scale) + np.float32(shift)).astype(np.float32)
    gamma = 0.1
    say("kernel_build bf16", kind, scale, shift)
    K = kqr.kqr_kernel_build(torch.from_numpy(X).to(dev), kind, gamma, "bf16").float().cpu().numpy()
    Kref, bound = entry_bound(X, kind, gamma)
    # BF16 round-to-nearest (unit roundoff 2^-8) of the FP32 value, whose
    # error is the FP32 bound plus, with three Gram products, their term
    extra = Kref * three_product_term(X, kind, gamma)
    err = np.abs(K[:, :n].astype(np.float64) - Kref)
    assert np.all(err <= 2.0 ** -8 * (Kref + bound + extra) + bound + extra)
    assert np.all(K[:, n:] == 0.0)
    assert np.all(np.diag(K[:, :n]) == 1.0)


# --------------------------------------------------------------------- K-apply
def _apply_bound(Kb, Kref, v, mode, bf16=False, otf=False):
    a = np.abs(v)
    if bf16:
        ent = BF16_REL * Kref + (1.0 + 2.0 ** -8) * Kb
    else:
        ent = Kb
    # rounding of v to FP32 (fast), FP32 products, FP32 partial sums of <= 64 terms
    if otf:
        arith = 70.0 * U32
    elif mode == kqr.KQR_APPLY_FAST:
        arith = 12.0 * U32
    else:
        arith = 1e-15
    return ent @ a + arith * (Kref @ a) + 1e-13


@pytest.mark.parametrize("kd", ["fp32", "bf16"])
@pytest.mark.parametrize("mode", [kqr.KQR_APPLY_FAST, kqr.KQR_APPLY_EXACT])
@pytest.mark.parametrize("n", [1337, 2048, 517])
def test_kernel_apply_materialised(dev, kd, mode, n):
    p = 10
    X, _ = inputs.smooth(n, p, (103, n))
    v = np.random.default_rng(n).standard_normal(n)
    gamma = 0.1
    say("kernel_apply materialised", kd, mode, n)
    Xt = torch.from_numpy(X).to(dev)
    K = kqr.kqr_kernel_build(Xt, "rbf", gamma, kd)
    u = kqr.kqr_kernel_apply(torch.from_numpy(v).to(dev), K=K, mode=mode).cpu().numpy()
    Kref, Kb = entry_bound(X, "rbf", gamma)
    bound = _apply_bound(Kb, Kref, v, mode, bf16=(kd == "bf16"))
    err = np.abs(u - Kref @ v)
    assert np.all(err <= bound), float((err / bound).max())


# p = 10: FP32 matrix-core Gram; 20 and 30: BF16x3 Gram with the norms in the
# spare coordinates; 32: BF16x3 Gram, norms added by the lanes
@pytest.mark.parametrize("kind", ["rbf", "laplacian"])
@pytest.mark.parametrize("mode", [kqr.KQR_APPLY_FAST, kqr.KQR_APPLY_EXACT])
@pytest.mark.parametrize("n,p", [(1337, 10), (1500, 20), (3000, 30), (2100, 32)])
def test_kernel_apply_on_the_fly(dev, kind, mode, n, p):
    X, _ = inputs.additive(n, p, (104, n))
    v = np.random.default_rng(1).standard_normal(n)
    gamma = 1.0 / p
    say("kernel_apply otf", kind, mode, n, p)
    u = kqr.kqr_kernel_apply(torch.from_numpy(v).to(dev), X=torch.from_numpy(X).to(dev), kernel=kind,
                             gamma=gamma, mode=mode).cpu().numpy()
    Kref, Kb = entry_bound(X, kind, gamma)
    bound = _apply_bound(Kb, Kref, v, kqr.KQR_APPLY_FAST, otf=True)
    err = np.abs(u - Kref @ v)
    assert np.all(err <= bound), float((err / bound).max())


def test_kernel_apply_multi_rhs(dev):
    n, p, m = 1500, 8, 3
    X, _ = inputs.additive(n, p, (105, 0))
    V = np.random.default_rng(2).standard_normal((n, m))
    say("kernel_apply multi-rhs", n, m)
    Xt = torch.from_numpy(X).to(dev)
    K = kqr.kqr_kernel_build(Xt, "rbf", 0.125, "fp32")
    U = kqr.kqr_kernel_apply(torch.from_numpy(V).to(dev), K=K, mode=kqr.KQR_APPLY_EXACT).cpu().numpy()
    Kref, Kb = entry_bound(X, "rbf", 0.125)
    for j in range(m):
        bound = _apply_bound(Kb, Kref, V[:, j], kqr.KQR_APPLY_EXACT)
        assert np.all(np.abs(U[:, j] - Kref @ V[:, j]) <= bound)


def test_predict(dev):
    n, m, p = 900, 333, 10
    X, y = inputs.smooth(n + m, p, (106, 0))
    a = np.random.default_rng(3).uniform(-0.5, 0.5, n)
    beta, lam, gamma = 0.3, 2.0, 0.1
    say("predict", n, m)
    f = kqr.kqr_predict(torch.from_numpy(X[:n]).to(dev), torch.from_numpy(a).to(dev), beta, lam, "rbf", gamma,
                        torch.from_numpy(X[n:]).to(dev)).cpu().numpy()
    Kv = okernel.kernel_block(X[n:], X[:n], "rbf", gamma)
    ref = beta + Kv @ a / lam
    err = np.abs(f - ref)
    assert np.all(err <= (70 * U32 + 1e-5) * (np.abs(Kv) @ np.abs(a)) / lam + 1e-12)


# --------------------------------------------------------------------- RPCholesky
@pytest.mark.parametrize("materialised", [True, False])
def test_rpcholesky_matches_oracle(dev, materialised):
    n, p, r = 600, 5, 40
    X, _ = inputs.smooth(n, p, (107, 0))
    gamma = 0.5
    u = inputs.pivot_uniforms(r, (107, 1))
    say("rpcholesky", materialised)
    Xt = torch.from_numpy(X).to(dev)
    K = kqr.kqr_kernel_build(Xt, "rbf", gamma, "fp32") if materialised else None
    F, piv, rout = kqr.kqr_rpcholesky(r, u, X=Xt, kernel="rbf", gamma=gamma, K=K)
    F = F.cpu().numpy()[:, :rout].astype(np.float64)
    op = okernel.DenseKernel(X, "rbf", gamma)
    Fo, pivo, _ = oprecond.rpcholesky(op, r, u)
    # pivots are an integer decision: equal unless the oracle's running sum sits
    # within rounding of the threshold at the first difference
    m = 0
    while m < min(rout, len(pivo)) and piv[m] == pivo[m]:
        m += 1
    if m < r:
        d = np.diag(op.K - Fo[:, :m] @ Fo[:, :m].T)
        d = np.maximum(d, 0)
        c = np.cumsum(d)
        thr = u[m] * c[-1]
        j = pivo[m]
        near = min(abs(c[j] - thr), abs(c[j - 1] - thr) if j > 0 else np.inf)
        assert near <= 1e-5 * c[-1], (m, near)
    assert m >= 1
    scale = np.abs(Fo[:, :m]).max()
    assert np.abs(F[:, :m] - Fo[:, :m]).max() <= 2e-4 * scale
    # whatever pivots were taken, F F^T interpolates K on them (Nystrom property)
    R = op.K - F @ F.T
    assert np.abs(R[np.ix_(piv, piv)]).max() < 1e-4


# --------------------------------------------------------------------- Woodbury
# r + 1 = 61: one 64-column block of the core factorisation; 64 / 65 and
# 128 / 129: block edges; 301: five blocks and a ragged one, two doubling
# levels of the inverse; 512: eight full blocks, three levels.
@pytest.mark.parametrize("lmin,r", [(1e-2, 60), (1e-7, 60), (1e-2, 63), (1e-2, 64), (1e-2, 127), (1e-2, 128),
                                    (1e-2, 300), (1e-2, 511)])
def test_woodbury_apply(dev, lmin, r):
    n = 1111
    g = np.random.default_rng(8)
    F = (g.standard_normal((n, r)) * 0.3).astype(np.float32)
    L = g.uniform(lmin, 2.0, n)
    L[::7] = lmin
    w = g.standard_normal(n)
    c = 0.7
    say("woodbury", lmin, r)
    Ft = torch.zeros((n, (r + 3) // 4 * 4), dtype=torch.float32)
    Ft[:, :r] = torch.from_numpy(F)
    out = kqr.kqr_woodbury_apply(Ft.to(dev), r, c, torch.from_numpy(L).to(dev), torch.from_numpy(w).to(dev)).cpu().numpy()
    W = oprecond.Woodbury(F.astype(np.float64), c, L)
    ref = W.apply(w)
    # FP64 throughout on exactly representable FP32 factors; error grows with cond(C)
    tol = 1e-10 if lmin > 1e-3 else 1e-5
    assert np.linalg.norm(out - ref) <= tol * np.linalg.norm(ref)
    # P (P^{-1} w) = w
    P = W.dense(F.astype(np.float64), c)
    assert np.linalg.norm(P @ out - w) <= (1e-9 if lmin > 1e-3 else 1e-4) * np.linalg.norm(w)


def test_woodbury_rank_zero(dev):
    n = 500
    g = np.random.default_rng(9)
    L = g.uniform(0.1, 1.0, n)
    w = g.standard_normal(n)
    say("woodbury r=0")
    out = kqr.kqr_woodbury_apply(None, 0, 2.0, torch.from_numpy(L).to(dev), torch.from_numpy(w).to(dev)).cpu().numpy()
    P = 2.0 * np.ones((n, n)) + np.diag(L)
    assert np.linalg.norm(out - np.linalg.solve(P, w)) <= 1e-11 * np.linalg.norm(w)


# --------------------------------------------------------------------- PCG
@pytest.mark.parametrize("rank", [0, 30])
def test_pcg_solve(dev, rank):
    n, p = 1200, 6
    X, y = inputs.smooth(n, p, (110, 0))
    gamma, c = 0.2, 0.5
    g = np.random.default_rng(10)
    L = g.uniform(0.5, 1.5, n)
    b = g.standard_normal(n)
    say("pcg", rank)
    Xt = torch.from_numpy(X).to(dev)
    K = kqr.kqr_kernel_build(Xt, "rbf", gamma, "fp32")
    F = None
    if rank:
        op = okernel.DenseKernel(X, "rbf", gamma)
        Fo, _, _ = oprecond.rpcholesky(op, rank, inputs.pivot_uniforms(rank, (110, 1)))
        F = torch.zeros((n, (rank + 3) // 4 * 4), dtype=torch.float32)
        F[:, :rank] = torch.from_numpy(Fo.astype(np.float32))
        F = F.to(dev)
    tol = 1e-8 * np.linalg.norm(b)
    x, it, res = kqr.kqr_pcg_solve(Xt, "rbf", gamma, c, torch.from_numpy(L).to(dev), torch.from_numpy(b).to(dev),
                                   tol, 500, K=K, F=F, r=rank)
    x = x.cpu().numpy()
    Kref = okernel.kernel_matrix(X, "rbf", gamma)
    A = Kref + c + np.diag(L)
    xs = np.linalg.solve(A, b)
    assert res <= tol and it > 0
    # the GPU system uses FP32 entries: ||dx|| <= ||A^-1|| ||dK|| ||x|| + ||A^-1|| tol
    dK = 2e-6 * np.abs(Kref).sum(1).max()
    assert np.linalg.norm(x - xs) <= (dK * np.linalg.norm(xs) + tol) / L.min() * 2
    if rank:
        _, it0, _ = kqr.kqr_pcg_solve(Xt, "rbf", gamma, c, torch.from_numpy(L).to(dev), torch.from_numpy(b).to(dev),
                                      tol, 500, K=K, r=0)
        assert it < it0  # the preconditioner helps


# --------------------------------------------------------------------- SSN set-up
def test_ssn_gradient(dev):
    n = 2345
    g = np.random.default_rng(11)
    tau, lam, beta, sigma = 0.3, 1.7, 0.25, 3.0
    alpha = g.uniform(-0.9, 0.5, n)
    Ka = g.standard_normal(n) * 5
    y = g.standard_normal(n)
    z = g.standard_normal(n)
    say("ssn_gradient")
    out = kqr.kqr_ssn_gradient(tau, lam, beta, sigma, *(torch.from_numpy(a).to(dev) for a in (alpha, Ka, y, z)))
    ref = oproblem.grad_phi(alpha, Ka, y, lam, tau, beta, z, sigma)
    w = alpha + z / sigma
    S = oproblem.jacobian_mask(w, tau)
    gn = np.linalg.norm(ref)
    et = max(0.1 * min(0.1, gn), 1e-12)
    assert np.allclose(out["grad"].cpu().numpy(), ref, rtol=1e-13, atol=1e-12)
    assert np.array_equal(out["S"].cpu().numpy().astype(np.float64), S)
    assert out["gnorm"] == pytest.approx(gn, rel=1e-13)
    assert out["eps_t"] == pytest.approx(et, rel=1e-13)
    assert np.allclose(out["Ldiag"].cpu().numpy(), lam * sigma * (1 - S) + lam * et, rtol=1e-15)
    assert np.allclose(out["rhs"].cpu().numpy(), -lam * ref, rtol=1e-13, atol=1e-12)


# --------------------------------------------------------------------- full fit
_ORACLE = {}


def oracle_fit(prob, **kw):
    key = (prob.name, prob.n, tuple(sorted(kw.items())))
    if key not in _ORACLE:
        _ORACLE[key] = osolver.fit(prob.X, prob.y, prob.tau, prob.lam, prob.kernel, prob.gamma,
                                   osolver.OracleOptions(tol=1e-10, **kw))
    return _ORACLE[key]


def alpha_tolerance(Kref, Kb, ref, lam, tau, y, level):
    """How far the GPU's alpha may lie from the FP64 optimum alpha*, to first
    order, relative to 1 + ||alpha*||.

    The GPU solves the problem with FP32 kernel entries, each within Kb of
    the FP64 one, to a KKT level `level`.  On a stable partition (L, E, R) of
    the optimum, alpha_N sits on its bounds and (alpha_E, beta) solve the
    bordered system G [alpha_E; beta] = [y_E - K_EN alpha_N / lambda;
    -1^T alpha_N] with G = [K_EE / lambda, 1; 1^T, 0] (the KKT conditions of
    (1.3)), so both the entry error and the residual the solver leaves move
    alpha_E by at most ||G^-1|| times their size on E: ||(Kb |alpha*|)_E|| /
    lambda for the entries, level (1 + ||y||) for the residual."""
    a = ref.alpha
    E = np.flatnonzero((a > tau - 1 + 1e-9) & (a < tau - 1e-9))
    if E.size == 0:
        return 0.0  # alpha* is fixed by the partition
    m = E.size
    G = np.zeros((m + 1, m + 1))
    G[:m, :m] = Kref[np.ix_(E, E)] / lam
    G[:m, m] = 1.0
    G[m, :m] = 1.0
    ginv = np.linalg.norm(np.linalg.inv(G), 2)
    r = np.linalg.norm(Kb[E] @ np.abs(a)) / lam + level * (1.0 + np.linalg.norm(y))
    return ginv * r / (1.0 + np.linalg.norm(a))


def certificate(prob, alpha, beta):
    """FP64 residuals of a returned (alpha, beta) with exact K: z = y - beta - K alpha/lambda, v = Pi_B(alpha)."""
    K = okernel.kernel_matrix(prob.X, prob.kernel, prob.gamma)
    Ka = K @ alpha
    z = prob.y - beta - Ka / prob.lam
    v = oproblem.proj_box(alpha, prob.tau)
    return oproblem.kkt(alpha, v, beta, z, Ka, prob.y, prob.lam, prob.tau)


@pytest.mark.parametrize("name,n,rank", [("c0", 2000, 0), ("c1", 3000, 200), ("c4", 2500, 0), ("c0", 901, -1)])
def test_fit_matches_oracle(dev, name, n, rank):
    prob = inputs.workload(name, n=n)
    say("fit", name, n, rank)
    X = torch.from_numpy(prob.X).to(dev)
    y = torch.from_numpy(prob.y).to(dev)
    alpha, beta, info, st = kqr.kqr_fit(X, y, prob.tau, prob.lam, prob.kernel, prob.gamma, rank=rank,
                                        uniforms=inputs.pivot_uniforms(max(rank, 64), (n, 5)), out_vz=True)
    a = alpha.cpu().numpy()
    say("  gpu info", {k: info[k] for k in ("eta_kkt", "eta_gap", "admm_iters", "alm_iters", "newton_iters",
                                            "pcg_iters", "kapply_calls", "rank_used", "t_total")})
    assert st == kqr.KQR_OK
    assert max(info["eta_kkt"], info["eta_gap"]) <= 1e-6
    ref = oracle_fit(prob)
    opt = ref.kkt["obj_p"]
    cert = certificate(prob, a, beta)
    rel_obj = abs(cert["obj_p"] - opt) / (1 + abs(opt))
    alpha_err = np.linalg.norm(a - ref.alpha) / (1 + np.linalg.norm(ref.alpha))
    # the Section 4 measures at the returned iterate (alpha, v, beta, z) with
    # the FP64 kernel: the fit's target, up to the FP32 entry error of K alpha
    Kref, Kb = entry_bound(prob.X, prob.kernel, prob.gamma)
    a_tol = alpha_tolerance(Kref, Kb, ref, prob.lam, prob.tau, prob.y, max(info["eta_kkt"], info["eta_gap"]))
    Ka = Kref @ a
    m64 = oproblem.kkt(a, info["v"].cpu().numpy(), beta, info["z"].cpu().numpy(), Ka, prob.y, prob.lam, prob.tau)
    dKa = Kb @ np.abs(a)
    shift_p = np.linalg.norm(dKa) / prob.lam / (1 + np.linalg.norm(prob.y))
    shift_gap = (np.abs(a) @ dKa / prob.lam) / (1 + abs(m64["obj_p"]) + abs(m64["obj_d"]))
    say(f"  rel_obj={rel_obj:.2e} alpha_err={alpha_err:.2e} (first-order bound {a_tol:.2e}) "
        f"FP64 eta_kkt={m64['eta_kkt']:.2e} eta_gap={m64['eta_gap']:.2e} beta={beta:.6f} beta*={ref.beta:.6f}")
    assert rel_obj <= 1e-6
    # alpha* is unique (K positive definite): within the first-order bound of
    # the FP32 entry error and the solver's residual (factor 2 for second
    # order), or the 1e-6 bar, whichever is larger
    assert alpha_err <= max(1e-6, 2 * a_tol)
    assert m64["eta_p"] <= 1e-6 + shift_p
    assert m64["eta_d"] <= 1e-6 and m64["eta_c"] <= 1e-6
    assert m64["eta_gap"] <= 1e-6 + shift_gap


def test_fit_is_deterministic(dev):
    prob = inputs.workload("c0", n=800)
    X = torch.from_numpy(prob.X).to(dev)
    y = torch.from_numpy(prob.y).to(dev)
    say("determinism")
    a1, b1, _, _ = kqr.kqr_fit(X, y, prob.tau, prob.lam, "rbf", prob.gamma)
    a2, b2, _, _ = kqr.kqr_fit(X, y, prob.tau, prob.lam, "rbf", prob.gamma)
    assert torch.equal(a1, a2) and b1 == b2


def test_fit_error_paths(dev):
    prob = inputs.workload("c0", n=300)
    X = torch.from_numpy(prob.X).to(dev)
    y = prob.y.copy()
    y[17] = np.nan
    say("error paths")
    with pytest.raises(kqr.KqrError) as e:
        kqr.kqr_fit(X, torch.from_numpy(y).to(dev), prob.tau, prob.lam, "rbf", prob.gamma)
    assert e.value.status == kqr.KQR_ENUMERIC
    yt = torch.from_numpy(prob.y).to(dev)
    _, _, info, st = kqr.kqr_fit(X, yt, prob.tau, prob.lam, "rbf", prob.gamma, admm_max_iter=2, alm_max_iter=1,
                                 tol=1e-12)
    assert st == kqr.KQR_NOT_CONVERGED and info["alm_iters"] == 1


# --------------------------------------------------------------------- full size, sampled
def test_kernel_apply_full_size_sampled(dev):
    """The benchmark's configuration: n = 50,000, p = 20, FP32 K (10 GB), fast apply.

    Rows are sampled and computed one by one by the oracle."""
    prob = inputs.workload("c1")
    n = prob.n
    say("full-size apply", n)
    X = torch.from_numpy(prob.X).to(dev)
    K = kqr.kqr_kernel_build(X, "rbf", prob.gamma, "fp32")
    v = np.random.default_rng(12).standard_normal(n)
    u = kqr.kqr_kernel_apply(torch.from_numpy(v).to(dev), K=K, mode=kqr.KQR_APPLY_FAST).cpu().numpy()
    ue = kqr.kqr_kernel_apply(torch.from_numpy(v).to(dev), K=K, mode=kqr.KQR_APPLY_EXACT).cpu().numpy()
    del K
    torch.cuda.empty_cache()
    rows = np.random.default_rng(13).choice(n, 48, replace=False)
    Xd = prob.X.astype(np.float64)
    q = (Xd * Xd).sum(1)
    for i in rows:
        d = okernel.distance_block(prob.X[i:i + 1], prob.X, "rbf")[0]
        k = np.exp(-prob.gamma * d)
        kb = k * (prob.gamma * (4.0 * 22 * U32 * (q[i] + q) + 2 * U32 * d) + 8 * U32)
        ref = k @ v
        assert abs(u[i] - ref) <= kb @ np.abs(v) + 12 * U32 * (k @ np.abs(v)) + 1e-12
        assert abs(ue[i] - ref) <= kb @ np.abs(v) + 1e-12
