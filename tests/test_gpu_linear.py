"""GPU parity of the linear kernel k(x, x') = x^T x' (Table 2): factored
K-apply, prediction, fits and lambda paths against the FP64 oracle.  K = X X^T
is only positive semidefinite, so alpha is not unique; the comparisons use
what is: the objective, K alpha (the fitted values) and the KKT residuals."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import kernel as okernel
from oracle import problem as oproblem
from oracle import solver as osolver
from paper_2510_07929_amd import inputs, kqr

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    kqr.lib()
    return torch.device("cuda:0")


def test_linear_apply_and_predict(dev):
    n, m, p = 3001, 257, 5
    X, _ = inputs.smooth(n + m, p, (150, 0))
    Xd = X.astype(np.float64)
    V = np.random.default_rng(1).standard_normal((n, 3))
    Xt = torch.from_numpy(X[:n].copy()).to(dev)
    U = kqr.kqr_kernel_apply(torch.from_numpy(V).to(dev), X=Xt, kernel="linear", gamma=1.0).cpu().numpy()
    ref = Xd[:n] @ (Xd[:n].T @ V)
    scale = np.abs(Xd[:n]) @ (np.abs(Xd[:n]).T @ np.abs(V))
    assert np.all(np.abs(U - ref) <= 1e-13 * scale + 1e-300)
    alpha = np.random.default_rng(2).uniform(-0.5, 0.5, n)
    f = kqr.kqr_predict(Xt, torch.from_numpy(alpha).to(dev), 0.7, 2.0, "linear", 1.0,
                        torch.from_numpy(X[n:].copy()).to(dev)).cpu().numpy()
    fref = 0.7 + Xd[n:] @ (Xd[:n].T @ alpha) / 2.0
    assert np.abs(f - fref).max() <= 1e-12 * (1 + np.abs(fref).max())


def _check(K, X, y, tau, lam, a, b, info, st, tol):
    ref = osolver.fit(X, y, tau, lam, "linear", 1.0, osolver.OracleOptions(tol=1e-10))
    Ka = K @ a
    obj = oproblem.primal_objective(y - b - Ka / lam, a, Ka, lam, tau)
    opt = ref.kkt["obj_p"]
    rel = abs(obj - opt) / (1 + abs(opt))
    fit_gpu, fit_ref = Ka / lam, ref.Kalpha / lam
    dfit = np.abs(fit_gpu - fit_ref).max() / (1 + np.abs(fit_ref).max())
    say(f"  tau={tau} lam={lam:.4g} status={st} rel_obj={rel:.2e} d_fit={dfit:.2e} kkt={info['eta_kkt']:.2e} "
        f"gap={info['eta_gap']:.2e} rank={info['rank_used']} pcg={info['pcg_iters'] + info['admm_pcg_iters']}")
    assert st == kqr.KQR_OK
    assert max(info["eta_kkt"], info["eta_gap"]) <= tol
    assert rel <= 1e-6
    assert dfit <= 1e-5


@pytest.mark.parametrize("tau", [0.1, 0.5, 0.9])
def test_linear_fit_matches_oracle(dev, tau):
    n, lam = 2000, 1.0
    X, y = inputs.paper2d(n, (151, int(10 * tau)))
    say("linear fit", n, tau)
    a, b, info, st = kqr.kqr_fit(torch.from_numpy(X).to(dev), torch.from_numpy(y).to(dev), tau, lam, "linear", 1.0,
                                 tol=1e-8)
    assert info["rank_used"] == 2
    K = okernel.kernel_matrix(X, "linear", 1.0)
    _check(K, X, y, tau, lam, a.cpu().numpy(), b, info, st, 1e-8)


def test_linear_fit_higher_dimension_and_plain_cg(dev):
    n, p, tau, lam = 1500, 10, 0.3, 2.0
    X, y = inputs.smooth(n, p, (152, 0))
    K = okernel.kernel_matrix(X, "linear", 1.0)
    for rank in (0, -1):
        say("linear fit p=10, rank option", rank)
        a, b, info, st = kqr.kqr_fit(torch.from_numpy(X).to(dev), torch.from_numpy(y).to(dev), tau, lam, "linear",
                                     1.0, tol=1e-8, rank=rank)
        assert info["rank_used"] == (p if rank >= 0 else 0)
        _check(K, X, y, tau, lam, a.cpu().numpy(), b, info, st, 1e-8)


def test_linear_path_matches_oracle(dev):
    n, tau = 1200, 0.5
    X, y = inputs.paper2d(n, (153, 0))
    lams = inputs.lambda_grid(18)
    say("linear path", n, len(lams))
    A, betas, infos, sts = kqr.kqr_fit_path(torch.from_numpy(X).to(dev), torch.from_numpy(y).to(dev), tau, lams,
                                            "linear", 1.0, tol=1e-8)
    A = A.cpu().numpy()
    K = okernel.kernel_matrix(X, "linear", 1.0)
    for t, lam in enumerate(lams):
        _check(K, X, y, tau, lam, A[t], betas[t], infos[t], sts[t], 1e-8)


def test_linear_kernel_rejections(dev):
    X = torch.zeros((10, 2), dtype=torch.float32, device=dev)
    y = torch.zeros(10, dtype=torch.float64, device=dev)
    with pytest.raises(kqr.KqrError):
        kqr.kqr_kernel_build(X, "linear", 1.0)
    with pytest.raises(kqr.KqrError):
        kqr.kqr_kernel_build_packed(X, "linear", 1.0)
    with pytest.raises(kqr.KqrError):
        kqr.kqr_fit_grad(X, y, 0.5, 1.0, "linear", 1.0, X, y)
