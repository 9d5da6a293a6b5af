"""GPU parity of the regularisation path (lambda sequences of Section 4.1):
every value of lambda against its own FP64 oracle fit."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import kernel as okernel
from oracle import problem as oproblem
from oracle import solver as osolver
from paper_2510_07929_amd import inputs, kqr
from tests.test_gpu_parity import alpha_tolerance, entry_bound

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


def _check_level(K, Kb, X, y, tau, lam, kind, gamma, alpha, beta, info, status, tol):
    ref = osolver.fit(X, y, tau, lam, kind, gamma, osolver.OracleOptions(tol=1e-10))
    Ka = K @ alpha
    z = y - beta - Ka / lam
    obj = oproblem.primal_objective(z, alpha, Ka, lam, tau)
    opt = ref.kkt["obj_p"]
    rel = abs(obj - opt) / (1 + abs(opt))
    da = np.linalg.norm(alpha - ref.alpha) / (1 + np.linalg.norm(ref.alpha))
    say(f"  lam={lam:.4g} rel_obj={rel:.2e} d_alpha={da:.2e} kkt={info['eta_kkt']:.2e} gap={info['eta_gap']:.2e} "
        f"|E|={ref.info['n_interior']} status={status}")
    assert status == kqr.KQR_OK
    assert max(info["eta_kkt"], info["eta_gap"]) <= tol
    assert rel <= 1e-6
    # alpha (unique: K positive definite) within the first-order move of the
    # optimum under the FP32 entry error and the solver's residual (factor 2
    # for second order), or 1e-6, whichever is larger
    a_tol = alpha_tolerance(K, Kb, ref, lam, tau, y, max(info["eta_kkt"], info["eta_gap"]))
    say(f"    alpha bound {a_tol:.2e}")
    assert da <= max(1e-6, 2 * a_tol)


@pytest.mark.parametrize("gamma", [0.1, 1e-3])
def test_path_matches_oracle(dev, gamma):
    # 18 values: more than the 16 that run at once, so workers take second values
    n, tau, tol = 900, 0.5, 1e-8
    X, y = inputs.paper2d(n, (41, int(1 / gamma)))
    lams = inputs.lambda_grid(18)
    say("path", n, gamma, len(lams))
    A, betas, infos, st = kqr.kqr_fit_path(torch.from_numpy(X).to(dev), torch.from_numpy(y).to(dev), tau, lams,
                                           "rbf", gamma, tol=tol, profile=1,
                                           uniforms=inputs.pivot_uniforms(64, (41, 1)))
    A = A.cpu().numpy()
    # the fast applies went out as shared K V launches
    assert infos[0]["kapply_fast_calls"] > 0 and infos[0]["t_kapply_fast"] > 0
    K, Kb = entry_bound(X, "rbf", gamma)
    # with gamma = 1e-3 on the unit square every eigenvalue of K after the third
    # (2e-5, 1e-5, 9e-6, then 2e-9 and below at n = 900) is under the spectral
    # size of the FP32 rounding of its entries (~n 6e-8 = 5e-5): along those
    # directions the objective is flat to rounding.  The interior points come
    # in near-duplicate pairs whose bordered system is nearly singular, so
    # the optimum of an FP32-entry problem moves by up to ~3e-4 in alpha
    # (measured on the oracle with the entries rounded, and with the norm
    # expansion in FP32) while the objective and the KKT residuals stay at
    # the tolerance; the alpha check takes its tolerance from the bordered
    # system's conditioning (alpha_tolerance)
    for t, lam in enumerate(lams):
        _check_level(K, Kb, X, y, tau, lam, "rbf", gamma, A[t], betas[t], infos[t], st[t], tol)


def test_path_on_the_fly_and_order(dev):
    # on-the-fly operator (no coalescing), values given in increasing order
    n, tau, gamma, tol = 700, 0.25, 0.1, 1e-8
    X, y = inputs.paper2d(n, (42, 0))
    lams = sorted(inputs.lambda_grid(5))
    say("path on the fly", n, lams)
    A, betas, infos, st = kqr.kqr_fit_path(torch.from_numpy(X).to(dev), torch.from_numpy(y).to(dev), tau, lams,
                                           "rbf", gamma, tol=tol, kmode=kqr.KQR_KMODE_ON_THE_FLY,
                                           uniforms=inputs.pivot_uniforms(64, (42, 1)))
    A = A.cpu().numpy()
    K, Kb = entry_bound(X, "rbf", gamma)
    for t, lam in enumerate(lams):
        _check_level(K, Kb, X, y, tau, lam, "rbf", gamma, A[t], betas[t], infos[t], st[t], tol)


def test_path_value_equals_single_fit(dev):
    # one value of the path against kqr_fit on the same value (cold starts both)
    prob = inputs.workload("path", n=1200)
    lams = inputs.lambda_grid(6)
    X = torch.from_numpy(prob.X).to(dev)
    y = torch.from_numpy(prob.y).to(dev)
    uni = inputs.pivot_uniforms(64, (43, 0))
    A, betas, infos, st = kqr.kqr_fit_path(X, y, prob.tau, lams, prob.kernel, prob.gamma, tol=1e-8, uniforms=uni)
    K = okernel.kernel_matrix(prob.X, prob.kernel, prob.gamma)
    for t in (0, 3, 5):
        a1, b1, inf1, s1 = kqr.kqr_fit(X, y, prob.tau, lams[t], prob.kernel, prob.gamma, tol=1e-8, uniforms=uni)
        a1 = a1.cpu().numpy()
        a0 = A[t].cpu().numpy()
        objs = []
        for a, b in ((a0, betas[t]), (a1, b1)):
            Ka = K @ a
            objs.append(oproblem.primal_objective(prob.y - b - Ka / lams[t], a, Ka, lams[t], prob.tau))
        say(f"  lam={lams[t]:.4g} path obj {objs[0]:.12g} single obj {objs[1]:.12g}")
        assert st[t] == kqr.KQR_OK and s1 == kqr.KQR_OK
        assert abs(objs[0] - objs[1]) / (1 + abs(objs[1])) <= 1e-7
        assert infos[t]["rank_used"] == inf1["rank_used"]


def test_path_rejects_bad_lambda(dev):
    X = torch.zeros((10, 2), dtype=torch.float32, device=dev)
    y = torch.zeros(10, dtype=torch.float64, device=dev)
    with pytest.raises(kqr.KqrError):
        kqr.kqr_fit_path(X, y, 0.5, [1.0, -1.0], "rbf", 0.1)
    with pytest.raises(kqr.KqrError):
        kqr.kqr_fit_path(X, y, 0.5, [], "rbf", 0.1)
