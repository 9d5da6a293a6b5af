"""Edge cases of the fit on the GPU against the FP64 oracle: the smallest n,
one feature and the largest p, extreme quantile levels, a penalty so large
that no coefficient is interior (beta then is not unique: only the objective
and alpha are compared), Phase I skipped, and the on-the-fly operator with
p beyond the matrix-core path."""
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


def _fit_and_compare(dev, X, y, tau, lam, kind, gamma, **kw):
    Xt = torch.from_numpy(X).to(dev)
    yt = torch.from_numpy(y).to(dev)
    alpha, beta, info, st = kqr.kqr_fit(Xt, yt, tau, lam, kind, gamma, **kw)
    assert st == kqr.KQR_OK
    a = alpha.cpu().numpy()
    ref = osolver.fit(X, y, tau, lam, kind, gamma, osolver.OracleOptions(tol=1e-10))
    K = okernel.kernel_matrix(X, kind, gamma)
    Ka = K @ a
    obj = oproblem.primal_objective(y - beta - Ka / lam, a, Ka, lam, tau)
    opt = ref.kkt["obj_p"]
    rel = abs(obj - opt) / (1 + abs(opt))
    say(f"  rel_obj={rel:.2e} kkt={info['eta_kkt']:.2e} |E|={info['n_interior']}")
    assert rel <= 1e-6
    return a, beta, ref


def test_two_points(dev):
    X = np.array([[0.0], [1.0]], dtype=np.float32)
    y = np.array([0.0, 1.0])
    say("n = 2")
    _fit_and_compare(dev, X, y, 0.3, 0.5, "rbf", 1.0)


@pytest.mark.parametrize("p", [1, 64])
def test_feature_count_limits(dev, p):
    X, y = inputs.smooth(700, p, (600, p))
    say("p =", p)
    _fit_and_compare(dev, X, y, 0.5, 0.7, "rbf", 1.0 / p)


@pytest.mark.parametrize("tau", [0.01, 0.99])
def test_extreme_quantile_levels(dev, tau):
    X, y = inputs.smooth(800, 5, (601, int(tau * 100)))
    say("tau =", tau)
    _fit_and_compare(dev, X, y, tau, 0.8, "rbf", 0.2)


def test_no_interior_coefficient(dev):
    # huge lambda: K alpha / lambda vanishes and every alpha sits on a bound
    # (tau n integral), so beta is any sample tau-quantile of y
    n = 400
    X, y = inputs.smooth(n, 3, (602, 0))
    tau = 0.25
    say("no interior coefficient")
    a, beta, ref = _fit_and_compare(dev, X, y, tau, 1e9, "rbf", 0.3)
    # the oracle's polished optimum has every alpha on a bound; the returned
    # ALM iterate is within its dual residual of it (||alpha - v|| <= eta_d (1 + ||alpha||))
    assert np.all((np.abs(ref.alpha - tau) < 1e-12) | (np.abs(ref.alpha - (tau - 1)) < 1e-12))
    assert np.max(np.abs(a - ref.alpha)) <= 1e-6 * (1 + np.linalg.norm(ref.alpha))
    lo, hi = np.sort(y)[int(tau * n) - 1], np.sort(y)[int(tau * n)]
    assert lo - 1e-6 <= beta <= hi + 1e-6


def test_phase_one_skipped(dev):
    prob = inputs.workload("c0", n=900)
    say("Phase I skipped")
    _fit_and_compare(dev, prob.X, prob.y, prob.tau, prob.lam, prob.kernel, prob.gamma, admm_max_iter=0)


def test_on_the_fly_rbf_beyond_matrix_core_path(dev):
    # p = 40 > 32: the on-the-fly RBF apply falls back to the VALU kernel
    X, y = inputs.smooth(1100, 40, (603, 0))
    say("on the fly, p = 40")
    _fit_and_compare(dev, X, y, 0.6, 1.1, "rbf", 1.0 / 40, kmode=kqr.KQR_KMODE_ON_THE_FLY)


# The square on-the-fly applies evaluate each distinct pair once over
# 128 x 128 upper-triangle tiles: one point, a partial single tile, exactly
# one tile, one tile and one column, and two tiles with a one-row tail
# (RBF p = 10: FP32 matrix-core Gram; 30 and 32: BF16x3 with and without the
# folded norms).
@pytest.mark.parametrize("kind,p", [("laplacian", 30), ("rbf", 10), ("rbf", 30), ("rbf", 32)])
@pytest.mark.parametrize("n", [1, 5, 127, 128, 129, 257])
@pytest.mark.parametrize("mode", [kqr.KQR_APPLY_FAST, kqr.KQR_APPLY_EXACT])
def test_on_the_fly_symmetric_apply_tile_edges(dev, kind, p, n, mode):
    X, _ = inputs.additive(n, p, (611, n))
    v = np.random.default_rng(n).standard_normal(n)
    gamma = 1.0 / p
    say("otf tile edges", kind, p, n, mode)
    u = kqr.kqr_kernel_apply(torch.from_numpy(v).to(dev), X=torch.from_numpy(X).to(dev), kernel=kind,
                             gamma=gamma, mode=mode).cpu().numpy()
    from tests.test_gpu_parity import _apply_bound, entry_bound  # the FP32 entry and sum bounds
    Kref, Kb = entry_bound(X, kind, gamma)
    bound = _apply_bound(Kb, Kref, v, mode, otf=True)
    err = np.abs(u - Kref @ v)
    assert np.all(err <= bound), float((err / bound).max())


@pytest.mark.parametrize("kind,p", [("laplacian", 30), ("rbf", 10), ("rbf", 30)])
@pytest.mark.parametrize("mode", [kqr.KQR_APPLY_FAST, kqr.KQR_APPLY_EXACT])
def test_on_the_fly_row_streamed_beyond_symmetric_limit(dev, kind, p, mode):
    # with no room for the symmetric form's partial sums the applies stream all
    # n^2 pairs; both forms agree with the oracle and with each other
    n = 1300
    X, _ = inputs.additive(n, p, (612, n))
    v = np.random.default_rng(3).standard_normal(n)
    gamma = 1.0 / p
    Xt, vt = torch.from_numpy(X).to(dev), torch.from_numpy(v).to(dev)
    say("otf row-streamed", kind, p, mode)
    sym = kqr.kqr_kernel_apply(vt, X=Xt, kernel=kind, gamma=gamma, mode=mode).cpu().numpy()
    try:
        kqr.kqr_set_otf_symmetric_limit(0)
        rows = kqr.kqr_kernel_apply(vt, X=Xt, kernel=kind, gamma=gamma, mode=mode).cpu().numpy()
    finally:
        kqr.kqr_set_otf_symmetric_limit(32 << 30)
    from tests.test_gpu_parity import _apply_bound, entry_bound
    Kref, Kb = entry_bound(X, kind, gamma)
    bound = _apply_bound(Kb, Kref, v, mode, otf=True)
    for u in (sym, rows):
        err = np.abs(u - Kref @ v)
        assert np.all(err <= bound), float((err / bound).max())
    assert np.all(np.abs(sym - rows) <= 2 * bound)
