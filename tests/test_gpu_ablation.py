"""GPU parity of the ablations of Section 4.1: the unpreconditioned variant
(plain CG, NALM-KQR), Phase I alone and Phase II alone, and the per-iteration
convergence trace."""
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


def _fit_vs_oracle(dev, prob, tol, **kw):
    X = torch.from_numpy(prob.X).to(dev)
    y = torch.from_numpy(prob.y).to(dev)
    a, b, info, st = kqr.kqr_fit(X, y, prob.tau, prob.lam, prob.kernel, prob.gamma, tol=tol,
                                 uniforms=inputs.pivot_uniforms(128, (50, prob.n)), trace=4000, **kw)
    a = a.cpu().numpy()
    ref = osolver.fit(prob.X, prob.y, prob.tau, prob.lam, prob.kernel, prob.gamma, osolver.OracleOptions(tol=1e-10))
    K = okernel.kernel_matrix(prob.X, prob.kernel, prob.gamma)
    Ka = K @ a
    obj = oproblem.primal_objective(prob.y - b - Ka / prob.lam, a, Ka, prob.lam, prob.tau)
    opt = ref.kkt["obj_p"]
    rel = abs(obj - opt) / (1 + abs(opt))
    say(f"  {kw} status={st} rel_obj={rel:.2e} kkt={info['eta_kkt']:.2e} gap={info['eta_gap']:.2e} "
        f"admm={info['admm_iters']} alm={info['alm_iters']} pcg={info['admm_pcg_iters'] + info['pcg_iters']}")
    assert st == kqr.KQR_OK
    assert max(info["eta_kkt"], info["eta_gap"]) <= tol
    assert rel <= 1e-6
    return info


def test_unpreconditioned_cg_matches_oracle(dev):
    prob = inputs.workload("c0", n=1000)
    say("plain CG (rank < 0)", prob.n)
    info = _fit_vs_oracle(dev, prob, 1e-6, rank=-1)
    assert info["rank_used"] == 0


def test_phase1_alone_matches_oracle(dev):
    prob = inputs.workload("c0", n=600)
    say("ADMM alone", prob.n)
    info = _fit_vs_oracle(dev, prob, 1e-6, admm_tol=1e-6, admm_max_iter=20000, alm_max_iter=0)
    assert info["alm_iters"] == 0 and info["newton_iters"] == 0
    tr = info["trace"]
    assert len(tr) == info["admm_iters"] and np.all(tr[:, 0] == 1)


def test_phase2_alone_matches_oracle(dev):
    prob = inputs.workload("c0", n=900)
    say("SSN-ALM alone", prob.n)
    info = _fit_vs_oracle(dev, prob, 1e-8, admm_max_iter=0)
    assert info["admm_iters"] == 0
    tr = info["trace"]
    assert len(tr) == info["alm_iters"] and np.all(tr[:, 0] == 2)


def test_trace_records_both_phases(dev):
    prob = inputs.workload("path", n=1500)
    X = torch.from_numpy(prob.X).to(dev)
    y = torch.from_numpy(prob.y).to(dev)
    uni = inputs.pivot_uniforms(128, (51, 0))
    a, b, info, st = kqr.kqr_fit(X, y, prob.tau, 0.1, prob.kernel, prob.gamma, tol=1e-8, uniforms=uni, trace=4000)
    tr = info["trace"]
    say("trace", len(tr), "records; last", tr[-1].tolist())
    assert st == kqr.KQR_OK
    n1, n2 = int(np.sum(tr[:, 0] == 1)), int(np.sum(tr[:, 0] == 2))
    assert (n1, n2) == (info["admm_iters"], info["alm_iters"]) and len(tr) == n1 + n2
    assert np.all(tr[:n1, 0] == 1) and np.all(tr[n1:, 0] == 2)
    assert np.array_equal(tr[:n1, 1], np.arange(1, n1 + 1)) and np.array_equal(tr[n1:, 1], np.arange(1, n2 + 1))
    assert np.all(np.diff(tr[:, 3]) >= 0) and tr[-1, 3] <= info["t_total"]
    # Phase I stops at its target; the last ALM record is the accepted iterate
    assert tr[n1 - 1, 2] <= 1e-3 and tr[-1, 2] <= 1e-8
    # a short buffer keeps the first records only
    _, _, info2, _ = kqr.kqr_fit(X, y, prob.tau, 0.1, prob.kernel, prob.gamma, tol=1e-8, uniforms=uni, trace=5)
    assert info2["trace_len"] == 5 and np.array_equal(info2["trace"][:, :3], tr[:5, :3])
