"""The error against FP64 of a full-size fit, certified without the optimum.

The benchmark's configuration (n = 50,000, p = 20, FP32 K of 10 GB, rank-500
preconditioner) is fitted on the GPU; the oracle's FP64 certificate
(oracle.certify: one pass of FP64 kernel products by direct differences)
then gives, at the returned point,

* the Section 4 measures at the returned iterate (alpha, v, beta, z) with the
  exact FP64 kernel, which must meet the fit's target up to the FP32 entry
  error of K alpha (bounded per row below), and agree with the fit's own
  report within that error;
* a weak-duality sandwich of the optimal value, whose width bounds the
  relative objective error of the returned point.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import certify
from paper_2510_07929_amd import inputs, kqr

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    kqr.lib()
    return torch.device("cuda:0")


def test_full_size_fit_certificate(dev):
    prob = inputs.workload("c1")
    n, p = prob.n, prob.p
    say("full-size certificate", prob.name, n)
    X = torch.from_numpy(prob.X).to(dev)
    y = torch.from_numpy(prob.y).to(dev)
    alpha, beta, info, st = kqr.kqr_fit(X, y, prob.tau, prob.lam, prob.kernel, prob.gamma, rank=prob.rank,
                                        uniforms=inputs.pivot_uniforms(prob.rank, (1, 5)), out_vz=True)
    assert st == kqr.KQR_OK
    a, v, z = alpha.cpu().numpy(), info["v"].cpu().numpy(), info["z"].cpu().numpy()
    del X, alpha
    torch.cuda.empty_cache()
    Xd = prob.X.astype(np.float64)
    q = (Xd * Xd).sum(1)
    # K |alpha| and K (q |alpha|) in the same pass: the FP32-entry error of the
    # GPU's K alpha is at most gamma u (4 (p + 2) (q_i + q_j) + 2 d_ij) K_ij + 8 u K_ij
    # per entry (norm expansion, then exp), and d_ij <= 2 (q_i + q_j)
    c = certify.certificate(prob.X, prob.y, prob.tau, prob.lam, prob.kernel, prob.gamma, a, beta, v=v, z=z,
                            extra=np.stack([np.abs(a), q * np.abs(a)], axis=1))
    w1, w2 = c["K_extra"][:, 0], c["K_extra"][:, 1]
    dKa = prob.gamma * U32 * (4.0 * (p + 2) + 4.0) * (q * w1 + w2) + 8.0 * U32 * w1
    ny = 1.0 + np.linalg.norm(prob.y)
    shift_p = np.linalg.norm(dKa) / prob.lam / ny
    dobj = np.abs(a) @ dKa / (2.0 * prob.lam)
    scale = 1.0 + abs(c["obj_p"]) + abs(c["obj_d"])
    say(f"  FP64 at the returned iterate: eta_p {c['eta_p']:.2e} eta_d {c['eta_d']:.2e} eta_c {c['eta_c']:.2e} "
        f"eta_gap {c['eta_gap']:.2e}; FP32-entry shift of eta_p <= {shift_p:.1e}")
    say(f"  GPU report: eta_p {info['eta_p']:.2e} eta_d {info['eta_d']:.2e} eta_c {info['eta_c']:.2e} "
        f"eta_gap {info['eta_gap']:.2e}")
    say(f"  sandwich: obj_P {c['obj_p_returned']:.12e} in [{c['lower']:.12e}, {c['upper']:.12e}], "
        f"relative objective error <= {c['rel_obj_err_bound']:.2e}; |E| = {c['n_interior']}")
    say(f"  residual form: eta_d {c['res_eta_d']:.2e} eta_c {c['res_eta_c']:.2e} eta_gap {c['res_eta_gap']:.2e}")
    # the stopping measures hold with the exact kernel, up to the entry error
    assert c["eta_p"] <= 1e-6 + shift_p
    assert c["eta_d"] <= 1e-6 and c["eta_c"] <= 1e-6
    assert c["eta_gap"] <= 1e-6 + 2 * dobj / scale
    # and the fit's own report is the FP64 one moved by at most that error
    assert abs(info["eta_p"] - c["eta_p"]) <= shift_p + 1e-12
    assert abs(info["eta_d"] - c["eta_d"]) <= 1e-12 * (1 + c["eta_d"]) and abs(info["eta_c"] - c["eta_c"]) <= 1e-12
    assert abs(info["obj_p"] - c["obj_p"]) <= dobj + 1e-12 * abs(c["obj_p"])
    # relative objective error of the returned (alpha, beta) against the optimum, bounded by the
    # sandwich (the primal objective at theta = alpha, beta minus a dual lower bound)
    assert c["lower"] <= c["upper"]
    assert c["rel_obj_err_bound"] <= 1e-6
