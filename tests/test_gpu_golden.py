"""GPU fits and adjoint gradients of the stored tiny problems
(tests/golden/tiny_fits.json, oracle values pinned by brute force in
tests/test_golden.py): the smallest sizes the path accepts, one 64-column
tile with a ragged tail."""
import json
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import kernel as okernel
from oracle import problem as oproblem
from paper_2510_07929_amd import kqr

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
CASES = json.load(open(os.path.join(HERE, "golden", "tiny_fits.json")))["cases"]


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    kqr.lib()
    return torch.device("cuda:0")


def _t(c, key, dtype, dev):
    return torch.tensor(np.asarray(c[key]), dtype=dtype, device=dev).contiguous()


@pytest.mark.parametrize("c", CASES, ids=lambda c: c["name"])
def test_tiny_fit_matches_golden(dev, c):
    say("golden fit", c["name"])
    X, y = _t(c, "X", torch.float32, dev), _t(c, "y", torch.float64, dev)
    alpha, beta, info, st = kqr.kqr_fit(X, y, c["tau"], c["lam"], c["kernel"], c["gamma"])
    assert st == kqr.KQR_OK
    a = alpha.cpu().numpy()
    Xd = np.asarray(c["X"])
    K = okernel.kernel_matrix(Xd, c["kernel"], c["gamma"])
    Ka = K @ a
    obj = oproblem.primal_objective(np.asarray(c["y"]) - beta - Ka / c["lam"], a, Ka, c["lam"], c["tau"])
    rel = abs(obj - c["obj_p"]) / (1 + abs(c["obj_p"]))
    say(f"  rel_obj={rel:.2e} kkt={info['eta_kkt']:.2e}")
    assert rel <= 1e-6
    # alpha is the ALM iterate (not its box projection): its distance to the
    # box and its sum are bounded by the dual and primal residuals reached
    assert abs(a.sum()) <= 1e-6 * (1 + np.abs(a).sum())
    assert max(0.0, a.max() - c["tau"], c["tau"] - 1 - a.min()) <= 1e-6 * (1 + np.linalg.norm(a))


@pytest.mark.parametrize("c", [c for c in CASES if "J" in c], ids=lambda c: c["name"])
def test_tiny_gradient_matches_golden(dev, c):
    say("golden gradient", c["name"])
    X, y = _t(c, "X", torch.float32, dev), _t(c, "y", torch.float64, dev)
    Xv, yv = _t(c, "Xval", torch.float32, dev), _t(c, "yval", torch.float64, dev)
    alpha, beta, J, (dg, dl), m, pol, info, st = kqr.kqr_fit_grad(X, y, c["tau"], c["lam"], c["kernel"], c["gamma"],
                                                                  Xv, yv, tol=1e-9)
    assert st == kqr.KQR_OK and pol and m == c["n_interior"]
    assert np.max(np.abs(alpha.cpu().numpy() - np.asarray(c["alpha"]))) <= 1e-9
    assert J == pytest.approx(c["J"], rel=1e-9)
    scale = abs(c["dJ_dlog_gamma"]) + abs(c["dJ_dlog_lambda"])
    assert abs(dg - c["dJ_dlog_gamma"]) <= 1e-9 * scale
    assert abs(dl - c["dJ_dlog_lambda"]) <= 1e-9 * scale
