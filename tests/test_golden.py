"""The stored tiny-problem fixtures (tests/golden/tiny_fits.json, written by
tests/golden/make_golden.py from the oracle) against method-independent
solutions: exhaustive partition enumeration for n = 9, SciPy SLSQP for n = 40,
and central differences of brute-force solutions for the stored gradients."""
import json
import math
import os

import numpy as np
import pytest

from oracle import kernel as okernel
from oracle import problem as oproblem
from tests import pins

HERE = os.path.dirname(os.path.abspath(__file__))
CASES = json.load(open(os.path.join(HERE, "golden", "tiny_fits.json")))["cases"]


def _arrays(c):
    return (np.asarray(c["X"]), np.asarray(c["y"]), np.asarray(c["Xval"]), np.asarray(c["yval"]),
            np.asarray(c["alpha"]))


@pytest.mark.parametrize("c", [c for c in CASES if c["n"] <= 9], ids=lambda c: c["name"])
def test_golden_matches_brute_force(c):
    X, y, _, _, alpha = _arrays(c)
    K = okernel.kernel_matrix(X, c["kernel"], c["gamma"])
    a_bf, b_lo, b_hi = pins.brute_force(K, y, c["lam"], c["tau"])
    assert np.max(np.abs(alpha - a_bf)) <= 1e-10
    assert b_lo - 1e-10 <= c["beta"] <= b_hi + 1e-10
    z = y - c["beta"] - K @ alpha / c["lam"]
    assert oproblem.primal_objective(z, alpha, K @ alpha, c["lam"], c["tau"]) == pytest.approx(c["obj_p"], rel=1e-12)


@pytest.mark.parametrize("c", [c for c in CASES if c["n"] > 9], ids=lambda c: c["name"])
def test_golden_matches_slsqp(c):
    X, y, _, _, alpha = _arrays(c)
    K = okernel.kernel_matrix(X, c["kernel"], c["gamma"])
    a_qp, _ = pins.slsqp_dual(K, y, c["lam"], c["tau"])
    dual = lambda a: a @ K @ a / (2 * c["lam"]) - y @ a
    # the stored point is at least as good as the generic QP solver's and feasible
    assert dual(alpha) <= dual(a_qp) + 1e-9 * (1 + abs(dual(a_qp)))
    assert np.max(np.abs(alpha - a_qp)) <= 1e-5
    assert abs(alpha.sum()) <= 1e-12 and alpha.min() >= c["tau"] - 1 and alpha.max() <= c["tau"]


@pytest.mark.parametrize("c", [c for c in CASES if c["n"] <= 9 and "J" in c], ids=lambda c: c["name"])
def test_golden_gradient_matches_brute_force_differences(c):
    X, y, Xv, yv, _ = _arrays(c)
    h = 1e-6

    def J(lg, ll):
        g, lam = math.exp(lg), math.exp(ll)
        K = okernel.kernel_matrix(X, c["kernel"], g)
        a, b, b2 = pins.brute_force(K, y, lam, c["tau"])
        assert b == b2  # unique beta (interior set non-empty)
        Kv = okernel.kernel_block(Xv, X, c["kernel"], g)
        return oproblem.check_loss(yv - b - Kv @ a / lam, c["tau"])

    lg, ll = math.log(c["gamma"]), math.log(c["lam"])
    assert J(lg, ll) == pytest.approx(c["J"], rel=1e-10)
    fd_g = (J(lg + h, ll) - J(lg - h, ll)) / (2 * h)
    fd_l = (J(lg, ll + h) - J(lg, ll - h)) / (2 * h)
    assert c["dJ_dlog_gamma"] == pytest.approx(fd_g, rel=1e-6, abs=1e-8)
    assert c["dJ_dlog_lambda"] == pytest.approx(fd_l, rel=1e-6, abs=1e-8)
