"""The Section 4 stopping measures of the GPU against the oracle's at the same iterate.

* kqr_kkt_residuals (the kernel every fit measures with) against
  oracle.problem.kkt on a random non-optimal iterate, with and without the
  multiplier step of Algorithms 1 and 2;
* at the iterate a fit returns (alpha, v, beta, z from kqr_fit's optional
  outputs): the GPU kernel fed the oracle's FP64 K alpha reproduces the
  oracle's measures up to FP64 rounding, and the fit's own reported measures
  (taken with FP32 kernel entries) differ from the oracle's only by the
  entry error of K alpha, bounded below.

Bounds: FP64 unit roundoff u = 2^-53; every measure is a sum of n terms, so
two evaluations in different orders differ by at most about n u times the sum
of the magnitudes of the terms (the `scale` of each check).
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import kernel as okernel
from oracle import problem as oproblem
from paper_2510_07929_amd import inputs, kqr
from tests.test_gpu_parity import entry_bound

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53
KEYS = ("eta_p", "eta_d", "eta_c", "eta_gap", "obj_p", "obj_d")


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    kqr.lib()
    return torch.device("cuda:0")


def _scales(alpha, v, beta, z, Ka, y, lam, tau):
    """Sum-of-magnitudes scale of each measure: the FP64 rounding of two
    evaluation orders differs by at most a few n u times this."""
    n = alpha.size
    ny = 1.0 + np.linalg.norm(y)
    mp = np.abs(z) + np.abs(y) + abs(beta) + np.abs(Ka) / lam
    na = 1.0 + np.linalg.norm(alpha)
    aKa = np.abs(alpha) @ np.abs(Ka) / (2.0 * lam)
    rho = np.sum(np.maximum(tau, 1.0 - tau) * np.abs(z))
    ya = np.abs(y) @ np.abs(alpha)
    return dict(
        eta_p=(np.linalg.norm(mp) + n * np.linalg.norm(mp)) / ny,
        eta_d=(n * np.abs(alpha).sum() + np.linalg.norm(alpha) + np.linalg.norm(v)) / na,
        eta_c=n * (np.linalg.norm(z) + np.linalg.norm(v)),
        obj_p=n * (rho + aKa),
        obj_d=n * (aKa + ya),
        eta_gap=n * (rho + 2 * aKa + ya),
    )


def _assert_close(got, ref, scales, what):
    for k in KEYS:
        tol = 8 * U64 * scales[k] + 1e-12 * abs(ref[k])
        say(f"  {what} {k}: gpu {got[k]:.15e} oracle {ref[k]:.15e} |d| {abs(got[k] - ref[k]):.2e} <= {tol:.2e}")
        assert abs(got[k] - ref[k]) <= tol, (k, got[k], ref[k], tol)


def test_kkt_residuals_random_iterate(dev):
    n = 3001
    g = np.random.default_rng(41)
    tau, lam, beta, sigma, step = 0.3, 2.5, 0.4, 3.0, 1.618
    alpha = g.uniform(-0.9, 0.5, n)  # partly outside B = [-0.7, 0.3]
    v = np.clip(alpha + 0.1 * g.standard_normal(n), tau - 1, tau)
    z = g.standard_normal(n)
    Ka = 3.0 * g.standard_normal(n)
    y = g.standard_normal(n)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    say("kkt_residuals random iterate", n)
    got = kqr.kqr_kkt_residuals(tau, lam, beta, T(alpha), T(Ka), T(y), T(z), T(v))
    ref = oproblem.kkt(alpha, v, beta, z, Ka, y, lam, tau)
    _assert_close(got, ref, _scales(alpha, v, beta, z, Ka, y, lam, tau), "as given")
    assert got["eta_kkt"] == max(got["eta_p"], got["eta_d"], got["eta_c"])

    # the multiplier step: v = Pi_B(alpha + z/sigma), z += step sigma (alpha - v)
    zt, vt = T(z), T(v)
    got = kqr.kqr_kkt_residuals(tau, lam, beta, T(alpha), T(Ka), T(y), zt, vt, sigma=sigma, step=step, update=True)
    v1 = oproblem.proj_box(alpha + z / sigma, tau)
    z1 = z + step * sigma * (alpha - v1)
    assert np.array_equal(vt.cpu().numpy(), v1)  # one division, one add, a clip: same rounding
    # a fused multiply-add on the GPU: at most one rounding of the product apart
    zb = 4 * U64 * (np.abs(z1) + step * sigma * np.abs(alpha - v1))
    assert np.all(np.abs(zt.cpu().numpy() - z1) <= zb)
    ref = oproblem.kkt(alpha, v1, beta, z1, Ka, y, lam, tau)
    _assert_close(got, ref, _scales(alpha, v1, beta, z1, Ka, y, lam, tau), "updated")


@pytest.mark.parametrize("name,n,rank", [("c0", 2000, 0), ("c1", 3000, 200), ("c4", 2500, 0)])
def test_fit_measures_match_oracle_at_the_returned_iterate(dev, name, n, rank):
    prob = inputs.workload(name, n=n)
    X = torch.from_numpy(prob.X).to(dev)
    y = torch.from_numpy(prob.y).to(dev)
    say("fit kkt", name, n, rank)
    alpha, beta, info, st = kqr.kqr_fit(X, y, prob.tau, prob.lam, prob.kernel, prob.gamma, rank=rank,
                                        uniforms=inputs.pivot_uniforms(max(rank, 64), (n, 5)), out_vz=True)
    assert st == kqr.KQR_OK
    a, v, z = alpha.cpu().numpy(), info["v"].cpu().numpy(), info["z"].cpu().numpy()
    Kref, Kb = entry_bound(prob.X, prob.kernel, prob.gamma)
    Ka = Kref @ a
    ref = oproblem.kkt(a, v, beta, z, Ka, prob.y, prob.lam, prob.tau)
    sc = _scales(a, v, beta, z, Ka, prob.y, prob.lam, prob.tau)

    # 1. the GPU's measuring kernel at the identical iterate and FP64 K alpha
    got = kqr.kqr_kkt_residuals(prob.tau, prob.lam, beta, alpha, torch.from_numpy(Ka).to(dev), y,
                                info["z"].clone(), info["v"].clone())
    _assert_close(got, ref, sc, "same K alpha")

    # 2. the fit's own report, measured with FP32 kernel entries: eta_d and
    # eta_c do not involve K; eta_p and the objectives move by at most the
    # entry error of K alpha, |dKa| <= Kb |alpha|
    dKa = Kb @ np.abs(a)
    ny = 1.0 + np.linalg.norm(prob.y)
    dobj = np.abs(a) @ dKa / (2.0 * prob.lam)
    bound = dict(eta_p=np.linalg.norm(dKa) / prob.lam / ny, eta_d=0.0, eta_c=0.0, obj_p=dobj, obj_d=dobj)
    for k in ("eta_p", "eta_d", "eta_c", "obj_p", "obj_d"):
        tol = bound[k] + 8 * U64 * sc[k] + 1e-12 * abs(ref[k])
        say(f"  own {k}: gpu {info[k]:.6e} oracle(FP64 K) {ref[k]:.6e} |d| {abs(info[k] - ref[k]):.2e} <= {tol:.2e}")
        assert abs(info[k] - ref[k]) <= tol, k
    gap_tol = 2 * dobj / (1 + abs(ref["obj_p"]) + abs(ref["obj_d"])) + 8 * U64 * sc["eta_gap"]
    assert abs(info["eta_gap"] - ref["eta_gap"]) <= gap_tol + 1e-13
    # the certificate the fit claims holds for the FP64 operator too, up to that error
    assert max(ref["eta_kkt"], ref["eta_gap"]) <= 1e-6 + bound["eta_p"] + gap_tol
    say(f"  FP64 eta_kkt {ref['eta_kkt']:.2e} eta_gap {ref['eta_gap']:.2e}; FP32-entry shift of eta_p "
        f"<= {bound['eta_p']:.1e}")
