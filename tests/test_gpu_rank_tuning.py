"""GPU checks of the rank heuristic, the K-apply tile shapes and the autotuner."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import kernel as okernel
from oracle import precond as oprecond
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


@pytest.mark.parametrize("name,n,xi", [("c0", 1500, 1e-3), ("c1", 2500, 1e-3), ("c0", 900, 1e-6)])
def test_adaptive_rank_matches_oracle(dev, name, n, xi):
    """Section 3 rule on the same F0: the integer r agrees unless an eigenvalue
    of F0^T F0 sits within rounding of xi * lambda_1."""
    prob = inputs.workload(name, n=n)
    r0 = int(np.ceil(np.sqrt(n)))
    op = okernel.DenseKernel(prob.X, prob.kernel, prob.gamma)
    F0, _, _ = oprecond.rpcholesky(op, r0, inputs.pivot_uniforms(r0, (n, 9)))
    ldf = (r0 + 3) // 4 * 4
    Ft = torch.zeros((n, ldf), dtype=torch.float32)
    Ft[:, :r0] = torch.from_numpy(F0.astype(np.float32))
    say("adaptive rank", name, n, xi)
    r_gpu, l1_gpu = kqr.kqr_adaptive_rank(Ft.to(dev), r0, xi)
    F32 = F0.astype(np.float32).astype(np.float64)  # the GPU sees the FP32-rounded factor
    ev = np.linalg.eigvalsh(F32.T @ F32)[::-1]
    r_ref = oprecond.adaptive_rank(F32, xi)
    assert l1_gpu == pytest.approx(ev[0], rel=1e-10)
    if r_gpu != r_ref:
        gap = np.min(np.abs(ev - xi * ev[0])) / ev[0]
        assert gap < 1e-9, (r_gpu, r_ref, gap)


@pytest.mark.parametrize("kd", ["fp32", "bf16"])
def test_apply_shapes_agree(dev, kd):
    """Every supported tile shape computes the same K v (up to summation order)."""
    n, p = 4099, 8
    X, _ = inputs.additive(n, p, (120, 0))
    Xt = torch.from_numpy(X).to(dev)
    K = kqr.kqr_kernel_build(Xt, "rbf", 0.125, kd)
    v = torch.from_numpy(np.random.default_rng(5).standard_normal(n)).to(dev)
    say("shapes", kd)
    ref = kqr.kqr_kernel_apply(v, K=K, mode=kqr.KQR_APPLY_EXACT).cpu().numpy()
    scale = np.abs(ref).max()
    try:
        for rows in (2, 4, 8):
            for unroll in (1, 2, 4):
                for segs in (1, 3, 16):
                    for mode in (kqr.KQR_APPLY_FAST, kqr.KQR_APPLY_EXACT):
                        kqr.kqr_set_apply_shape(kd, mode, n, rows, unroll, segs)
                        u = kqr.kqr_kernel_apply(v, K=K, mode=mode).cpu().numpy()
                        tol = 1e-12 if mode == kqr.KQR_APPLY_EXACT else 2e-5
                        assert np.abs(u - ref).max() <= tol * scale * (1 + np.sqrt(n)), (rows, unroll, segs, mode)
    finally:
        for mode in (kqr.KQR_APPLY_FAST, kqr.KQR_APPLY_EXACT):
            kqr.kqr_set_apply_shape(kd, mode, n, 8, 2, 4)
    with pytest.raises(kqr.KqrError):
        kqr.kqr_set_apply_shape(kd, 0, n, 3, 1, 1)


def test_autotuner_reports_and_installs(dev):
    n, p = 6000, 10
    X, _ = inputs.smooth(n, p, (121, 0))
    K = kqr.kqr_kernel_build(torch.from_numpy(X).to(dev), "rbf", 0.1, "fp32")
    say("autotune")
    rep = kqr.kqr_autotune_apply(K, kqr.KQR_APPLY_FAST, reps=2)
    assert rep["n"] == n and len(rep["shapes"]) == 45
    best = rep["best"]
    assert best["us"] == min(s["us"] for s in rep["shapes"])
    v = torch.from_numpy(np.random.default_rng(6).standard_normal(n)).to(dev)
    u = kqr.kqr_kernel_apply(v, K=K).cpu().numpy()
    ref = okernel.kernel_matrix(X, "rbf", 0.1) @ v.cpu().numpy()
    assert np.abs(u - ref).max() <= 1e-4 * np.abs(ref).max()
