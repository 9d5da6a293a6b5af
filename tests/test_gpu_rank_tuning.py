"""GPU checks of the rank heuristic, the K-apply tile shapes, the autotuners
and the tuning file."""
import json
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import kernel as okernel
from oracle import precond as oprecond
from paper_2510_07929_amd import inputs, kqr
from tests.test_gpu_parity import _apply_bound, entry_bound

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
    """Every supported tile shape computes K v against the oracle: within the
    entry bound of the storage type (FP64 kernel matrix), and in exact mode
    equal to the stored entries times v up to FP64 summation order."""
    n, p = 4099, 8
    X, _ = inputs.additive(n, p, (120, 0))
    Xt = torch.from_numpy(X).to(dev)
    K = kqr.kqr_kernel_build(Xt, "rbf", 0.125, kd)
    vn = np.random.default_rng(5).standard_normal(n)
    v = torch.from_numpy(vn).to(dev)
    say("shapes", kd)
    Kref, Kb = entry_bound(X, "rbf", 0.125)
    Ks = K.float().cpu().numpy()[:, :n].astype(np.float64)
    stored = Ks @ vn
    stored_scale = np.abs(Ks) @ np.abs(vn)
    try:
        for rows in (2, 4, 8):
            for unroll in (1, 2, 4):
                for segs in (1, 3, 16):
                    for mode in (kqr.KQR_APPLY_FAST, kqr.KQR_APPLY_EXACT):
                        kqr.kqr_set_apply_shape(kd, mode, n, rows, unroll, segs)
                        u = kqr.kqr_kernel_apply(v, K=K, mode=mode).cpu().numpy()
                        bound = _apply_bound(Kb, Kref, vn, mode, bf16=(kd == "bf16"))
                        assert np.all(np.abs(u - Kref @ vn) <= bound), (rows, unroll, segs, mode)
                        if mode == kqr.KQR_APPLY_EXACT:
                            assert np.all(np.abs(u - stored) <= 4 * n * 2.0 ** -53 * stored_scale)
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
    Kref, Kb = entry_bound(X, "rbf", 0.1)
    vn = v.cpu().numpy()
    assert np.all(np.abs(u - Kref @ vn) <= _apply_bound(Kb, Kref, vn, kqr.KQR_APPLY_FAST))


def test_on_the_fly_autotuner(dev):
    n, p = 3100, 20
    X, _ = inputs.additive(n, p, (122, 0))
    Xt = torch.from_numpy(X).to(dev)
    say("autotune on the fly")
    try:
        rep = kqr.kqr_autotune_otf(Xt, "rbf", 1.0 / p, kqr.KQR_APPLY_FAST, reps=2)
        strips = [s["strip"] for s in rep["strips"]]
        assert strips == [1, 2, 4, 8, 16, 32]
        assert rep["best"]["strip"] in strips
        assert rep["best"]["us"] == min(s["us"] for s in rep["strips"])
        assert rep["best"]["wgs"] in [w["wgs"] for w in rep["wgs"]]
        # the installed shape computes the same operator
        vn = np.random.default_rng(7).standard_normal(n)
        u = kqr.kqr_kernel_apply(torch.from_numpy(vn).to(dev), X=Xt, kernel="rbf", gamma=1.0 / p).cpu().numpy()
        Kref, Kb = entry_bound(X, "rbf", 1.0 / p)
        assert np.all(np.abs(u - Kref @ vn) <= _apply_bound(Kb, Kref, vn, kqr.KQR_APPLY_FAST, otf=True))
    finally:
        kqr.kqr_set_otf_shape(0, 0)


def test_tuning_file_round_trip(dev, tmp_path):
    """Shapes installed in this process are written keyed by the GPU
    architecture and read back; a file tuned on another architecture installs
    nothing; a malformed entry is rejected."""
    n = 5000
    X, _ = inputs.smooth(n, 8, (123, 0))
    K = kqr.kqr_kernel_build(torch.from_numpy(X).to(dev), "rbf", 0.125, "fp32")
    say("tuning file")
    kqr.kqr_autotune_apply(K, kqr.KQR_APPLY_FAST, reps=1)
    kqr.kqr_set_kv_shape("fp32", n, 0, 1, 2)
    f1, f2, f3 = tmp_path / "a.json", tmp_path / "b.json", tmp_path / "c.json"
    written = kqr.kqr_tune_save(f1)
    assert written >= 2
    text = f1.read_text()
    arch = json.loads(text)["arch"]
    assert arch.startswith("gfx")
    assert kqr.kqr_tune_load(f1) == written
    kqr.kqr_tune_save(f2)
    assert json.loads(f2.read_text()) == json.loads(text)
    f3.write_text(text.replace(f'"arch": "{arch}"', '"arch": "gfx000"'))
    assert kqr.kqr_tune_load(f3) == 0
    f3.write_text(text.replace('"kind": "kv"', '"kind": "warp"'))
    with pytest.raises(kqr.KqrError) as e:
        kqr.kqr_tune_load(f3)
    assert e.value.status == kqr.KQR_EINVAL
    kqr.kqr_set_kv_shape("fp32", n, 0, 1, 4)
