"""kqr_kernel_apply_static (no allocation) against kqr_kernel_apply.

Two calls in a row on one device, the second with a smaller input (the
fixed scratch array then holds the first call's contents), FP32 and BF16 K,
fast and exact, contiguous and strided vectors: the results equal those of
kqr_kernel_apply (same kernels and launch shape, so the same bits), and lie
within the FP32/BF16 entry bound of the FP64 oracle.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

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


@pytest.mark.parametrize("kd", ["fp32", "bf16"])
@pytest.mark.parametrize("mode", [kqr.KQR_APPLY_FAST, kqr.KQR_APPLY_EXACT])
def test_static_apply_equals_kernel_apply(dev, kd, mode):
    for n, stride in ((20011, 1), (3001, 3)):  # second call smaller (and strided)
        p = 8
        X, _ = inputs.additive(n, p, (950, n))
        vn = np.random.default_rng(n).standard_normal(n)
        say("static apply", kd, mode, n, stride)
        K = kqr.kqr_kernel_build(torch.from_numpy(X).to(dev), "rbf", 1.0 / p, kd)
        vbig = torch.zeros(n * stride, dtype=torch.float64, device=dev)
        vbig[::stride] = torch.from_numpy(vn).to(dev)
        v = vbig[::stride]
        ubig = torch.full((n * stride,), float("nan"), dtype=torch.float64, device=dev)
        u = ubig[::stride]
        kqr.kqr_kernel_apply_static(v, K, mode, u=u)
        ref = kqr.kqr_kernel_apply(v.contiguous(), K=K, mode=mode)
        torch.cuda.synchronize()
        assert torch.equal(u.contiguous(), ref), float((u - ref).abs().max())
        if stride > 1:  # entries between the strided outputs are untouched
            mask = torch.ones(n * stride, dtype=torch.bool, device=dev)
            mask[::stride] = False
            assert torch.isnan(ubig[mask]).all()
        if n <= 5000:
            Kref, Kb = entry_bound(X, "rbf", 1.0 / p)
            bound = _apply_bound(Kb, Kref, vn, mode, bf16=(kd == "bf16"))
            assert np.all(np.abs(u.cpu().numpy() - Kref @ vn) <= bound)
        del K
        torch.cuda.empty_cache()


def test_static_apply_rejects_sizes_beyond_the_array(dev):
    K = torch.zeros((8, 8), dtype=torch.float32, device=dev)
    v = torch.zeros(8, dtype=torch.float64, device=dev)
    lib = kqr.lib()
    # n = 4 million needs 80 MB of scratch (> 64 MiB): rejected before any device work
    st = lib.kqr_kernel_apply_static(K.data_ptr(), kqr.KQR_FP32, 4_000_000, 4_000_000, v.data_ptr(), 1,
                                     v.data_ptr(), 1, 0, None)
    assert st == kqr.KQR_EINVAL and "static" in kqr.last_error()
