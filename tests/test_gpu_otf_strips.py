"""The symmetric on-the-fly K-applies at every strip width they run with, and
at the full sizes of the precision workloads, against the FP64 oracle.

The square apply K(X, X) v evaluates each distinct pair once over 128 x 128
tiles; a workgroup walks a strip of tiles of one tile-row.  The strip is 2,
8, 16 or 32 tiles by size (32 from n = 130,945 on, which the n = 150,000 RBF
and n = 300,000 Laplacian workloads use).  Here every strip is forced at a
ragged size through kqr_set_otf_shape, for the three kernels (Laplacian in
fixed point, RBF p <= 16 with the FP32 matrix-core Gram, RBF 16 < p <= 32
with the BF16x3 Gram, with and without the norms in the spare coordinates),
fast and exact; then the size rule itself is checked at full size on sampled
rows, each computed one by one by the oracle.

Also: EXACT multi-column applies on a materialised K are FP64 throughout
(every case that is not the one-pass FP32-K path of up to four columns runs
column by column).
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import kernel as okernel
from paper_2510_07929_amd import inputs, kqr
from tests.test_gpu_parity import U32, _apply_bound, entry_bound

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    kqr.lib()
    yield torch.device("cuda:0")
    kqr.kqr_set_otf_shape(0, 0)


_REF = {}


def _reference(kind, n, p):
    key = (kind, n, p)
    if key not in _REF:
        X, _ = inputs.additive(n, p, (910, n, p))
        _REF[key] = (X,) + entry_bound(X, kind, 1.0 / p)
    return _REF[key]


# 33 tile-rows: strips of 8, 16 and 32 leave ragged last strips; the last tile is ragged too
@pytest.mark.parametrize("strip", [1, 2, 8, 16, 32])
@pytest.mark.parametrize("kind,p", [("laplacian", 30), ("rbf", 8), ("rbf", 20), ("rbf", 30), ("rbf", 32)])
@pytest.mark.parametrize("mode", [kqr.KQR_APPLY_FAST, kqr.KQR_APPLY_EXACT])
def test_symmetric_on_the_fly_every_strip(dev, strip, kind, p, mode):
    n = 4100
    X, Kref, Kb = _reference(kind, n, p)
    v = np.random.default_rng(strip).standard_normal(n)
    say("otf strip", strip, kind, p, mode)
    kqr.kqr_set_otf_shape(strip, 0)
    try:
        u = kqr.kqr_kernel_apply(torch.from_numpy(v).to(dev), X=torch.from_numpy(X).to(dev), kernel=kind,
                                 gamma=1.0 / p, mode=mode).cpu().numpy()
    finally:
        kqr.kqr_set_otf_shape(0, 0)
    bound = _apply_bound(Kb, Kref, v, kqr.KQR_APPLY_FAST, otf=True)
    err = np.abs(u - Kref @ v)
    assert np.all(err <= bound), float((err / bound).max())


def _sampled_rows_check(X, kind, gamma, v, u, rows, exact):
    Xd = X.astype(np.float64)
    p = X.shape[1]
    q = (Xd * Xd).sum(1)
    worst = 0.0
    for i in rows:
        d = okernel.distance_block(X[i:i + 1], X, kind)[0]
        k = np.exp(-gamma * d)
        if kind == "rbf":
            dd = 4.0 * (p + 2) * U32 * (q[i] + q) + 2.0 * U32 * d
        else:
            dd = 2.0 * (p + 2) * U32 * d + 1e-30
        kb = k * (gamma * dd + 8.0 * U32)
        ref = k @ v
        # FP32 products summed in FP32 within a tile in fast mode; FP64 in exact mode
        arith = (1e-15 if exact else 70.0 * U32) * (k @ np.abs(v))
        bound = kb @ np.abs(v) + arith + 1e-12
        worst = max(worst, abs(u[i] - ref) / bound)
        assert abs(u[i] - ref) <= bound, (int(i), u[i], ref, bound)
    return worst


# the sizes of the precision workloads: strip 32 by the size rule for all three kernels
@pytest.mark.parametrize("kind,n,p", [("laplacian", 300000, 30), ("rbf", 150000, 30), ("rbf", 140000, 8)])
def test_symmetric_on_the_fly_full_size_sampled(dev, kind, n, p):
    X, _ = inputs.additive(n, p, (911, n, p))
    gamma = 1.0 / p
    v = np.random.default_rng(n).standard_normal(n)
    say("otf full size", kind, n, p)
    Xt = torch.from_numpy(X).to(dev)
    vt = torch.from_numpy(v).to(dev)
    uf = kqr.kqr_kernel_apply(vt, X=Xt, kernel=kind, gamma=gamma, mode=kqr.KQR_APPLY_FAST).cpu().numpy()
    ue = kqr.kqr_kernel_apply(vt, X=Xt, kernel=kind, gamma=gamma, mode=kqr.KQR_APPLY_EXACT).cpu().numpy()
    rows = np.random.default_rng(n + 1).choice(n, 48, replace=False)
    rows[:2] = [0, n - 1]  # the first tile-row's diagonal tile and the ragged last tile
    wf = _sampled_rows_check(X, kind, gamma, v, uf, rows, exact=False)
    we = _sampled_rows_check(X, kind, gamma, v, ue, rows, exact=True)
    say(f"  worst error / bound: fast {wf:.3f} exact {we:.3f}")


@pytest.mark.parametrize("kd,m", [("fp32", 3), ("fp32", 5), ("fp32", 16), ("bf16", 2), ("bf16", 7)])
def test_exact_multi_column_is_fp64(dev, kd, m):
    n, p = 1337, 8
    X, _ = inputs.additive(n, p, (912, m))
    V = np.random.default_rng(m).standard_normal((n, m))
    say("exact multi-column", kd, m)
    Xt = torch.from_numpy(X).to(dev)
    K = kqr.kqr_kernel_build(Xt, "rbf", 0.125, kd)
    U = kqr.kqr_kernel_apply(torch.from_numpy(V).to(dev), K=K, mode=kqr.KQR_APPLY_EXACT)
    # the stored entries are the operator: FP64 products and sums of them
    Ks = K.float().cpu().numpy()[:, :n].astype(np.float64)
    ref = Ks @ V
    scale = np.abs(Ks) @ np.abs(V)
    Un = U.cpu().numpy()
    assert np.all(np.abs(Un - ref) <= 4 * n * 2.0 ** -53 * scale + 1e-300)
    if not (kd == "fp32" and m <= 4):  # column by column: the same launches as single-column calls
        for j in range(m):
            uj = kqr.kqr_kernel_apply(torch.from_numpy(np.ascontiguousarray(V[:, j])).to(dev), K=K,
                                      mode=kqr.KQR_APPLY_EXACT)
            assert torch.equal(U[:, j].contiguous(), uj)
    # and the kernel matrix within the entry bound of the storage type
    Kref, Kb = entry_bound(X, "rbf", 0.125)
    for j in range(m):
        b = _apply_bound(Kb, Kref, V[:, j], kqr.KQR_APPLY_EXACT, bf16=(kd == "bf16"))
        assert np.all(np.abs(Un[:, j] - Kref @ V[:, j]) <= b)
