"""GPU parity of the symmetric packed layout (upper-triangle tiles): the
stored entries against the documented layout, the K-apply against the oracle
and against the full layout, and whole fits against the oracle."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import kernel as okernel
from oracle import problem as oproblem
from oracle import solver as osolver
from paper_2510_07929_amd import inputs, kqr
from tests.test_gpu_parity import BF16_REL  # BF16-stored entry: relative part of its bound

pytestmark = pytest.mark.gpu
U32 = 2.0 ** -24
T = 128


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    kqr.lib()
    return torch.device("cuda:0")


def unpack(flat, n):
    """Dense n x n matrix from the packed buffer, by the documented layout."""
    nt = -(-n // T)
    tiles = flat.reshape(-1, T, T)
    assert tiles.shape[0] == nt * (nt + 1) // 2
    full = np.zeros((nt * T, nt * T), dtype=np.float64)
    t = 0
    for I in range(nt):
        for J in range(I, nt):
            full[I * T:(I + 1) * T, J * T:(J + 1) * T] = tiles[t]
            if J > I:
                full[J * T:(J + 1) * T, I * T:(I + 1) * T] = tiles[t].T
            t += 1
    # padding beyond n is zero
    assert not full[n:, :].any() and not full[:, n:].any()
    return full[:n, :n]


@pytest.mark.parametrize("kd", ["fp32", "bf16"])
@pytest.mark.parametrize("n", [1, 130, 1000])
def test_packed_entries_match_full_layout(dev, kd, n):
    p = 6
    X, _ = inputs.smooth(n, p, (140, n))
    Xt = torch.from_numpy(X).to(dev)
    say("packed build", kd, n)
    Kp = kqr.kqr_kernel_build_packed(Xt, "rbf", 1.0 / p, kd)
    Kf = kqr.kqr_kernel_build(Xt, "rbf", 1.0 / p, kd)
    dense = unpack(Kp.float().cpu().numpy().astype(np.float64), n)
    ref = Kf.float().cpu().numpy().astype(np.float64)[:, :n]
    # same entry formula on both layouts: the stored upper triangle is
    # bit-identical; the lower triangle is mirrored from it (the full layout
    # evaluates K[j][i] itself, with the operands of each product swapped)
    iu = np.triu_indices(n)
    assert np.array_equal(dense[iu], ref[iu])
    tol = 4 * (U32 if kd == "fp32" else 2.0 ** -8)
    assert np.abs(dense - ref).max() <= tol
    assert np.all(np.diag(dense) == 1.0)


def _bound(X, gamma, kd, v):
    Xd = X.astype(np.float64)
    p = X.shape[1]
    D = okernel.distance_block(Xd, Xd, "rbf")
    K = np.exp(-gamma * D)
    q = (Xd * Xd).sum(1)
    dd = 4.0 * (p + 2) * U32 * (q[:, None] + q[None, :]) + 2.0 * U32 * D
    Kb = K * (gamma * dd + 8.0 * U32)
    if kd == "bf16":
        Kb = BF16_REL * K + (1.0 + 2.0 ** -8) * Kb
    return K, Kb @ np.abs(v) + 300 * U32 * (K @ np.abs(v))


@pytest.mark.parametrize("kd", ["fp32", "bf16"])
@pytest.mark.parametrize("mode", [kqr.KQR_APPLY_FAST, kqr.KQR_APPLY_EXACT])
@pytest.mark.parametrize("n", [1, 257, 3001])
def test_packed_apply_matches_oracle(dev, kd, mode, n):
    p = 8
    X, _ = inputs.additive(n, p, (141, n))
    gamma = 1.0 / p
    v = np.random.default_rng(n).standard_normal(n)
    say("packed apply", kd, mode, n)
    Kp = kqr.kqr_kernel_build_packed(torch.from_numpy(X).to(dev), "rbf", gamma, kd)
    u = kqr.kqr_kernel_apply_packed(torch.from_numpy(v).to(dev), Kp, n, mode).cpu().numpy()
    K, bound = _bound(X, gamma, kd, v)
    err = np.abs(u - K @ v)
    assert np.all(err <= bound), float(np.max(err / bound))
    if mode == kqr.KQR_APPLY_EXACT:
        # FP64 arithmetic on the stored entries: equal to the stored matrix times v
        dense = unpack(Kp.float().cpu().numpy().astype(np.float64), n)
        ref = dense @ v
        assert np.abs(u - ref).max() <= 1e-12 * (np.abs(dense) @ np.abs(v)).max()


@pytest.mark.parametrize("kd", ["fp32", "bf16"])
def test_every_packed_shape_and_autotuner(dev, kd):
    # every (map, strip) computes the same K v up to summation order; the
    # autotuner reports each shape and installs a supported one
    n, p = 2900, 8
    X, _ = inputs.additive(n, p, (143, 0))
    Kp = kqr.kqr_kernel_build_packed(torch.from_numpy(X).to(dev), "rbf", 0.125, kd)
    v = torch.from_numpy(np.random.default_rng(9).standard_normal(n)).to(dev)
    say("packed shapes", kd)
    vn = v.cpu().numpy()
    K, bound = _bound(X, 0.125, kd, vn)  # the oracle's FP64 K and the storage bound
    dense = unpack(Kp.float().cpu().numpy().astype(np.float64), n)
    stored, stored_scale = dense @ vn, np.abs(dense) @ np.abs(vn)
    shapes = [(mp, strip) for mp in (0, 1, 2, 3) for strip in (1, 2, 3, 4, 8, 16, 32)] + [(4, 2), (4, 4), (5, 2), (5, 4)]
    for mode in (kqr.KQR_APPLY_FAST, kqr.KQR_APPLY_EXACT):
        for mp, strip in shapes:
            kqr.kqr_set_packed_shape(kd, mode, mp, strip)
            u = kqr.kqr_kernel_apply_packed(v, Kp, n, mode).cpu().numpy()
            assert np.all(np.abs(u - K @ vn) <= bound), (mode, mp, strip)
            if mode == kqr.KQR_APPLY_EXACT:  # FP64 on the stored entries
                assert np.all(np.abs(u - stored) <= 4 * n * 2.0 ** -53 * stored_scale), (mp, strip)
        rep = kqr.kqr_autotune_packed(Kp, n, mode, reps=2)
        assert len(rep["shapes"]) == 24 and rep["best"]["map"] in (0, 1, 2, 3, 4, 5) and 1 <= rep["best"]["strip"] <= 16
    with pytest.raises(kqr.KqrError):
        kqr.kqr_set_packed_shape(kd, kqr.KQR_APPLY_FAST, 6, 4)
    with pytest.raises(kqr.KqrError):
        kqr.kqr_set_packed_shape(kd, kqr.KQR_APPLY_FAST, 4, 3)
    with pytest.raises(kqr.KqrError):
        kqr.kqr_set_packed_shape(kd, kqr.KQR_APPLY_FAST, 0, 33)


@pytest.mark.parametrize("kd", ["fp32", "bf16"])
def test_packed_block_map_ragged_sizes(dev, kd):
    # maps 4 and 5 (square blocks of B x B tiles): one tile (n = 1, 100, 128), a
    # block grid whose last block row and column are partial (n = 129: two
    # tile-rows; 640: five; 1153: ten), and B = 2 and 4 in both modes, against
    # the oracle's K and (exact) FP64 on the stored entries
    p = 5
    for n in (1, 100, 128, 129, 640, 1153):
        X, _ = inputs.smooth(n, p, (145, n))
        Kp = kqr.kqr_kernel_build_packed(torch.from_numpy(X).to(dev), "rbf", 1.0 / p, kd)
        vn = np.random.default_rng(n + 1).standard_normal(n)
        v = torch.from_numpy(vn).to(dev)
        K, bound = _bound(X, 1.0 / p, kd, vn)
        dense = unpack(Kp.float().cpu().numpy().astype(np.float64), n)
        stored, stored_scale = dense @ vn, np.abs(dense) @ np.abs(vn)
        for mode in (kqr.KQR_APPLY_FAST, kqr.KQR_APPLY_EXACT):
            for mp in (4, 5):
                for B in (2, 4):
                    say("packed blocks", kd, n, mode, mp, B)
                    kqr.kqr_set_packed_shape(kd, mode, mp, B)
                    u = kqr.kqr_kernel_apply_packed(v, Kp, n, mode).cpu().numpy()
                    assert np.all(np.abs(u - K @ vn) <= bound), (n, mode, mp, B)
                    if mode == kqr.KQR_APPLY_EXACT:
                        assert np.all(np.abs(u - stored) <= 4 * n * 2.0 ** -53 * stored_scale), (n, mp, B)


def test_packed_apply_full_size_against_full_layout(dev):
    # the c1 shape: n = 50,000, p = 20, in the launch shapes the fits use
    # (compiled defaults and the tuned table: exact map 5 with blocks of 4 x 4
    # and 2 x 2 tiles, fast map 4 with 4 x 4) and the strip maps before them;
    # exact applies of both layouts use the same FP32 entries with FP64
    # products, so they differ by summation order
    prob = inputs.workload("c1")
    n = prob.n
    Xt = torch.from_numpy(prob.X).to(dev)
    v = torch.from_numpy(np.random.default_rng(7).standard_normal(n)).to(dev)
    say("full-size packed vs full", n)
    Kp = kqr.kqr_kernel_build_packed(Xt, "rbf", prob.gamma, "fp32")
    exact_shapes, fast_shapes = [(5, 4), (5, 2), (0, 4)], [(4, 4), (5, 4), (2, 4)]
    ups, upfs = [], []
    for mp, s in exact_shapes:
        kqr.kqr_set_packed_shape("fp32", kqr.KQR_APPLY_EXACT, mp, s)
        ups.append(kqr.kqr_kernel_apply_packed(v, Kp, n, kqr.KQR_APPLY_EXACT).cpu().numpy())
    for mp, s in fast_shapes:
        kqr.kqr_set_packed_shape("fp32", kqr.KQR_APPLY_FAST, mp, s)
        upfs.append(kqr.kqr_kernel_apply_packed(v, Kp, n, kqr.KQR_APPLY_FAST).cpu().numpy())
    del Kp
    Kf = kqr.kqr_kernel_build(Xt, "rbf", prob.gamma, "fp32")
    uf = kqr.kqr_kernel_apply(v, K=Kf, mode=kqr.KQR_APPLY_EXACT).cpu().numpy()
    # sampled rows against the oracle's FP64 entries
    rows = np.random.default_rng(8).choice(n, 64, replace=False)
    Krows = okernel.kernel_block(prob.X[rows], prob.X, "rbf", prob.gamma)
    del Kf
    torch.cuda.empty_cache()
    scale = np.abs(v.cpu().numpy()).sum()
    ref = Krows @ v.cpu().numpy()
    for (mp, s), up in zip(exact_shapes, ups):
        # equal entries up to the mirrored triangle (see the entry test); the
        # rest is summation order
        assert np.abs(up - uf).max() <= 8 * U32 * scale, (mp, s)
        assert np.abs(up[rows] - ref).max() <= 64 * U32 * scale, (mp, s)
    for (mp, s), upf in zip(fast_shapes, upfs):
        assert np.abs(upf - ups[0]).max() <= 300 * U32 * scale, (mp, s)
        assert np.abs(upf[rows] - ref).max() <= 300 * U32 * scale, (mp, s)
    say(f"  max |packed - full| = {max(np.abs(u - uf).max() for u in ups):.3e}, "
        f"fast-exact {max(np.abs(u - ups[0]).max() for u in upfs):.3e}")
    _install_default_shapes()


def _install_default_shapes():
    """The compiled default packed shapes (what a process uses untuned), so
    that the fits below run on them after the shape tests above."""
    F, E = kqr.KQR_APPLY_FAST, kqr.KQR_APPLY_EXACT
    kqr.kqr_set_packed_shape("fp32", F, 4, 4)
    kqr.kqr_set_packed_shape("fp32", E, 5, 4)
    kqr.kqr_set_packed_shape("bf16", F, 5, 4)
    kqr.kqr_set_packed_shape("bf16", E, 0, 16)


@pytest.mark.parametrize("kd", ["fp32", "bf16"])
def test_packed_fit_matches_oracle(dev, kd):
    prob = inputs.workload("c0", n=2500)
    X = torch.from_numpy(prob.X).to(dev)
    y = torch.from_numpy(prob.y).to(dev)
    say("packed fit", kd, prob.n)
    a, b, info, st = kqr.kqr_fit(X, y, prob.tau, prob.lam, prob.kernel, prob.gamma, k_layout=1,
                                 k_dtype=kqr.KDTYPES[kd], kmode=kqr.KQR_KMODE_MATERIALIZE,
                                 uniforms=inputs.pivot_uniforms(128, (142, 0)))
    a = a.cpu().numpy()
    ref = osolver.fit(prob.X, prob.y, prob.tau, prob.lam, prob.kernel, prob.gamma, osolver.OracleOptions(tol=1e-10))
    K = okernel.kernel_matrix(prob.X, prob.kernel, prob.gamma)
    Ka = K @ a
    obj = oproblem.primal_objective(prob.y - b - Ka / prob.lam, a, Ka, prob.lam, prob.tau)
    opt = ref.kkt["obj_p"]
    rel = abs(obj - opt) / (1 + abs(opt))
    say(f"  status={st} rel_obj={rel:.2e} kkt={info['eta_kkt']:.2e} gap={info['eta_gap']:.2e}")
    assert st == kqr.KQR_OK
    assert max(info["eta_kkt"], info["eta_gap"]) <= 1e-6
    assert rel <= 1e-6


def test_packed_layout_rejected_by_joint_fits(dev):
    prob = inputs.workload("c0", n=300)
    X = torch.from_numpy(prob.X).to(dev)
    y = torch.from_numpy(prob.y).to(dev)
    with pytest.raises(kqr.KqrError):
        kqr.kqr_fit_multi_tau(X, y, [0.3, 0.7], prob.lam, "rbf", prob.gamma, k_layout=1)
    with pytest.raises(kqr.KqrError):
        kqr.kqr_fit_path(X, y, 0.5, [1.0, 0.5], "rbf", prob.gamma, k_layout=1)
    with pytest.raises(kqr.KqrError):
        kqr.kqr_fit(X, y, 0.5, prob.lam, "rbf", prob.gamma, k_layout=2)
