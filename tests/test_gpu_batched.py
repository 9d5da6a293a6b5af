"""GPU parity of the batched forms: K V on the matrix cores, the joint
multi-tau fit, and the uneven batch of independent problems."""
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


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    kqr.lib()
    return torch.device("cuda:0")


def entry_bound(X, gamma):
    Xd = X.astype(np.float64)
    p = X.shape[1]
    D = okernel.distance_block(Xd, Xd, "rbf")
    K = np.exp(-gamma * D)
    q = (Xd * Xd).sum(1)
    dd = 4.0 * (p + 2) * U32 * (q[:, None] + q[None, :]) + 2.0 * U32 * D
    return K, K * (gamma * dd + 8.0 * U32)


@pytest.mark.parametrize("kd", ["fp32", "bf16"])
@pytest.mark.parametrize("n,m", [(3001, 9), (700, 16), (1500, 2)])
def test_kv_multi_rhs_matches_oracle(dev, kd, n, m):
    p = 8
    X, _ = inputs.additive(n, p, (130, n))
    gamma = 1.0 / p
    V = np.random.default_rng(m).standard_normal((n, m))
    say("K V", kd, n, m)
    K = kqr.kqr_kernel_build(torch.from_numpy(X).to(dev), "rbf", gamma, kd)
    U = kqr.kqr_kernel_apply(torch.from_numpy(V).to(dev), K=K).cpu().numpy()
    Kref, Kb = entry_bound(X, gamma)
    A = np.abs(V)
    if kd == "fp32":
        # FP32 entries, V rounded to FP32, FP32 accumulation over 256-column stages
        bound = Kb @ A + 300 * U32 * (Kref @ A)
    else:
        # BF16 entries (BF16_REL), V split into hi + lo BF16 parts (2^-16)
        bound = (BF16_REL * Kref + (1.0 + 2.0 ** -8) * Kb) @ A + (2.0 ** -15 + 300 * U32) * (Kref @ A)
    err = np.abs(U - Kref @ V)
    assert np.all(err <= bound + 1e-12), float((err / (bound + 1e-12)).max())


@pytest.mark.parametrize("kd", ["fp32", "bf16"])
def test_kv_every_launch_shape_and_autotuner(dev, kd):
    # every shape the autotuner may choose meets the same bound; ragged n so the
    # last step of the last segment is partial for every step width
    n, m, p = 2777, 9, 8
    X, _ = inputs.additive(n, p, (131, n))
    gamma = 1.0 / p
    V = np.random.default_rng(7).standard_normal((n, m))
    K = kqr.kqr_kernel_build(torch.from_numpy(X).to(dev), "rbf", gamma, kd)
    Vt = torch.from_numpy(V).to(dev)
    Kref, Kb = entry_bound(X, gamma)
    A = np.abs(V)
    if kd == "fp32":
        bound = Kb @ A + 300 * U32 * (Kref @ A)
    else:
        bound = (BF16_REL * Kref + (1.0 + 2.0 ** -8) * Kb) @ A + (2.0 ** -15 + 300 * U32) * (Kref @ A)
    ref = Kref @ V
    say("K V shapes", kd)
    outs = []
    for nld in (0, 4, 8):
        for pf in (0, 1):
            for segs in (1, 2, 4, 8):
                if nld == 0 and pf == 0:
                    continue
                kqr.kqr_set_kv_shape(kd, n, nld, pf, segs)
                U = kqr.kqr_kernel_apply(Vt, K=K).cpu().numpy()
                err = np.abs(U - ref)
                assert np.all(err <= bound + 1e-12), (nld, pf, segs, float((err / (bound + 1e-12)).max()))
                outs.append(U)
    rep = kqr.kqr_autotune_apply(K, kqr.KQR_APPLY_KV, reps=2)
    assert rep["n"] == n and len(rep["shapes"]) == 20
    assert rep["best"]["us"] == min(s["us"] for s in rep["shapes"])
    U = kqr.kqr_kernel_apply(Vt, K=K).cpu().numpy()
    assert np.all(np.abs(U - ref) <= bound + 1e-12)
    with pytest.raises(kqr.KqrError):
        kqr.kqr_set_kv_shape(kd, n, 6, 0, 1)


@pytest.mark.parametrize("n,m", [(3001, 4), (700, 2), (129, 3)])
def test_exact_multi_column_apply(dev, n, m):
    # exact columns from one pass over an FP32 K (the path the joint fits use
    # for their exact applies) against column-by-column exact applies and the
    # oracle: FP64 products of the same FP32 entries, so only summation order
    # separates the two GPU forms
    p = 8
    X, _ = inputs.additive(n, p, (131, n))
    gamma = 1.0 / p
    V = np.random.default_rng(m).standard_normal((n, m))
    say("exact multi-column", n, m)
    K = kqr.kqr_kernel_build(torch.from_numpy(X).to(dev), "rbf", gamma, "fp32")
    Vt = torch.from_numpy(V).to(dev)
    U = kqr.kqr_kernel_apply(Vt, K=K, mode=kqr.KQR_APPLY_EXACT).cpu().numpy()
    cols = np.stack([kqr.kqr_kernel_apply(Vt[:, j].contiguous(), K=K, mode=kqr.KQR_APPLY_EXACT).cpu().numpy().ravel()
                     for j in range(m)], axis=1)
    Kf = K.cpu().numpy().astype(np.float64)[:, :n]
    scale = np.abs(Kf) @ np.abs(V)
    assert np.all(np.abs(U - cols) <= 1e-13 * scale)
    assert np.all(np.abs(U - Kf @ V) <= 1e-13 * scale)
    Kref, Kb = entry_bound(X, gamma)
    assert np.all(np.abs(U - Kref @ V) <= Kb @ np.abs(V) + 1e-13 * scale)


def _oracle_obj(prob, tau, alpha, beta):
    K = okernel.kernel_matrix(prob.X, prob.kernel, prob.gamma)
    Ka = K @ alpha
    z = prob.y - beta - Ka / prob.lam
    return oproblem.primal_objective(z, alpha, Ka, prob.lam, tau)


def test_fit_multi_tau_matches_oracle(dev):
    prob = inputs.workload("c3a", n=2500)
    taus = prob.extras["taus"]
    say("multi-tau", prob.n, len(taus))
    X = torch.from_numpy(prob.X).to(dev)
    y = torch.from_numpy(prob.y).to(dev)
    A, betas, infos, st = kqr.kqr_fit_multi_tau(X, y, taus, prob.lam, prob.kernel, prob.gamma, profile=1,
                                                uniforms=inputs.pivot_uniforms(128, (3, 1)))
    A = A.cpu().numpy()
    assert all(s == kqr.KQR_OK for s in st), st
    # every level used the shared K V launches
    assert infos[0]["kapply_fast_calls"] > 0 and infos[0]["t_kapply_fast"] > 0
    for t, tau in enumerate(taus):
        ref = osolver.fit(prob.X, prob.y, tau, prob.lam, prob.kernel, prob.gamma, osolver.OracleOptions(tol=1e-10))
        opt = ref.kkt["obj_p"]
        rel = abs(_oracle_obj(prob, tau, A[t], betas[t]) - opt) / (1 + abs(opt))
        say(f"  tau={tau} rel_obj={rel:.2e} kkt={infos[t]['eta_kkt']:.2e}")
        assert max(infos[t]["eta_kkt"], infos[t]["eta_gap"]) <= 1e-6
        assert rel <= 1e-6


def test_fit_multi_tau_single_level_equals_fit(dev):
    prob = inputs.workload("c0", n=1200)
    X = torch.from_numpy(prob.X).to(dev)
    y = torch.from_numpy(prob.y).to(dev)
    uni = inputs.pivot_uniforms(64, (4, 2))
    say("multi-tau with one level")
    A, b, _, st = kqr.kqr_fit_multi_tau(X, y, [prob.tau], prob.lam, "rbf", prob.gamma, uniforms=uni)
    a1, b1, _, st1 = kqr.kqr_fit(X, y, prob.tau, prob.lam, "rbf", prob.gamma, uniforms=uni)
    # one level has nothing to coalesce: the same code path, bitwise
    assert st == [st1] and torch.equal(A[0], a1) and b[0] == b1


def test_fit_batch_matches_oracle(dev):
    probs = inputs.uneven_batch(count=6, lo=300, hi=1400, seed=3)
    say("uneven batch", [p.n for p in probs])
    Xs = [torch.from_numpy(p.X).to(dev) for p in probs]
    ys = [torch.from_numpy(p.y).to(dev) for p in probs]
    alphas, betas, infos, st = kqr.kqr_fit_batch(Xs, ys, [p.tau for p in probs], [p.lam for p in probs],
                                                 [p.gamma for p in probs], profile=1,
                                                 uniforms=inputs.pivot_uniforms(64, (5, 1)))
    assert all(s == kqr.KQR_OK for s in st), st
    assert infos[0]["kapply_fast_calls"] > 0
    for i, prob in enumerate(probs):
        a = alphas[i].cpu().numpy()
        ref = osolver.fit(prob.X, prob.y, prob.tau, prob.lam, "rbf", prob.gamma, osolver.OracleOptions(tol=1e-10))
        opt = ref.kkt["obj_p"]
        rel = abs(_oracle_obj(prob, prob.tau, a, betas[i]) - opt) / (1 + abs(opt))
        say(f"  n={prob.n} rel_obj={rel:.2e} kkt={infos[i]['eta_kkt']:.2e}")
        assert max(infos[i]["eta_kkt"], infos[i]["eta_gap"]) <= 1e-6
        assert rel <= 1e-6


def test_batched_pcg_steps_equal_per_problem_kernels(dev):
    """kqr_fit_batch with the PCG iterations' vector and preconditioner work in
    batched launches gives bitwise the results of the same work launched per
    problem (same device code per problem, same order).  Problems with a
    preconditioner rank below 128 take the batched form; their F^T g and F s
    passes span several workgroups each."""
    probs = inputs.uneven_batch(count=10, lo=300, hi=6000, seed=9)
    Xs = [torch.from_numpy(p.X).to(dev) for p in probs]
    ys = [torch.from_numpy(p.y).to(dev) for p in probs]
    runs = {}
    try:
        for on in (True, False):
            kqr.kqr_test_batch_steps(on)
            a, b, inf, st = kqr.kqr_fit_batch(Xs, ys, [p.tau for p in probs], [p.lam for p in probs],
                                              [p.gamma for p in probs], uniforms=inputs.pivot_uniforms(64, (5, 4)))
            assert all(s == kqr.KQR_OK for s in st), st
            runs[on] = ([x.cpu() for x in a], list(b), [i["kapply_calls"] for i in inf],
                        [i["pcg_iters"] + i["admm_pcg_iters"] for i in inf], [i["rank_used"] for i in inf])
            say("batched steps", on, "ranks", runs[on][4], "pcg iterations", sum(runs[on][3]))
    finally:
        kqr.kqr_test_batch_steps(True)
    (a1, b1, k1, i1, r1), (a0, b0, k0, i0, r0) = runs[True], runs[False]
    assert any(0 < r < 128 for r in r1)  # the batched form ran
    assert r1 == r0 and k1 == k0 and i1 == i0
    assert all(torch.equal(x, y) for x, y in zip(a1, a0))
    assert b1 == b0


def test_batched_pcg_steps_on_long_vectors_equal_per_problem_kernels(dev):
    """An uneven batch with a problem longer than one workgroup (n = 17,000):
    its PCG iterations' vector work in batched launches (several workgroups
    per problem, partial sums finished per problem) beside the one-workgroup
    problems gives bitwise the results of the same work launched per problem."""
    big = inputs.workload("c0", n=17000)
    probs = [big] + inputs.uneven_batch(count=3, lo=500, hi=2000, seed=19)
    Xs = [torch.from_numpy(p.X).to(dev) for p in probs]
    ys = [torch.from_numpy(p.y).to(dev) for p in probs]
    uni = inputs.pivot_uniforms(64, (5, 9))
    runs = {}
    try:
        for on in (True, False):
            kqr.kqr_test_batch_steps(on)
            # a fixed rank below 128 (the adaptive rule picks 131 for the long problem)
            a, b, inf, st = kqr.kqr_fit_batch(Xs, ys, [p.tau for p in probs], [p.lam for p in probs],
                                              [p.gamma for p in probs], rank=64, uniforms=uni)
            assert all(s == kqr.KQR_OK for s in st), st
            runs[on] = ([x.cpu() for x in a], list(b), [i["kapply_calls"] for i in inf],
                        [i["pcg_iters"] + i["admm_pcg_iters"] for i in inf])
            say("long-vector batched steps", on, "pcg iterations", runs[on][3])
    finally:
        kqr.kqr_test_batch_steps(True)
    (a1, b1, k1, i1), (a0, b0, k0, i0) = runs[True], runs[False]
    assert k1 == k0 and i1 == i0
    assert all(torch.equal(x, y) for x, y in zip(a1, a0))
    assert b1 == b0


def test_fit_batch_mixed_sizes_matches_lone_fits(dev):
    """An uneven batch where one problem's preconditioner core is too large for
    the batched PCG steps (n = 17,000, adaptive rank 131 >= 128: its vector work
    runs per problem and it resumes on the round's completion event) beside
    problems that take them: every problem reaches
    the optimum its lone kqr_fit reaches (the K-apply kernels differ, so the
    comparison is of objectives and KKT levels, not bits)."""
    big = inputs.workload("c0", n=17000)
    small = inputs.uneven_batch(count=4, lo=400, hi=3000, seed=11)
    probs = [big] + small
    Xs = [torch.from_numpy(p.X).to(dev) for p in probs]
    ys = [torch.from_numpy(p.y).to(dev) for p in probs]
    uni = inputs.pivot_uniforms(64, (5, 6))
    say("mixed batch", [p.n for p in probs])
    a, b, inf, st = kqr.kqr_fit_batch(Xs, ys, [p.tau for p in probs], [p.lam for p in probs],
                                      [p.gamma for p in probs], uniforms=uni)
    assert all(s == kqr.KQR_OK for s in st), st
    for i, prob in enumerate(probs):
        a1, b1, i1, s1 = kqr.kqr_fit(Xs[i], ys[i], prob.tau, prob.lam, "rbf", prob.gamma, uniforms=uni)
        assert s1 == kqr.KQR_OK
        rel = abs(inf[i]["obj_p"] - i1["obj_p"]) / (1.0 + abs(i1["obj_p"]))
        say(f"  n={prob.n} rel_obj={rel:.2e} kkt={inf[i]['eta_kkt']:.2e}/{i1['eta_kkt']:.2e}")
        assert max(inf[i]["eta_kkt"], inf[i]["eta_gap"]) <= 1e-6
        assert rel <= 2e-6  # both within 1e-6 of the optimum (each certified by its own KKT level)


def test_fit_batch_bf16_matches_oracle(dev):
    """An uneven batch with BF16 storage: the inner PCG solves on the BF16 K
    take the batched steps and open rounds, the refinement residuals use the
    exact operator per problem; every problem reaches its oracle optimum."""
    probs = inputs.uneven_batch(count=5, lo=300, hi=1600, seed=17)
    Xs = [torch.from_numpy(p.X).to(dev) for p in probs]
    ys = [torch.from_numpy(p.y).to(dev) for p in probs]
    say("uneven batch, BF16 K", [p.n for p in probs])
    alphas, betas, infos, st = kqr.kqr_fit_batch(Xs, ys, [p.tau for p in probs], [p.lam for p in probs],
                                                 [p.gamma for p in probs], k_dtype=kqr.KQR_BF16,
                                                 kmode=kqr.KQR_KMODE_MATERIALIZE,
                                                 uniforms=inputs.pivot_uniforms(64, (5, 8)))
    assert all(s == kqr.KQR_OK for s in st), st
    assert sum(i["refinements"] for i in infos) > 0
    for i, prob in enumerate(probs):
        a = alphas[i].cpu().numpy()
        ref = osolver.fit(prob.X, prob.y, prob.tau, prob.lam, "rbf", prob.gamma, osolver.OracleOptions(tol=1e-10))
        opt = ref.kkt["obj_p"]
        rel = abs(_oracle_obj(prob, prob.tau, a, betas[i]) - opt) / (1 + abs(opt))
        say(f"  n={prob.n} rel_obj={rel:.2e} kkt={infos[i]['eta_kkt']:.2e} refinements={infos[i]['refinements']}")
        assert max(infos[i]["eta_kkt"], infos[i]["eta_gap"]) <= 1e-6
        assert rel <= 1e-6


def test_batched_entry_points_validate(dev):
    prob = inputs.workload("c0", n=100)
    X = torch.from_numpy(prob.X).to(dev)
    y = torch.from_numpy(prob.y).to(dev)
    with pytest.raises(kqr.KqrError) as e:
        kqr.kqr_fit_multi_tau(X, y, [0.5, 1.5], prob.lam, "rbf", prob.gamma)
    assert e.value.status == kqr.KQR_EINVAL
    with pytest.raises(kqr.KqrError) as e:
        kqr.kqr_fit_multi_tau(X, y, [0.5] * 17, prob.lam, "rbf", prob.gamma)
    assert e.value.status == kqr.KQR_EINVAL


def test_batched_results_do_not_depend_on_host_threads(dev):
    """The batched launches of a round carry the same requests whatever the
    number of host threads, and every fit issues the same kernels in the same
    order: the results are bitwise the same."""
    probs = inputs.uneven_batch(count=12, lo=300, hi=2500, seed=5)
    Xs = [torch.from_numpy(p.X).to(dev) for p in probs]
    ys = [torch.from_numpy(p.y).to(dev) for p in probs]
    path = inputs.workload("c0", n=1500)
    Xp = torch.from_numpy(path.X).to(dev)
    yp = torch.from_numpy(path.y).to(dev)
    lams = list(np.geomspace(0.3, 30.0, 7) * path.lam)
    runs = {}
    try:
        for T in (1, 5):
            kqr.kqr_set_batch_threads(T)
            a, b, inf, st = kqr.kqr_fit_batch(Xs, ys, [p.tau for p in probs], [p.lam for p in probs],
                                              [p.gamma for p in probs], uniforms=inputs.pivot_uniforms(64, (5, 2)))
            ap, bp, infp, stp = kqr.kqr_fit_path(Xp, yp, path.tau, lams, "rbf", path.gamma,
                                                 uniforms=inputs.pivot_uniforms(64, (5, 3)))
            assert all(s == kqr.KQR_OK for s in st + stp)
            runs[T] = ([x.cpu() for x in a], list(b), [i["kapply_calls"] for i in inf], ap.cpu(), list(bp))
            say("threads", T, "batch kapply calls", sum(runs[T][2]))
    finally:
        kqr.kqr_set_batch_threads(0)
    (a1, b1, k1, p1, q1), (a5, b5, k5, p5, q5) = runs[1], runs[5]
    assert all(torch.equal(x, y) for x, y in zip(a1, a5))
    assert b1 == b5 and k1 == k5
    assert torch.equal(p1, p5) and q1 == q5
