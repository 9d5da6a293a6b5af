"""GPU parity of the implicit adjoint (gradient of the validation check loss
with respect to log gamma and log lambda) against the FP64 oracle, and against
central finite differences of polished GPU fits.

The GPU adjoint forms every kernel entry in FP64 from the FP32 inputs, so it
and the oracle differ only by summation order and by the conditioning of the
bordered system on K_EE: the gradients are compared at 1e-6 relative.
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import adjoint as oadj
from oracle import kernel as okernel
from oracle import solver as osolver
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


def _problem(n, kind="rbf", seed=0):
    prob = inputs.workload("c4", seed=seed, n=n)
    gamma = prob.gamma if kind == "rbf" else 0.5 / prob.X.shape[1]
    return prob, gamma


def _gpu(prob, dev, kind, gamma, lam=None, **kw):
    X = torch.from_numpy(prob.X).to(dev)
    y = torch.from_numpy(prob.y).to(dev)
    Xv = torch.from_numpy(prob.extras["Xval"]).to(dev)
    yv = torch.from_numpy(prob.extras["yval"]).to(dev)
    lam = prob.lam if lam is None else lam
    return kqr.kqr_fit_grad(X, y, prob.tau, lam, kind, gamma, Xv, yv, **kw)


@pytest.mark.parametrize("kind,n", [("rbf", 1500), ("laplacian", 1200), ("rbf", 777)])
def test_adjoint_matches_oracle(dev, kind, n):
    prob, gamma = _problem(n, kind)
    say("adjoint vs oracle", kind, n)
    alpha, beta, J, (dg, dl), m, polished, info, st = _gpu(prob, dev, kind, gamma, tol=1e-8)
    assert st == kqr.KQR_OK and polished
    ref = osolver.fit(prob.X, prob.y, prob.tau, prob.lam, kind, gamma, osolver.OracleOptions(tol=1e-10))
    assert ref.info["polished"]
    Xv, yv = prob.extras["Xval"], prob.extras["yval"]
    J0, dg0, dl0, m0 = oadj.adjoint_gradient(prob.X, ref.alpha, ref.beta, Xv, yv, prob.lam, prob.tau, kind, gamma)
    a = alpha.cpu().numpy()
    say(f"  |E|={m} (oracle {m0}) J={J:.12g} ({J0:.12g}) dg={dg:.10g} ({dg0:.10g}) dl={dl:.10g} ({dl0:.10g})")
    assert m == m0
    # the polished point solves the same FP64 bordered system as the oracle's
    assert np.max(np.abs(a - ref.alpha)) <= 1e-7
    assert abs(beta - ref.beta) <= 1e-7 * (1 + abs(ref.beta))
    assert J == pytest.approx(J0, rel=1e-9, abs=1e-9)
    scale_g = abs(dg0) + abs(dl0)
    assert abs(dg - dg0) <= 1e-6 * scale_g
    assert abs(dl - dl0) <= 1e-6 * scale_g


def _signs(prob, alpha, beta, kind, gamma, lam):
    """Validation residual signs and the interior set of a polished fit (FP64 on the CPU)."""
    Kv = okernel.kernel_block(prob.extras["Xval"], prob.X, kind, gamma)
    r = prob.extras["yval"] - beta - Kv @ alpha / lam
    E = np.flatnonzero((alpha > prob.tau - 1.0) & (alpha < prob.tau))
    return np.sign(r), E


@pytest.mark.parametrize("kind", ["rbf", "laplacian"])
def test_adjoint_matches_central_differences(dev, kind):
    prob, gamma = _problem(1000, kind, seed=1)
    h = 1e-4
    say("adjoint vs central FD", kind)
    a0, b0, J0, (dg, dl), m0, pol, _, st = _gpu(prob, dev, kind, gamma, tol=1e-9)
    assert st == kqr.KQR_OK and pol
    s0, E0 = _signs(prob, a0.cpu().numpy(), b0, kind, gamma, prob.lam)
    for which, g_an in (("gamma", dg), ("lambda", dl)):
        vals, kink = [], False
        for sgn in (+1, -1):
            gg = gamma * math.exp(sgn * h) if which == "gamma" else gamma
            ll = prob.lam * math.exp(sgn * h) if which == "lambda" else prob.lam
            a, b, J, _, _, pol, _, st = _gpu(prob, dev, kind, gg, lam=ll, tol=1e-9)
            assert st == kqr.KQR_OK and pol
            s, E = _signs(prob, a.cpu().numpy(), b, kind, gg, ll)
            kink |= not (np.array_equal(s, s0) and np.array_equal(E, E0))
            vals.append(J)
        fd = (vals[0] - vals[1]) / (2 * h)
        rel = abs(fd - g_an) / max(abs(g_an), 1e-12)
        say(f"  d/dlog {which}: adjoint {g_an:.10g} fd {fd:.10g} rel {rel:.2e} kink={kink}")
        # kink-free interval: 1e-6; a partition or validation sign change inside it: 1e-3
        assert rel <= (1e-3 if kink else 1e-6)


def test_autograd_function(dev):
    prob, gamma = _problem(600, "rbf", seed=2)
    X = torch.from_numpy(prob.X).to(dev)
    y = torch.from_numpy(prob.y).to(dev)
    Xv = torch.from_numpy(prob.extras["Xval"]).to(dev)
    yv = torch.from_numpy(prob.extras["yval"]).to(dev)
    lg = torch.tensor(math.log(gamma), dtype=torch.float64, requires_grad=True)
    ll = torch.tensor(math.log(prob.lam), dtype=torch.float64, requires_grad=True)
    say("autograd function")
    loss = kqr.kqr_validation_loss(lg, ll, X, y, Xv, yv, prob.tau, "rbf", tol=1e-8)
    (3.0 * loss).backward()
    # same (gamma, lambda) as the Function saw after the exp of the logs: bitwise the same fit
    g_in = float(torch.exp(lg.detach()))
    l_in = float(torch.exp(ll.detach()))
    _, _, J, (dg, dl), _, _, _, _ = _gpu(prob, dev, "rbf", g_in, lam=l_in, tol=1e-8)
    assert float(loss.detach()) == J
    assert float(lg.grad) == pytest.approx(3.0 * dg, rel=1e-12)
    assert float(ll.grad) == pytest.approx(3.0 * dl, rel=1e-12)


def test_adjoint_argument_errors(dev):
    prob, gamma = _problem(300)
    X = torch.from_numpy(prob.X).to(dev)
    y = torch.from_numpy(prob.y).to(dev)
    say("adjoint errors")
    Xv = torch.zeros((0, X.shape[1]), dtype=torch.float32, device=dev)
    yv = torch.zeros(0, dtype=torch.float64, device=dev)
    with pytest.raises(kqr.KqrError) as e:
        kqr.kqr_fit_grad(X, y, prob.tau, prob.lam, "rbf", gamma, Xv, yv)
    assert e.value.status == kqr.KQR_EINVAL
    with pytest.raises(ValueError):
        kqr.kqr_fit_grad(X, y, prob.tau, prob.lam, "rbf", gamma, X[:, :3].contiguous(), y[:10])


def test_adjoint_full_size_against_kink_free_differences(dev):
    # the c4 workload at its full size (n = 20000 + 5000 validation), in the
    # configuration bench.py times: the adjoint against central differences of
    # polished fits, with the step shrunk until the interval crosses no kink
    prob, gamma = _problem(20000, "rbf", seed=0)
    X = torch.from_numpy(prob.X).to(dev)
    Xv = torch.from_numpy(prob.extras["Xval"]).to(dev)
    yv = torch.from_numpy(prob.extras["yval"]).to(dev)
    say("adjoint full size")
    _, _, J0, (dg, dl), m, pol, _, st = _gpu(prob, dev, "rbf", gamma, rank=0)
    assert st == kqr.KQR_OK and pol and m > 0

    def probe(gg, ll):
        a, b, J, _, _, pol, _, st = _gpu(prob, dev, "rbf", gg, lam=ll, rank=0)
        assert st == kqr.KQR_OK and pol
        f = kqr.kqr_predict(X, a, b, ll, "rbf", gg, Xv)
        ac = a.cpu().numpy()
        return J, torch.sign(yv - f).cpu().numpy(), (ac > prob.tau - 1) & (ac < prob.tau)

    _, s0, E0 = probe(gamma, prob.lam)
    checked = 0
    for which, g_an in (("gamma", dg), ("lambda", dl)):
        for h in (1e-4, 3e-5, 1e-5, 3e-6, 1e-6):
            vals, kink = [], False
            for sgn in (1, -1):
                gg = gamma * math.exp(sgn * h) if which == "gamma" else gamma
                ll = prob.lam * math.exp(sgn * h) if which == "lambda" else prob.lam
                J, s, E = probe(gg, ll)
                kink |= not (np.array_equal(s, s0) and np.array_equal(E, E0))
                vals.append(J)
            fd = (vals[0] - vals[1]) / (2 * h)
            rel = abs(fd - g_an) / abs(g_an)
            say(f"  d/dlog {which} h={h:g}: adjoint {g_an:.10g} fd {fd:.10g} rel {rel:.2e} kink={kink}")
            if not kink:
                assert rel <= 1e-6
                checked += 1
                break
    say(f"  kink-free checks: {checked} of 2")
    assert checked == 2  # each derivative compared with central differences on a kink-free interval
