"""Seeded synthetic workloads for kernel quantile regression.

This module holds random draws and the response surfaces that define each
workload, and nothing of the solver's arithmetic.  The GPU path (tests, bench)
and the FP64 CPU oracle both take their inputs from here, so the two sides see
the same bits: X is drawn in float64 and rounded to float32 once; y stays
float64.

Workloads (the paper's own experiments use a 2-D surface, Section 4.1, and an
energy-load dataset, Section 4.2, that is not available here; the shapes below
are synthetic stand-ins sized for one MI355X):

* ``smooth``  : x ~ U[-1,1]^p, y = sin(pi*||x||_2) + 0.3*(0.5+|x_1|)*e with
                e ~ N(0,1) (or Student-t(2) for the heavy-tailed variant).
* ``additive``: x ~ N(0, I_p), y = sum_j sin(x_j)/sqrt(p) + (1+|x_1|)*t_3.
* ``paper2d`` : the two-dimensional ratio-of-exponentials surface of
                Section 4.1 with N(0,1) noise (used for regularisation paths).

Random numbers the method itself draws (the RPCholesky pivot samples) are
produced here as well, as a vector of uniforms, and passed to both sides.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Problem",
    "workload",
    "smooth",
    "additive",
    "paper2d",
    "lambda_grid",
    "pivot_uniforms",
    "uneven_batch",
    "WORKLOADS",
]


def _rng(*key: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(k) for k in key]))


@dataclass
class Problem:
    """One KQR instance: data plus (tau, lambda, kernel, gamma)."""

    name: str
    X: np.ndarray  # (n, p) float32, row-major
    y: np.ndarray  # (n,) float64
    tau: float
    lam: float
    kernel: str  # "rbf" | "laplacian"
    gamma: float
    rank: int = 0  # 0: adaptive rank; >0: fixed rank
    kdtype: str = "fp32"  # storage type of a materialised K
    extras: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.X.shape[0])

    @property
    def p(self) -> int:
        return int(self.X.shape[1])


def smooth(n: int, p: int, key: tuple, heavy_tail: bool = False):
    """x ~ U[-1,1]^p ; y = sin(pi ||x||) + 0.3 (0.5+|x1|) e."""
    g = _rng(*key)
    x = g.uniform(-1.0, 1.0, size=(n, p))
    e = g.standard_t(2, size=n) if heavy_tail else g.standard_normal(n)
    X = x.astype(np.float32)
    xd = X.astype(np.float64)
    y = np.sin(np.pi * np.sqrt((xd * xd).sum(1))) + 0.3 * (0.5 + np.abs(xd[:, 0])) * e
    return X, y


def additive(n: int, p: int, key: tuple):
    """x ~ N(0, I) ; y = sum_j sin(x_j)/sqrt(p) + (1+|x1|) t_3."""
    g = _rng(*key)
    x = g.standard_normal((n, p))
    e = g.standard_t(3, size=n)
    X = x.astype(np.float32)
    xd = X.astype(np.float64)
    y = np.sin(xd).sum(1) / np.sqrt(p) + (1.0 + np.abs(xd[:, 0])) * e
    return X, y


def paper2d(n: int, key: tuple):
    """Section 4.1 surface on [0,1]^2 with standard normal noise."""
    g = _rng(*key)
    x = g.uniform(0.0, 1.0, size=(n, 2))
    e = g.standard_normal(n)
    X = x.astype(np.float32)
    a = X[:, 0].astype(np.float64)
    b = X[:, 1].astype(np.float64)
    num = 40.0 * np.exp(8.0 * ((a - 0.5) ** 2 + (b - 0.5) ** 2))
    den = np.exp(8.0 * ((a - 0.2) ** 2 + (b - 0.7) ** 2)) + np.exp(
        8.0 * ((a - 0.7) ** 2 + (b - 0.2) ** 2)
    )
    return X, num / den + e


def pivot_uniforms(count: int, key: tuple) -> np.ndarray:
    """Uniforms in [0,1) that drive RPCholesky's pivot draws (one per step)."""
    return _rng(*key, 7919).uniform(0.0, 1.0, size=count)


# name -> (default n, description)
WORKLOADS = {
    "c0": (2000, "smooth, n=2000, p=10, RBF gamma=1/p, tau=0.5, lambda=1e-3 n, FP32 K"),
    "c1": (50000, "additive, n=50000, p=20, RBF gamma=1/(2p), tau=0.25, lambda=1e-4 n, FP32 K, rank 500"),
    "c2": (150000, "additive, n=150000, p=30, RBF gamma=1/p, tau=0.75, lambda=1e-4 n, BF16 K"),
    "c2lap": (300000, "additive, n=300000, p=30, Laplacian gamma=1/p, tau=0.75, lambda=1e-4 n, on the fly"),
    "c3a": (100000, "additive, n=100000, p=8, RBF gamma=1/p, 9 tau levels 0.1..0.9, lambda=1e-4 n"),
    "c4": (20000, "smooth with t(2) noise, n=20000 train + 5000 validation, p=10, RBF gamma=0.1, tau=0.5, lambda=1e-3 n"),
    "ablation": (10000, "paper2d, n=10000, p=2, RBF gamma=1e-3, tau=0.1, lambda=10, tol 1e-8"),
    "linear": (20000, "paper2d, n=20000, p=2, linear kernel x^T x', tau=0.5, 50 lambda log-spaced over [1e-2, 1], tol 1e-8"),
    "path": (20000, "paper2d, n=20000, p=2, RBF gamma=0.1, tau=0.5, 50 lambda log-spaced over [1e-2, 1], tol 1e-8"),
}


def lambda_grid(count: int = 50, lo: float = 1e-2, hi: float = 1.0) -> list:
    """``count`` values of lambda log-spaced over [lo, hi], largest first (the
    sequences of Section 4.1)."""
    return [float(v) for v in np.logspace(np.log10(hi), np.log10(lo), count)]


def workload(name: str, seed: int = 0, n: int | None = None) -> Problem:
    """Build a named workload; ``n`` overrides the size (lambda follows n)."""
    if name not in WORKLOADS:
        raise KeyError(f"unknown workload {name!r}; have {sorted(WORKLOADS)}")
    n = int(n if n is not None else WORKLOADS[name][0])
    if name == "c0":
        p = 10
        X, y = smooth(n, p, (0, seed))
        return Problem(name, X, y, 0.5, 1e-3 * n, "rbf", 1.0 / p)
    if name == "c1":
        p = 20
        X, y = additive(n, p, (1, seed))
        return Problem(name, X, y, 0.25, 1e-4 * n, "rbf", 1.0 / (2 * p), rank=500)
    if name == "c2":
        p = 30
        X, y = additive(n, p, (2, seed))
        return Problem(name, X, y, 0.75, 1e-4 * n, "rbf", 1.0 / p, kdtype="bf16")
    if name == "c2lap":
        p = 30
        X, y = additive(n, p, (20, seed))
        return Problem(name, X, y, 0.75, 1e-4 * n, "laplacian", 1.0 / p)
    if name == "c3a":
        p = 8
        X, y = additive(n, p, (3, seed))
        taus = [round(0.1 * k, 1) for k in range(1, 10)]
        return Problem(name, X, y, 0.5, 1e-4 * n, "rbf", 1.0 / p, extras={"taus": taus})
    if name == "c4":
        p = 10
        nval = max(1, n // 4)
        X, y = smooth(n + nval, p, (4, seed), heavy_tail=True)
        return Problem(
            name, X[:n].copy(), y[:n].copy(), 0.5, 1e-3 * n, "rbf", 0.1,
            extras={"Xval": X[n:].copy(), "yval": y[n:].copy()},
        )
    if name == "ablation":
        X, y = paper2d(n, (44, seed))
        return Problem(name, X, y, 0.1, 10.0, "rbf", 1e-3, extras={"tol": 1e-8})
    if name == "linear":
        X, y = paper2d(n, (47, seed))
        lams = lambda_grid()
        return Problem(name, X, y, 0.5, lams[0], "linear", 1.0, extras={"lams": lams, "tol": 1e-8})
    if name == "path":
        X, y = paper2d(n, (40, seed))
        lams = lambda_grid()
        return Problem(name, X, y, 0.5, lams[0], "rbf", 0.1, extras={"lams": lams, "tol": 1e-8})
    raise AssertionError(name)


def uneven_batch(count: int = 64, lo: int = 500, hi: int = 8000, p: int = 10, seed: int = 0):
    """``count`` independent problems with n_i ~ U{lo..hi}, smooth generator,
    RBF gamma=1/p, tau=0.5, lambda_i=1e-3 n_i."""
    sizes = _rng(30, seed).integers(lo, hi + 1, size=count)
    probs = []
    for i, ni in enumerate(sizes):
        X, y = smooth(int(ni), p, (31, seed, i))
        probs.append(Problem(f"c3b[{i}]", X, y, 0.5, 1e-3 * int(ni), "rbf", 1.0 / p))
    return probs
