"""Kernel matrices in float64 by direct differences.

Section 1 defines the two kernels used by the method:
RBF  k(x, x') = exp(-gamma ||x - x'||_2^2) and
Laplacian k(x, x') = exp(-gamma ||x - x'||_1).
The oracle sums coordinate differences directly (never the norm expansion
||x||^2 + ||x'||^2 - 2 x.x'), so that it does not share a formula with the
GPU path.  The linear kernel of Table 2, k(x, x') = x^T x', is the plain
product X X^T.
"""
from __future__ import annotations

import numpy as np

KINDS = ("rbf", "laplacian", "linear")


def distance_block(Xa: np.ndarray, Xb: np.ndarray, kind: str) -> np.ndarray:
    """Squared Euclidean (rbf) or L1 (laplacian) distances, (ma, mb) float64."""
    if kind not in ("rbf", "laplacian"):
        raise ValueError(kind)
    Xa = np.asarray(Xa, dtype=np.float64)
    Xb = np.asarray(Xb, dtype=np.float64)
    D = np.zeros((Xa.shape[0], Xb.shape[0]))
    for f in range(Xa.shape[1]):
        diff = Xa[:, f, None] - Xb[None, :, f]
        if kind == "rbf":
            D += diff * diff
        else:
            D += np.abs(diff)
    return D


def kernel_block(Xa, Xb, kind: str, gamma: float) -> np.ndarray:
    """K(Xa, Xb) in float64: the RBF and Laplacian kernels of Section 1, or
    the linear kernel k(x, x') = x^T x' of Table 2 (gamma unused)."""
    if kind == "linear":
        return np.asarray(Xa, dtype=np.float64) @ np.asarray(Xb, dtype=np.float64).T
    return np.exp(-gamma * distance_block(Xa, Xb, kind))


def kernel_matrix(X, kind: str, gamma: float, block: int = 2048) -> np.ndarray:
    """Full n x n kernel matrix, built block by block."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    K = np.empty((n, n))
    for i in range(0, n, block):
        K[i : i + block] = kernel_block(X[i : i + block], X, kind, gamma)
    return K


def kernel_apply(X, V, kind: str, gamma: float, Xrows=None, block: int = 1024) -> np.ndarray:
    """U = K(Xrows, X) @ V without storing K (rows of K built per block).

    ``V`` may be a vector (n,) or a matrix (n, m).  ``Xrows`` defaults to X.
    """
    X = np.asarray(X, dtype=np.float64)
    Xr = X if Xrows is None else np.asarray(Xrows, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    out = np.empty((Xr.shape[0],) + V.shape[1:])
    for i in range(0, Xr.shape[0], block):
        out[i : i + block] = kernel_block(Xr[i : i + block], X, kind, gamma) @ V
    return out


class DenseKernel:
    """A materialised float64 kernel matrix with the operations the solver uses."""

    def __init__(self, X, kind: str, gamma: float):
        self.X = np.asarray(X, dtype=np.float64)
        self.kind = kind
        self.gamma = float(gamma)
        self.K = kernel_matrix(self.X, kind, gamma)
        self.n = self.K.shape[0]
        self.applies = 0

    def apply(self, v):
        self.applies += 1
        return self.K @ v

    def column(self, j: int) -> np.ndarray:
        return self.K[:, j].copy()

    def diag(self) -> np.ndarray:
        return np.diag(self.K).copy()


class ImplicitKernel:
    """Kernel operator that never stores K (for sizes whose float64 K does not fit)."""

    def __init__(self, X, kind: str, gamma: float, block: int = 1024):
        self.X = np.asarray(X, dtype=np.float64)
        self.kind = kind
        self.gamma = float(gamma)
        self.n = self.X.shape[0]
        self.block = block
        self.applies = 0

    def apply(self, v):
        self.applies += 1
        return kernel_apply(self.X, v, self.kind, self.gamma, block=self.block)

    def column(self, j: int) -> np.ndarray:
        return kernel_block(self.X, self.X[j : j + 1], self.kind, self.gamma)[:, 0]

    def diag(self) -> np.ndarray:
        if self.kind == "linear":
            return (self.X * self.X).sum(1)
        return np.ones(self.n)  # RBF and Laplacian have k(x, x) = exp(0) = 1
