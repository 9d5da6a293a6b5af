"""Writes tiny_fits.json: FP64 oracle solutions of small seeded problems.

Run from the repository root:  python tests/golden/make_golden.py
Only the oracle and the seeded input generators are called.  The stored
values are checked against brute-force partition enumeration by
tests/test_golden.py (CPU) and used as expected values by the GPU tests.
"""
from __future__ import annotations

import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import adjoint as oadj  # noqa: E402
from oracle import solver as osolver  # noqa: E402
from paper_2510_07929_amd import inputs  # noqa: E402

CASES = [
    # name, n, p, kernel, gamma, tau, lambda, seed
    ("rbf_n9", 9, 2, "rbf", 0.5, 0.3, 0.7, 1),
    ("laplacian_n9", 9, 3, "laplacian", 0.4, 0.5, 1.3, 2),
    ("rbf_n9_tau09", 9, 2, "rbf", 1.5, 0.9, 0.2, 3),
    ("rbf_n40", 40, 3, "rbf", 0.3, 0.25, 2.0, 4),
]


def main():
    out = []
    for name, n, p, kind, gamma, tau, lam, seed in CASES:
        X, y = inputs.smooth(n + 10, p, (500, seed))
        Xtr, ytr, Xv, yv = X[:n], y[:n], X[n:], y[n:]
        r = osolver.fit(Xtr, ytr, tau, lam, kind, gamma, osolver.OracleOptions(tol=1e-12))
        rec = dict(name=name, n=n, p=p, kernel=kind, gamma=gamma, tau=tau, lam=lam, seed=seed,
                   X=Xtr.astype(float).tolist(), y=ytr.tolist(), Xval=Xv.astype(float).tolist(), yval=yv.tolist(),
                   alpha=r.alpha.tolist(), beta=float(r.beta), obj_p=float(r.kkt["obj_p"]),
                   polished=bool(r.info["polished"]), n_interior=int(r.info["n_interior"]))
        if r.info["n_interior"] > 0:
            J, dg, dl, m = oadj.adjoint_gradient(Xtr, r.alpha, r.beta, Xv, yv, lam, tau, kind, gamma)
            rec.update(J=J, dJ_dlog_gamma=dg, dJ_dlog_lambda=dl)
        out.append(rec)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tiny_fits.json")
    with open(path, "w") as f:
        json.dump({"generator": "tests/golden/make_golden.py", "cases": out}, f, indent=1)
    print(f"wrote {path} ({len(out)} cases)")


if __name__ == "__main__":
    main()
