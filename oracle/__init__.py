"""FP64 CPU oracle for kernel quantile regression solved by PALM-KQR.

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke check
and the CPU-baseline leg of the benchmark may import or run anything in this
package.  The GPU library never calls it and shares no code with it.

Everything here is plain NumPy/SciPy in float64, written from the paper:

* ``kernel``   -- kernel matrices by direct differences (Section 1).
* ``problem``  -- check loss, box projection, objectives, KKT residuals and
                  the relative duality gap (Section 1, Section 4).
* ``precond``  -- randomly pivoted Cholesky and the Woodbury form of the
                  preconditioner (Section 3, Lemma 1).
* ``solver``   -- PCG, Phase I inexact ADMM (Algorithm 1), Phase II SSN-ALM
                  (Algorithms 2 and 3), the two-phase driver and an
                  active-set polish.
* ``adjoint``  -- implicit gradient of a validation check loss with respect
                  to log(gamma) and log(lambda) (not in the paper; derived
                  from the KKT system of the dual problem (1.3)).
* ``certify``  -- FP64 certificate of a returned (alpha, beta) at any n: the
                  Section 4 measures with the exact kernel and a weak-duality
                  sandwich of the optimal value.  Its kernel products come
                  from ``kapply.c`` (plain C, FP64, direct differences, rows
                  over OpenMP threads), compiled by ``build_c``.

Points the paper leaves open are fixed by the constants in
``solver.OracleOptions``; each default states its reading.
"""
from . import kernel, problem, precond, solver, adjoint  # noqa: F401
# certify loads the C library on first use; import it explicitly: from oracle import certify
