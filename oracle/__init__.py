"""Correctness oracle for the parallel Riccati Newton-step solver.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import, call or execute anything in this
package.  The GPU library never depends on it, and this package shares no code
with the GPU library: the two meet only through the seeded synthetic inputs.

Contents (each function cites the passage of the paper it follows):

* ``riccati``   - serial FP64 Riccati recursion (Alg. 1-3), written in C.
* ``kkt``       - dense KKT assembly and LU solve of P(N), the blockwise KKT
                  residual and direct evaluation of the objective.
* ``exact``     - the KKT system solved in exact rational arithmetic (tiny
                  problems; golden fixtures).
* ``reduction`` - closed-form reduced subproblem of Theorem 1 and the master
                  problem of Sec. 4.3, built from the preliminary Riccati
                  solution by the paper's product and sum formulas; the
                  rank-revealing form with the U_1 basis (n_uo <= n_x
                  inputs per master stage) and a dense KKT solve of master
                  problems whose stages have different input dimensions.
* ``mhe``       - MHE problem to UFTOC conversion (Sec. 2) and the RTS
                  smoother, used as an independent closed-form pin.
* ``boxqp``     - minimiser of P(N) with bounds on the inputs (the
                  inequality-constrained problem of Sec. 3) by condensing and
                  bounded-variable least squares.

Problems are dicts of float64 numpy arrays, row-major blocks:
``Qx (N,nx,nx)  Qw (N,nu,nu)  Qxw (N,nx,nu)  A (N,nx,nx)  B (N,nx,nu)
a (N,nx)  lx (N,nx)  lw (N,nu)  c (N,)  QxN (nx,nx)  lN (nx,)  cN ()
x0 (nx,)``.
"""
