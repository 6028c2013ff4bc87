"""FP64 CPU oracle for the even-odd Wilson(-clover) operator and its solvers.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links this package; only the tests, the package's smoke check and the
CPU-baseline leg of the benchmark use it.  It shares no code with the HIP
library (no kernels, headers, tables or helpers); the only thing both sides
consume is the seeded input arrays made by ``gen.fields``.

What it computes follows the paper's statement of the problem (section 3,
eq. "linear": solve M phi = b or M^dagger M phi = b for Wilson or clover
fermions) and of the solvers (section 5: CG on the normal operator,
even-odd Schur complement CG, FGCR == FGMRES as a flexible outer method,
mixed precision by iterative refinement).  The paper does not write down the
Dirac operator, the gamma basis, the clover term or the solver recurrences;
the readings used here are stated in each module's header and pinned by the
``-m "not gpu"`` tests (free-field spectrum, gamma5-hermiticity, gauge
covariance, point-source stencil, abelian clover closed form, dense solves).

Everything is complex128 NumPy with plain whole-lattice array operations:
no blocking, fusion or reordering beyond the definitions.

Modules:
    dirac    gamma matrices, hopping term H, Wilson operator M_W = 1 - kappa H
    clover   clover leaves Q, field strength F, clover term A, A^{-1}
    evenodd  parity split, Schur operator, source preparation, reconstruction
    solvers  CGNR, BiCGStab, FGMRES(m), flexible CG
    dense    dense matrix of an operator (tiny lattices only)
    net      gauge-covariant linear preconditioner net: forward, backward
"""
