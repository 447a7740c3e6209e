"""CPU oracle for the shifted-HSS Helmholtz solver (Cotter, Hope-Collins and
Knook, "Shifted HSS solvers for the indefinite Helmholtz equation").

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, complex-FP64
re-statement of what the GPU path computes: element-by-element finite-element
assembly into CSR matrices, the operators of the gamma=k HSS iteration, the
shifted-HSS preconditioner, a CSR geometric-multigrid V-cycle, and flexible
GMRES.  Only the test-suite, the smoke check of the package entry point and
the CPU-baseline leg of the benchmark may import it.  The product path never
routes through it, and it shares no code, tables or constants with the HIP
library.

Modules
-------
fem        meshes, element matrices, global assembly, interpolation, and the
           elimination of Dirichlet faces (Sec. 2)
operators  B_delta, the H inner product, A_S, and the HSS operators L, N
           (Sec. 3.1 and the shifted-HSS definition of Sec. 4)
hss        the gamma=k HSS iteration in its literal and correction forms, and
           the shifted-HSS preconditioner (Sec. 3.1, Sec. 4)
multigrid  CSR V(nu1,nu2) cycle with scaled-Jacobi smoothing (Sec. 5.3)
krylov     right-preconditioned flexible GMRES and preconditioned
           Richardson for the outer iteration (Sec. 5.1)
solver     the assembled end-to-end solve used as the parity reference

Parity status: every function above is pinned by a CPU test against a
closed form, an invariant of the discretisation, a textbook convergence rate,
an independent library routine, or a value printed in the paper.  The
two-grid contraction of the V(2,2)-Jacobi cycle is pinned by local Fourier
analysis on meshes with every face Dirichlet.  Two quantities have no exact
pin ("parity unpinned"): the outer iteration count of the V(2,2)-Jacobi
preconditioned solve at the benchmark settings and the multigrid
contraction factor there (impedance faces, many levels); the paper prints
neither.
"""

from . import fem, operators, hss, multigrid, krylov, solver  # noqa: F401
