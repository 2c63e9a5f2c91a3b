"""FP64 CPU oracle for the fast-diagonalisation preconditioned CG method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) imports, links or calls this package; only the tests, the
smoke check and the benchmark's CPU-baseline leg do.  It shares no code with
the GPU path: the only common module is `synth`, which generates seeded inputs
and does none of the method's arithmetic.

The oracle is written to be read against the paper (Sangalli & Tani,
"Isogeometric preconditioners based on fast solvers for the Sylvester
equation"): plain NumPy, float64, every function citing the passage it
follows.  Library primitives (matmul, Cholesky, symmetric eigensolver,
Gauss-Legendre nodes, sparse matrix-vector product) serve as single steps.

Modules
    splines     open knot vectors, Cox-de Boor basis and derivatives,
                Gauss rule, 1D mass/stiffness matrices (Sec. 2.1, Sec. 3)
    geometry    the maps F, their Jacobians, Q = |det J| J^-1 K J^-T,
                right-hand sides (Sec. 2.1 eq. A, eq. Q)
    assembly    Galerkin stiffness A and load vector b by an element loop
                over Gauss points (Sec. 2.1 eq. A)
    fd          generalised eigendecomposition and the fast diagonalisation
                apply of P^-1 (Sec. 4.1 Alg. 1, Sec. 5.1 Alg. 3), the
                explicit Kronecker form of P (Sec. 3 eq. prec)
    pcg         preconditioned CG, flexible CG, scaled preconditioner
    adi         three-variable ADI of Douglas as an inexact P^-1 (Sec. 5.2
                Alg. '3D ADI method'), its parameters and closed form
    multipatch  L-shaped three-patch domain with C^0 interfaces and the
                overlapping additive Schwarz preconditioners P_EAS, P_IAS
                (Sec. 6 eq. Peas, eq. Pias)
    mlp         FP64 reference of the learned diagonal scaling network

Parity status: every function has a pin in tests/test_oracle_*.py except
the mixed-precision solves (no exact value exists: parity unpinned; they are
judged by the FP64 true residual) -- see the module headers.
"""
