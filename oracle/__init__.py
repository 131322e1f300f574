"""CPU FP64 oracle for the space-time Galerkin discretisation of the linear
Schroedinger equation and its Kronecker-structured solvers.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link anything in this package; only
the test-suite, the smoke check and the CPU-baseline leg of the benchmark use
it.  It shares no code with the GPU path: assembly, quadrature, the temporal
decomposition and every solver here are written independently, in plain
numpy/scipy, in double precision, following the paper's definitions in the
paper's order:

* model problem and sesquilinear form            -- Sec. 3, eq. (VF_inhomogen)
* homogenisation by the initial datum            -- Sec. 3 (psi_hat = psi - psi_0)
* tensor-product P1/P2 spaces, Galerkin system    -- Sec. 3, eqs. (VF_FEM), (LGS)
* spatial and temporal matrices                   -- Sec. 3, eqs. (matrix_x), (matrix_t)
* Kronecker solver: Bartels-Stewart / fast diag.  -- Sec. 3, solver steps 1-4, eq. (LGS_x)
* space-time error norms and kappa_2(X_t)         -- Sec. 4, Tables 1-3

Modules
-------
quadrature  Gauss-Legendre and collapsed (Duffy) triangle rules
fem         meshes, element loops, global matrices, load vectors, interpolation
problems    manufactured solutions and their right-hand sides
solvers     dense/sparse global solves, paper-form FDM and Bartels-Stewart, adjoint
norms       L2(Q) and H1(Q)-seminorm errors by quadrature, eoc
baseline    the time-parallel oracle FDM used as the CPU throughput baseline
"""
