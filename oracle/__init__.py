"""FP64 CPU oracle for the exponential-integrator Q1 finite element (EIFE) method.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, deliberately
straightforward NumPy/SciPy implementation of what the GPU library computes.
It exists to check the GPU library, never to stand in for it: only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import
it.  It shares no code, tables or constants with the HIP library.

What it computes (Huang, Ju, Xu, "Efficient Exponential Integrator Finite
Element Method for Semilinear Parabolic Equations"):

* ``fem``       -- Q1 mass and stiffness matrices on a uniform tensor grid of a
                   rectangle with homogeneous Dirichlet data (Section 2.1,
                   eq. (2.5); Section 4, eq. (4.1)), assembled from element
                   matrices, plus an independent Gauss-quadrature assembly.
* ``phi``       -- the functions phi_k(z) of Section 2.2.
* ``spectral``  -- three bases that diagonalise the pair (K, M): dense
                   generalised eigendecomposition (tier A), per-axis dense
                   eigendecomposition applied as Kronecker mode products
                   (tier B), and the sine transform with closed-form
                   eigenvalues (tier C, Section 4).
* ``stepper``   -- EIFE1 (eq. (2.13)) and EIFE2 (eq. (2.14)).
* ``problems``  -- reaction terms and exact solutions of the test problems.
* ``norms``     -- discrete and quadrature L2/H1 norms, Allen-Cahn energy.

Every function names the passage of the paper it follows.
"""
