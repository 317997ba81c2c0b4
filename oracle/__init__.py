"""CPU FP64 oracle for the H(div)-DG Stokes multigrid of Cui & Kanschat,
"Multigrid methods for the Stokes problem on GPU systems" (arXiv 2410.09497).

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import it.  The product library
(``paper_2410_09497_amd``) never imports, links or calls anything here, and
nothing here imports the product library: the two share no code.

Everything is computed from the plain definitions, in float64:

* ``fe1d``     -- quadrature rules and 1D Lagrange bases (Sec. 2.1).
* ``stokes``   -- the DoF layout, element-by-element 3D quadrature of the
                  bilinear form (Eq. bilinear) and the divergence form
                  (Eq. weak_form), global sparse assembly, matrix-free apply
                  by local element matrices, right-hand sides, error norms and
                  a direct solve (the discrete problem of Sec. 2).
* ``patches``  -- vertex patches, colours, patch matrices taken as the
                  Galerkin restriction K[X_j, X_j] and the dense
                  pseudo-inverse local solver (Sec. 3.1, the "Direct solver" of
                  Sec. 3.3), plus the Schur/fast-diagonalization route of
                  Sec. 3.2 written out with dense matrices.
* ``mg``       -- transfers, the colourized vertex-patch smoother (Alg. 2),
                  the V-cycle (Sec. 3) and right-preconditioned FGMRES.
* ``mlp``      -- the per-patch network of the learned local solver (not in
                  the paper): forward, loss, backward, Adam, and smoother
                  callbacks for pair capture and learned solves.

Where the paper is silent or garbled, each module states the reading it
applies next to the code that applies it (bases and quadrature, the sign of
B, the penalty and face terms, the restriction, the pseudo-inverse).
"""
