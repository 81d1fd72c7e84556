"""Plain CPU oracle for the matrix-free DG operators (test infrastructure only).

This package is the checker, not the product.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  It shares no code with the HIP path: it evaluates the weak forms
of the paper's Section 3.2 element by element with explicit three-dimensional
basis tables (dense matrices over all (k+1)^3 basis functions and all
quadrature points), with no sum factorisation, in float64.

Modules
-------
basis       1D Legendre-Gauss-Lobatto / Gauss rules and Lagrange tables (Sec. 3.2)
mesh        periodic Cartesian mesh, element numbering and neighbours (Sec. 4)
tables      explicit 3D cell and face tables built from the 1D ones
laplace     SIPG negative Laplacian l_h (Sec. 3.2, weak form of l_h)
convective  convective term c_h with local Lax-Friedrichs flux, its explicit
            Jacobian, JVP and VJP (Sec. 3.2, weak form of c_h)
divergence  velocity divergence d_h with central flux (Sec. 3.2, weak form of d_h)
solvers     CG (Jacobi / Chebyshev preconditioned), Chebyshev iteration and
            the fast-diagonalisation direct solve (Sec. 3.3)
"""
