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
gradient    pressure gradient g_h in the velocity space (Sec. 3.2)
mass        mass matrix, its inverse and the Helmholtz operator (Sec. 3.3)
projection  the projection-step operator M + A_D + A_C (Sec. 3.2, 3.3)
transfer    h-multigrid level transfers (Sec. 3.3)
multigrid   the geometric multigrid V-cycle (Sec. 3.3)
mixed       divergence and gradient between the degree-k velocity and the
            degree-(k-1) pressure (Sec. 3.2, mixed-order spaces)
dual_splitting  one BDF1/BDF2 dual-splitting step composed from the operators
            above, the penalty parameters and the Taylor-Green diagnostics
            e_k and eps (Sec. 3.1, 3.2, 4.2)
"""
