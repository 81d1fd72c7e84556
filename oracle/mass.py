"""Mass matrix of the DG space and its inverse, evaluated the plain way (test
infrastructure only).

Sec. 3.3: the mass matrix of a discontinuous Galerkin space is
block-diagonal, one dense (k+1)^3 x (k+1)^3 block per element,
M_e[i, j] = (phi_i, phi_j)_K, and its inverse is applied element by element.
Here each block is assembled as an explicit Gauss sum over the (k+1)^3 cell
points against the dense 3D basis table (exact: the integrand has degree 2k
in each direction), and the inverse is applied by a dense solve.
"""
import numpy as np

from .tables import tables


def mass_block(k, mesh):
    """M_e of one element (all elements of the Cartesian mesh share it)."""
    T = tables(k, k + 1)
    vol = float(np.prod(mesh.h))
    return vol * (T.B.T * T.W) @ T.B


def mass_apply(u, k, mesh, elems=None):
    """y = M u; u has shape [..., N_el, (k+1)^3]."""
    M = mass_block(k, mesh)
    u = np.asarray(u, dtype=np.float64)
    ue = u if elems is None else u[..., np.asarray(elems), :]
    return ue @ M.T


def inverse_mass_apply(u, k, mesh, elems=None):
    """x = M^-1 u, element by element; u has shape [..., N_el, (k+1)^3]."""
    M = mass_block(k, mesh)
    u = np.asarray(u, dtype=np.float64)
    ue = u if elems is None else u[..., np.asarray(elems), :]
    flat = ue.reshape(-1, ue.shape[-1])
    return np.linalg.solve(M, flat.T).T.reshape(ue.shape)


def helmholtz_apply(u, k, mesh, mass_factor, scale=1.0, penalty_factor=1.0, n_q=0):
    """mass_factor M u + scale L u: the operator of the viscous step (Sec. 3.3,
    gamma_0/dt M + nu L), each term evaluated by its own oracle."""
    from .laplace import laplace_apply
    return mass_factor * mass_apply(u, k, mesh) + laplace_apply(u, k, mesh, n_q=n_q,
                                                                penalty_factor=penalty_factor, scale=scale)
