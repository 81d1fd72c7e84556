"""1D nodal basis and quadrature for the oracle (test infrastructure only).

Sec. 3.2: shape functions are tensor products of 1D Lagrange polynomials whose
support points are the Legendre-Gauss-Lobatto (LGL) nodes; integrals are
evaluated with Gauss quadrature on the reference interval [0, 1].

Everything here is the plain definition: LGL nodes are the end points plus the
roots of P_k' (found from NumPy's Legendre module and polished by Newton
steps), Gauss rules come from ``numpy.polynomial.legendre.leggauss``, Lagrange
values and derivatives are the product formula evaluated term by term.
"""
import numpy as np
from numpy.polynomial import legendre as npleg


def lgl_nodes(k):
    """The k+1 LGL nodes of degree k on [0, 1], ascending (Sec. 3.2).

    Interior nodes are the roots of the derivative of the Legendre polynomial
    P_k on [-1, 1]; the end points are exactly 0 and 1.
    """
    if k < 1:
        raise ValueError("degree must be >= 1")
    ck = np.zeros(k + 1)
    ck[k] = 1.0
    d1 = npleg.legder(ck)
    d2 = npleg.legder(d1)
    if k >= 2:
        r = np.sort(np.real(npleg.legroots(d1)))
        for _ in range(3):  # Newton polish of the roots of P_k'
            r = r - npleg.legval(r, d1) / npleg.legval(r, d2)
    else:
        r = np.zeros(0)
    # symmetrise: the node set is symmetric about 0 on [-1, 1]
    r = 0.5 * (r - r[::-1])
    x = np.concatenate(([-1.0], r, [1.0]))
    return 0.5 * (x + 1.0)


def gauss_rule(m):
    """m-point Gauss-Legendre rule on [0, 1]: (points, weights)."""
    x, w = npleg.leggauss(m)
    return 0.5 * (x + 1.0), 0.5 * w


def lagrange_values(nodes, x):
    """L[q, a] = l_a(x_q), the Lagrange polynomial of node a at point x_q."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    L = np.ones((len(x), n))
    for a in range(n):
        for j in range(n):
            if j != a:
                L[:, a] *= (x - nodes[j]) / (nodes[a] - nodes[j])
    return L


def lagrange_derivs(nodes, x):
    """G[q, a] = l_a'(x_q), by the product rule applied to the product formula."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    G = np.zeros((len(x), n))
    for a in range(n):
        for j in range(n):
            if j == a:
                continue
            term = np.full(len(x), 1.0 / (nodes[a] - nodes[j]))
            for l in range(n):
                if l != a and l != j:
                    term = term * (x - nodes[l]) / (nodes[a] - nodes[l])
            G[:, a] += term
    return G


def default_laplace_nq(k):
    """Gauss points per direction for the Laplace form: k+1 (exact on affine cells)."""
    return k + 1


def default_convective_nq(k):
    """Gauss points for the convective form: floor(3k/2)+1, the 3/2 rule (Sec. 3.2).

    The cell integrand grad(v) : (u x u) has degree (k-1) + 2k = 3k-1 per
    direction and the face integrand 3k, so floor(3k/2)+1 points integrate
    both exactly.
    """
    return (3 * k) // 2 + 1
