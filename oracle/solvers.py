"""Solvers for the SPD systems of Sec. 3.3 (test infrastructure only).

* ``pcg``: preconditioned conjugate gradients (Sec. 3.3 uses PCG for every
  SPD system).  The Polak-Ribiere (flexible) beta is used so that a slightly
  non-symmetric single-precision preconditioner is tolerated.  On periodic
  meshes the Laplacian annihilates constants; with ``project=True`` the
  residual and the preconditioned residual are kept at zero Euclidean mean.
* ``chebyshev``: the polynomial smoother of Adams et al. (2003) cited in
  Sec. 3.3 (degree 5, smoothing range 20 there), in the three-term form of
  Saad's Chebyshev acceleration, started from zero.
* ``sipg_1d`` / ``mass_1d``: textbook periodic 1D SIPG and DG mass matrices.
* ``fdm_solve``: fast diagonalisation (Lynch, Rice & Thomas 1964) of the 3D
  Kronecker-sum operator A = K(x)M(x)M + M(x)K(x)M + M(x)M(x)K, exact on
  uniform periodic Cartesian meshes.
"""
import numpy as np
import scipy.linalg as sla

from .basis import gauss_rule, lagrange_derivs, lagrange_values, lgl_nodes


def pcg(apply_A, b, precond=None, x0=None, rtol=1e-10, atol=0.0, max_iter=10000,
        project=False, flexible=True):
    """Returns (x, info) with info = dict(iterations, rel_res, history)."""
    def proj(v):
        return v - v.mean() if project else v
    if precond is None:
        precond = lambda r: r.copy()
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = proj(b - apply_A(x))
    bnorm = np.linalg.norm(proj(b))
    z = proj(precond(r))
    p = z.copy()
    rz = float(np.vdot(r, z))
    hist = [np.linalg.norm(r) / bnorm]
    it = 0
    while it < max_iter and np.linalg.norm(r) > max(rtol * bnorm, atol):
        q = apply_A(p)
        pq = float(np.vdot(p, q))
        if not pq > 0:
            raise FloatingPointError("p.Ap <= 0: breakdown")
        alpha = rz / pq
        x = x + alpha * p
        r = proj(r - alpha * q)
        z_new = proj(precond(r))
        rz_new = float(np.vdot(r, z_new))
        beta = (rz_new - float(np.vdot(r, z))) / rz if flexible else rz_new / rz
        p = z_new + beta * p
        z, rz = z_new, rz_new
        it += 1
        hist.append(np.linalg.norm(r) / bnorm)
    return x, dict(iterations=it, rel_res=hist[-1], history=hist)


def chebyshev(apply_A, dinv, b, degree, lam_min, lam_max):
    """Chebyshev iteration for A x = b preconditioned by D^-1, from x = 0.

    theta = (lmax+lmin)/2 is the centre and delta = (lmax-lmin)/2 the half
    width of the target interval; the first step is a damped Jacobi step
    D^-1 b / theta and each later step adds rho_k rho_{k-1} d_{k-1} +
    (2 rho_k / delta) D^-1 r_k with rho_k = 1/(2 theta/delta - rho_{k-1}).
    ``degree`` steps cost degree-1 operator applications; the error
    polynomial after them is T_degree((theta-l)/delta) / T_degree(theta/delta).
    """
    theta = 0.5 * (lam_max + lam_min)
    delta = 0.5 * (lam_max - lam_min)
    d = dinv * b / theta
    x = d.copy()
    rho_prev = delta / theta
    for _ in range(1, degree):
        r = b - apply_A(x)
        rho = 1.0 / (2.0 * theta / delta - rho_prev)
        d = rho * rho_prev * d + (2.0 * rho / delta) * dinv * r
        x = x + d
        rho_prev = rho
    return x


def lanczos_max_eig(apply_A, dinv, n, steps=20, seed=0, project=False):
    """Largest eigenvalue of D^-1 A from the Lanczos tridiagonal of Jacobi-PCG."""
    rng = np.random.default_rng(seed)
    b = rng.standard_normal(n)
    if project:
        b -= b.mean()
    # plain Jacobi-PCG, recording its alpha and beta coefficients
    r = b.copy()
    z = dinv * r
    if project:
        z -= z.mean()
    p = z.copy()
    rz = r @ z
    alphas, betas = [], []
    for _ in range(steps):
        q = apply_A(p)
        a = rz / (p @ q)
        r = r - a * q
        if project:
            r -= r.mean()
        z = dinv * r
        if project:
            z -= z.mean()
        rz_new = r @ z
        bt = rz_new / rz
        alphas.append(a)
        betas.append(bt)
        p = z + bt * p
        rz = rz_new
    m = len(alphas)
    Tm = np.zeros((m, m))
    for i in range(m):
        Tm[i, i] = 1.0 / alphas[i] + (betas[i - 1] / alphas[i - 1] if i > 0 else 0.0)
        if i + 1 < m:
            Tm[i, i + 1] = Tm[i + 1, i] = np.sqrt(betas[i]) / alphas[i]
    return float(np.linalg.eigvalsh(Tm).max())


def mass_1d(k, N, h, n_q=0):
    """Block-diagonal 1D DG mass matrix on N periodic elements of size h."""
    m = n_q or (k + 1)
    z, w = gauss_rule(m)
    L = lagrange_values(lgl_nodes(k), z)
    Me = h * (L.T * w) @ L
    return np.kron(np.eye(N), Me)


def sipg_1d(k, N, h, penalty_factor=1.0, n_q=0):
    """Textbook periodic 1D SIPG matrix:

    a(v, u) = sum_K (v', u')_K + sum_faces ( -{v'}[u] - [v]{u'} + tau [v][u] ),
    [u] = u_left - u_right, {u'} = average of the one-sided derivatives,
    tau = penalty_factor * (k+1)^2 / h.
    """
    n = k + 1
    m = n_q or n
    nodes = lgl_nodes(k)
    z, w = gauss_rule(m)
    Ld = lagrange_derivs(nodes, z) / h
    Ke = h * (Ld.T * w) @ Ld
    K = np.kron(np.eye(N), Ke)
    v0 = lagrange_values(nodes, [0.0])[0]
    v1 = lagrange_values(nodes, [1.0])[0]
    g0 = lagrange_derivs(nodes, [0.0])[0] / h
    g1 = lagrange_derivs(nodes, [1.0])[0] / h
    tau = penalty_factor * (k + 1) ** 2 / h
    for e in range(N):
        L, R = e, (e + 1) % N
        # face between element L (its right end) and R (its left end);
        # [u] = u_L(1) - u_R(0) and {u'} as coefficient rows of each side
        sides = [(L, v1, 0.5 * g1), (R, -v0, 0.5 * g0)]
        for ea, ja, ga in sides:
            for eb, jb, gb in sides:
                blk = -np.outer(ga, jb) - np.outer(ja, gb) + tau * np.outer(ja, jb)
                K[ea * n:ea * n + n, eb * n:eb * n + n] += blk
    return K


def to_tensor(v, mesh, k):
    """[N_el, n^3] element-major -> [Nz*n, Ny*n, Nx*n] global tensor (x fastest)."""
    n = k + 1
    Nx, Ny, Nz = mesh.n_el
    t = np.asarray(v).reshape(Nz, Ny, Nx, n, n, n)      # ez, ey, ex, c, b, a
    return t.transpose(0, 3, 1, 4, 2, 5).reshape(Nz * n, Ny * n, Nx * n)


def from_tensor(t, mesh, k):
    n = k + 1
    Nx, Ny, Nz = mesh.n_el
    v = np.asarray(t).reshape(Nz, n, Ny, n, Nx, n).transpose(0, 2, 4, 1, 3, 5)
    return v.reshape(mesh.N, n ** 3)


def fdm_solve(b, k, mesh, penalty_factor=1.0, scale=1.0):
    """x with A x = b (zero mode dropped) by fast diagonalisation.

    1D generalised eigenproblems K_d S_d = M_d S_d Lambda_d with
    S_d^T M_d S_d = I give A^-1 = (S_z(x)S_y(x)S_x) diag(1/(l_i+l_j+l_l)) (...)^T.
    """
    h = mesh.h
    S, lam = [], []
    for d in range(3):
        K = sipg_1d(k, mesh.n_el[d], h[d], penalty_factor)
        M = mass_1d(k, mesh.n_el[d], h[d])
        w, V = sla.eigh(K, M)
        S.append(V)
        lam.append(w)
    t = to_tensor(b, mesh, k)
    t = np.einsum('zc,yb,xa,zyx->cba', S[2], S[1], S[0], t, optimize=True)
    den = scale * (lam[2][:, None, None] + lam[1][None, :, None] + lam[0][None, None, :])
    zero = np.abs(den) < 1e-10 * np.abs(den).max()
    t = np.where(zero, 0.0, t / np.where(zero, 1.0, den))
    t = np.einsum('zc,yb,xa,cba->zyx', S[2], S[1], S[0], t, optimize=True)
    return from_tensor(t, mesh, k)
