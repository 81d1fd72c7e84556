"""Seeded synthetic inputs shared by the checker and the GPU path.

This module holds none of the method's arithmetic: it draws random numbers
and evaluates the closed-form Taylor-Green initial velocity (Sec. 4) at
caller-supplied points.  Reference node positions on [0, 1] are passed in by
the caller (each side computes its own).

Layouts: scalar [N_el, n^3], vector [3, N_el, n^3]; element
e = ex + Nx*(ey + Ny*ez), local node i = a + n*(b + n*c), x fastest.
The box is [-length/2, length/2] per direction ([-pi L, pi L]^3 with L = 1
for the Taylor-Green vortex).
"""
import numpy as np

FIELD_SEED_BASE = 100      # seed of configuration j is FIELD_SEED_BASE + j
COTANGENT_OFFSET = 1000    # cotangents and directions use seed + 1000


def rng(seed):
    return np.random.default_rng(seed)


def uniform(shape, seed, lo=-1.0, hi=1.0):
    """U[lo, hi] samples in float64."""
    return rng(seed).uniform(lo, hi, size=shape)


def normal(shape, seed, std=1.0):
    return rng(seed).normal(0.0, std, size=shape)


def node_positions(ref_nodes, n_el, length):
    """Physical coordinates (x, y, z), each [N_el, n^3], of all nodes.

    ref_nodes: the n nodes on [0, 1] of the 1D basis (supplied by the caller).
    """
    ref = np.asarray(ref_nodes, dtype=np.float64)
    n = len(ref)
    Nx, Ny, Nz = n_el
    h = [length[d] / n_el[d] for d in range(3)]
    e = np.arange(Nx * Ny * Nz)
    ex, ey, ez = e % Nx, (e // Nx) % Ny, e // (Nx * Ny)
    i = np.arange(n ** 3)
    a, b, c = i % n, (i // n) % n, i // (n * n)
    x = -0.5 * length[0] + (ex[:, None] + ref[a][None, :]) * h[0]
    y = -0.5 * length[1] + (ey[:, None] + ref[b][None, :]) * h[1]
    z = -0.5 * length[2] + (ez[:, None] + ref[c][None, :]) * h[2]
    return x, y, z


def taylor_green(x, y, z, U0=1.0, L=1.0):
    """Taylor-Green initial velocity (Sec. 4): [3, ...] array."""
    return np.stack([
        U0 * np.sin(x / L) * np.cos(y / L) * np.cos(z / L),
        -U0 * np.cos(x / L) * np.sin(y / L) * np.cos(z / L),
        np.zeros_like(x),
    ])


def tgv_plus_noise(ref_nodes, n_el, length, seed, noise_std=0.01):
    """Taylor-Green velocity at the nodes plus N(0, noise_std^2) on all 3 components."""
    x, y, z = node_positions(ref_nodes, n_el, length)
    u = taylor_green(x, y, z)
    return u + normal(u.shape, seed, noise_std)
