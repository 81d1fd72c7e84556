"""Periodic Cartesian hexahedral mesh for the oracle (test infrastructure only).

Sec. 4: the Taylor-Green vortex domain is a box with periodic boundaries in
all directions, discretised by a uniform Cartesian grid of hexahedra mapped
affinely from [0,1]^3 (Sec. 3.2, k_m = 1).

Numbering: element e = ex + Nx*(ey + Ny*ez); local node i = a + n*(b + n*c)
with a the x index (fastest).  Scalar fields are stored [N_el, n^3], vector
fields [3, N_el, n^3].
"""
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Mesh:
    n_el: tuple   # elements per direction (Nx, Ny, Nz)
    length: tuple  # box edge per direction

    @property
    def N(self):
        return int(np.prod(self.n_el))

    @property
    def h(self):
        return np.asarray(self.length, dtype=np.float64) / np.asarray(self.n_el, dtype=np.float64)

    def coords(self):
        """(ex, ey, ez) integer coordinates of every element, shape [N_el, 3]."""
        Nx, Ny, Nz = self.n_el
        e = np.arange(self.N)
        return np.stack([e % Nx, (e // Nx) % Ny, e // (Nx * Ny)], axis=1)

    def index(self, ijk):
        Nx, Ny, Nz = self.n_el
        ijk = np.asarray(ijk)
        return ijk[..., 0] + Nx * (ijk[..., 1] + Ny * ijk[..., 2])

    def neighbor(self, d, s, elems=None):
        """Neighbour across face (d, s) with periodic wrap.

        s = 0 is the face at reference coordinate xi_d = 0 (outward normal -e_d),
        s = 1 the face at xi_d = 1 (outward normal +e_d).
        """
        c = self.coords() if elems is None else self.coords()[np.asarray(elems)]
        c = c.copy()
        c[:, d] = (c[:, d] + (1 if s == 1 else -1)) % self.n_el[d]
        return self.index(c)


def cube(N, length=2.0 * np.pi):
    return Mesh((N, N, N), (length, length, length))
