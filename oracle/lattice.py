"""Cuboid lattice indexing (oracle; test infrastructure).

Sec. 3.4 (Geometry): cuboid domains of arbitrary size, periodic boundary
conditions selectable per spatial dimension; vector entries addressed by
(x, y, z, basis place) and a vector-block index.

Conventions (x fastest):
    site  s = x + Lx*(y + Ly*z)
    row   r = s*n_orb + o
    elem  e = r*nb + c
A neighbour coordinate x+dx is wrapped modulo Lx when that dimension is
periodic and dropped when it leaves [0, Lx) otherwise.
"""

from __future__ import annotations

import numpy as np


class Lattice:
    def __init__(self, L, periodic, n_orb: int):
        L = list(L) + [1] * (3 - len(L))
        periodic = list(periodic) + [True] * (3 - len(periodic))
        self.L = tuple(int(v) for v in L)
        self.periodic = tuple(bool(p) for p in periodic)
        self.n_orb = int(n_orb)
        if min(self.L) < 1:
            raise ValueError("extents must be >= 1")

    @property
    def n_sites(self) -> int:
        return self.L[0] * self.L[1] * self.L[2]

    @property
    def n_rows(self) -> int:
        return self.n_sites * self.n_orb

    def site(self, x, y, z):
        return x + self.L[0] * (y + self.L[1] * z)

    def coords(self, s):
        s = np.asarray(s, dtype=np.int64)
        x = s % self.L[0]
        y = (s // self.L[0]) % self.L[1]
        z = s // (self.L[0] * self.L[1])
        return x, y, z

    def shift(self, s, d):
        """Site index of s + d for every entry of s, and a validity mask
        (False where an open boundary drops the neighbour)."""
        coords = self.coords(s)
        valid = np.ones(np.shape(s), dtype=bool)
        out = []
        for dim in range(3):
            c = coords[dim] + int(d[dim])
            if self.periodic[dim]:
                c = np.mod(c, self.L[dim])
            else:
                valid &= (c >= 0) & (c < self.L[dim])
                c = np.clip(c, 0, self.L[dim] - 1)
            out.append(c)
        return self.site(out[0], out[1], out[2]), valid
