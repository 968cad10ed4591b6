"""Model Hamiltonians of Sec. 2 as hopping terms (oracle; test infrastructure).

A model is described exactly as the paper writes its Hamiltonians:

    H = sum_n sum_terms ( Psi^dag_{n+e} A Psi_n + h.c. ) + sum_n Psi^dag_n (E0 + V_n) Psi_n

``Model.hops`` is the list of (e, A): the displacement e in lattice units and
the n_orb x n_orb complex matrix A that carries an electron from cell n to
cell n+e.  ``Model.onsite`` is E0.  ``Model.pot`` says how the real on-site
field enters: "site" (V_n times the identity, as V_n Gamma^0 for the TI and
the Weyl model) or "orbital" (diag(v_{n,0..n_orb-1}), as V_n of the graphene
four-site cell).

Readings of the paper (also listed in the design notes):
* TI Gamma matrices: G1 = tau_z (x) sigma_0, G_{j+1} = tau_x (x) sigma_j,
  G5 = tau_y (x) sigma_0, G15 = [G1, G5]/(2i); orbital index o = 2*tau + sigma.
  Any irreducible representation of the Clifford algebra gives the same
  spectrum; the paper's printed choice differs by a unitary.
* TI hopping: the term Psi^dag_{n+e_j} (-(t/2))(G1 - i G_{j+1}) Psi_n of the
  TI equation, with the hopping amplitude t kept explicit (t = 1 in the paper).
* Graphene two-site cell: A(i,j) bonds to B(i,j), B(i-1,j), B(i,j-1) with
  amplitude -t (honeycomb in brick-wall index form, Sec. 2.1 dispersion).
* Graphene four-site cell: the matrices T_x, T_y, T_n of the graphene model
  equation, used as printed.
* Weyl: the two-band model equation with k0 = pi/2.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

S0 = np.eye(2, dtype=np.complex128)
SX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
SY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
SZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)


@dataclass
class Model:
    name: str
    dim: int
    n_orb: int
    hops: list = field(default_factory=list)   # [(e (3-tuple), A (n_orb x n_orb))]
    onsite: np.ndarray = None
    pot: str = "site"                          # "site" | "orbital" | "none"


def ti_gammas():
    """G1..G5 and G15 in the tau (x) sigma convention."""
    G1 = np.kron(SZ, S0)
    G2 = np.kron(SX, SX)
    G3 = np.kron(SX, SY)
    G4 = np.kron(SX, SZ)
    G5 = np.kron(SY, S0)
    G15 = (G1 @ G5 - G5 @ G1) / 2j
    return G1, G2, G3, G4, G5, G15


def topological_insulator(t: float = 1.0, m: float = 2.0, delta1: float = 0.0,
                          delta2: float = 0.0) -> Model:
    """3D TI, Sec. 2.2 Eq. (TB_H_topi): on-site m G1 + D1 G5 + D2 G15 + V_n G0,
    hopping -(t/2)(G1 - i G_{j+1}) from n to n+e_j, j = x, y, z."""
    G1, G2, G3, G4, G5, G15 = ti_gammas()
    Gj = [G2, G3, G4]
    hops = []
    for j in range(3):
        e = [0, 0, 0]
        e[j] = 1
        hops.append((tuple(e), -(t / 2.0) * (G1 - 1j * Gj[j])))
    onsite = m * G1 + delta1 * G5 + delta2 * G15
    return Model("ti", 3, 4, hops, onsite.astype(np.complex128), "site")


def graphene_two_site(t: float = 1.0) -> Model:
    """Honeycomb with a two-atom (A=0, B=1) cell on an (i, j) index grid.
    H[(n,A),(n,B)] = H[(n,A),(n-e_i,B)] = H[(n,A),(n-e_j,B)] = -t, plus h.c.
    Written as hops from n to n+e: the bond A(n+e_i)-B(n) carries -t from B(n)
    into A(n+e_i), i.e. A_e[A, B] = -t for e = e_i and e = e_j."""
    A = np.zeros((2, 2), dtype=np.complex128)
    A[0, 1] = -t
    onsite = np.array([[0, -t], [-t, 0]], dtype=np.complex128)
    hops = [((1, 0, 0), A.copy()), ((0, 1, 0), A.copy())]
    return Model("graphene2", 2, 2, hops, onsite, "site")


def graphene_four_site(t: float = 1.0) -> Model:
    """Graphene four-site rectangular cell, Sec. 2.1 Eq. (graphene_model):
    hops T_x (n -> n+e_x), T_y (n -> n+e_y), intra-cell T_n, V_n = diag(v_{n,j})."""
    Tx = np.zeros((4, 4), dtype=np.complex128)
    Tx[1, 0] = -t
    Tx[2, 3] = -t
    Ty = np.zeros((4, 4), dtype=np.complex128)
    Ty[0, 3] = -t
    Tn = np.zeros((4, 4), dtype=np.complex128)
    for a in range(3):
        Tn[a, a + 1] = -t
        Tn[a + 1, a] = -t
    hops = [((1, 0, 0), Tx), ((0, 1, 0), Ty)]
    return Model("graphene4", 2, 4, hops, Tn, "orbital")


def weyl_semimetal(k0: float = math.pi / 2.0) -> Model:
    """Weyl semimetal, Sec. 2.3 Eq. (TB_H_wsm): hop sigma_x/2 along x,
    (sigma_x + i sigma_j)/2 along j = y, z; on-site V_n - sigma_x (2 + cos k0)."""
    hops = [((1, 0, 0), SX / 2.0),
            ((0, 1, 0), (SX + 1j * SY) / 2.0),
            ((0, 0, 1), (SX + 1j * SZ) / 2.0)]
    onsite = -SX * (2.0 + math.cos(k0))
    return Model("weyl", 3, 2, hops, onsite.astype(np.complex128), "site")
