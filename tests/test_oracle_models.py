"""Pins of the oracle's Hamiltonians against what the paper and the
mathematics fix: closed-form band energies, Hermiticity, the chiral symmetry
of the clean TI, spectral bounds, and brute-force lattice indexing."""

import json
import math
import os

import numpy as np
import pytest

from oracle import hamiltonian, lattice, models
import workloads as W

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")))


def dense(model, L, periodic, V=None):
    lat = lattice.Lattice(L, periodic, model.n_orb)
    return hamiltonian.assemble(model, lat, V).toarray(), lat


def ti_bloch_energies(L, m=2.0, t=1.0):
    """Sec. 2.2 band matrix, with the sign of the printed k-space form corrected
    so that it is Hermitian: h(k) = (m - t sum cos k_j) G1 + t sum sin k_j G_{j+1},
    E = +-sqrt((m - t sum cos)^2 + t^2 sum sin^2), each twofold (Kramers)."""
    out = []
    ks = [2 * np.pi * np.arange(n) / n for n in L]
    for kx in ks[0]:
        for ky in ks[1]:
            for kz in ks[2]:
                e = math.sqrt((m - t * (math.cos(kx) + math.cos(ky) + math.cos(kz))) ** 2
                              + t * t * (math.sin(kx) ** 2 + math.sin(ky) ** 2 + math.sin(kz) ** 2))
                out += [e, e, -e, -e]
    return np.sort(out)


def graphene_paper_dispersion(kx, ky):
    """Sec. 2.1 Eq. (graphene_e_k), a = 1."""
    return math.sqrt(max(0.0, 3 + 2 * math.cos(math.sqrt(3) * ky)
                         + 4 * math.cos(math.sqrt(3) * ky / 2) * math.cos(1.5 * kx)))


@pytest.mark.parametrize("L", [(4, 4, 4), (3, 5, 4), (6, 3, 3)])
@pytest.mark.parametrize("m", [2.0, 0.5, 3.5])
def test_ti_spectrum_matches_bloch_energies(L, m):
    H, _ = dense(models.topological_insulator(m=m), L, (1, 1, 1))
    assert np.abs(H - H.conj().T).max() == 0.0
    ev = np.linalg.eigvalsh(H)
    assert np.abs(ev - ti_bloch_energies(L, m=m)).max() < 1e-13


def test_ti_bulk_gap_and_bandwidth():
    # m = 2: the periodic spectrum touches |E| = 1 exactly at k = 0 (bulk gap, Sec. 2.2)
    H, _ = dense(models.topological_insulator(m=2.0), (4, 4, 4), (1, 1, 1))
    ev = np.linalg.eigvalsh(H)
    assert abs(np.abs(ev).min() - GOLDEN["ti_bulk_gap_m2"]["value"]) < 1e-12
    assert ev.max() <= 5 + 1e-12 and ev.min() >= -5 - 1e-12


def test_ti_disordered_spectrum_in_paper_range():
    # W = 1 disorder: ||H|| <= 5 + W/2, the [-5.5, 5.5] of Table fd_cases
    V = W.uniform_potential(4 * 4 * 4, 1.0, W.generator(0, 1))
    H, _ = dense(models.topological_insulator(), (4, 4, 4), (1, 1, 1), V)
    ev = np.linalg.eigvalsh(H)
    lo, hi = GOLDEN["ti_fd_spectrum_range"]["value"]
    assert ev.min() >= lo and ev.max() <= hi


def test_ti_kramers_degeneracy_with_disorder():
    V = W.uniform_potential(3 * 3 * 3, 2.0, W.generator(0, 1))
    H, _ = dense(models.topological_insulator(), (3, 3, 3), (1, 1, 1), V)
    ev = np.linalg.eigvalsh(H)
    assert np.abs(ev[0::2] - ev[1::2]).max() < 1e-12


def test_ti_chiral_symmetry_clean():
    """V = 0, Delta = 0: C H C = -H with C = I (x) tau_y (x) sigma_0, since every
    term is built from G1..G4, which anticommute with G5."""
    H, lat = dense(models.topological_insulator(), (3, 4, 3), (1, 1, 1))
    G5 = np.kron(np.array([[0, -1j], [1j, 0]]), np.eye(2))
    C = np.kron(np.eye(lat.n_sites), G5)
    assert np.abs(C @ H @ C + H).max() < 1e-14


def test_ti_block_structure():
    # seven 4x4 blocks per block row (Sec. 2.2), 13 nonzeros per row
    H, lat = dense(models.topological_insulator(), (4, 4, 4), (1, 1, 1))
    nb = GOLDEN["ti_subdiagonals"]
    blocks = set()
    for r in range(4):
        for c in np.nonzero(H[r])[0]:
            blocks.add(c // 4)
    assert len(blocks) == nb["blocks_per_row"]
    assert all(np.count_nonzero(H[r]) == 13 for r in range(lat.n_rows))


@pytest.mark.parametrize("L", [(6, 5), (4, 7), (3, 3)])
def test_graphene_two_site_matches_paper_dispersion(L):
    H, _ = dense(models.graphene_two_site(), L, (1, 1))
    ev = np.linalg.eigvalsh(H)
    E = []
    for p in range(L[0]):
        for q in range(L[1]):
            t1, t2 = 2 * np.pi * p / L[0], 2 * np.pi * q / L[1]
            # lattice vectors a1 = (3/2, sqrt3/2), a2 = (3/2, -sqrt3/2): k.a1 = t1, k.a2 = t2
            e = graphene_paper_dispersion((t1 + t2) / 3, (t1 - t2) / math.sqrt(3))
            E += [e, -e]
    assert np.abs(np.sort(E) - ev).max() < 1e-13
    assert ev.max() <= GOLDEN["graphene_bandwidth"]["value"] + 1e-12


@pytest.mark.parametrize("L", [(3, 4), (4, 2), (5, 3)])
def test_graphene_four_site_matches_paper_dispersion(L):
    """The four-site cell (zigzag chains along x) is the honeycomb of
    Eq. (graphene_e_k) with x and y exchanged; its Lx x Ly torus carries the
    momenta kx = 2 pi p/(sqrt3 Lx), ky = 2 pi q/(3 Ly), p < Lx, q < 2 Ly."""
    H, _ = dense(models.graphene_four_site(), L, (1, 1))
    ev = np.linalg.eigvalsh(H)
    E = []
    for p in range(L[0]):
        for q in range(2 * L[1]):
            e = graphene_paper_dispersion(2 * np.pi * q / (3 * L[1]), 2 * np.pi * p / (math.sqrt(3) * L[0]))
            E += [e, -e]
    assert np.abs(np.sort(E) - ev).max() < 1e-13


def test_weyl_matches_band_matrix():
    """Sec. 2.3 Eq. (band_h_wsm), V = 0: E = +-|d(k)| with
    d = (cos kx - cos k0 + cos ky + cos kz - 2, sin ky, sin kz)."""
    L = (5, 4, 3)
    H, _ = dense(models.weyl_semimetal(), L, (1, 1, 1))
    ev = np.linalg.eigvalsh(H)
    k0 = GOLDEN["weyl_nodes"]["k0"]
    E = []
    for kx in 2 * np.pi * np.arange(L[0]) / L[0]:
        for ky in 2 * np.pi * np.arange(L[1]) / L[1]:
            for kz in 2 * np.pi * np.arange(L[2]) / L[2]:
                d = (math.cos(kx) - math.cos(k0) + math.cos(ky) + math.cos(kz) - 2, math.sin(ky), math.sin(kz))
                e = math.sqrt(sum(v * v for v in d))
                E += [e, -e]
    assert np.abs(np.sort(E) - ev).max() < 1e-13


def test_weyl_nodes_are_gapless():
    # at the node momenta (+-k0, 0, 0) the band matrix vanishes
    k0 = GOLDEN["weyl_nodes"]["k0"]
    for kx, _, _ in GOLDEN["weyl_nodes"]["nodes"]:
        d = math.cos(kx) - math.cos(k0)
        assert abs(d) < 1e-15


@pytest.mark.parametrize("model,L,periodic", [
    (models.topological_insulator(), (3, 4, 5), (1, 1, 1)),
    (models.topological_insulator(), (3, 4, 5), (0, 1, 0)),
    (models.graphene_two_site(), (5, 4), (0, 1)),
    (models.graphene_four_site(), (3, 4), (1, 0)),
    (models.weyl_semimetal(), (4, 3, 3), (1, 1, 0)),
])
def test_hermitian_and_open_boundaries(model, L, periodic):
    H, lat = dense(model, L, periodic, W.uniform_potential(int(np.prod(L)) * (model.n_orb if model.pot == "orbital" else 1), 1.0, W.generator(9, 1)))
    assert np.abs(H - H.conj().T).max() < 1e-15
    # brute-force neighbour check: every nonzero couples sites at lattice distance <= 1
    # per dimension, respecting open boundaries (no wrap where not periodic)
    rows, cols = np.nonzero(H)
    xs, ys, zs = lat.coords(rows // model.n_orb)
    xc, yc, zc = lat.coords(cols // model.n_orb)
    for d, (a, b) in enumerate([(xs, xc), (ys, yc), (zs, zc)]):
        diff = np.abs(a - b)
        if periodic[d] if d < len(periodic) else True:
            diff = np.minimum(diff, lat.L[d] - diff)
        assert diff.max() <= 1


def test_rows_of_sites_match_full_matrix():
    model = models.topological_insulator()
    lat = lattice.Lattice((4, 3, 5), (1, 0, 1), 4)
    V = W.uniform_potential(lat.n_sites, 1.5, W.generator(3, 1))
    H = hamiltonian.assemble(model, lat, V).toarray()
    sites = np.array([0, 7, 11, 59])
    R = hamiltonian.rows_of_sites(model, lat, V, sites).toarray()
    rows = (sites[:, None] * 4 + np.arange(4)[None, :]).reshape(-1)
    assert np.array_equal(R, H[rows])


def _bloch_vector(lat, k, u):
    n = np.arange(lat.n_sites)
    x, y, z = lat.coords(n)
    ph = np.exp(1j * (k[0] * x + k[1] * y + k[2] * z))
    return (ph[:, None] * u[None, :]).reshape(-1)


@pytest.mark.parametrize("k", [(1, 2, 0), (3, 1, 2), (0, 0, 1)])
def test_ti_bloch_eigenvectors_fix_hopping_direction(k):
    """psi = exp(i k.n) u(k), u an eigenvector of h(k) = (m - sum cos k_j) G1 +
    sum sin k_j G_{j+1}, is an eigenvector of H.  Reversing the hopping
    direction would replace h(k) by h(-k) and fail this."""
    L = (4, 5, 3)
    lat = lattice.Lattice(L, (1, 1, 1), 4)
    H = hamiltonian.assemble(models.topological_insulator(m=2.0), lat, None)
    kv = [2 * np.pi * k[d] / L[d] for d in range(3)]
    G1, G2, G3, G4, _, _ = models.ti_gammas()
    h = (2.0 - sum(np.cos(kv))) * G1 + np.sin(kv[0]) * G2 + np.sin(kv[1]) * G3 + np.sin(kv[2]) * G4
    E, U = np.linalg.eigh(h)
    for i in range(4):
        psi = _bloch_vector(lat, kv, U[:, i])
        assert np.abs(H @ psi - E[i] * psi).max() < 1e-13


@pytest.mark.parametrize("k", [(1, 1, 0), (2, 3, 1)])
def test_weyl_bloch_eigenvectors(k):
    L = (5, 4, 3)
    lat = lattice.Lattice(L, (1, 1, 1), 2)
    H = hamiltonian.assemble(models.weyl_semimetal(), lat, None)
    kv = [2 * np.pi * k[d] / L[d] for d in range(3)]
    k0 = np.pi / 2
    h = (models.SX * (np.cos(kv[0]) - np.cos(k0) + np.cos(kv[1]) + np.cos(kv[2]) - 2)
         + models.SY * np.sin(kv[1]) + models.SZ * np.sin(kv[2]))
    E, U = np.linalg.eigh(h)
    for i in range(2):
        psi = _bloch_vector(lat, kv, U[:, i])
        assert np.abs(H @ psi - E[i] * psi).max() < 1e-13
