"""Pins of the host-parallel oracle (oracle/omp/cheb_omp.cpp, C++ with
OpenMP): the fused Chebyshev step against the dense definition
alpha (H x - beta x) + gamma z with numpy's dense product, its dot products
against their sums, and KPM moments against the spectral formula
mu_n = sum_i |<v_i, r>|^2 T_n(lambda~_i) / D from dense eigendecomposition
and against the Python oracle's doubling.  Tolerances: 1e-13 relative
(summation order), moments 1e-12."""

import numpy as np
import pytest

from oracle import hamiltonian, kpm, lattice, models, omp_sweep
import workloads as W


@pytest.fixture(scope="module", autouse=True)
def built():
    import os
    if not os.path.exists(omp_sweep.LIB_PATH):
        pytest.skip("liboracle_omp.so not built")


def case(name, L, periodic, Wd, seed):
    model = {"ti": models.topological_insulator(1.0, 2.0), "graphene2": models.graphene_two_site(1.0),
             "weyl": models.weyl_semimetal()}[name]
    olat = lattice.Lattice(L, periodic, model.n_orb)
    n = olat.n_sites if model.pot == "site" else olat.n_rows
    V = W.uniform_potential(n, Wd, W.generator(seed, W.STREAM_POTENTIAL))
    return hamiltonian.assemble(model, olat, V), olat


@pytest.mark.parametrize("name,L,periodic", [("ti", (5, 4, 3), (1, 1, 1)), ("ti", (6, 3, 4), (0, 1, 0)),
                                             ("graphene2", (9, 7), (0, 1)), ("weyl", (4, 4, 3), (1, 1, 0))])
@pytest.mark.parametrize("nb", [1, 3, 8])
def test_sweep_matches_dense_definition(name, L, periodic, nb):
    H, olat = case(name, L, periodic, 1.5, nb)
    Hd = H.toarray()
    g = W.generator(3, 7, nb)
    x = W.gaussian_block(olat.n_rows, nb, g)
    z = W.gaussian_block(olat.n_rows, nb, g)
    A = omp_sweep.Csr(H)
    for alpha, beta, gamma in ((1.0, 0.0, 0.0), (2.0 / 7.0, 0.3, -1.0), (0.4, -0.2, 0.7)):
        y, d = omp_sweep.sweep(A, x, alpha, beta, gamma, z if gamma else None)
        ref = alpha * (Hd @ x - beta * x) + gamma * z
        assert np.abs(y - ref).max() < 1e-13 * np.abs(ref).max()
        xx = np.sum(np.abs(x) ** 2, axis=0)
        xy = np.sum(np.conj(x) * ref, axis=0)
        yy = np.sum(np.abs(ref) ** 2, axis=0)
        assert np.abs(d[:, 0] - xx).max() < 1e-13 * xx.max()
        assert np.abs(d[:, 1] + 1j * d[:, 2] - xy).max() < 1e-13 * max(np.abs(xy).max(), xx.max())
        assert np.abs(d[:, 3] - yy).max() < 1e-13 * yy.max()


def test_sweep_without_gamma_never_reads_z():
    H, olat = case("ti", (4, 3, 3), (1, 1, 1), 1.0, 1)
    x = W.gaussian_block(olat.n_rows, 2, W.generator(1, 2))
    y, _ = omp_sweep.sweep(omp_sweep.Csr(H), x, 0.5, 0.1, 0.0, None)
    assert np.abs(y - 0.5 * (H @ x - 0.1 * x)).max() < 1e-13 * np.abs(y).max()


def test_kpm_moments_match_spectral_formula_and_doubling():
    H, olat = case("ti", (4, 3, 3), (1, 0, 1), 1.0, 2)
    r = W.random_phase_block(olat.n_rows, 3, W.generator(2, 2))
    a, b, M = 7.0, 0.2, 40
    mu = omp_sweep.kpm_moments(omp_sweep.Csr(H), r, M, a, b)
    lam, U = np.linalg.eigh(H.toarray())
    wts = np.abs(U.conj().T @ r) ** 2                 # [states][columns]
    T = np.cos(np.arange(M)[:, None] * np.arccos((lam - b) / a)[None, :])
    ref = (T @ wts).T / olat.n_rows
    assert np.abs(mu - ref).max() < 1e-12
    assert np.abs(mu - kpm.moments_doubling(H, r, M, a, b)).max() < 1e-13
    assert np.abs(mu[:, 0] - 1.0).max() < 1e-14


def test_thread_count_changes_only_rounding():
    H, olat = case("ti", (8, 8, 4), (1, 1, 1), 2.0, 3)
    x = W.random_phase_block(olat.n_rows, 4, W.generator(3, 2))
    A = omp_sweep.Csr(H)
    n0 = omp_sweep.threads()
    try:
        omp_sweep.set_threads(1)
        y1, d1 = omp_sweep.sweep(A, x, 0.3, 0.0, 0.0)
        omp_sweep.set_threads(max(2, n0))
        y2, d2 = omp_sweep.sweep(A, x, 0.3, 0.0, 0.0)
    finally:
        omp_sweep.set_threads(n0)
    assert np.array_equal(y1, y2)                     # rows are independent
    assert np.abs(d1 - d2).max() < 1e-12 * np.abs(d1).max()
