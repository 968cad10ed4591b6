"""Pins of the oracle's trLanczosFD: the filter is the Jackson-damped
Chebyshev expansion of a delta peak (equal to the KPM DOS reconstruction of
the moments T_k(x_c), up to the weight and normalisation), and the solver
finds exactly the eigenvalues of a disordered TI inside a window (dense
eigendecomposition), with orthonormal Ritz vectors and small residuals."""

import numpy as np
import pytest

from oracle import hamiltonian, kpm, lattice, models, trlanczos
import workloads as W


def test_filter_is_a_damped_delta_peak():
    lam_l, lam_r, a, b, K = 0.9, 1.3, 7.0, 0.1, 150
    coef, tau = trlanczos.delta_filter(lam_l, lam_r, a, b, K)
    xc = ((lam_l + lam_r) / 2 - b) / a
    E = np.linspace(-6.8, 6.9, 301)
    x = (E - b) / a
    p = np.polynomial.chebyshev.chebval(x, coef)
    mu = np.cos(np.arange(K + 1) * np.arccos(xc))         # moments of delta(x - xc)
    rho = kpm.dos(mu, E, a, b)                              # Jackson-damped reconstruction
    ref = rho * np.pi * a * np.sqrt(1 - x * x)
    ref = ref / (kpm.dos(mu, np.array([(lam_l + lam_r) / 2]), a, b)[0] * np.pi * a * np.sqrt(1 - xc * xc))
    assert np.abs(p - ref).max() < 1e-12
    assert abs(np.polynomial.chebyshev.chebval(xc, coef) - 1.0) < 1e-14
    assert 0 < tau < 1


@pytest.mark.parametrize("centre,half", [(1.2, 0.06), (-1.5, 0.1)])
def test_finds_the_window_eigenvalues(centre, half):
    L = (6, 6, 6)
    lat = lattice.Lattice(L, (1, 1, 1), 4)
    V = W.uniform_potential(lat.n_sites, 2.0, W.generator(9, W.STREAM_POTENTIAL))
    H = hamiltonian.assemble(models.topological_insulator(1.0, 2.0), lat, V)
    ev = np.linalg.eigvalsh(H.toarray())
    inside = ev[np.abs(ev - centre) < half]
    V0 = W.gaussian_block(lat.n_rows, 2, W.generator(9, W.STREAM_VECTORS))
    m = 2 * inside.size + 12
    th, U, res, it = trlanczos.trlanczos_fd(H, V0, 7.0, 0.0, centre - half, centre + half, 160, m=m, tol=1e-9)
    assert th.size == inside.size
    assert np.abs(th - inside).max() < 1e-10 * 7.0
    assert res.max() <= 1e-9
    assert np.abs(U.conj().T @ U - np.eye(th.size)).max() < 1e-10
