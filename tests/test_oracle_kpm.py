"""Pins of the oracle's SpMMV, dot products and KPM moments."""

import numpy as np
import pytest

from oracle import hamiltonian, kpm, lattice, models, spmmv
import workloads as W


def ti(L=(3, 3, 3), periodic=(1, 1, 1), Wd=1.0, seed=0):
    lat = lattice.Lattice(L, periodic, 4)
    V = W.uniform_potential(lat.n_sites, Wd, W.generator(seed, 1))
    return hamiltonian.assemble(models.topological_insulator(), lat, V), lat, V


def test_spmmv_definition_against_dense():
    H, lat, _ = ti((3, 4, 2), (1, 0, 1))
    g = W.generator(0, 2)
    x = W.gaussian_block(lat.n_rows, 3, g)
    z = W.gaussian_block(lat.n_rows, 3, g)
    alpha, beta, gamma = np.array([0.5, 2.0, -1.0]), np.array([0.0, 0.3, -1.2]), np.array([0.0, -1.0, 0.25])
    y = spmmv.spmmv(H, x, alpha, beta, gamma, z)
    Hd = H.toarray()
    for c in range(3):
        ref = alpha[c] * (Hd @ x[:, c] - beta[c] * x[:, c]) + gamma[c] * z[:, c]
        assert np.abs(y[:, c] - ref).max() < 1e-13


def test_spmmv_gamma_zero_never_reads_z():
    H, lat, _ = ti()
    x = W.gaussian_block(lat.n_rows, 2, W.generator(0, 2))
    z = np.full_like(x, np.nan)
    y = spmmv.spmmv(H, x, 1.0, 0.0, 0.0, z)
    assert np.isfinite(y).all()


def test_delta_vectors_pick_matrix_columns_exactly():
    """H e_j is column j of H, bit for bit (one product per entry)."""
    H, lat, _ = ti((3, 3, 4), (1, 1, 1))
    cols = [0, 5, 17, 100, lat.n_rows - 1]
    X = W.basis_block(lat.n_rows, cols)
    Y = spmmv.spmmv(H, X, 1.0, 0.0, 0.0)
    Hd = H.toarray()
    for c, j in enumerate(cols):
        assert np.array_equal(Y[:, c], Hd[:, j])


def test_block_dots():
    g = W.generator(0, 2)
    x = W.gaussian_block(50, 2, g)
    y = W.gaussian_block(50, 2, g)
    xx, xy, yy = spmmv.block_dots(x, y)
    for c in range(2):
        assert abs(xx[c] - np.vdot(x[:, c], x[:, c]).real) < 1e-12
        assert abs(xy[c] - np.vdot(x[:, c], y[:, c])) < 1e-12
        assert abs(yy[c] - np.vdot(y[:, c], y[:, c]).real) < 1e-12


def test_mu0_is_one_for_random_phases():
    H, lat, _ = ti()
    r = W.random_phase_block(lat.n_rows, 4, W.generator(0, 2))
    mu = kpm.moments_doubling(H, r, 16, 7.0, 0.0)
    assert np.abs(mu[:, 0] - 1.0).max() < 1e-15
    assert np.abs(mu).max() <= 1.0 + 1e-12


@pytest.mark.parametrize("M", [2, 4, 32, 64])
def test_doubling_equals_direct(M):
    H, lat, _ = ti((3, 2, 4), (1, 0, 1), Wd=2.0)
    r = W.random_phase_block(lat.n_rows, 3, W.generator(0, 2))
    a = kpm.moments_doubling(H, r, M, 7.0, 0.1)
    b = kpm.moments_direct(H, r, M, 7.0, 0.1)
    assert np.abs(a - b).max() < 1e-13


def test_moments_from_dense_eigendecomposition():
    """mu_n = sum_i |<v_i, r>|^2 T_n(lambda_i~) / D with T_n = cos(n arccos)."""
    H, lat, _ = ti((2, 3, 3), (1, 1, 0), Wd=1.0)
    r = W.random_phase_block(lat.n_rows, 2, W.generator(0, 2))
    a, b = 7.0, 0.2
    mu = kpm.moments_doubling(H, r, 40, a, b)
    lam, U = np.linalg.eigh(H.toarray())
    w = np.abs(U.conj().T @ r) ** 2
    T = np.cos(np.arange(40)[:, None] * np.arccos((lam - b) / a)[None, :])
    ref = (T @ w).T / lat.n_rows
    assert np.abs(mu - ref).max() < 1e-13


def test_clean_trace_from_bloch_energies():
    """Exact trace (all basis vectors) of the clean periodic TI equals
    (1/D) sum_k T_n(E_k/a) over the closed-form band energies."""
    from test_oracle_models import ti_bloch_energies
    L = (3, 3, 2)
    lat = lattice.Lattice(L, (1, 1, 1), 4)
    H = hamiltonian.assemble(models.topological_insulator(), lat, None)
    R = np.eye(lat.n_rows, dtype=np.complex128)
    mu = kpm.moments_doubling(H, R, 24, 7.0, 0.0).sum(axis=0)
    E = ti_bloch_energies(L)
    ref = np.cos(np.arange(24)[:, None] * np.arccos(E / 7.0)[None, :]).sum(axis=1) / lat.n_rows
    assert np.abs(mu - ref).max() < 1e-13
    # chiral symmetry: odd trace moments vanish
    assert np.abs(mu[1::2]).max() < 1e-14


def test_stochastic_estimate_near_trace():
    """Random-phase estimate within a few standard deviations of the exact trace."""
    L = (6, 6, 6)
    lat = lattice.Lattice(L, (1, 1, 1), 4)
    H = hamiltonian.assemble(models.topological_insulator(), lat, None)
    r = W.random_phase_block(lat.n_rows, 1, W.generator(0, 2))
    mu = kpm.moments_doubling(H, r, 16, 7.0, 0.0)[0]
    from test_oracle_models import ti_bloch_energies
    E = ti_bloch_energies(L)
    ref = np.cos(np.arange(16)[:, None] * np.arccos(E / 7.0)[None, :]).sum(axis=1) / lat.n_rows
    sigma = 1.0 / np.sqrt(lat.n_rows)
    assert np.abs(mu - ref).max() < 5 * sigma


def test_jackson_and_dos_normalisation():
    g = kpm.jackson(64)
    assert abs(g[0] - 1.0) < 1e-14 and np.all(np.diff(g) < 0) and g[-1] > 0
    H, lat, _ = ti((4, 4, 4), (1, 1, 1), Wd=1.0)
    r = W.random_phase_block(lat.n_rows, 2, W.generator(0, 2))
    mu = kpm.moments_doubling(H, r, 64, 7.0, 0.0).mean(axis=0)
    # integrate rho(E) dE with x = cos(theta) (Chebyshev-Gauss nodes) -> g0 mu0 = 1
    n = 4000
    th = (np.arange(n) + 0.5) * np.pi / n
    E = 7.0 * np.cos(th)
    rho = kpm.dos(mu, E, 7.0, 0.0)
    integral = (rho * 7.0 * np.sin(th)).sum() * np.pi / n
    assert abs(integral - 1.0) < 1e-12
    assert (rho > -1e-12).all()


@pytest.mark.parametrize("M", [2, 16, 64, 257, 1024])
def test_jackson_factors_are_the_normalised_autocorrelation(M):
    """Jackson's construction (Weisse et al. 2006, the KPM reference of the
    paper, Sec. 2.2): g_n is the autocorrelation at lag n of
    a_k = sin(pi (k + 1)/(M + 1)), k = 0..M-1, divided by its value at lag 0.
    Built here by brute-force sums over the sequence, independent of the
    closed form; it fixes every g_n (g_1 = cos(pi/(M + 1)))."""
    g = kpm.jackson(M)
    a = np.sin(np.pi * (np.arange(M) + 1) / (M + 1))
    ac = np.array([sum(a[k] * a[k + n] for k in range(M - n)) for n in range(M)]) / np.dot(a, a)
    assert np.abs(g - ac).max() < 1e-14
    if M > 1:
        assert abs(g[1] - np.cos(np.pi / (M + 1))) < 1e-15


@pytest.mark.parametrize("M,tol", [(64, 2e-3), (256, 1.2e-4), (1024, 8e-6)])
def test_dos_reconstructs_uniform_density(M, tol):
    """A density uniform on [b - a, b + a] (value 1/(2a)) has the Chebyshev
    moments mu_n = (1/2) int_{-1}^{1} T_n(x) dx: mu_0 = 1,
    mu_{2k} = -1/(4k^2 - 1), odd moments 0.  The Jackson-damped series must
    return 1/(2a) away from the band edges, with an error that falls as 1/M^2
    (the kernel's resolution pi/M, squared for a smooth density)."""
    mu = np.zeros(M)
    mu[0] = 1.0
    k = np.arange(1, M // 2)
    mu[2 * k] = -1.0 / (4.0 * k * k - 1.0)
    a, b = 2.5, 0.3
    E = b + a * np.linspace(-0.9, 0.9, 181)
    rho = kpm.dos(mu, E, a, b)
    assert np.abs(rho * 2 * a - 1.0).max() < tol


@pytest.mark.parametrize("x0", [0.0, 0.37, -0.81])
def test_dos_of_a_delta_peak_has_the_kernels_moments(x0):
    """A single level at E0 = b + a x0 has moments mu_n = T_n(x0).  Integrals
    of the reconstructed density against 1, x and x^2 (Gauss-Chebyshev
    quadrature in E) follow from Chebyshev orthogonality alone:
    int rho = g_0, <x> = g_1 x0, <x^2> = (g_0 + g_2 T_2(x0))/2.  A dropped
    factor 2 on the n >= 1 terms, a wrong T_n argument or a wrong a, b
    mapping breaks one of them; the maximum sits at E0 within the kernel's
    resolution."""
    M, a, b = 128, 3.0, -0.4
    mu = np.cos(np.arange(M) * np.arccos(x0))
    g = kpm.jackson(M)
    n = 20000
    th = (np.arange(n) + 0.5) * np.pi / n
    x = np.cos(th)
    rho = kpm.dos(mu, b + a * x, a, b)
    w = a * np.sin(th) * np.pi / n
    assert abs((rho * w).sum() - 1.0) < 1e-13
    assert abs((rho * x * w).sum() - g[1] * x0) < 1e-13
    assert abs((rho * x * x * w).sum() - 0.5 * (1.0 + g[2] * (2 * x0 * x0 - 1.0))) < 1e-13
    assert abs(x[np.argmax(rho)] - x0) < np.pi / M
