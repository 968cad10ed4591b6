"""Pins of the oracle's filter diagonalisation and of its adjoints."""

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import adjoint, chebfd, chebtp, hamiltonian, kpm, lattice, models
import workloads as W


def ti(L, periodic=(1, 1, 1), Wd=1.0, seed=0):
    lat = lattice.Lattice(L, periodic, 4)
    V = W.uniform_potential(lat.n_sites, Wd, W.generator(seed, 1))
    return hamiltonian.assemble(models.topological_insulator(), lat, V), lat, V


# --------------------------------------------------------------- ChebFD

def test_window_series_converges_to_indicator():
    c = chebfd.window_coefficients(-0.2, 0.1, 4000)
    x = np.array([-0.9, -0.5, -0.1, 0.0, 0.05, 0.5, 0.95])
    p = chebfd.filter_polynomial(x, c)
    inside = (x > -0.2) & (x < 0.1)
    assert np.abs(p - inside).max() < 0.01


def test_filter_block_equals_polynomial_at_eigenvalues():
    H, lat, _ = ti((3, 3, 3), Wd=2.0)
    coef = chebfd.filter_coefficients(-0.8, 0.8, 7.0, 0.0, 60)
    lam, U = np.linalg.eigh(H.toarray())
    X = W.random_phase_block(lat.n_rows, 3, W.generator(2, 2))
    Y = chebtp.cheb_series(H, X, 7.0, 0.0, coef)
    p = chebfd.filter_polynomial((lam - 0.0) / 7.0, coef)
    ref = U @ (p[:, None] * (U.conj().T @ X))
    assert np.abs(Y - ref).max() < 1e-12


def test_cholesky_qr_orthonormal():
    X = W.gaussian_block(300, 12, W.generator(2, 2))
    Q = chebfd.cholesky_qr(chebfd.cholesky_qr(X))
    assert np.abs(Q.conj().T @ Q - np.eye(12)).max() < 1e-14
    # same column space
    assert np.abs(Q @ (Q.conj().T @ X) - X).max() < 1e-12


@pytest.mark.parametrize("ns", [48, 64, 128])
def test_chebfd_finds_interior_eigenvalues(ns):
    """TI 6x6x6, W = 2, a window holding exactly the 16 eigenvalues closest
    to E = 0 (8 Kramers pairs; its edges halfway to the 17th): they agree
    with dense diagonalisation, residuals below tolerance, for search spaces
    of 3, 4 and 8 times the count (the larger ones hold Ritz values in the
    window that belong to no eigenvector)."""
    H, lat, _ = ti((6, 6, 6), Wd=2.0, seed=2)
    ev = np.linalg.eigvalsh(H.toarray())
    lam = np.sort(np.abs(ev))
    assert lam[16] - lam[15] > 1e-3
    w = 0.5 * (lam[15] + lam[16])
    X0 = W.random_phase_block(lat.n_rows, ns, W.generator(2, 2))
    th, Q, res, it = chebfd.chebfd(H, X0, 7.0, 0.0, -w, w, 300, 16, 7e-9, max_iter=15)
    near = np.sort(ev[np.argsort(np.abs(ev))][:16])
    assert it < 15
    assert np.abs(np.sort(th) - near).max() < 1e-10 * 7.0
    assert res.max() <= 7e-9
    assert np.abs(Q.conj().T @ Q - np.eye(16)).max() < 1e-12


# --------------------------------------------------------------- KPM adjoint

def test_kpm_vjp_against_finite_differences():
    H, lat, V = ti((3, 3, 3), Wd=1.0)
    model = models.topological_insulator()
    r = W.random_phase_block(lat.n_rows, 3, W.generator(4, 2))
    gbar = W.generator(4, 5).standard_normal((3, 32))
    grad = adjoint.kpm_vjp(H, 4, "site", r, 32, 7.0, 0.0, gbar)
    sites = W.sample_sites(lat.n_sites, 6, W.generator(4, 4))
    fd = adjoint.central_fd(adjoint.kpm_loss(model, lat, r, 32, 7.0, 0.0, gbar), V, sites, 1e-6)
    assert np.abs(grad[sites] - fd).max() < 1e-6 * np.abs(grad).max()


def test_kpm_vjp_trace_closed_form():
    """Exact trace (identity start block): d/dV_m (1/D) Tr T_n(H~) =
    (n/(a D)) sum_o [U_{n-1}(H~)]_{mo,mo}, U the Chebyshev polynomial of the
    second kind, evaluated through the eigendecomposition."""
    H, lat, V = ti((2, 2, 3), Wd=1.0)
    D = lat.n_rows
    a, b, M = 7.0, 0.1, 12
    R = np.eye(D, dtype=np.complex128)
    n_sel = 9
    gbar = np.zeros((D, M))
    gbar[:, n_sel] = 1.0
    grad = adjoint.kpm_vjp(H, 4, "site", R, M, a, b, gbar)
    lam, U = np.linalg.eigh(H.toarray())
    th = np.arccos((lam - b) / a)
    Un1 = np.sin(n_sel * th) / np.sin(th)
    diag = (np.abs(U) ** 2) @ Un1
    ref = (n_sel / (a * D)) * diag.reshape(-1, 4).sum(axis=1)
    assert np.abs(grad - ref).max() < 1e-13


def test_kpm_vjp_orbital_potential_fd():
    model = models.graphene_four_site()
    lat = lattice.Lattice((3, 3), (1, 0), 4)
    V = W.uniform_potential(lat.n_rows, 0.5, W.generator(5, 1))
    H = hamiltonian.assemble(model, lat, V)
    r = W.random_phase_block(lat.n_rows, 2, W.generator(5, 2))
    gbar = W.generator(5, 5).standard_normal((2, 16))
    grad = adjoint.kpm_vjp(H, 4, "orbital", r, 16, 3.5, 0.0, gbar)
    rows = [0, 5, 17, 30]
    fd = adjoint.central_fd(adjoint.kpm_loss(model, lat, r, 16, 3.5, 0.0, gbar), V, rows, 1e-6)
    assert np.abs(grad[rows] - fd).max() < 1e-6 * np.abs(grad).max()


# --------------------------------------------------------------- propagation adjoint

def graphene(L=(6, 5), periodic=(0, 1), Wd=0.3, seed=6):
    lat = lattice.Lattice(L, periodic, 2)
    V = W.uniform_potential(lat.n_sites, Wd, W.generator(seed, 1))
    return hamiltonian.assemble(models.graphene_two_site(), lat, V), lat, V


def test_propagate_vjp_against_matrix_exponential_derivative():
    """T = sum_{i in R} |psi_i(t)|^2 with psi(t) = exp(-i H t) psi_0: the exact
    derivative uses the Frechet derivative of expm, independent of the
    Chebyshev machinery (truncation error ~1e-15)."""
    H, lat, V = graphene()
    a, b, dt, M, S = 3.6, 0.05, 5.0, 48, 2
    psi0 = W.gaussian_block(lat.n_rows, 1, W.generator(6, 2))
    psi0 /= np.linalg.norm(psi0)
    region = np.zeros(lat.n_rows, dtype=bool)
    region[lat.n_rows // 2:] = True
    psiT = chebtp.propagate(H, psi0, a, b, dt, M, S)
    psibar = 2.0 * np.where(region[:, None], psiT, 0)
    _, grad = adjoint.propagate_vjp(H, 2, "site", psi0, a, b, dt, M, S, psibar)
    Hd = H.toarray()
    A = -1j * Hd * dt * S
    for m in [0, 7, 21]:
        E = np.zeros_like(Hd)
        E[2 * m, 2 * m] = E[2 * m + 1, 2 * m + 1] = 1.0
        _, dU = sla.expm_frechet(A, -1j * dt * S * E)
        dpsi = dU @ psi0
        ref = np.real(np.vdot(psibar, dpsi))
        assert abs(grad[m] - ref) < 1e-11


def test_series_vjp_dot_product_test():
    """<Ybar, J Xdot> = <J^H Ybar, Xdot> for the linear map X -> Y."""
    H, lat, _ = graphene()
    eta = chebtp.step_coefficients(3.6, 0.05, 5.0, 40)
    g = W.generator(6, 7)
    X = W.gaussian_block(lat.n_rows, 2, g)
    Xd = W.gaussian_block(lat.n_rows, 2, g)
    Yb = W.gaussian_block(lat.n_rows, 2, g)
    Xbar, _ = adjoint.series_vjp(H, 2, "site", X, 3.6, 0.05, eta, Yb)
    lhs = np.vdot(Yb, chebtp.cheb_series(H, Xd, 3.6, 0.05, eta))
    rhs = np.vdot(Xbar, Xd)
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)


def test_propagate_vjp_finite_differences():
    H, lat, V = graphene()
    model = models.graphene_two_site()
    a, b, dt, M, S = 3.6, 0.05, 5.0, 48, 2
    psi0 = W.gaussian_block(lat.n_rows, 1, W.generator(6, 2))
    psibar = W.gaussian_block(lat.n_rows, 1, W.generator(6, 5))
    _, grad = adjoint.propagate_vjp(H, 2, "site", psi0, a, b, dt, M, S, psibar)

    def loss(Vv):
        Hh = hamiltonian.assemble(model, lat, Vv)
        return float(np.real(np.vdot(psibar, chebtp.propagate(Hh, psi0, a, b, dt, M, S))))
    sites = [1, 9, 20]
    fd = adjoint.central_fd(loss, V, sites, 1e-6)
    assert np.abs(grad[sites] - fd).max() < 1e-6 * np.abs(grad).max()
