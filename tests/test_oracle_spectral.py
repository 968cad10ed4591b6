"""Pins of the oracle's spectral function (Eq. ak): closed-form moments of
Bloch columns on the clean periodic Weyl lattice from the 2 x 2 band matrix
of Eq. (band_h_wsm), completeness of the Bloch basis (the sum over the
momentum grid gives the trace moments, with disorder), surface-layer states,
peak positions and the integral of A."""

import math

import numpy as np

from oracle import hamiltonian, kpm, lattice, models, spectral
import workloads as W

K0 = math.pi / 2


def band_matrix(k):
    return (models.SX * (math.cos(k[0]) - math.cos(K0) + math.cos(k[1]) + math.cos(k[2]) - 2)
            + models.SY * math.sin(k[1]) + models.SZ * math.sin(k[2]))


def test_clean_bloch_moments_closed_form():
    L = (6, 5, 4)
    lat = lattice.Lattice(L, (1, 1, 1), 2)
    H = hamiltonian.assemble(models.weyl_semimetal(), lat, None)
    ks = [(2 * math.pi * i / L[0], 2 * math.pi * j / L[1], 2 * math.pi * l / L[2])
          for (i, j, l) in [(0, 0, 0), (1, 2, 3), (3, 1, 0), (5, 4, 1)]]
    kk = [k for k in ks for _ in (0, 1)]
    nu = [n for _ in ks for n in (0, 1)]
    R = spectral.bloch_block(lat, 2, kk, nu)
    M, a = 40, 7.0
    mu = kpm.moments_doubling(H, R, M, a, 0.0)
    T = np.polynomial.chebyshev.chebvander
    for c, (k, n) in enumerate(zip(kk, nu)):
        e, U = np.linalg.eigh(band_matrix(k))
        ref = sum(abs(U[n, i]) ** 2 * T(np.array([e[i] / a]), M - 1)[0] for i in range(2))
        ref *= lat.n_sites / lat.n_rows
        assert np.abs(mu[c] - ref).max() < 1e-12


def test_completeness_gives_trace_moments_with_disorder():
    L = (4, 3, 3)
    lat = lattice.Lattice(L, (1, 1, 1), 2)
    V = W.uniform_potential(lat.n_sites, 2.0, W.generator(1, W.STREAM_POTENTIAL))
    H = hamiltonian.assemble(models.weyl_semimetal(), lat, V)
    grid = [(2 * math.pi * i / L[0], 2 * math.pi * j / L[1], 2 * math.pi * l / L[2])
            for i in range(L[0]) for j in range(L[1]) for l in range(L[2])]
    kk = [k for k in grid for _ in (0, 1)]
    nu = [n for _ in grid for n in (0, 1)]
    R = spectral.bloch_block(lat, 2, kk, nu)
    M, a = 30, 7.0
    mu = kpm.moments_doubling(H, R, M, a, 0.0).sum(axis=0)
    ev = np.linalg.eigvalsh(H.toarray())
    trace = np.polynomial.chebyshev.chebvander(ev / a, M - 1).sum(axis=0)
    assert np.abs(mu - lat.n_sites * trace / lat.n_rows).max() < 1e-10


def test_surface_layer_state():
    L = (5, 4, 3)
    lat = lattice.Lattice(L, (1, 1, 0), 2)
    R = spectral.bloch_block(lat, 2, [(0.3, -0.2, 0.0)], [1], layer=(2, 0))
    x, y, z = lat.coords(np.arange(lat.n_sites))
    col = R.reshape(lat.n_sites, 2)
    assert np.all(col[z != 0] == 0) and np.all(col[:, 0] == 0)
    assert np.allclose(np.abs(col[z == 0, 1]), 1.0)
    assert abs(np.vdot(R[:, 0], R[:, 0]).real - L[0] * L[1]) < 1e-12


def test_spectral_function_peaks_and_integral():
    L = (8, 6, 4)
    lat = lattice.Lattice(L, (1, 1, 1), 2)
    H = hamiltonian.assemble(models.weyl_semimetal(), lat, None)
    k = (2 * math.pi * 2 / L[0], 2 * math.pi * 1 / L[1], 0.0)
    R = spectral.bloch_block(lat, 2, [k, k], [0, 1])
    M, a = 256, 7.0
    mu = kpm.moments_doubling(H, R, M, a, 0.0)
    E = np.linspace(-6.9, 6.9, 4001)
    A = spectral.spectral_function(mu, E, a, 0.0, lat.n_rows / lat.n_sites)
    e = np.linalg.eigvalsh(band_matrix(k))
    width = math.pi * a / M
    for ei in e:
        win = np.abs(E - ei) < 3 * width
        assert E[win][np.argmax(A[win])] == E[np.argmax(np.where(np.abs(E - ei) < 10 * width, A, 0))]
    assert abs(np.trapezoid(A, E) - 2.0) < 1e-2
