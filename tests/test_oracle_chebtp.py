"""Pins of the oracle's Bessel functions and Chebyshev time propagation."""

import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.special as sps

from oracle import chebtp, hamiltonian, lattice, models
import workloads as W


@pytest.mark.parametrize("z", [0.0, 0.5, 3.0, 30.6, 61.2, -35.0])
def test_bessel_against_library(z):
    J = chebtp.bessel_j(z, 80)
    ref = sps.jv(np.arange(81), z)
    assert np.abs(J - ref).max() < 1e-14


def test_bessel_identity_and_asymptotics():
    J = chebtp.bessel_j(30.6, 120)
    assert abs(J[0] + 2 * J[2::2].sum() - 1.0) < 1e-15
    # Sec. 4.1 asymptotic decay for k -> infinity (z fixed); the form is also
    # an upper bound where z^2 is not small against k
    J3 = chebtp.bessel_j(3.0, 60)
    for k in (30, 40, 50):
        asym = (1 / math.sqrt(2 * math.pi * k)) * (math.e * 3.0 / (2 * k)) ** k
        assert 0.85 < abs(J3[k]) / asym < 1.0
    for k in (70, 90, 110):
        asym = (1 / math.sqrt(2 * math.pi * k)) * (math.e * 30.6 / (2 * k)) ** k
        assert abs(J[k]) < asym
    assert chebtp.truncation_bound(3.06, 10.0, 64) < 1e-14


def test_coefficients_integral_definition():
    """c_k = int T_k(x) exp(-i x a dt) / (pi sqrt(1-x^2)) dx, by Gauss-Chebyshev."""
    n = 400
    th = (np.arange(n) + 0.5) * np.pi / n
    x = np.cos(th)
    adt = 7.3
    c = chebtp.tp_coefficients(1.0, adt, 20)
    for k in range(21):
        ref = (np.cos(k * th) * np.exp(-1j * x * adt)).sum() / n
        assert abs(c[k] - ref) < 1e-13


def graphene(L=(8, 6), periodic=(0, 1), Wd=0.3, seed=1):
    lat = lattice.Lattice(L, periodic, 2)
    V = W.uniform_potential(lat.n_sites, Wd, W.generator(seed, 1))
    return hamiltonian.assemble(models.graphene_two_site(), lat, V), lat, V


def test_propagation_matches_matrix_exponential():
    H, lat, _ = graphene()
    psi = W.gaussian_block(lat.n_rows, 2, W.generator(1, 2))
    out = chebtp.propagate(H, psi, 3.5, 0.1, 10.0, 64, 3)
    ref = sla.expm(-1j * H.toarray() * 30.0) @ psi
    assert np.abs(out - ref).max() / np.abs(ref).max() < 1e-10


def test_unitarity_and_time_reversal():
    H, lat, _ = graphene()
    psi = W.gaussian_block(lat.n_rows, 1, W.generator(1, 2))
    fwd = chebtp.propagate(H, psi, 3.5, 0.1, 5.0, 64, 5)
    assert abs(np.linalg.norm(fwd) - np.linalg.norm(psi)) < 1e-11 * np.linalg.norm(psi)
    back = chebtp.propagate(H, fwd, 3.5, 0.1, -5.0, 64, 5)
    assert np.abs(back - psi).max() < 1e-11


def test_bloch_eigenstate_gains_phase():
    """On a clean periodic two-site honeycomb, a Bloch eigenstate of energy E
    evolves as exp(-i E t)."""
    Li, Lj = 6, 9
    lat = lattice.Lattice((Li, Lj), (1, 1), 2)
    H = hamiltonian.assemble(models.graphene_two_site(), lat, None)
    k1, k2 = 2 * np.pi * 1 / Li, 2 * np.pi * 2 / Lj
    f = 1 + np.exp(-1j * k1) + np.exp(-1j * k2)
    E = abs(f)
    ii, jj = np.meshgrid(np.arange(Li), np.arange(Lj))
    ph = np.exp(1j * (k1 * ii + k2 * jj)).reshape(-1)
    psi = np.stack([ph, -np.conj(f) / abs(f) * ph], axis=1).reshape(-1, 1) / math.sqrt(2 * Li * Lj)
    assert np.abs(H @ psi - E * psi).max() < 1e-14
    out = chebtp.propagate(H, psi, 3.1, 0.0, 7.0, 64, 4)
    assert np.abs(out - np.exp(-1j * E * 28.0) * psi).max() < 1e-12
