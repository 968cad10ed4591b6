"""Chebyshev filter diagonalisation (oracle; test infrastructure).

Sec. 4.2: a polynomial filter adapted to a target interval is applied to a
block of vectors; after each filter pass the search space is checked with a
Rayleigh-Ritz step.  The paper defers details to its ChebFD reference; the
steps here are the standard ones that description implies:

1. target window [lam_l, lam_r] mapped to x_l, x_r in the scaled spectrum;
2. Chebyshev series of the window indicator:
     c_0 = (arccos x_l - arccos x_r)/pi,
     c_k = 2 (sin(k arccos x_l) - sin(k arccos x_r)) / (k pi);
3. damping g_k (Jackson, as for KPM);
4. filter  Y = sum_{k=0}^{K} g_k c_k T_k(H~) X;
5. orthonormalise Y (Cholesky QR, applied twice), in float64;
6. Rayleigh-Ritz: H_S = Q^H H Q, H_S = U diag(theta) U^H, Q <- Q U;
7. residuals ||H q_i - theta_i q_i||;
8. a Ritz pair counts as converged when its value lies in the window and
   its residual is <= tol; the iteration ends when n_target pairs have
   converged, and returns those closest to the window centre; otherwise
   X <- Q and repeat.  A search space larger than the window's count holds
   Ritz values in the window that belong to no eigenvector (residuals of
   order one); they never count, so they can not stall the iteration.
"""

from __future__ import annotations

import numpy as np

from .chebtp import cheb_series
from .kpm import jackson


def window_coefficients(x_l: float, x_r: float, K: int) -> np.ndarray:
    """Chebyshev coefficients c_0..c_K of the indicator of [x_l, x_r] in [-1, 1]."""
    al, ar = np.arccos(x_l), np.arccos(x_r)
    k = np.arange(1, K + 1, dtype=np.float64)
    c = np.empty(K + 1)
    c[0] = (al - ar) / np.pi
    c[1:] = 2.0 * (np.sin(k * al) - np.sin(k * ar)) / (k * np.pi)
    return c


def filter_coefficients(lam_l: float, lam_r: float, a: float, b: float, K: int) -> np.ndarray:
    """g_k c_k, k = 0..K, for the window [lam_l, lam_r] in energy units."""
    c = window_coefficients((lam_l - b) / a, (lam_r - b) / a, K)
    return jackson(K + 1) * c


def filter_polynomial(x, coef) -> np.ndarray:
    """p(x) = sum_k coef_k T_k(x) evaluated directly with T_k = cos(k arccos x)."""
    x = np.asarray(x, dtype=np.float64)
    k = np.arange(len(coef))
    return np.cos(k[None, :] * np.arccos(np.clip(x, -1, 1))[:, None]) @ np.asarray(coef)


def cholesky_qr(Y: np.ndarray) -> np.ndarray:
    G = Y.conj().T @ Y
    R = np.linalg.cholesky(G).conj().T          # G = R^H R
    return np.linalg.solve(R.T, Y.T).T          # Y R^{-1}


def rayleigh_ritz(H, Q):
    HQ = H @ Q
    Hs = Q.conj().T @ HQ
    Hs = 0.5 * (Hs + Hs.conj().T)
    theta, U = np.linalg.eigh(Hs)
    return theta, Q @ U, HQ @ U


def chebfd(H, X0, a: float, b: float, lam_l: float, lam_r: float, K: int,
           n_target: int, tol: float, max_iter: int = 20):
    """Returns (theta, Q, residuals, iterations) for n_target Ritz pairs:
    the converged ones (value in the window, residual <= tol) closest to the
    window centre first, then the others closest to the centre."""
    coef = filter_coefficients(lam_l, lam_r, a, b, K)
    centre = 0.5 * (lam_l + lam_r)
    X = np.asarray(X0, dtype=np.complex128)
    for it in range(1, max_iter + 1):
        Y = cheb_series(H, X, a, b, coef)
        Q = cholesky_qr(cholesky_qr(Y))
        theta, Q, HQ = rayleigh_ritz(H, Q)
        res = np.linalg.norm(HQ - Q * theta[None, :], axis=0)
        conv = (theta >= lam_l) & (theta <= lam_r) & (res <= tol)
        dist = np.abs(theta - centre)
        order = np.lexsort((dist, ~conv))[:n_target]     # converged first, then by distance
        sel_t, sel_r = theta[order], res[order]
        if conv.sum() >= n_target:
            return sel_t, Q[:, order], sel_r, it
        X = Q
    return sel_t, Q[:, order], sel_r, max_iter
