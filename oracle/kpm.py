"""Kernel polynomial method (oracle; test infrastructure).

Sec. 2.2 (DOS equation) and Sec. 4 (KPM, stochastic trace with random
vectors, Chebyshev moments formed from partial dot products).  The spectrum is
mapped into [-1, 1] by H~ = (H - b)/a (Sec. 4.1).

Moments per start column r (D = number of rows):

    mu_n = Re <r, T_n(H~) r> / D

``moments_direct`` evaluates this definition with w_n = T_n(H~) r from the
three-term recurrence w_{n+1} = 2 H~ w_n - w_{n-1}, w_1 = H~ w_0, w_0 = r.
``moments_doubling`` uses T_{2n} = 2 T_n^2 - T_0 and
T_{2n+1} = 2 T_{n+1} T_n - T_1 (H~ Hermitian), so that M moments need only
M/2 products:

    mu_{2n}   = 2 <w_n, w_n>/D - mu_0,     mu_{2n+1} = 2 Re <w_n, w_{n+1}>/D - mu_1

with mu_0 = <w_0, w_0>/D and mu_1 = Re <w_0, w_1>/D.  This is the quantity the
fused dot products of the stencil sweep deliver.
"""

from __future__ import annotations

import numpy as np


def _apply_scaled(H, w, a, b):
    return (H @ w - b * w) / a


def moments_direct(H, r, M: int, a: float, b: float) -> np.ndarray:
    """mu[c, n] for n = 0..M-1, straight from the definition."""
    r = np.asarray(r, dtype=np.complex128)
    D = r.shape[0]
    mu = np.zeros((r.shape[1], M))
    w_prev = r.copy()
    mu[:, 0] = np.einsum("rc,rc->c", np.conj(r), w_prev).real / D
    if M == 1:
        return mu
    w = _apply_scaled(H, r, a, b)
    mu[:, 1] = np.einsum("rc,rc->c", np.conj(r), w).real / D
    for n in range(2, M):
        w_next = 2.0 * _apply_scaled(H, w, a, b) - w_prev
        w_prev, w = w, w_next
        mu[:, n] = np.einsum("rc,rc->c", np.conj(r), w).real / D
    return mu


def chebyshev_vectors(H, r, N: int, a: float, b: float):
    """[w_0, ..., w_N] with w_n = T_n(H~) r."""
    r = np.asarray(r, dtype=np.complex128)
    ws = [r.copy()]
    if N >= 1:
        ws.append(_apply_scaled(H, r, a, b))
    for n in range(2, N + 1):
        ws.append(2.0 * _apply_scaled(H, ws[-1], a, b) - ws[-2])
    return ws


def moments_doubling(H, r, M: int, a: float, b: float) -> np.ndarray:
    """mu[c, n] for n = 0..M-1 (M even) from w_0..w_{M/2}."""
    if M < 2 or M % 2:
        raise ValueError("M must be even and >= 2")
    r = np.asarray(r, dtype=np.complex128)
    D = r.shape[0]
    N = M // 2
    ws = chebyshev_vectors(H, r, N, a, b)
    mu = np.zeros((r.shape[1], M))
    dot = lambda u, v: np.einsum("rc,rc->c", np.conj(u), v)
    mu[:, 0] = dot(ws[0], ws[0]).real / D
    mu[:, 1] = dot(ws[0], ws[1]).real / D
    for n in range(1, N):
        mu[:, 2 * n] = 2.0 * dot(ws[n], ws[n]).real / D - mu[:, 0]
        mu[:, 2 * n + 1] = 2.0 * dot(ws[n], ws[n + 1]).real / D - mu[:, 1]
    return mu


def jackson(M: int) -> np.ndarray:
    """Jackson damping factors g_n, n = 0..M-1 (Weisse et al., Rev. Mod. Phys.
    78, 275 (2006), the KPM reference of the paper)."""
    n = np.arange(M, dtype=np.float64)
    q = np.pi / (M + 1)
    return ((M - n + 1) * np.cos(q * n) + np.sin(q * n) / np.tan(q)) / (M + 1)


def dos(mu: np.ndarray, E, a: float, b: float, kernel: str = "jackson") -> np.ndarray:
    """Density of states per row from moments mu[0..M-1] (one column or the
    column mean):  rho(E) = [g_0 mu_0 + 2 sum_{n>=1} g_n mu_n T_n(x)] /
    (pi a sqrt(1 - x^2)),  x = (E - b)/a.  Integrates to mu_0."""
    mu = np.asarray(mu, dtype=np.float64)
    M = mu.shape[-1]
    g = jackson(M) if kernel == "jackson" else np.ones(M)
    x = (np.asarray(E, dtype=np.float64) - b) / a
    n = np.arange(M)
    T = np.cos(n[None, :] * np.arccos(np.clip(x, -1.0, 1.0))[:, None])
    wts = g * mu
    wts[1:] *= 2.0
    return (T @ wts) / (np.pi * a * np.sqrt(1.0 - x * x))
