"""Chebyshev time propagation (oracle; test infrastructure).

Sec. 4.1, Eq. (U_1):

    U(dt) = exp(-i b dt) [ c_0 + 2 sum_{k=1}^{M} c_k T_k(H~) ],
    c_k = (-i)^k J_k(a dt),   H~ = (H - b)/a,

with w_k = T_k(H~) psi from w_{k+1} = 2 H~ w_k - w_{k-1}, w_1 = H~ w_0,
w_0 = psi: M matrix-vector products per time step.

Bessel functions J_k(z) of the first kind are evaluated with Miller's
backward recurrence J_{k-1} = (2k/z) J_k - J_{k+1}, normalised by the
identity J_0 + 2 sum_{k>=1} J_{2k} = 1 (Abramowitz & Stegun 9.1.27 and
9.1.46).
"""

from __future__ import annotations

import numpy as np


def bessel_j(z: float, kmax: int) -> np.ndarray:
    """J_0(z) .. J_kmax(z) for real z; negative z via J_k(-z) = (-1)^k J_k(z)."""
    z = float(z)
    out = np.zeros(kmax + 1)
    if z == 0.0:
        out[0] = 1.0
        return out
    if z < 0.0:
        return bessel_j(-z, kmax) * (-1.0) ** np.arange(kmax + 1)
    start = kmax + int(z) + 60
    start += start % 2
    vals = np.zeros(start + 2)
    vals[start + 1] = 0.0
    vals[start] = 1e-30
    for k in range(start, 0, -1):
        vals[k - 1] = (2.0 * k / z) * vals[k] - vals[k + 1]
        if abs(vals[k - 1]) > 1e250:           # rescale to stay finite
            vals[k - 1:] *= 1e-250
    norm = vals[0] + 2.0 * vals[2:start + 1:2].sum()
    return vals[:kmax + 1] / norm


def tp_coefficients(a: float, dt: float, M: int) -> np.ndarray:
    """c_k = (-i)^k J_k(a dt), k = 0..M (complex128)."""
    J = bessel_j(a * dt, M)
    k = np.arange(M + 1)
    return ((-1j) ** k) * J


def cheb_series(H, X, a: float, b: float, coef) -> np.ndarray:
    """Y = sum_k coef[k] T_k(H~) X for a block X [D, nb]."""
    X = np.asarray(X, dtype=np.complex128)
    coef = np.asarray(coef)
    w_prev = X
    Y = coef[0] * X
    if coef.size == 1:
        return Y
    w = (H @ X - b * X) / a
    Y = Y + coef[1] * w
    for k in range(2, coef.size):
        w_next = 2.0 * (H @ w - b * w) / a - w_prev
        w_prev, w = w, w_next
        Y = Y + coef[k] * w
    return Y


def step_coefficients(a: float, b: float, dt: float, M: int) -> np.ndarray:
    """Series coefficients of one propagation step: exp(-i b dt) * c_0 and
    exp(-i b dt) * 2 c_k for k >= 1."""
    c = tp_coefficients(a, dt, M)
    eta = c * np.exp(-1j * b * dt)
    eta[1:] *= 2.0
    return eta


def propagate(H, psi, a: float, b: float, dt: float, M: int, nsteps: int) -> np.ndarray:
    """psi(t0 + nsteps*dt) for a block psi [D, nb]."""
    eta = step_coefficients(a, b, dt, M)
    psi = np.asarray(psi, dtype=np.complex128)
    if psi.ndim == 1:
        psi = psi[:, None]
    for _ in range(nsteps):
        psi = cheb_series(H, psi, a, b, eta)
    return psi


def truncation_bound(a: float, dt: float, M: int) -> float:
    """|J_{M+1}(a dt)|: size of the first neglected expansion coefficient."""
    return abs(bessel_j(a * dt, M + 1)[M + 1])
