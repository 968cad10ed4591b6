"""Discrete adjoints with respect to the on-site potential (oracle; test
infrastructure).

The forward computations are the KPM moments obtained by the product
doubling (``kpm.moments_doubling``) and the Chebyshev propagation steps
(``chebtp.propagate``).  H~ = (H - b)/a depends on the on-site field through
dH~/dV_m = P_m / a, where P_m is the projector on the rows of site m
("site" potential: all orbitals of the site) or on row m ("orbital"
potential).  a and b are fixed numbers, not differentiated.

KPM, scalar L = sum_{c,n} gbar[c,n] mu[c,n].  With N = M/2, the gradient of L
with respect to w_k (dL = Re <G_k, dw_k>) is, for k = 1..N,

    G_k = ( 4 gbar_{2k} w_k [k<N] + 2 gbar_{2k+1} w_{k+1} [k<N]
          + 2 gbar_{2k-1} w_{k-1} [k>=2] + ghat_1 w_0 [k=1] ) / D,
    ghat_1 = gbar_1 - sum_{n=1}^{N-1} gbar_{2n+1}

(the last because every odd moment subtracts mu_1).  The adjoint vectors
follow the transposed recurrence

    lambda_k = G_k + 2 H~ lambda_{k+1} - lambda_{k+2},  lambda_{N+1} = lambda_{N+2} = 0,

and

    dL/dV_m = (1/a) Re [ <lambda_1, P_m w_0> + 2 sum_{k=1}^{N-1} <lambda_{k+1}, P_m w_k> ].

Chebyshev series Y = sum_{k=0}^{K} eta_k w_k with cotangent Ybar: G_k =
conj(eta_k) Ybar, lambda_K = G_K, lambda_{K-1} = G_{K-1} + 2 H~ lambda_K,
lambda_k = G_k + 2 H~ lambda_{k+1} - lambda_{k+2} (k >= 1), and the input
cotangent lambda_0 = G_0 + H~ lambda_1 - lambda_2; the V-gradient has the
same form as above with N replaced by K.
"""

from __future__ import annotations

import numpy as np

from .chebtp import step_coefficients
from .hamiltonian import assemble
from .kpm import chebyshev_vectors, moments_doubling


def _scaled(H, w, a, b):
    return (H @ w - b * w) / a


def _project(u, v, n_orb, pot):
    """Per site (or row) sum over orbitals and columns of Re(conj(u) v)."""
    prod = (np.conj(u) * v).real.sum(axis=1)
    if pot == "site":
        return prod.reshape(-1, n_orb).sum(axis=1)
    return prod


def kpm_vjp(H, n_orb: int, pot: str, r, M: int, a: float, b: float, gbar) -> np.ndarray:
    """dL/dV for L = sum gbar[c, n] mu[c, n] (mu from the product doubling)."""
    r = np.asarray(r, dtype=np.complex128)
    gbar = np.asarray(gbar, dtype=np.float64)
    D = r.shape[0]
    N = M // 2
    ws = chebyshev_vectors(H, r, N, a, b)
    G = [None] + [np.zeros_like(r) for _ in range(N)]
    for k in range(1, N + 1):
        if k < N:
            G[k] += 4.0 * gbar[:, 2 * k][None, :] * ws[k]
            G[k] += 2.0 * gbar[:, 2 * k + 1][None, :] * ws[k + 1]
        if k >= 2:
            G[k] += 2.0 * gbar[:, 2 * k - 1][None, :] * ws[k - 1]
    ghat1 = gbar[:, 1] - gbar[:, 3:M:2].sum(axis=1)
    G[1] += ghat1[None, :] * ws[0]
    for k in range(1, N + 1):
        G[k] /= D
    lam = [None] * (N + 3)
    lam[N + 1] = np.zeros_like(r)
    lam[N + 2] = np.zeros_like(r)
    for k in range(N, 0, -1):
        lam[k] = G[k] + 2.0 * _scaled(H, lam[k + 1], a, b) - lam[k + 2]
    grad = _project(lam[1], ws[0], n_orb, pot)
    for k in range(1, N):
        grad = grad + 2.0 * _project(lam[k + 1], ws[k], n_orb, pot)
    return grad / a


def series_vjp(H, n_orb: int, pot: str, X, a: float, b: float, eta, Ybar):
    """For Y = sum_k eta_k T_k(H~) X: returns (Xbar, dL/dV) given Ybar."""
    X = np.asarray(X, dtype=np.complex128)
    K = len(eta) - 1
    ws = chebyshev_vectors(H, X, K, a, b)
    G = [np.conj(eta[k]) * Ybar for k in range(K + 1)]
    lam = [None] * (K + 3)
    lam[K + 1] = np.zeros_like(X)
    lam[K + 2] = np.zeros_like(X)
    for k in range(K, 0, -1):
        lam[k] = G[k] + 2.0 * _scaled(H, lam[k + 1], a, b) - lam[k + 2]
    Xbar = G[0] + _scaled(H, lam[1], a, b) - lam[2]
    grad = _project(lam[1], ws[0], n_orb, pot) if K >= 1 else 0.0
    for k in range(1, K):
        grad = grad + 2.0 * _project(lam[k + 1], ws[k], n_orb, pot)
    return Xbar, grad / a


def propagate_vjp(H, n_orb: int, pot: str, psi0, a, b, dt, M, nsteps, psibar):
    """Cotangent of psi0 and dL/dV for psi_final = U(dt)^nsteps psi0, given
    the cotangent psibar of psi_final (dL = Re <psibar, d psi_final>)."""
    from .chebtp import cheb_series
    eta = step_coefficients(a, b, dt, M)
    psi = np.asarray(psi0, dtype=np.complex128)
    if psi.ndim == 1:
        psi = psi[:, None]
    states = [psi]
    for _ in range(nsteps):
        states.append(cheb_series(H, states[-1], a, b, eta))
    ybar = np.asarray(psibar, dtype=np.complex128).reshape(states[-1].shape)
    grad = 0.0
    for s in range(nsteps, 0, -1):
        ybar, g = series_vjp(H, n_orb, pot, states[s - 1], a, b, eta, ybar)
        grad = grad + g
    return ybar, grad


def central_fd(loss, V: np.ndarray, sites, h: float = 1e-6) -> np.ndarray:
    """(loss(V + h e_m) - loss(V - h e_m)) / (2h) for m in sites."""
    out = np.zeros(len(sites))
    for i, m in enumerate(sites):
        Vp = V.copy()
        Vp[m] += h
        Vm = V.copy()
        Vm[m] -= h
        out[i] = (loss(Vp) - loss(Vm)) / (2.0 * h)
    return out


def kpm_loss(model, lat, r, M, a, b, gbar):
    """V -> sum gbar * mu(V), for finite differences."""
    def f(V):
        H = assemble(model, lat, V)
        return float((np.asarray(gbar) * moments_doubling(H, r, M, a, b)).sum())
    return f
