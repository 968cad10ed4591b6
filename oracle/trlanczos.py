"""Thick-restart block Lanczos with polynomial filtering for interior
eigenvalues (oracle; test infrastructure).

Sec. 4.2 compares ChebFD with trLanczosFD, the thick-restart Lanczos method
with polynomial filters of Li, Xi, Vecharynski, Yang and Saad (SIAM J. Sci.
Comput. 38, 2016), without describing it; the paper notes that it works with
smaller blocks of vectors than ChebFD.  This module follows that method with
a block size nbl (>= 2 resolves the Kramers pairs of the TI, which a single
start vector cannot):

1. Filter.  p(x) = sum_k g_k (2 - delta_k0) T_k(x_c) T_k(x), the Jackson-
   damped Chebyshev expansion of a delta peak at the centre x_c of the
   target window [x_l, x_r] (scaled units x = (E - b)/a), normalised to
   p(x_c) = 1.  Eigenvalues of H inside the window map to values of p(H~)
   above the threshold tau = min(p(x_l), p(x_r)).
2. Block Lanczos on A = p(H~): W = A V_j, full reorthogonalisation against
   the basis (classical Gram-Schmidt, twice; the first pass gives the
   diagonal block A_j), QR of the rest, W = V_{j+1} B_j, giving the block
   tridiagonal projected matrix.
3. Thick restart once the basis holds m vectors: the Ritz vectors of A with
   values above tau are kept (their number rounded up to whole blocks with
   the next Ritz vectors), the last block continues the basis, and the
   projected matrix starts as diag(kept values) with the couplings
   B_last * (last block rows of the kept eigenvectors).
4. Convergence: for the kept Ritz vectors u, theta = u^H H u and the true
   residual ||H u - theta u||; the run ends when every Ritz value above tau
   belongs to a pair with residual <= tol and that number of pairs did not
   change since the previous restart.
5. Result: the pairs with theta inside [lam_l, lam_r] (eigenvalues just
   outside the window can pass the threshold tau).
"""

from __future__ import annotations

import numpy as np

from . import kpm
from .chebtp import cheb_series


def delta_filter(lam_l: float, lam_r: float, a: float, b: float, K: int):
    """Coefficients of p (degree K, in H~ = (H - b)/a) and the threshold tau."""
    xl, xr = (lam_l - b) / a, (lam_r - b) / a
    xc = 0.5 * (xl + xr)
    g = kpm.jackson(K + 1)
    k = np.arange(K + 1)
    Tc = np.cos(k * np.arccos(xc))
    coef = g * np.where(k == 0, 1.0, 2.0) * Tc
    pc = float(np.polynomial.chebyshev.chebval(xc, coef))
    coef = coef / pc
    tau = min(float(np.polynomial.chebyshev.chebval(xl, coef)), float(np.polynomial.chebyshev.chebval(xr, coef)))
    return coef, tau


def trlanczos_fd(H, V0, a: float, b: float, lam_l: float, lam_r: float, K: int, m: int, tol: float,
                 max_restarts: int = 60):
    """V0: start block [n, nbl]; m: basis size (a multiple of nbl).  Returns
    (theta ascending, U, residuals, restarts) for the pairs found inside
    [lam_l, lam_r]."""
    coef, tau = delta_filter(lam_l, lam_r, a, b, K)
    V0 = np.asarray(V0, dtype=np.complex128)
    if V0.ndim == 1:
        V0 = V0[:, None]
    nbl = V0.shape[1]
    assert m % nbl == 0 and m >= 2 * nbl

    def apply(X):
        return cheb_series(H, X, a, b, coef)

    n = H.shape[0]
    V = np.zeros((n, m + nbl), dtype=np.complex128)
    V[:, :nbl] = np.linalg.qr(V0)[0]
    k, kept, S = 0, np.zeros(0), np.zeros((nbl, 0), dtype=np.complex128)
    last_count = -1
    theta = res = U = None
    for restart in range(1, max_restarts + 1):
        T = np.zeros((m, m), dtype=np.complex128)
        if k:
            T[:k, :k] = np.diag(kept)
            T[k:k + nbl, :k] = S
            T[:k, k:k + nbl] = S.conj().T
        B = None
        for j0 in range(k, m, nbl):
            j1 = j0 + nbl
            W = apply(V[:, j0:j1])
            C = V[:, :j1].conj().T @ W
            Aj = C[j0:j1]
            W = W - V[:, :j1] @ C
            W = W - V[:, :j1] @ (V[:, :j1].conj().T @ W)
            T[j0:j1, j0:j1] = 0.5 * (Aj + Aj.conj().T)
            Q, B = np.linalg.qr(W)
            if j1 < m:
                T[j1:j1 + nbl, j0:j1] = B
                T[j0:j1, j1:j1 + nbl] = B.conj().T
            V[:, j1:j1 + nbl] = Q
        mu, Y = np.linalg.eigh(T)
        want = np.where(mu > tau)[0]
        U = V[:, :m] @ Y[:, want]
        HU = H @ U
        theta = np.einsum("ij,ij->j", U.conj(), HU).real
        res = np.linalg.norm(HU - U * theta[None, :], axis=0)
        if want.size and (res <= tol).all() and want.size == last_count:
            return _inside(theta, U, res, lam_l, lam_r) + (restart,)
        last_count = want.size
        # thick restart: the wanted Ritz vectors, rounded up to whole blocks
        nk = min(-(-want.size // nbl) * nbl, m - nbl)
        keep = np.arange(m - nk, m)                 # the nk largest Ritz values of A
        V[:, :nk] = V[:, :m] @ Y[:, keep]
        S = B @ Y[m - nbl:m, keep]
        V[:, nk:nk + nbl] = V[:, m:m + nbl]
        k, kept = nk, mu[keep]
    return _inside(theta, U, res, lam_l, lam_r) + (max_restarts,)


def _inside(theta, U, res, lam_l, lam_r):
    sel = np.where((theta >= lam_l) & (theta <= lam_r))[0]
    sel = sel[np.argsort(theta[sel])]
    return theta[sel], U[:, sel], res[sel]
