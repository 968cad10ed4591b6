"""Sparse matrix-multiple-vector product with Chebyshev scale/shift and the
partial dot products (oracle; test infrastructure).

Sec. 3.2, generated-code listing for the graphene stencil: every column k of
the vector block is updated as

    y_k <- scale_z[k] * y_k + scale_h[k] * ( H x_k - shift_h[k] * x_k )

and, on request, the partial dot products xx, xy, yy of the same columns are
formed in the same sweep.  Here alpha = scale_h, beta = shift_h, gamma =
scale_z, and the old y may come from a separate block z.  gamma = 0 means z
is not read at all.  The dot products use <a, b> = sum conj(a) b:
    xx = <x, x>,  xy = <x, y>,  yy = <y, y>   (xy is complex; KPM uses Re xy).
"""

from __future__ import annotations

import numpy as np


def spmmv(H, x, alpha, beta, gamma, z=None):
    x = np.asarray(x)
    nb = x.shape[1]
    alpha = np.broadcast_to(np.asarray(alpha, dtype=np.float64), (nb,))
    beta = np.broadcast_to(np.asarray(beta, dtype=np.float64), (nb,))
    gamma = np.broadcast_to(np.asarray(gamma, dtype=np.float64), (nb,))
    Hx = H @ x
    y = alpha[None, :] * (Hx - beta[None, :] * x)
    for c in range(nb):
        if gamma[c] != 0.0:
            y[:, c] += gamma[c] * z[:, c]
    return y


def block_dots(x, y):
    """Per column: (<x,x>, <x,y>, <y,y>) with <a,b> = sum conj(a) b."""
    xx = np.einsum("rc,rc->c", np.conj(x), x).real
    xy = np.einsum("rc,rc->c", np.conj(x), y)
    yy = np.einsum("rc,rc->c", np.conj(y), y).real
    return xx, xy, yy
