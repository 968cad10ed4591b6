"""Momentum-resolved spectral function A(k, E) (oracle; test infrastructure).

Sec. 2.2, Eq. (ak): A(k, E) = sum_nu sum_l |<l|psi(k, nu)>|^2 delta(E - E_l)
with the Bloch state <n, nu'|psi(k, nu)> = exp(i k . r_n) delta_{nu nu'}.
Its Chebyshev moments are <psi|T_n(H~)|psi>, so A follows from the KPM with
Bloch start vectors.  The state may be restricted to one layer of sites (a
surface, as for the Fermi arcs of the Weyl semimetal in Sec. 4.3).

Normalisation: moments per column are divided by D = n_rows (as for the DOS);
A(E) = norm * sum_c rho_c(E) with norm = D / (sites carrying the state), so A
integrates to the number of columns.
"""

from __future__ import annotations

import numpy as np

from . import kpm


def bloch_block(lat, n_orb: int, k, orbital, layer=None) -> np.ndarray:
    """Columns c = exp(i k_c . r) on orbital[c]; layer = (axis, index) keeps
    only the sites with that coordinate.  Shape [n_rows, nb]."""
    k = np.asarray(k, dtype=np.float64).reshape(-1, 3)
    orbital = np.asarray(orbital).reshape(-1)
    s = np.arange(lat.n_sites)
    r = np.stack(lat.coords(s), axis=1).astype(np.float64)
    out = np.zeros((lat.n_sites, n_orb, k.shape[0]), dtype=np.complex128)
    on = np.ones(lat.n_sites, dtype=bool) if layer is None else (r[:, layer[0]] == layer[1])
    for c in range(k.shape[0]):
        out[on, orbital[c], c] = np.exp(1j * (r[on] @ k[c]))
    return out.reshape(lat.n_sites * n_orb, k.shape[0])


def spectral_function(mu, E, a: float, b: float, norm: float) -> np.ndarray:
    """A(E) = norm * sum over columns of the Jackson-damped reconstruction."""
    mu = np.atleast_2d(np.asarray(mu, dtype=np.float64))
    return norm * sum(kpm.dos(m, E, a, b) for m in mu)
