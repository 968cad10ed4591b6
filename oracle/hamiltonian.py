"""Explicit sparse Hamiltonian from the model terms (oracle; test infrastructure).

This is the matrix the paper's matrix-free stencil applies implicitly
(Sec. 3, the spMVM "lattice sweep").  Entries, for every target cell m:

    hop (e, A), forward:   H[(m, o), (m-e, o')] += A[o, o']          (if m-e exists)
    hop (e, A), h.c.:      H[(m, p), (m+e, q)]  += conj(A[q, p])      (if m+e exists)
    on-site:               H[(m, o), (m, o')]  += E0[o, o'] + V-term

with m +- e wrapped or dropped per dimension (Sec. 3.4).  Duplicates (e.g.
extent 1 or 2 along a periodic dimension) are summed, which is what the
operator sum in the model equations means.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .lattice import Lattice
from .models import Model


def _entries(model: Model, lat: Lattice, V, targets):
    targets = np.asarray(targets, dtype=np.int64)
    no = model.n_orb
    rows, cols, vals = [], [], []
    for e, A in model.hops:
        e = np.asarray(e, dtype=np.int64)
        src, ok = lat.shift(targets, -e)
        for o in range(no):
            for o2 in range(no):
                if A[o, o2] != 0:
                    rows.append(targets[ok] * no + o)
                    cols.append(src[ok] * no + o2)
                    vals.append(np.full(int(ok.sum()), A[o, o2], dtype=np.complex128))
        dst, ok = lat.shift(targets, e)
        AH = A.conj().T
        for p in range(no):
            for q in range(no):
                if AH[p, q] != 0:
                    rows.append(targets[ok] * no + p)
                    cols.append(dst[ok] * no + q)
                    vals.append(np.full(int(ok.sum()), AH[p, q], dtype=np.complex128))
    E0 = model.onsite
    for o in range(no):
        for o2 in range(no):
            if E0[o, o2] != 0:
                rows.append(targets * no + o)
                cols.append(targets * no + o2)
                vals.append(np.full(targets.size, E0[o, o2], dtype=np.complex128))
    if V is not None and model.pot != "none":
        V = np.asarray(V, dtype=np.float64)
        for o in range(no):
            rows.append(targets * no + o)
            cols.append(targets * no + o)
            if model.pot == "site":
                vals.append(V[targets].astype(np.complex128))
            else:
                vals.append(V[targets * no + o].astype(np.complex128))
    return np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)


def assemble(model: Model, lat: Lattice, V=None) -> sp.csr_matrix:
    """Full sparse H (complex128, CSR) on the lattice."""
    if lat.n_orb != model.n_orb:
        raise ValueError("lattice n_orb does not match the model")
    r, c, v = _entries(model, lat, V, np.arange(lat.n_sites, dtype=np.int64))
    D = lat.n_rows
    return sp.coo_matrix((v, (r, c)), shape=(D, D)).tocsr()


def rows_of_sites(model: Model, lat: Lattice, V, sites) -> sp.csr_matrix:
    """The rows of H belonging to the given sites, as a CSR matrix of shape
    [len(sites)*n_orb, D] (row k*n_orb + o is H's row sites[k]*n_orb + o)."""
    sites = np.asarray(sites, dtype=np.int64)
    r, c, v = _entries(model, lat, V, sites)
    no = model.n_orb
    # map global row -> local row
    local = {int(s): k for k, s in enumerate(sites)}
    site_of_row = r // no
    lr = np.fromiter((local[int(s)] for s in site_of_row), dtype=np.int64, count=r.size) * no + r % no
    return sp.coo_matrix((v, (lr, c)), shape=(sites.size * no, lat.n_rows)).tocsr()
