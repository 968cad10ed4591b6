"""GPU parity of the fused stencil sweep (pv_spmmv) against the oracle.

Tolerances: complex128 -- 1e-13 relative to max|y| (different summation
order, FMA contraction on both sides); delta vectors -- bit-exact (one
nonzero product per entry); complex64 vectors -- 2e-6 relative (FP32 stencil
arithmetic, unit round-off 6e-8 times at most ~20 accumulated terms of
comparable size)."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1708_09689_amd as pv  # noqa: E402
from oracle import spmmv  # noqa: E402
import workloads as W  # noqa: E402

from gpu_common import Case, dev, host, rel_err  # noqa: E402


@pytest.mark.parametrize("name,L,periodic", [
    ("ti", (5, 4, 3), (1, 1, 1)),
    ("ti", (7, 3, 4), (0, 1, 0)),
    ("ti_delta", (4, 3, 3), (1, 0, 1)),
    ("graphene2", (9, 5), (0, 1)),
    ("graphene4", (6, 5), (1, 0)),
    ("weyl", (5, 4, 3), (1, 1, 0)),
])
def test_delta_vectors_bit_exact(name, L, periodic):
    c = Case(name, L, periodic, Wd=1.0)
    cols = [0, 1, c.D // 3, c.D // 2 + 1, c.D - 1, 7, 11, c.D - 5]
    X = W.basis_block(c.D, cols)
    y = torch.empty((c.D, len(cols)), dtype=torch.complex128, device="cuda")
    pv.pv_spmmv(c.lat, dev(X), y, 1.0, 0.0, 0.0)
    ref = spmmv.spmmv(c.H, X, 1.0, 0.0, 0.0)
    assert np.array_equal(host(y), ref)


@pytest.mark.parametrize("name,L,periodic", [
    ("ti", (37, 5, 4), (1, 1, 1)),      # ragged x-rows for every tile width
    ("ti", (16, 9, 7), (0, 0, 1)),
    ("ti", (1, 2, 3), (1, 1, 1)),       # extents 1 and 2 along periodic axes
    ("ti_delta", (12, 6, 5), (1, 1, 0)),
    ("graphene2", (70, 9), (0, 1)),
    ("graphene4", (21, 10), (1, 1)),
    ("weyl", (19, 6, 5), (1, 1, 0)),
])
@pytest.mark.parametrize("nb", [1, 4, 32])
def test_sweep_matches_oracle_c128(name, L, periodic, nb):
    c = Case(name, L, periodic, Wd=2.0, seed=nb)
    x = c.block(nb, seed=1)
    z = c.block(nb, seed=2)
    g = W.generator(5, 7, nb)
    alpha, beta, gamma = 0.5 + g.random(nb), g.standard_normal(nb), g.standard_normal(nb)
    y = dev(z.copy())
    dots = pv.pv_spmmv(c.lat, dev(x), y, alpha, beta, gamma, z=y, dot_flags=7)
    ref = spmmv.spmmv(c.H, x, alpha, beta, gamma, z)
    out = host(y)
    assert rel_err(out, ref) < 1e-13
    xx, xy, yy = spmmv.block_dots(x, ref)
    d = host(dots)
    assert np.abs(d[:, 0] - xx).max() < 1e-12 * xx.max()
    assert np.abs(d[:, 1] + 1j * d[:, 2] - xy).max() < 1e-12 * np.sqrt(xx.max() * yy.max())
    assert np.abs(d[:, 3] - yy).max() < 1e-12 * yy.max()


@pytest.mark.parametrize("nb", [1, 2, 8, 16, 64])
def test_sweep_all_block_widths(nb):
    c = Case("ti", (11, 6, 5), (1, 1, 1), Wd=1.0)
    x = c.block(nb)
    y = torch.empty((c.D, nb), dtype=torch.complex128, device="cuda")
    pv.pv_spmmv(c.lat, dev(x), y, 0.25, 0.1, 0.0)
    assert rel_err(host(y), spmmv.spmmv(c.H, x, 0.25, 0.1, 0.0)) < 1e-13


@pytest.mark.parametrize("name", ["ti", "graphene2", "weyl"])
@pytest.mark.parametrize("vdtype", [np.float64, np.float32])
def test_sweep_c64_error_bound(name, vdtype):
    L = {"ti": (13, 6, 5), "graphene2": (40, 12), "weyl": (9, 6, 5)}[name]
    c = Case(name, L, (1, 1, 1), Wd=2.0, vdtype=vdtype)
    nb = 4
    x = c.block(nb, dtype=np.complex64)
    z = c.block(nb, seed=2, dtype=np.complex64)
    y = dev(z.copy())
    dots = pv.pv_spmmv(c.lat, dev(x), y, 2.0 / 7.0, 0.0, -1.0, z=y, dot_flags=7)
    Vq = c.V.astype(vdtype).astype(np.float64)
    import oracle.hamiltonian as oh
    Hq = oh.assemble(c.model, c.olat, Vq)
    ref = spmmv.spmmv(Hq, x.astype(np.complex128), 2.0 / 7.0, 0.0, -1.0, z.astype(np.complex128))
    assert rel_err(host(y).astype(np.complex128), ref) < 2e-6
    # dots accumulate in FP64 from the FP32 values
    xx, _, _ = spmmv.block_dots(x.astype(np.complex128), x.astype(np.complex128))
    assert np.abs(host(dots)[:, 0] - xx).max() < 1e-12 * xx.max()


def test_per_column_and_gamma_zero_semantics():
    c = Case("ti", (9, 4, 4), (1, 1, 1))
    nb = 4
    x = c.block(nb)
    z = np.full((c.D, nb), np.nan + 0j)
    y = dev(z)
    alpha = np.array([1.0, 0.5, 2.0, 1.0])
    beta = np.array([0.0, 1.0, -2.0, 0.5])
    pv.pv_spmmv(c.lat, dev(x), y, alpha, beta, np.zeros(nb))   # gamma = 0: y is write-only
    out = host(y)
    assert np.isfinite(out).all()
    assert rel_err(out, spmmv.spmmv(c.H, x, alpha, beta, 0.0)) < 1e-13


@pytest.mark.parametrize("name,L,periodic", [("ti", (21, 6, 5), (1, 1, 1)), ("ti", (9, 7, 6), (0, 1, 0)),
                                             ("weyl", (13, 5, 4), (1, 0, 1)), ("graphene2", (37, 11), (0, 1))])
@pytest.mark.parametrize("nb", [1, 4, 16])
@pytest.mark.parametrize("sh", [{"kernel": 1}, {"kernel": 2}, {"kernel": 2, "elems_per_lane": 2},
                                {"kernel": 2, "elems_per_lane": 2, "workgroup_size": 512}])
def test_plain_sweep_gamma_zero_uniform(name, L, periodic, nb, sh):
    """Uniform alpha, beta and gamma = 0 take the plain staged kernel that
    loads no z: y starts as NaN and must come out as alpha (H x - beta x)."""
    c = Case(name, L, periodic, Wd=1.5, seed=nb)
    pv.pv_lattice_set_tuning(c.lat, pv.PV_C128, nb, sh)
    x = c.block(nb, seed=5)
    y = dev(np.full((c.D, nb), np.nan + 0j))
    pv.pv_spmmv(c.lat, dev(x), y, 0.6, -0.3, 0.0)
    out = host(y)
    assert np.isfinite(out).all()
    assert rel_err(out, spmmv.spmmv(c.H, x, 0.6, -0.3, 0.0)) < 1e-13


def test_sweep_is_deterministic():
    c = Case("ti", (33, 17, 9), (1, 1, 1))
    x = dev(c.block(4))
    y1 = torch.empty_like(x)
    y2 = torch.empty_like(x)
    d1 = pv.pv_spmmv(c.lat, x, y1, 1.0, 0.0, 0.0, dot_flags=7)
    d2 = pv.pv_spmmv(c.lat, x, y2, 1.0, 0.0, 0.0, dot_flags=7)
    assert torch.equal(y1, y2) and torch.equal(d1, d2)


def _explicit_matrix(L, per, no, offsets, blocks, E0, V, pot_orbital):
    """Sparse H straight from a stencil definition: (H x)[s] += B_t x[s + d_t],
    on-site block plus the field (per orbital row or per site)."""
    import scipy.sparse as sp
    from oracle import lattice as olat_mod
    ol = olat_mod.Lattice(L, per, no)
    rows, cols, vals = [], [], []
    s = np.arange(ol.n_sites)
    for o, B in zip(offsets, blocks):
        nbr, ok = ol.shift(s, o)
        for a in range(no):
            for b in range(no):
                rows.append(s[ok] * no + a)
                cols.append(nbr[ok] * no + b)
                vals.append(np.full(ok.sum(), B[a, b]))
    for a in range(no):
        for b in range(no):
            fv = (V[s * no + a] if pot_orbital else V[s]) if a == b else 0.0
            rows.append(s * no + a)
            cols.append(s * no + b)
            vals.append(np.full(s.size, E0[a, b]) + fv)
    H = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(ol.n_rows, ol.n_rows)).tocsr()
    return ol, H


def test_generic_family_random_hermitian_stencil():
    """A stencil with diagonal offsets and dense random blocks (no compiled
    family): generic kernel against the explicit matrix of the same stencil."""
    g = np.random.default_rng(11)
    offs = [(1, 0, 0), (0, 1, 0), (1, 1, 0), (1, -1, 1), (0, 0, 1)]
    no = 2
    blocks, offsets = [], []
    for o in offs:
        B = g.standard_normal((no, no)) + 1j * g.standard_normal((no, no))
        offsets += [o, tuple(-v for v in o)]
        blocks += [B, B.conj().T]
    E0 = g.standard_normal((no, no)) + 1j * g.standard_normal((no, no))
    E0 = E0 + E0.conj().T
    st = {"dim": 3, "n_orb": no, "offsets": np.array(offsets), "blocks": np.array(blocks), "onsite": E0,
          "pot_mode": pv.PV_POT_ORBITAL}
    L, per = (6, 5, 4), (1, 0, 1)
    lat = pv.Lattice(L, per, st)
    assert lat.family == 0
    V = W.uniform_potential(L[0] * L[1] * L[2] * no, 1.0, W.generator(3, 1))
    lat.set_potential(dev(V))
    ol, H = _explicit_matrix(L, per, no, offsets, blocks, E0, V, True)
    x = W.gaussian_block(ol.n_rows, 8, W.generator(3, 2))
    y = torch.empty((ol.n_rows, 8), dtype=torch.complex128, device="cuda")
    pv.pv_spmmv(lat, dev(x), y, 1.0, 0.3, 0.0)
    assert rel_err(host(y), spmmv.spmmv(H, x, 1.0, 0.3, 0.0)) < 1e-13


GENERIC_OFFSETS = {
    # a y step together with a z step: direct kernel only
    "diagonal": [(1, 0, 0), (0, 1, 0), (0, 0, 1), (0, 1, 1), (1, 0, -1)],
    # y steps alone, x and z steps combined: the staged kernel takes it too
    "stageable": [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 0, -1), (1, 0, 1)],
    # y steps with x steps (side rows with the x halo) and x with z steps
    "xy": [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, -1, 0), (1, 0, 1)],
}


@pytest.mark.parametrize("no,nb,dtype", [(4, 4, np.complex128), (4, 1, np.complex128), (1, 8, np.complex128),
                                         (4, 16, np.complex64), (2, 32, np.complex128)])
@pytest.mark.parametrize("shape", ["diagonal", "stageable", "xy"])
@pytest.mark.parametrize("kernel", [1, 2])
@pytest.mark.parametrize("per", [(1, 1, 0), (0, 0, 1)])
def test_generic_family_sparse_blocks(no, nb, dtype, shape, kernel, per):
    """Generic stencils whose blocks are mostly zero, with rows of different
    entry counts (some empty) and an on-site block with off-diagonal entries:
    the kernels walk only the nonzero entries.  Chebyshev step with dots, on
    the direct kernel and (where the offsets allow it) the staged one, with
    open and periodic x and y boundaries."""
    g = np.random.default_rng(12 + no + nb)
    offs = GENERIC_OFFSETS[shape]
    blocks, offsets = [], []
    for i, o in enumerate(offs):
        B = (g.standard_normal((no, no)) + 1j * g.standard_normal((no, no))) * (g.random((no, no)) < 0.4)
        if no > 1:
            B[i % no, :] = 0.0                       # an empty row
        offsets += [o, tuple(-v for v in o)]
        blocks += [B, B.conj().T]
    E0 = (g.standard_normal((no, no)) + 1j * g.standard_normal((no, no))) * (g.random((no, no)) < 0.5)
    E0 = E0 + E0.conj().T
    st = {"dim": 3, "n_orb": no, "offsets": np.array(offsets), "blocks": np.array(blocks), "onsite": E0,
          "pot_mode": pv.PV_POT_SITE}
    L = (7, 5, 4)
    lat = pv.Lattice(L, per, st)
    assert lat.family == 0
    code = pv.PV_C128 if dtype == np.complex128 else pv.PV_C64
    pv.pv_lattice_set_tuning(lat, code, nb, {"kernel": kernel})
    n_sites = L[0] * L[1] * L[2]
    V = W.uniform_potential(n_sites, 1.0, W.generator(4, 1))
    vdt = np.float64 if dtype == np.complex128 else np.float32
    lat.set_potential(dev(V.astype(vdt)))
    ol, H = _explicit_matrix(L, per, no, offsets, blocks, E0, V.astype(vdt).astype(np.float64), False)
    x = W.gaussian_block(ol.n_rows, nb, W.generator(4, 2), dtype)
    z = W.gaussian_block(ol.n_rows, nb, W.generator(4, 3), dtype)
    y = dev(z.copy())
    d = host(pv.pv_spmmv(lat, dev(x), y, 0.4, 0.2, -1.0, z=y, dot_flags=7))
    x64, z64 = x.astype(np.complex128), z.astype(np.complex128)
    ref = spmmv.spmmv(H, x64, 0.4, 0.2, -1.0, z64)
    tol = 1e-13 if dtype == np.complex128 else 2e-6
    assert rel_err(host(y).astype(np.complex128), ref) < tol
    xx = np.sum(np.abs(x64) ** 2, axis=0)
    assert np.abs(d[:, 0] - xx).max() < (1e-12 if dtype == np.complex128 else 1e-5) * xx.max()


@pytest.mark.parametrize("shape", ["diagonal", "stageable", "xy"])
@pytest.mark.parametrize("nb", [1, 8])
def test_generic_plain_sweep_gamma_zero(shape, nb):
    """Generic stencils, uniform coefficients and gamma = 0 on the staged
    kernel where the offsets allow it (the plain kernel without a z stream,
    with or without halo side rows): y starts as NaN and is written only."""
    g = np.random.default_rng(50 + nb)
    no = 2
    blocks, offsets = [], []
    for o in GENERIC_OFFSETS[shape]:
        B = (g.standard_normal((no, no)) + 1j * g.standard_normal((no, no))) * (g.random((no, no)) < 0.6)
        offsets += [o, tuple(-v for v in o)]
        blocks += [B, B.conj().T]
    E0 = np.array([[0.1, 0.3j], [-0.3j, -0.2]])
    st = {"dim": 3, "n_orb": no, "offsets": np.array(offsets), "blocks": np.array(blocks), "onsite": E0,
          "pot_mode": pv.PV_POT_SITE}
    L, per = (11, 6, 5), (0, 1, 1)
    lat = pv.Lattice(L, per, st)
    pv.pv_lattice_set_tuning(lat, pv.PV_C128, nb, {"kernel": 2})
    V = W.uniform_potential(L[0] * L[1] * L[2], 1.0, W.generator(6, 1))
    lat.set_potential(dev(V))
    ol, H = _explicit_matrix(L, per, no, offsets, blocks, E0, V, False)
    x = W.gaussian_block(ol.n_rows, nb, W.generator(6, 2))
    y = dev(np.full((ol.n_rows, nb), np.nan + 0j))
    pv.pv_spmmv(lat, dev(x), y, 0.8, 0.25, 0.0)
    out = host(y)
    assert np.isfinite(out).all()
    assert rel_err(out, spmmv.spmmv(H, x, 0.8, 0.25, 0.0)) < 1e-13


@pytest.mark.parametrize("kernel", [1, 2])
@pytest.mark.parametrize("shape", ["stageable", "xy"])
def test_generic_stageable_open_x_orbital_field_series(kernel, shape):
    """Staged generic path with an open x boundary, a per-orbital field and
    the series epilogue (Chebyshev series of degree 9) against the oracle's
    series on the explicit matrix."""
    from oracle import chebtp
    g = np.random.default_rng(31)
    no = 2
    offs = GENERIC_OFFSETS[shape]
    blocks, offsets = [], []
    for o in offs:
        B = (g.standard_normal((no, no)) + 1j * g.standard_normal((no, no))) * (g.random((no, no)) < 0.7)
        offsets += [o, tuple(-v for v in o)]
        blocks += [B, B.conj().T]
    E0 = np.array([[0.3, 0.2 - 0.1j], [0.2 + 0.1j, -0.4]])
    st = {"dim": 3, "n_orb": no, "offsets": np.array(offsets), "blocks": np.array(blocks), "onsite": E0,
          "pot_mode": pv.PV_POT_ORBITAL}
    L, per = (9, 4, 5), (0, 1, 1)
    lat = pv.Lattice(L, per, st)
    assert lat.family == 0
    nb = 4
    pv.pv_lattice_set_tuning(lat, pv.PV_C128, nb, {"kernel": kernel})
    V = W.uniform_potential(L[0] * L[1] * L[2] * no, 1.0, W.generator(5, 1))
    lat.set_potential(dev(V))
    ol, H = _explicit_matrix(L, per, no, offsets, blocks, E0, V, True)
    a = float(np.abs(H).sum(axis=1).max()) * 1.05
    X = W.gaussian_block(ol.n_rows, nb, W.generator(5, 2))
    coef = W.generator(5, 3).standard_normal(10) + 1j * W.generator(5, 4).standard_normal(10)
    Y = torch.empty((ol.n_rows, nb), dtype=torch.complex128, device="cuda")
    pv.pv_cheb_series(lat, dev(X), Y, a, 0.1, coef)
    assert rel_err(host(Y), chebtp.cheb_series(H, X, a, 0.1, coef)) < 1e-12


@pytest.mark.parametrize("nb,dtype", [(1, np.complex64), (2, np.complex64), (1, np.complex128)])
@pytest.mark.parametrize("per", [(1, 1, 1), (0, 1, 0)])
@pytest.mark.parametrize("kernel", [0, 2])
def test_generic_single_orbital_narrow_sites(nb, dtype, per, kernel):
    """Single-orbital generic stencil (simple-cubic hops with next-nearest x-z
    hops) with sites narrower than or equal to one 16-byte chunk: complex64
    at nb = 1 (half a chunk per site, where a staged ring row would start
    inside a chunk, so the launch takes the direct kernel even when the
    staged one is requested), complex64 at nb = 2 and complex128 at nb = 1
    (one chunk per site, staged).  Open and periodic x; Chebyshev step with
    dots against the oracle on the explicit matrix."""
    g = np.random.default_rng(70 + nb)
    no = 1
    blocks, offsets = [], []
    for o in GENERIC_OFFSETS["stageable"]:
        B = g.standard_normal((1, 1)) + 1j * g.standard_normal((1, 1))
        offsets += [o, tuple(-v for v in o)]
        blocks += [B, B.conj().T]
    E0 = np.array([[0.25]])
    st = {"dim": 3, "n_orb": no, "offsets": np.array(offsets), "blocks": np.array(blocks), "onsite": E0,
          "pot_mode": pv.PV_POT_SITE}
    L = (67, 5, 6)          # ragged: 67 sites per row
    lat = pv.Lattice(L, per, st)
    assert lat.family == 0
    code = pv.PV_C128 if dtype == np.complex128 else pv.PV_C64
    if kernel:
        pv.pv_lattice_set_tuning(lat, code, nb, {"kernel": kernel})
    V = W.uniform_potential(L[0] * L[1] * L[2], 1.0, W.generator(7, 1))
    vdt = np.float64 if dtype == np.complex128 else np.float32
    lat.set_potential(dev(V.astype(vdt)))
    ol, H = _explicit_matrix(L, per, no, offsets, blocks, E0, V.astype(vdt).astype(np.float64), False)
    x = W.gaussian_block(ol.n_rows, nb, W.generator(7, 2), dtype)
    z = W.gaussian_block(ol.n_rows, nb, W.generator(7, 3), dtype)
    y = dev(z.copy())
    pv.pv_spmmv(lat, dev(x), y, 0.4, 0.2, -1.0, z=y, dot_flags=7)
    ref = spmmv.spmmv(H, x.astype(np.complex128), 0.4, 0.2, -1.0, z.astype(np.complex128))
    tol = 1e-13 if dtype == np.complex128 else 2e-6
    assert rel_err(host(y).astype(np.complex128), ref) < tol
