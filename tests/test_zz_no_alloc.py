"""The allocation-free sweep (pv_spmmv_noalloc) against pv_spmmv, through the
C ABI: two calls in a row on one GPU's static scratch, the second with a
smaller block, each compared with pv_spmmv on the same inputs (bitwise: the
same kernels in the same launch shapes) and with the oracle (complex128,
1e-13 relative to max|y|; dots 1e-12 relative)."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1708_09689_amd as pv  # noqa: E402
from oracle import spmmv  # noqa: E402
import workloads as W  # noqa: E402

from gpu_common import Case, dev, host, rel_err  # noqa: E402


def _both(c, nb, alpha, beta, gamma, seed):
    x = c.block(nb, seed=seed)
    z = c.block(nb, seed=seed + 1)
    # reference: pv_spmmv with a workspace (y starts as z: in-place recurrence)
    y_ref = dev(z.copy())
    d_ref = pv.pv_spmmv(c.lat, dev(x), y_ref, alpha, beta, gamma, z=y_ref, dot_flags=7)
    # allocation-free call; y starts as z, dots start as NaN (every entry written)
    y = dev(z.copy())
    dots = torch.full((nb, 4), float("nan"), dtype=torch.float64, device="cuda")
    pv.pv_spmmv_noalloc(c.lat, dev(x), y, alpha, beta, gamma, z=y, dot_flags=7, dots=dots)
    ref = spmmv.spmmv(c.H, x, np.broadcast_to(alpha, (nb,)), np.broadcast_to(beta, (nb,)),
                      np.broadcast_to(gamma, (nb,)), z)
    return host(y), host(dots), host(y_ref), host(d_ref), ref, x


def test_noalloc_sweep_matches_pv_spmmv_two_calls():
    # first call: a block of 2^22 elements (staged kernel, 512-lane shape by
    # default for c128 is not forced: whatever pv_spmmv takes, both take)
    big = Case("ti", (64, 32, 32), (1, 1, 1), Wd=2.0, seed=3)
    pv.pv_spmmv(big.lat, dev(big.block(8, seed=9)), torch.empty((big.D, 8), dtype=torch.complex128, device="cuda"),
                1.0, 0.0, 0.0)   # creates the lattice's device tables (the only allocation)
    y, d, y_ref, d_ref, ref, x = _both(big, 8, 2.0 / 7.0, 0.1, -1.0, 11)
    assert np.array_equal(y, y_ref)
    assert np.array_equal(d, d_ref)
    assert rel_err(y, ref) < 1e-13
    xx = np.sum(np.abs(x) ** 2, axis=0)
    assert np.abs(d[:, 0] - xx).max() < 1e-12 * xx.max()
    assert np.abs(d[:, 3] - np.sum(np.abs(ref) ** 2, axis=0)).max() < 1e-12 * xx.max() * 10

    # second call, smaller block, per-column scales (scratch holds the table)
    small = Case("ti", (9, 7, 5), (1, 0, 1), Wd=1.0, seed=4)
    pv.pv_spmmv(small.lat, dev(small.block(4, seed=2)),
                torch.empty((small.D, 4), dtype=torch.complex128, device="cuda"), 1.0, 0.0, 0.0)
    g = W.generator(8, 7, 4)
    alpha, beta, gamma = 0.5 + g.random(4), g.standard_normal(4), g.standard_normal(4)
    y, d, y_ref, d_ref, ref, x = _both(small, 4, alpha, beta, gamma, 21)
    assert np.array_equal(y, y_ref)
    assert np.array_equal(d, d_ref)
    assert rel_err(y, ref) < 1e-13
    assert np.isfinite(d).all()


def test_noalloc_sweep_needs_device_tables_and_bounds_scratch():
    c = Case("ti", (6, 5, 4), (1, 1, 1), Wd=1.0, seed=5)   # no sweep has run on this lattice
    x = dev(c.block(2, seed=1))
    y = torch.empty_like(x)
    with pytest.raises(pv.PvError) as e:
        pv.pv_spmmv_noalloc(c.lat, x, y, 1.0, 0.0, 0.0)
    assert e.value.status == 1
    assert b"no device tables" in pv.lib().pv_last_error()
    # after one other sweep the same call runs
    pv.pv_spmmv(c.lat, x, torch.empty_like(x), 1.0, 0.0, 0.0)
    pv.pv_spmmv_noalloc(c.lat, x, y, 1.0, 0.0, 0.0)
    assert rel_err(host(y), spmmv.spmmv(c.H, host(x), 1.0, 0.0, 0.0)) < 1e-13


def _generic_case(seed, L, per):
    """A two-orbital generic stencil (no built-in family) with diagonal hops,
    its lattice with a site field, and the oracle's explicit matrix."""
    from test_gpu_sweep import _explicit_matrix
    g = np.random.default_rng(seed)
    offsets, blocks = [], []
    for o in [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (0, 1, -1)]:
        B = (g.standard_normal((2, 2)) + 1j * g.standard_normal((2, 2))) * (g.random((2, 2)) < 0.7)
        offsets += [o, tuple(-v for v in o)]
        blocks += [B, B.conj().T]
    E0 = np.array([[0.2, 0.1 - 0.3j], [0.1 + 0.3j, -0.4]])
    st = {"dim": 3, "n_orb": 2, "offsets": np.array(offsets), "blocks": np.array(blocks), "onsite": E0,
          "pot_mode": pv.PV_POT_SITE}
    lat = pv.Lattice(L, per, st)
    assert lat.family == 0 and pv.pv_lattice_get_codegen(lat)
    V = W.uniform_potential(int(np.prod(L)), 1.0, W.generator(seed, 1))
    lat.set_potential(dev(V))
    _, H = _explicit_matrix(L, per, 2, offsets, blocks, E0, V, False)
    return lat, H


def test_noalloc_generic_stencil_takes_loaded_generated_kernels_only():
    """Generic stencils: the allocation-free sweep takes a generated kernel
    only when an earlier call on the GPU loaded that instance (bitwise equal
    to pv_spmmv then), else the interpreted kernel (same result up to the
    summation order), and never compiles."""
    nb = 4
    lat, H = _generic_case(41, (12, 6, 5), (1, 1, 0))
    D = H.shape[0]
    x = W.gaussian_block(D, nb, W.generator(41, 2))
    z = W.gaussian_block(D, nb, W.generator(41, 3))
    ref = spmmv.spmmv(H, x, 0.3, 0.2, -1.0, z)
    # loaded: pv_spmmv with the same arguments first (compiles the instance)
    n0 = pv.pv_codegen_instances()
    y_ref = dev(z.copy())
    d_ref = pv.pv_spmmv(lat, dev(x), y_ref, 0.3, 0.2, -1.0, z=y_ref, dot_flags=7)
    assert pv.pv_codegen_instances() == n0 + 1
    y = dev(z.copy())
    dots = torch.full((nb, 4), float("nan"), dtype=torch.float64, device="cuda")
    pv.pv_spmmv_noalloc(lat, dev(x), y, 0.3, 0.2, -1.0, z=y, dot_flags=7, dots=dots)
    assert pv.pv_codegen_instances() == n0 + 1
    assert np.array_equal(host(y), host(y_ref))
    assert np.array_equal(host(dots), host(d_ref))
    assert rel_err(host(y), ref) < 1e-13
    # not loaded: another pattern whose only earlier sweep had another epilogue
    lat2, H2 = _generic_case(43, (9, 7, 6), (0, 1, 1))
    D2 = H2.shape[0]
    x2 = W.gaussian_block(D2, nb, W.generator(43, 2))
    z2 = W.gaussian_block(D2, nb, W.generator(43, 3))
    pv.pv_spmmv(lat2, dev(x2), torch.empty((D2, nb), dtype=torch.complex128, device="cuda"), 1.0, 0.0, 0.0)
    y2 = dev(z2.copy())
    n1 = pv.pv_codegen_instances()
    pv.pv_spmmv_noalloc(lat2, dev(x2), y2, 0.3, 0.2, -1.0, z=y2, dot_flags=7, dots=dots)
    assert pv.pv_codegen_instances() == n1   # nothing compiled
    assert rel_err(host(y2), spmmv.spmmv(H2, x2, 0.3, 0.2, -1.0, z2)) < 1e-13
    assert np.isfinite(host(dots)).all()
