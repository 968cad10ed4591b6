"""Launch shapes of the sweep (direct / staged kernels, elements per lane,
lanes per workgroup, strip, walk and workgroup counts) and the autotuner.

Every shape runs the same per-element arithmetic (the stencil slots in the
same order), so y is bitwise identical across shapes; the fused dot products
differ only in summation order (1e-12 relative).  complex128 results are also
checked against the oracle (1e-13 relative to max|y|)."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1708_09689_amd as pv  # noqa: E402
from oracle import chebtp, spmmv  # noqa: E402
import workloads as W  # noqa: E402

from gpu_common import Case, dev, host, rel_err  # noqa: E402

SHAPES_C128 = [
    {"kernel": 1},
    {"kernel": 1, "tiles_per_group": 64, "slab_rows": 1},
    {"kernel": 2, "elems_per_lane": 1},
    {"kernel": 2, "elems_per_lane": 2},
    {"kernel": 2, "elems_per_lane": 1, "strip_rows": 3, "walk_planes": 2, "groups_per_xcd": 5},
    {"kernel": 2, "elems_per_lane": 2, "strip_rows": 1, "walk_planes": 1, "groups_per_xcd": 1},
    {"kernel": 2, "elems_per_lane": 2, "workgroup_size": 512},
    {"kernel": 2, "elems_per_lane": 1, "workgroup_size": 512, "strip_rows": 3, "walk_planes": 2, "groups_per_xcd": 5},
]
SHAPES_C64 = [
    {"kernel": 1},
    {"kernel": 2, "elems_per_lane": 2},
    {"kernel": 2, "elems_per_lane": 4},
    {"kernel": 2, "elems_per_lane": 2, "strip_rows": 5, "walk_planes": 3, "groups_per_xcd": 3},
    {"kernel": 2, "elems_per_lane": 4, "workgroup_size": 512},
    {"kernel": 2, "elems_per_lane": 2, "workgroup_size": 512, "groups_per_xcd": 3},
]

CASES = [
    ("ti", (37, 5, 4), (1, 1, 1)),
    ("ti", (9, 11, 6), (0, 0, 1)),
    ("ti", (3, 1, 2), (1, 1, 1)),
    ("graphene2", (70, 9), (0, 1)),
    ("graphene2", (33, 17), (1, 0)),
    ("graphene4", (21, 10), (1, 1)),
    ("weyl", (19, 6, 5), (1, 1, 0)),
]


def run_shapes(c, shapes, dtype, nb, x, z, alpha, beta, gamma):
    outs, dots = [], []
    for sh in shapes:
        pv.pv_lattice_set_tuning(c.lat, dtype, nb, sh)
        y = z.clone()
        d = pv.pv_spmmv(c.lat, x, y, alpha, beta, gamma, z=y, dot_flags=7)
        outs.append(host(y))
        dots.append(host(d))
    pv.pv_lattice_set_tuning(c.lat, dtype, nb, None)
    return outs, dots


@pytest.mark.parametrize("name,L,periodic", CASES)
@pytest.mark.parametrize("nb", [1, 4, 16])
def test_shapes_c128_identical_and_match_oracle(name, L, periodic, nb):
    c = Case(name, L, periodic, Wd=2.0, seed=nb + 3)
    x = c.block(nb, seed=1)
    z = c.block(nb, seed=2)
    g = W.generator(6, 7, nb)
    alpha, beta, gamma = 0.5 + g.random(nb), g.standard_normal(nb), g.standard_normal(nb)
    outs, dots = run_shapes(c, SHAPES_C128, pv.PV_C128, nb, dev(x), dev(z), alpha, beta, gamma)
    ref = spmmv.spmmv(c.H, x, alpha, beta, gamma, z)
    assert rel_err(outs[0], ref) < 1e-13
    for o, d in zip(outs[1:], dots[1:]):
        assert np.array_equal(o, outs[0])
        assert np.abs(d - dots[0]).max() <= 1e-12 * np.abs(dots[0]).max()


@pytest.mark.parametrize("name,L,periodic", CASES)
@pytest.mark.parametrize("nb", [4, 16])
def test_shapes_c128_uniform_coefficients(name, L, periodic, nb):
    """Uniform alpha, beta, gamma take the specialised epilogues (per-column
    ones take the run-time epilogue): every shape gives the same y as the
    direct kernel, which matches the oracle, and dots within rounding."""
    c = Case(name, L, periodic, Wd=2.0, seed=nb + 11)
    x = c.block(nb, seed=3)
    z = c.block(nb, seed=4)
    outs, dots = run_shapes(c, SHAPES_C128, pv.PV_C128, nb, dev(x), dev(z), 0.7, -0.2, -1.0)
    ref = spmmv.spmmv(c.H, x, 0.7, -0.2, -1.0, z)
    assert rel_err(outs[0], ref) < 1e-13
    dref = np.stack([np.einsum("ij,ij->j", x.conj(), x).real, (x.conj() * ref).sum(0).real,
                     (x.conj() * ref).sum(0).imag, np.einsum("ij,ij->j", ref.conj(), ref).real], axis=1)
    for o, d in zip(outs, dots):
        assert np.array_equal(o, outs[0])
        assert np.abs(d - dref).max() <= 1e-11 * np.abs(dref).max()


@pytest.mark.parametrize("name,L,periodic", CASES)
@pytest.mark.parametrize("nb", [1, 8])
def test_shapes_c64_identical(name, L, periodic, nb):
    c = Case(name, L, periodic, Wd=2.0, seed=nb + 5, vdtype=np.float32)
    x = c.block(nb, seed=1, dtype=np.complex64)
    z = c.block(nb, seed=2, dtype=np.complex64)
    outs, dots = run_shapes(c, SHAPES_C64, pv.PV_C64, nb, dev(x), dev(z), 0.3, 0.1, -1.0)
    for o, d in zip(outs[1:], dots[1:]):
        assert np.array_equal(o, outs[0])
        assert np.abs(d - dots[0]).max() <= 1e-10 * np.abs(dots[0]).max()


def test_misaligned_block_falls_back_to_direct():
    """A complex64 block at an 8-byte offset cannot take the staged kernel's
    16-byte chunk loads; the sweep still matches the aligned result."""
    c = Case("ti", (10, 4, 3), (1, 1, 1), Wd=1.0, vdtype=np.float32)
    x = c.block(1, dtype=np.complex64)
    buf = torch.zeros(c.D + 1, dtype=torch.complex64, device="cuda")
    buf[1:] = dev(x)[:, 0]
    xs = buf[1:]
    assert xs.data_ptr() % 16 == 8
    y1 = torch.empty(c.D, dtype=torch.complex64, device="cuda")
    y2 = torch.empty(c.D, dtype=torch.complex64, device="cuda")
    pv.pv_spmmv(c.lat, xs, y1, 0.5, 0.0, 0.0, nb=1)
    pv.pv_spmmv(c.lat, dev(x), y2, 0.5, 0.0, 0.0, nb=1)
    assert np.array_equal(host(y1), host(y2))


def test_autotune_applies_and_caches(tmp_path):
    cache = tmp_path / "tune.jsonl"
    c = Case("ti", (24, 24, 16), (1, 1, 1), Wd=1.0)
    shape, ms = pv.pv_autotune(c.lat, 4, pv.PV_C128, cache_path=str(cache))
    assert ms > 0.0
    assert shape == pv.pv_lattice_get_tuning(c.lat, pv.PV_C128, 4)
    assert shape["kernel"] in (1, 2)
    lines = cache.read_text().strip().splitlines()
    assert len(lines) == 1 and '"key": "family=1 orb=4 L=24x24x16' in lines[0]
    assert '"acc_kernel": ' in lines[0]          # the series step's own shape
    # a fresh lattice of the same shape takes the cached entry without timing
    c2 = Case("ti", (24, 24, 16), (1, 1, 1), Wd=1.0)
    shape2, ms2 = pv.pv_autotune(c2.lat, 4, pv.PV_C128, cache_path=str(cache))
    assert ms2 == 0.0 and shape2 == shape
    assert len(cache.read_text().strip().splitlines()) == 1
    # the tuned lattice still computes the oracle's sweep
    x = c2.block(4)
    y = torch.empty((c2.D, 4), dtype=torch.complex128, device="cuda")
    pv.pv_spmmv(c2.lat, dev(x), y, 0.25, 0.0, 0.0)
    assert rel_err(host(y), spmmv.spmmv(c2.H, x, 0.25, 0.0, 0.0)) < 1e-13
    # and the oracle's Chebyshev series through the series step's shape
    g = W.generator(8, 2, 4)
    coef = g.standard_normal(12) + 1j * g.standard_normal(12)
    pv.pv_cheb_series(c2.lat, dev(x), y, 7.0, 0.1, coef)
    assert rel_err(host(y), chebtp.cheb_series(c2.H, x, 7.0, 0.1, coef)) < 1e-12


def test_concurrent_host_threads():
    """Four host threads, each with its own lattice, stream and block width,
    sweep at the same time (the launchers' one-time set-up is shared): every
    result equals the one computed alone."""
    import threading
    cases = [("ti", (20, 9, 6), (1, 1, 1), 4), ("ti", (17, 8, 7), (1, 0, 1), 16),
             ("weyl", (11, 6, 5), (1, 1, 0), 8), ("graphene2", (40, 12), (0, 1), 2)]
    setups = []
    for i, (name, L, per, nb) in enumerate(cases):
        c = Case(name, L, per, Wd=1.0, seed=40 + i)
        setups.append((c, nb, dev(c.block(nb, seed=1)), dev(c.block(nb, seed=2))))

    def run(c, nb, x, z):
        y = z.clone()
        d = pv.pv_spmmv(c.lat, x, y, 0.3, 0.1, -1.0, z=y, dot_flags=3)
        torch.cuda.current_stream().synchronize()
        return host(y), host(d)

    alone = [run(*s) for s in setups]
    out = [None] * len(setups)
    errs = []

    def worker(k):
        try:
            with torch.cuda.stream(torch.cuda.Stream()):
                for _ in range(5):
                    out[k] = run(*setups[k])
        except Exception as e:  # reported below
            errs.append(e)

    threads = [threading.Thread(target=worker, args=(k,)) for k in range(len(setups))]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errs, errs
    for (y0, d0), (y1, d1) in zip(alone, out):
        assert np.array_equal(y0, y1)
        assert np.array_equal(d0, d1)
