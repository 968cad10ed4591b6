"""On-the-fly disorder: the sweep kernels generate the on-site field from the
counter-based generator instead of reading it.  Parity against the oracle
with the oracle's own implementation of the same generator (oracle.rng), and
bitwise agreement with the same field passed as a stored array (the field
values are one rounded product on both sides).  Tolerances as in the sweep,
KPM, batch and adjoint parity tests."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1708_09689_amd as pv  # noqa: E402
from oracle import adjoint, hamiltonian, kpm, rng, spmmv  # noqa: E402
import workloads as W  # noqa: E402

from gpu_common import Case, dev, host, rel_err, SHAPE_KINDS, shape  # noqa: E402

SEED = 0x5EED_1708


def rng_case(name, L, periodic, Wd, seed=SEED):
    c = Case(name, L, periodic, with_field=False)
    n = c.olat.n_sites if c.model.pot == "site" else c.olat.n_rows
    c.V = rng.field(seed, Wd, n)
    c.H = hamiltonian.assemble(c.model, c.olat, c.V)
    c.lat.set_random_potential(seed, Wd)
    return c


@pytest.mark.parametrize("name,L,periodic", [
    ("ti", (37, 9, 6), (1, 1, 1)),
    ("ti", (12, 7, 5), (0, 1, 0)),
    ("graphene2", (70, 9), (0, 1)),
    ("graphene4", (21, 10), (1, 1)),      # per-orbital field
    ("weyl", (19, 6, 5), (1, 1, 0)),
])
@pytest.mark.parametrize("kernel", SHAPE_KINDS)
def test_sweep_with_generated_field(name, L, periodic, kernel):
    nb = 4
    c = rng_case(name, L, periodic, 2.0)
    pv.pv_lattice_set_tuning(c.lat, pv.PV_C128, nb, shape(kernel))
    x = c.block(nb, seed=1)
    z = c.block(nb, seed=2)
    y = dev(z.copy())
    pv.pv_spmmv(c.lat, dev(x), y, 0.3, 0.1, -1.0, z=y)
    ref = spmmv.spmmv(c.H, x, 0.3, 0.1, -1.0, z)
    assert rel_err(host(y), ref) < 1e-13
    # the same field as a stored array gives the same bits
    y2 = dev(z.copy())
    c.lat.set_potential(dev(c.V))
    pv.pv_spmmv(c.lat, dev(x), y2, 0.3, 0.1, -1.0, z=y2)
    assert np.array_equal(host(y), host(y2))


def test_generated_field_c64():
    c = rng_case("ti", (24, 10, 6), (1, 1, 1), 1.5)
    x = c.block(8, seed=3, dtype=np.complex64)
    y = torch.empty((c.D, 8), dtype=torch.complex64, device="cuda")
    pv.pv_spmmv(c.lat, dev(x), y, 0.25, 0.0, 0.0)
    ref = spmmv.spmmv(c.H, x.astype(np.complex128), 0.25, 0.0, 0.0)
    assert rel_err(host(y).astype(np.complex128), ref) < 2e-6


def test_kpm_and_batch_with_generated_fields():
    cases = [rng_case("ti", L, (1, 1, 1), Wd, seed=SEED + i)
             for i, (L, Wd) in enumerate([((6, 5, 4), 1.0), ((8, 8, 8), 2.5), ((5, 7, 3), 0.5)])]
    rs = [c.block(2, seed=10 + i, kind="phase") for i, c in enumerate(cases)]
    for c, r in zip(cases, rs):
        mu = host(pv.pv_kpm_moments(c.lat, dev(r), 48, 7.0, 0.0))
        assert np.abs(mu - kpm.moments_doubling(c.H, r, 48, 7.0, 0.0)).max() < 1e-12
    batch = pv.Batch([c.lat for c in cases])
    mu = host(pv.pv_batch_kpm_moments(batch, [dev(r) for r in rs], 48, 7.0, 0.0))
    for i, c in enumerate(cases):
        assert np.abs(mu[i] - kpm.moments_doubling(c.H, rs[i], 48, 7.0, 0.0)).max() < 1e-12


def test_gradient_with_generated_field():
    c = rng_case("ti", (5, 4, 4), (1, 1, 1), 1.0)
    r = c.block(2, kind="phase")
    gbar = W.generator(9, W.STREAM_COTANGENT).standard_normal((2, 32))
    g = host(pv.pv_kpm_moments_vjp(c.lat, dev(r), 32, 7.0, 0.0, dev(gbar), ckpt_every=8))
    ref = adjoint.kpm_vjp(c.H, 4, "site", r, 32, 7.0, 0.0, gbar)
    assert np.abs(g - ref).max() < 1e-10 * np.abs(ref).max()


def test_dsl_program_end_to_end():
    """A DSL program with random per-site coefficients (the Weyl model file of
    the DSL tests) drives the KPM on the GPU with the on-the-fly field."""
    import os
    from oracle import lattice, models
    text = open(os.path.join(os.path.dirname(__file__), "golden", "dsl", "weyl.dsl")).read()
    st = pv.pv_dsl_stencil(text)
    assert st["field"] == 2
    L = (10, 6, 5)
    lat = pv.Lattice(L, (1, 1, 0), st)
    lat.set_random_potential(SEED + 7, 1.5)
    olat = lattice.Lattice(L, (1, 1, 0), 2)
    H = hamiltonian.assemble(models.weyl_semimetal(), olat, rng.field(SEED + 7, 1.5, olat.n_sites))
    r = W.random_phase_block(olat.n_rows, 4, W.generator(7, W.STREAM_VECTORS))
    mu = host(pv.pv_kpm_moments(lat, dev(r), 64, 7.5, 0.0))
    assert np.abs(mu - kpm.moments_doubling(H, r, 64, 7.5, 0.0)).max() < 1e-12
