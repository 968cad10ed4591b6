"""GPU parity of the batched, graph-captured KPM over ragged disorder
realisations: every instance equals its own oracle run (complex128 to 1e-12,
complex64 vectors with FP64 dots to 1e-4), the graph is captured once and
replayed, and replays are bitwise identical."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1708_09689_amd as pv  # noqa: E402
from oracle import kpm  # noqa: E402
import workloads as W  # noqa: E402

from gpu_common import Case, dev, host  # noqa: E402


def instances(dtype=np.complex128, vdtype=np.float64, nb=4):
    sizes = [(3, 4, 5), (5, 5, 5), (8, 3, 6), (6, 7, 4), (9, 9, 9), (2, 2, 2)]
    cases, rs = [], []
    for i, L in enumerate(sizes):
        c = Case("ti", L, (1, 1, 1), Wd=0.5 + 0.5 * i, seed=30 + i, vdtype=vdtype)
        cases.append(c)
        rs.append(c.block(nb, seed=40 + i, kind="phase", dtype=dtype))
    a = np.array([7.0, 7.5, 8.0, 7.0, 9.0, 7.2])
    b = np.array([0.0, 0.1, -0.2, 0.05, 0.0, 0.3])
    return cases, rs, a, b


def test_batched_kpm_c128_matches_each_instance_and_replays():
    cases, rs, a, b = instances()
    batch = pv.Batch([c.lat for c in cases])
    rd = [dev(r) for r in rs]
    mu1 = host(pv.pv_batch_kpm_moments(batch, rd, 64, a, b)).copy()
    for i, c in enumerate(cases):
        ref = kpm.moments_doubling(c.H, rs[i], 64, a[i], b[i])
        assert np.abs(mu1[i] - ref).max() < 1e-12, i
    mu2 = host(pv.pv_batch_kpm_moments(batch, rd, 64, a, b))
    assert np.array_equal(mu1, mu2)
    assert batch.stats() == (1, 1)
    # the output buffer may move between calls without a new capture
    keep = [torch.empty(n, device="cuda") for n in (1000, 3000)]
    out = torch.full((len(cases), 4, 64), np.nan, dtype=torch.float64, device="cuda")
    pv.pv_batch_kpm_moments(batch, rd, 64, a, b, mu=out)
    assert np.array_equal(mu1, host(out))
    assert batch.stats() == (1, 2)
    del keep
    # a different start block pointer forces a new capture
    rd[2] = dev(rs[2] * 1.0)
    mu3 = host(pv.pv_batch_kpm_moments(batch, rd, 64, a, b))
    assert np.array_equal(mu1, mu3)
    assert batch.stats() == (2, 2)


@pytest.mark.parametrize("M", [2, 6, 10])
def test_batched_kpm_short_runs(M):
    """One step (only the final reduction) and odd step counts (the last
    step's partials in the other buffer of the pair): every instance equals
    its oracle run."""
    cases, rs, a, b = instances(nb=2)
    batch = pv.Batch([c.lat for c in cases])
    mu = host(pv.pv_batch_kpm_moments(batch, [dev(r) for r in rs], M, a, b))
    for i, c in enumerate(cases):
        ref = kpm.moments_doubling(c.H, rs[i], M, a[i], b[i])
        assert np.abs(mu[i] - ref).max() < 1e-12, (M, i)


def test_batched_kpm_c64_stated_error():
    cases, rs, a, b = instances(np.complex64, np.float32, nb=16)
    batch = pv.Batch([c.lat for c in cases])
    mu = host(pv.pv_batch_kpm_moments(batch, [dev(r) for r in rs], 128, a, b))
    import oracle.hamiltonian as oh
    for i, c in enumerate(cases):
        Hq = oh.assemble(c.model, c.olat, c.V.astype(np.float32).astype(np.float64))
        ref = kpm.moments_doubling(Hq, rs[i].astype(np.complex128), 128, a[i], b[i])
        assert np.abs(mu[i] - ref).max() < 1e-4, i


def test_batched_equals_single_lattice_path():
    cases, rs, a, b = instances(nb=2)
    batch = pv.Batch([c.lat for c in cases])
    rd = [dev(r) for r in rs]
    mu = host(pv.pv_batch_kpm_moments(batch, rd, 32, a, b))
    for i, c in enumerate(cases):
        single = host(pv.pv_kpm_moments(c.lat, rd[i], 32, a[i], b[i]))
        assert np.abs(mu[i] - single).max() < 1e-14


@pytest.mark.parametrize("dtype", [np.complex128, np.complex64])
def test_batched_direct_and_staged_kernels_agree(dtype):
    """Lattice 0's tuning selects the kernel of the whole batch; both give the
    same moments up to the summation order of the dots."""
    vd = np.float64 if dtype == np.complex128 else np.float32
    cases, rs, a, b = instances(dtype, vd, nb=8)
    code = pv.PV_C128 if dtype == np.complex128 else pv.PV_C64
    batch = pv.Batch([c.lat for c in cases])
    rd = [dev(r) for r in rs]
    pv.pv_lattice_set_tuning(cases[0].lat, code, 8, {"kernel": 2})
    mu_s = host(pv.pv_batch_kpm_moments(batch, rd, 48, a, b)).copy()
    pv.pv_lattice_set_tuning(cases[0].lat, code, 8, {"kernel": 1})
    mu_d = host(pv.pv_batch_kpm_moments(batch, rd, 48, a, b)).copy()
    pv.pv_lattice_set_tuning(cases[0].lat, code, 8, None)
    assert batch.stats()[0] == 2          # the kernel change forced a new capture
    tol = 1e-13 if dtype == np.complex128 else 1e-6
    assert np.abs(mu_s - mu_d).max() < tol


@pytest.mark.parametrize("dtype,elems", [(np.complex128, 1), (np.complex128, 2),
                                         (np.complex64, 2), (np.complex64, 4)])
def test_batched_staged_elements_per_lane(dtype, elems):
    """Lattice 0's elements per lane set the staged tile length of the whole
    batch: every instance equals its oracle run (complex64 vectors and field
    against the oracle on the FP32-rounded field, to the stated 1e-4)."""
    vd = np.float64 if dtype == np.complex128 else np.float32
    cases, rs, a, b = instances(dtype, vd, nb=16)
    code = pv.PV_C128 if dtype == np.complex128 else pv.PV_C64
    batch = pv.Batch([c.lat for c in cases])
    pv.pv_lattice_set_tuning(cases[0].lat, code, 16, {"kernel": 2, "elems_per_lane": elems})
    try:
        mu = host(pv.pv_batch_kpm_moments(batch, [dev(r) for r in rs], 40, a, b))
    finally:
        pv.pv_lattice_set_tuning(cases[0].lat, code, 16, None)
    import oracle.hamiltonian as oh
    for i, c in enumerate(cases):
        H = c.H if dtype == np.complex128 else oh.assemble(c.model, c.olat, c.V.astype(np.float32).astype(np.float64))
        ref = kpm.moments_doubling(H, rs[i].astype(np.complex128), 40, a[i], b[i])
        tol = 1e-12 if dtype == np.complex128 else 1e-4
        assert np.abs(mu[i] - ref).max() < tol, (elems, i)


@pytest.mark.parametrize("dtype,elems,wg", [(np.complex128, 1, 512), (np.complex128, 2, 512), (np.complex128, 2, 0),
                                            (np.complex64, 2, 512), (np.complex64, 4, 512), (np.complex64, 4, 0)])
def test_batch_shape_set_on_the_batch(dtype, elems, wg):
    """A shape set on the batch (pv_batch_set_tuning), 256- or 512-lane
    workgroups, serves every instance: each equals its oracle run (complex64
    to the stated 1e-4 on the FP32-rounded field), and lattice 0's own
    tuning no longer matters."""
    vd = np.float64 if dtype == np.complex128 else np.float32
    cases, rs, a, b = instances(dtype, vd, nb=16)
    code = pv.PV_C128 if dtype == np.complex128 else pv.PV_C64
    batch = pv.Batch([c.lat for c in cases])
    shape = {"kernel": 2, "elems_per_lane": elems, "workgroup_size": wg}
    pv.pv_batch_set_tuning(batch, code, 16, shape)
    assert {k: v for k, v in pv.pv_batch_get_tuning(batch, code, 16).items() if v} == \
        {k: v for k, v in shape.items() if v}
    pv.pv_lattice_set_tuning(cases[0].lat, code, 16, {"kernel": 1})    # ignored by the batch
    try:
        mu = host(pv.pv_batch_kpm_moments(batch, [dev(r) for r in rs], 40, a, b))
    finally:
        pv.pv_lattice_set_tuning(cases[0].lat, code, 16, None)
    import oracle.hamiltonian as oh
    for i, c in enumerate(cases):
        H = c.H if dtype == np.complex128 else oh.assemble(c.model, c.olat, c.V.astype(np.float32).astype(np.float64))
        ref = kpm.moments_doubling(H, rs[i].astype(np.complex128), 40, a[i], b[i])
        tol = 1e-12 if dtype == np.complex128 else 1e-4
        assert np.abs(mu[i] - ref).max() < tol, (elems, wg, i)


def test_batch_autotune_picks_a_candidate_and_keeps_results():
    """pv_batch_autotune times the batch's candidate shapes on its own steps,
    keeps the fastest, and the batch then gives the same moments as with the
    direct kernel (to the dots' summation order)."""
    cases, rs, a, b = instances(nb=8)
    batch = pv.Batch([c.lat for c in cases])
    rd = [dev(r) for r in rs]
    pv.pv_batch_set_tuning(batch, pv.PV_C128, 8, {"kernel": 1})
    mu_d = host(pv.pv_batch_kpm_moments(batch, rd, 32, a, b)).copy()
    shape, ms = pv.pv_batch_autotune(batch, rd, a, b)
    assert ms > 0.0
    assert shape["kernel"] in (1, 2) and shape["workgroup_size"] in (0, 512)
    assert pv.pv_batch_get_tuning(batch, pv.PV_C128, 8) == shape
    mu_t = host(pv.pv_batch_kpm_moments(batch, rd, 32, a, b))
    assert np.abs(mu_t - mu_d).max() < 1e-13
    pv.pv_batch_set_tuning(batch, pv.PV_C128, 8, None)
    assert pv.pv_batch_get_tuning(batch, pv.PV_C128, 8)["workgroup_size"] == 0
