"""Parity at the full benchmark size: TI 256 x 256 x 64 periodic (D =
16,777,216 rows), W = 2, the Chebyshev step with fused dots in the launch
configurations the benchmark times: the autotuner's shape (as bench.py
obtains it) and every shape whose traffic bench.py reports.

The oracle cannot assemble H at this size, so the output is checked on
sampled sites: the oracle builds the explicit rows of H for those sites, the
test gathers the x entries those rows touch from the device, and compares
alpha (H x - beta x) + gamma z there.  Sites include every face, edge and
corner of the periodic box.  The dot products are checked against the closed
form <x, x> = D of random-phase columns.  Tolerances as in the small parity
tests (complex128 1e-13, complex64 2e-6 relative to the sampled maximum)."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import bench  # noqa: E402
import paper_1708_09689_amd as pv  # noqa: E402
from oracle import hamiltonian, lattice, models  # noqa: E402
import workloads as W  # noqa: E402

L = (256, 256, 64)
A_SCALE = 7.0


def sampled_sites(olat):
    g = W.generator(2, W.STREAM_FD_SITES)
    rnd = W.sample_sites(olat.n_sites, 96, g)
    Lx, Ly, Lz = L
    corners = [x + Lx * (y + Ly * z) for x in (0, Lx - 1) for y in (0, Ly - 1) for z in (0, Lz - 1)]
    faces = [0 + Lx * (17 + Ly * 9), Lx - 1 + Lx * (200 + Ly * 33), 77 + Lx * (0 + Ly * 5),
             130 + Lx * (Ly - 1 + Ly * 40), 5 + Lx * (6 + Ly * 0), 250 + Lx * (251 + Ly * (Lz - 1))]
    # sites at column-tile and strip boundaries of the staged traversal
    tiles = [63 + Lx * (31 + Ly * 20), 64 + Lx * (32 + Ly * 21), 127 + Lx * (95 + Ly * 63), 128 + Lx * (160 + Ly * 1)]
    return np.unique(np.concatenate([rnd, corners, faces, tiles]).astype(np.int64))


def launch_shapes(dtype, nb):
    """None (the autotuner's choice) and the shapes with counted traffic."""
    return [None] + [sh for sh, _ in bench.COUNTED_TRAFFIC.get((dtype, nb), [])]


@pytest.mark.parametrize("dtype,nb,k", [("c128", 32, k) for k in range(len(launch_shapes("c128", 32)))] +
                                       [("c64", 16, k) for k in range(len(launch_shapes("c64", 16)))])
def test_fullsize_chebyshev_step_sampled(dtype, nb, k):
    dev = torch.device("cuda:0")
    c128 = dtype == "c128"
    model = models.topological_insulator(1.0, 2.0)
    olat = lattice.Lattice(L, (1, 1, 1), 4)
    V = W.uniform_potential(olat.n_sites, 2.0, W.generator(2, W.STREAM_POTENTIAL))
    lat = pv.Lattice(L, (1, 1, 1), pv.pv_model_stencil(pv.PV_MODEL_TI, [1.0, 2.0, 0.0, 0.0]))
    Vd = torch.from_numpy(V if c128 else V.astype(np.float32)).to(dev)
    lat.set_potential(Vd)
    code = pv.PV_C128 if c128 else pv.PV_C64
    shape = launch_shapes(dtype, nb)[k]
    if shape is None:
        shape, _ = pv.pv_autotune(lat, nb, code)
    else:
        pv.pv_lattice_set_tuning(lat, code, nb, shape)
    assert pv.pv_lattice_get_tuning(lat, code, nb) == {**{f: 0 for f in pv.TUNING_FIELDS}, **shape}
    tname = "complex128" if c128 else "complex64"
    x = W.random_phase_device(lat.n_rows, nb, 900 + nb, dev, tname)
    y = W.random_phase_device(lat.n_rows, nb, 901 + nb, dev, tname)
    z_sites = sampled_sites(olat)
    rows = (z_sites[:, None] * 4 + np.arange(4)[None, :]).ravel()
    z_before = y[torch.from_numpy(rows).to(dev)].cpu().numpy().astype(np.complex128)
    alpha, beta, gamma = 2.0 / A_SCALE, 0.0, -1.0
    dots = pv.pv_spmmv(lat, x, y, alpha, beta, gamma, z=y, dot_flags=pv.PV_DOT_XX | pv.PV_DOT_XY)
    torch.cuda.synchronize()
    Vq = V if c128 else V.astype(np.float32).astype(np.float64)
    Hs = hamiltonian.rows_of_sites(model, olat, Vq, z_sites).tocsr()
    cols = np.unique(Hs.indices)
    xg = x[torch.from_numpy(cols).to(dev)].cpu().numpy().astype(np.complex128)
    Hc = Hs[:, cols]
    xs = x[torch.from_numpy(rows).to(dev)].cpu().numpy().astype(np.complex128)
    ref = alpha * (Hc @ xg - beta * xs) + gamma * z_before
    out = y[torch.from_numpy(rows).to(dev)].cpu().numpy().astype(np.complex128)
    tol = 1e-13 if c128 else 2e-6
    assert np.abs(out - ref).max() < tol * np.abs(ref).max()
    d = dots.cpu().numpy()
    assert np.abs(d[:, 0] - lat.n_rows).max() < (1e-12 if c128 else 1e-6) * lat.n_rows
