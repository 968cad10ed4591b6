"""GPU parity of the generated stencil kernels (Sec. 3.2: kernels generated
from a stencil's own block structure, compiled at run time) against the
oracle on the explicit matrix of the same stencil, and against the
interpreted generic kernels.

Stencils: the TI plus next-nearest-neighbour hops -(t'/2) G1 (t' = 0.1)
along (+-1, 0, +-1), along (+-1, +-1, 0) (halo side rows), along
(0, +-1, +-1) (y steps with z steps: side rows at w -+ 1 as well) and along
+-(1, 1, 1) with +-(1, -1, 0) (both), and a 2D two-orbital stencil with
complex blocks and diagonal hops.  The staged kernel takes all of them on
the generated path; the interpreted generic path stages only the first two.

Tolerances: complex128 1e-13 relative to max|y| (the generated kernels sum a
row's terms in slot order, the oracle in matrix order); complex64 vectors
2e-6 relative (FP32 stencil arithmetic, as for the built-in families)."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1708_09689_amd as pv  # noqa: E402
from oracle import chebtp, kpm, spmmv  # noqa: E402
import workloads as W  # noqa: E402

from gpu_common import dev, host, rel_err  # noqa: E402
from test_gpu_sweep import _explicit_matrix  # noqa: E402

G1 = np.diag([1.0, 1.0, -1.0, -1.0]).astype(np.complex128)
NNN = {
    "xz": [(1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1)],
    "xy": [(1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0)],
    "yz": [(0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)],
    "xyz": [(1, 1, 1), (-1, -1, -1), (1, -1, 0), (-1, 1, 0)],
}


def stencil(name):
    """(stencil dict, offsets, blocks, on-site block) of a test stencil."""
    if name == "2d":
        g = np.random.default_rng(17)
        offsets, blocks = [], []
        for o in [(1, 0, 0), (0, 1, 0), (1, 1, 0), (1, -1, 0)]:
            B = (g.standard_normal((2, 2)) + 1j * g.standard_normal((2, 2))) * np.array([[1, 0], [1, 1]])
            offsets += [o, tuple(-v for v in o)]
            blocks += [B, B.conj().T]
        E0 = np.array([[0.3, 0.2 - 0.5j], [0.2 + 0.5j, -0.1]])
        dim, no = 2, 2
    else:
        ti = pv.pv_model_stencil(pv.PV_MODEL_TI, [1.0, 2.0, 0.0, 0.0])
        offsets = [tuple(int(v) for v in o) for o in np.asarray(ti["offsets"]).reshape(-1, 3)] + NNN[name]
        blocks = list(np.asarray(ti["blocks"]).reshape(-1, 4, 4)) + [-0.05 * G1] * 4
        E0 = np.asarray(ti["onsite"]).reshape(4, 4)
        dim, no = 3, 4
    st = {"dim": dim, "n_orb": no, "offsets": np.array(offsets), "blocks": np.array(blocks), "onsite": E0,
          "pot_mode": pv.PV_POT_SITE}
    return st, offsets, blocks, E0


class GenCase:
    def __init__(self, name, L, per, vdtype=np.float64, seed=3):
        self.st, offsets, blocks, E0 = stencil(name)
        self.lat = pv.Lattice(L, per, self.st)
        assert self.lat.family == 0 and pv.pv_lattice_get_codegen(self.lat)
        n_sites = int(np.prod(L))
        V = W.uniform_potential(n_sites, 1.0, W.generator(seed, W.STREAM_POTENTIAL)).astype(vdtype)
        self.lat.set_potential(dev(V))
        self.ol, self.H = _explicit_matrix(L, per, self.st["n_orb"], offsets, blocks, E0, V.astype(np.float64), False)
        self.D = self.ol.n_rows


CASES = [("xz", (13, 6, 5), (1, 1, 1)), ("xy", (11, 7, 4), (0, 1, 1)), ("yz", (9, 6, 5), (1, 0, 1)),
         ("xyz", (10, 5, 6), (0, 1, 0)), ("2d", (37, 9), (0, 1))]


@pytest.mark.parametrize("name,L,per", CASES)
@pytest.mark.parametrize("dtype,nb", [(np.complex128, 1), (np.complex128, 4), (np.complex128, 16),
                                      (np.complex64, 16)])
@pytest.mark.parametrize("kernel", [1, 2])
def test_generated_step_matches_oracle_and_interpreted(name, L, per, dtype, nb, kernel):
    """Chebyshev step with dots, y = alpha (H - beta) x + gamma z, on the
    generated kernels (direct, or staged where the offsets allow it) against
    the oracle; then the same launch on the interpreted generic kernels."""
    c = GenCase(name, L, per, np.float64 if dtype == np.complex128 else np.float32)
    code = pv.PV_C128 if dtype == np.complex128 else pv.PV_C64
    pv.pv_lattice_set_tuning(c.lat, code, nb, {"kernel": kernel})
    x = W.gaussian_block(c.D, nb, W.generator(4, 2, nb), dtype)
    z = W.gaussian_block(c.D, nb, W.generator(4, 3, nb), dtype)
    x64, z64 = x.astype(np.complex128), z.astype(np.complex128)
    ref = spmmv.spmmv(c.H, x64, 0.4, 0.2, -1.0, z64)
    tol = 1e-13 if dtype == np.complex128 else 2e-6
    outs = []
    for gen in (True, False):
        pv.pv_lattice_set_codegen(c.lat, gen)
        assert pv.pv_lattice_get_codegen(c.lat) == gen
        n0 = pv.pv_codegen_instances()
        y = dev(z.copy())
        d = host(pv.pv_spmmv(c.lat, dev(x), y, 0.4, 0.2, -1.0, z=y, dot_flags=7))
        out = host(y).astype(np.complex128)
        assert rel_err(out, ref) < tol, gen
        xx = np.sum(np.abs(x64) ** 2, axis=0)
        assert np.abs(d[:, 0] - xx).max() < (1e-12 if dtype == np.complex128 else 1e-5) * xx.max()
        outs.append(out)
        assert pv.pv_codegen_instances() >= n0 and (pv.pv_codegen_instances() > 0 or not gen)
    assert rel_err(outs[0], outs[1]) < tol


@pytest.mark.parametrize("name,L,per", CASES)
@pytest.mark.parametrize("dtype", [np.complex128, np.complex64])
def test_generated_512_lane_shapes(name, L, per, dtype):
    """The longer tiles of the built-in families (512-lane workgroups, two
    complex128 or four complex64 elements per lane) on generated kernels:
    Chebyshev step with dots, the series step and the plain sweep without z
    (where six side rows would overflow the LDS, the launch takes the
    shortest tile instead)."""
    c = GenCase(name, L, per, np.float64 if dtype == np.complex128 else np.float32, seed=8)
    nb = 8
    code = pv.PV_C128 if dtype == np.complex128 else pv.PV_C64
    pv.pv_lattice_set_tuning(c.lat, code, nb, {"kernel": 2, "elems_per_lane": 2 if dtype == np.complex128 else 4,
                                               "workgroup_size": 512})
    tol = 1e-13 if dtype == np.complex128 else 2e-6
    x = W.gaussian_block(c.D, nb, W.generator(9, 2), dtype)
    z = W.gaussian_block(c.D, nb, W.generator(9, 3), dtype)
    x64, z64 = x.astype(np.complex128), z.astype(np.complex128)
    y = dev(z.copy())
    pv.pv_spmmv(c.lat, dev(x), y, 0.7, -0.1, -1.0, z=y, dot_flags=7)
    assert rel_err(host(y).astype(np.complex128), spmmv.spmmv(c.H, x64, 0.7, -0.1, -1.0, z64)) < tol
    y = dev(np.full(x.shape, np.nan, dtype=dtype))
    pv.pv_spmmv(c.lat, dev(x), y, 0.5, 0.3, 0.0)
    out = host(y).astype(np.complex128)
    assert np.isfinite(out).all()
    assert rel_err(out, spmmv.spmmv(c.H, x64, 0.5, 0.3, 0.0)) < tol
    a = float(np.abs(c.H).sum(axis=1).max()) * 1.05
    coef = W.generator(9, 4).standard_normal(9) + 1j * W.generator(9, 5).standard_normal(9)
    Y = torch.empty(x.shape, dtype=torch.complex128 if dtype == np.complex128 else torch.complex64, device="cuda")
    pv.pv_cheb_series(c.lat, dev(x), Y, a, 0.1, coef)
    ref = chebtp.cheb_series(c.H, x64, a, 0.1, coef)
    assert rel_err(host(Y).astype(np.complex128), ref) < (1e-12 if dtype == np.complex128 else 2e-5)


@pytest.mark.parametrize("name,L,per", CASES[:4])
@pytest.mark.parametrize("kernel", [1, 2])
def test_generated_per_column_coefficients(name, L, per, kernel):
    """Per-column alpha, beta, gamma take the kernels that read their
    epilogue at run time (one complex128 element per lane)."""
    c = GenCase(name, L, per, seed=11)
    nb = 4
    pv.pv_lattice_set_tuning(c.lat, pv.PV_C128, nb, {"kernel": kernel, "elems_per_lane": 2})
    g = W.generator(11, 7)
    alpha, beta, gamma = 0.5 + g.random(nb), g.standard_normal(nb), g.standard_normal(nb)
    x = W.gaussian_block(c.D, nb, W.generator(11, 2))
    z = W.gaussian_block(c.D, nb, W.generator(11, 3))
    y = dev(z.copy())
    pv.pv_spmmv(c.lat, dev(x), y, alpha, beta, gamma, z=y, dot_flags=7)
    assert rel_err(host(y), spmmv.spmmv(c.H, x, alpha, beta, gamma, z)) < 1e-13


@pytest.mark.parametrize("name,L,per", CASES[1:])
def test_generated_kpm_moments(name, L, per):
    """KPM moments (Chebyshev steps with fused dots, the reduction folded into
    the next sweep) on the generated kernels against the oracle's moments by
    the product doubling on the explicit matrix."""
    c = GenCase(name, L, per, seed=13)
    nb, M = 4, 48
    a = float(np.abs(c.H).sum(axis=1).max()) * 1.05
    r = W.random_phase_block(c.D, nb, W.generator(13, 2))
    mu = pv.pv_kpm_moments(c.lat, dev(r), M, a, 0.05)
    ref = kpm.moments_doubling(c.H, r, M, a, 0.05)
    assert np.abs(host(mu) - ref).max() < 1e-12


def test_generated_kernels_replay_in_a_captured_graph():
    """A sweep on generated kernels captured into a graph (after an eager call
    compiled and loaded the instance) replays correctly, several times, with
    eager work on the same buffers between the replays."""
    c = GenCase("xy", (11, 7, 4), (0, 1, 1), seed=21)
    nb = 4
    xh = W.gaussian_block(c.D, nb, W.generator(21, 2))
    x = dev(xh)
    y = torch.empty_like(x)
    dots = torch.empty((nb, 4), dtype=torch.float64, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        pv.pv_spmmv(c.lat, x, y, 0.5, 0.1, 0.0, dot_flags=7, dots=dots)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    eager_y, eager_d = host(y).copy(), host(dots).copy()
    assert rel_err(eager_y, spmmv.spmmv(c.H, xh, 0.5, 0.1, 0.0)) < 1e-13
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        pv.pv_spmmv(c.lat, x, y, 0.5, 0.1, 0.0, dot_flags=7, dots=dots)
    for k in range(3):
        y.fill_(float("nan"))
        dots.fill_(float("nan"))
        pv.pv_spmmv(c.lat, x, torch.empty_like(x), 1.0, 0.0, 0.0)   # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(y), eager_y), k
        assert np.array_equal(host(dots), eager_d), k


_CACHE_RUN = r"""
import sys, numpy as np, torch
sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
import paper_1708_09689_amd as pv, workloads as W
from test_gpu_codegen import stencil
st, _, _, _ = stencil("xz")
st["blocks"] = np.array(st["blocks"]) * 1.0
st["onsite"] = np.asarray(st["onsite"]) + np.diag([0.01, 0.02, 0.03, 0.04])   # a pattern no other test compiles
lat = pv.Lattice((9, 6, 5), (1, 1, 1), st)
x = torch.from_numpy(W.gaussian_block(lat.n_rows, 4, W.generator(77, 2))).cuda()
y = torch.empty_like(x)
pv.pv_lattice_set_tuning(lat, pv.PV_C128, 4, {{"kernel": 2}})
assert pv.pv_lattice_get_codegen(lat)
pv.pv_spmmv(lat, x, y, 0.5, 0.1, 0.0)
assert pv.pv_codegen_instances() == 1
np.save({out!r}, y.cpu().numpy())
"""


def test_codegen_disk_cache_across_processes(tmp_path):
    """PV_CODEGEN_CACHE keeps generated code objects across processes: the
    first process writes one, a file that is not a code object is compiled
    again and replaced, and every process computes the same result."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    cache = tmp_path / "cache"
    cache.mkdir()
    env = dict(os.environ, PV_CODEGEN_CACHE=str(cache))
    outs = []
    for k in range(3):
        out = str(tmp_path / f"y{k}.npy")
        code = _CACHE_RUN.format(root=root, tests=os.path.join(root, "tests"), out=out)
        r = subprocess.run([sys.executable, "-c", code], env=env, timeout=150, capture_output=True, text=True)
        assert r.returncode == 0, r.stdout + r.stderr
        outs.append(np.load(out))
        files = sorted(cache.glob("pvcg_*.co"))
        assert len(files) == 1, (k, sorted(p.name for p in cache.iterdir()), r.stderr[-2000:])
        body = files[0].read_bytes()
        assert b"\x7fELF" in body[:512]
        if k == 0:
            files[0].write_bytes(b"not a code object\n" + b"x" * 100)   # damaged entry: compiled again
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


def test_sweeps_compile_each_generated_instance_once():
    """The first sweep of a pattern, launch shape and epilogue compiles and
    loads one generated instance; repeating it, or running the interpreted
    kernels, loads none; another epilogue loads one more."""
    g = np.random.default_rng(99)
    offsets, blocks = [], []
    for o in [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 1)]:
        B = (g.standard_normal((2, 2)) + 1j * g.standard_normal((2, 2))) * np.array([[1, 1], [0, 1]])
        offsets += [o, tuple(-v for v in o)]
        blocks += [B, B.conj().T]
    E0 = np.array([[0.5, 0.25j], [-0.25j, 0.0]])
    st = {"dim": 3, "n_orb": 2, "offsets": np.array(offsets), "blocks": np.array(blocks), "onsite": E0,
          "pot_mode": pv.PV_POT_SITE}
    L, per = (10, 6, 5), (1, 0, 1)
    lat = pv.Lattice(L, per, st)
    V = W.uniform_potential(int(np.prod(L)), 1.0, W.generator(99, 1))
    lat.set_potential(dev(V))
    _, H = _explicit_matrix(L, per, 2, offsets, blocks, E0, V, False)
    nb = 2
    pv.pv_lattice_set_tuning(lat, pv.PV_C128, nb, {"kernel": 2})
    xh = W.gaussian_block(H.shape[0], nb, W.generator(99, 2))
    x, y = dev(xh), torch.empty((H.shape[0], nb), dtype=torch.complex128, device="cuda")
    n0 = pv.pv_codegen_instances()
    pv.pv_spmmv(lat, x, y, 0.5, 0.1, 0.0)
    assert pv.pv_codegen_instances() == n0 + 1
    assert rel_err(host(y), spmmv.spmmv(H, xh, 0.5, 0.1, 0.0)) < 1e-13
    pv.pv_spmmv(lat, x, y, 0.5, 0.1, 0.0)
    assert pv.pv_codegen_instances() == n0 + 1
    pv.pv_lattice_set_codegen(lat, False)
    pv.pv_spmmv(lat, x, y, 0.5, 0.1, 0.0)
    assert pv.pv_codegen_instances() == n0 + 1
    pv.pv_lattice_set_codegen(lat, True)
    dots = torch.empty((nb, 4), dtype=torch.float64, device="cuda")
    pv.pv_spmmv(lat, x, y, 0.5, 0.1, 0.0, dot_flags=7, dots=dots)   # the Chebyshev-step epilogue
    assert pv.pv_codegen_instances() == n0 + 2


@pytest.mark.parametrize("dtype,shape", [(np.complex128, {"kernel": 1}),
                                         (np.complex128, {"kernel": 2, "elems_per_lane": 1}),
                                         (np.complex128, {"kernel": 2, "elems_per_lane": 2, "workgroup_size": 512}),
                                         (np.complex64, {"kernel": 2, "elems_per_lane": 4, "workgroup_size": 512})])
def test_batched_kpm_on_generated_kernels(dtype, shape):
    """A batch of lattices sharing one generated pattern (ragged sizes, the
    xy stencil with halo side rows) runs its graph-captured KPM on generated
    kernels, compiled before the capture; every instance equals its oracle
    run (complex128 1e-12, complex64 vectors with FP64 moments 1e-4), and a
    replay is bitwise identical."""
    from oracle import kpm as okpm
    vd = np.float64 if dtype == np.complex128 else np.float32
    sizes = [((6, 5, 4), (1, 1, 1)), ((7, 6, 5), (0, 1, 1)), ((5, 5, 5), (1, 1, 0)), ((8, 4, 6), (1, 1, 1))]
    cases = [GenCase("xy", L, per, vd, seed=60 + i) for i, (L, per) in enumerate(sizes)]
    nb, M = 8, 24
    rs = [W.random_phase_block(c.D, nb, W.generator(61, i), dtype) for i, c in enumerate(cases)]
    a = np.array([float(np.abs(c.H).sum(axis=1).max()) * 1.05 for c in cases])
    b = np.array([0.0, 0.05, -0.1, 0.02])
    batch = pv.Batch([c.lat for c in cases])
    code = pv.PV_C128 if dtype == np.complex128 else pv.PV_C64
    pv.pv_batch_set_tuning(batch, code, nb, shape)
    n0 = pv.pv_codegen_instances()
    rd = [dev(r) for r in rs]
    mu = host(pv.pv_batch_kpm_moments(batch, rd, M, a, b)).copy()
    assert pv.pv_codegen_instances() >= n0 + 1 or n0 > 0
    tol = 1e-12 if dtype == np.complex128 else 1e-4
    for i, c in enumerate(cases):
        ref = okpm.moments_doubling(c.H, rs[i].astype(np.complex128), M, a[i], b[i])
        assert np.abs(mu[i] - ref).max() < tol, (shape, i)
    assert np.array_equal(host(pv.pv_batch_kpm_moments(batch, rd, M, a, b)), mu)
    assert batch.stats() == (1, 1)


def test_batch_of_different_patterns_takes_interpreted_kernels():
    """Lattices with different generic patterns share no generated kernel:
    their batch runs the interpreted kernels (512-lane shapes are refused)
    and every instance still equals its oracle run."""
    from oracle import kpm as okpm
    cases = [GenCase("xy", (6, 5, 4), (1, 1, 1), seed=70), GenCase("xz", (5, 6, 4), (1, 1, 1), seed=71)]
    nb, M = 4, 16
    rs = [W.random_phase_block(c.D, nb, W.generator(72, i)) for i, c in enumerate(cases)]
    a = np.array([float(np.abs(c.H).sum(axis=1).max()) * 1.05 for c in cases])
    b = np.zeros(2)
    batch = pv.Batch([c.lat for c in cases])
    with pytest.raises(pv.PvError):
        pv.pv_batch_set_tuning(batch, pv.PV_C128, nb, {"kernel": 2, "elems_per_lane": 1, "workgroup_size": 512})
    n0 = pv.pv_codegen_instances()
    mu = host(pv.pv_batch_kpm_moments(batch, [dev(r) for r in rs], M, a, b))
    assert pv.pv_codegen_instances() == n0
    for i, c in enumerate(cases):
        assert np.abs(mu[i] - okpm.moments_doubling(c.H, rs[i], M, a[i], b[i])).max() < 1e-12


@pytest.mark.parametrize("kernel", [1, 2])
def test_generated_kernels_with_the_on_the_fly_field(kernel):
    """Generated kernels evaluate the counter-based disorder field inside the
    sweep like the built-in families: KPM moments of the xy stencil with the
    field W (u_i - 1/2) generated on the fly equal the oracle's on the
    explicit matrix with the same field."""
    from oracle import rng
    st, offsets, blocks, E0 = stencil("xy")
    L, per = (11, 6, 5), (1, 1, 0)
    lat = pv.Lattice(L, per, st)
    lat.set_random_potential(4321, 1.5)
    V = rng.field(4321, 1.5, int(np.prod(L)))
    _, H = _explicit_matrix(L, per, 4, offsets, blocks, E0, V, False)
    nb, M = 4, 32
    pv.pv_lattice_set_tuning(lat, pv.PV_C128, nb, {"kernel": kernel})
    a = float(np.abs(H).sum(axis=1).max()) * 1.05
    r = W.random_phase_block(H.shape[0], nb, W.generator(43, 2))
    mu = host(pv.pv_kpm_moments(lat, dev(r), M, a, 0.0))
    assert pv.pv_codegen_instances() > 0
    assert np.abs(mu - kpm.moments_doubling(H, r, M, a, 0.0)).max() < 1e-12


@pytest.mark.parametrize("name", ["xy", "yz"])
def test_generated_kernels_kpm_gradient(name):
    """The adjoint sweeps (the source-term and gradient epilogues) run on the
    generated direct kernel: the field gradient of sum gbar mu equals the
    oracle's discrete adjoint on the explicit matrix, with checkpoints."""
    from oracle import adjoint
    c = GenCase(name, (7, 5, 4), (1, 0, 1), seed=80)
    nb, M = 4, 24
    a = float(np.abs(c.H).sum(axis=1).max()) * 1.05
    r = W.random_phase_block(c.D, nb, W.generator(81, 2))
    gbar = W.generator(81, 3).standard_normal((nb, M))
    g = host(pv.pv_kpm_moments_vjp(c.lat, dev(r), M, a, 0.05, dev(gbar), ckpt_every=5))
    ref = adjoint.kpm_vjp(c.H, 4, "site", r, M, a, 0.05, gbar)
    assert np.abs(g - ref).max() < 1e-10 * np.abs(ref).max()


def test_failed_compilation_is_an_error_and_the_lattice_stays_usable(monkeypatch):
    """A generated kernel that does not compile (forced with the test hook)
    fails the sweep with PV_ERR_HIP and the compiler's message; the same
    lattice then runs on the interpreted kernels, and on generated ones once
    compilation works again."""
    g = np.random.default_rng(123)
    offsets, blocks = [], []
    for o in [(1, 0, 0), (0, 1, 0), (0, 0, 1), (0, 1, 1)]:
        B = (g.standard_normal((2, 2)) + 1j * g.standard_normal((2, 2))) * np.array([[0, 1], [1, 1]])
        offsets += [o, tuple(-v for v in o)]
        blocks += [B, B.conj().T]
    E0 = np.array([[0.1, 0.0], [0.0, -0.3]])
    st = {"dim": 3, "n_orb": 2, "offsets": np.array(offsets), "blocks": np.array(blocks), "onsite": E0,
          "pot_mode": pv.PV_POT_SITE}
    L, per = (6, 5, 4), (1, 1, 1)
    lat = pv.Lattice(L, per, st)
    V = W.uniform_potential(int(np.prod(L)), 1.0, W.generator(123, 1))
    lat.set_potential(dev(V))
    _, H = _explicit_matrix(L, per, 2, offsets, blocks, E0, V, False)
    xh = W.gaussian_block(H.shape[0], 2, W.generator(123, 2))
    x, y = dev(xh), torch.empty((H.shape[0], 2), dtype=torch.complex128, device="cuda")
    n0 = pv.pv_codegen_instances()
    monkeypatch.setenv("PV_TEST_FAIL_CODEGEN", "1")
    with pytest.raises(pv.PvError) as e:
        pv.pv_spmmv(lat, x, y, 0.5, 0.0, 0.0)
    assert e.value.status == 6 and "PV_TEST_FAIL_CODEGEN" in str(e.value)
    assert pv.pv_codegen_instances() == n0
    pv.pv_lattice_set_codegen(lat, False)
    pv.pv_spmmv(lat, x, y, 0.5, 0.0, 0.0)
    assert rel_err(host(y), spmmv.spmmv(H, xh, 0.5, 0.0, 0.0)) < 1e-13
    monkeypatch.delenv("PV_TEST_FAIL_CODEGEN")
    pv.pv_lattice_set_codegen(lat, True)
    y.zero_()
    pv.pv_spmmv(lat, x, y, 0.5, 0.0, 0.0)
    assert pv.pv_codegen_instances() == n0 + 1
    assert rel_err(host(y), spmmv.spmmv(H, xh, 0.5, 0.0, 0.0)) < 1e-13


def test_batch_autotune_on_generated_kernels():
    """pv_batch_autotune on a batch sharing one generated pattern times the
    staged candidates too (512 lanes included) and keeps results equal to
    the direct generated kernel's up to the dots' summation order."""
    cases = [GenCase("xz", L, (1, 1, 1), seed=90 + i) for i, L in enumerate([(6, 5, 4), (7, 6, 5), (8, 4, 6)])]
    nb, M = 8, 16
    rs = [dev(W.random_phase_block(c.D, nb, W.generator(91, i))) for i, c in enumerate(cases)]
    a = np.array([float(np.abs(c.H).sum(axis=1).max()) * 1.05 for c in cases])
    b = np.zeros(3)
    batch = pv.Batch([c.lat for c in cases])
    pv.pv_batch_set_tuning(batch, pv.PV_C128, nb, {"kernel": 1})
    mu_d = host(pv.pv_batch_kpm_moments(batch, rs, M, a, b)).copy()
    shape, ms = pv.pv_batch_autotune(batch, rs, a, b)
    assert ms > 0.0 and shape["kernel"] in (1, 2) and shape["workgroup_size"] in (0, 512)
    mu_t = host(pv.pv_batch_kpm_moments(batch, rs, M, a, b))
    assert np.abs(mu_t - mu_d).max() < 1e-13


def _extra_case(name, L, per, vdtype):
    """A generated-kernel lattice with a per-orbital field ("2d_orbital": the
    2D two-orbital stencil) or a single-orbital 3D stencil with complex
    diagonal hops ("cubic1"), and the oracle's explicit matrix."""
    if name == "2d_orbital":
        st, offsets, blocks, E0 = stencil("2d")
        st = dict(st, pot_mode=pv.PV_POT_ORBITAL)
    else:
        g = np.random.default_rng(23)
        offsets, blocks = [], []
        for o in [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (0, 1, -1), (1, 0, 1)]:
            B = np.array([[g.standard_normal() + 1j * g.standard_normal()]])
            offsets += [o, tuple(-v for v in o)]
            blocks += [B, B.conj().T]
        E0 = np.array([[0.25 + 0j]])
        st = {"dim": 3, "n_orb": 1, "offsets": np.array(offsets), "blocks": np.array(blocks), "onsite": E0,
              "pot_mode": pv.PV_POT_SITE}
    lat = pv.Lattice(L, per, st)
    assert lat.family == 0 and pv.pv_lattice_get_codegen(lat)
    orbital = st["pot_mode"] == pv.PV_POT_ORBITAL
    n = int(np.prod(L)) * (st["n_orb"] if orbital else 1)
    V = W.uniform_potential(n, 1.0, W.generator(29, W.STREAM_POTENTIAL)).astype(vdtype)
    lat.set_potential(dev(V))
    ol, H = _explicit_matrix(L, per, st["n_orb"], offsets, blocks, E0, V.astype(np.float64), orbital)
    return lat, H, ol.n_rows


@pytest.mark.parametrize("name,L,per", [("2d_orbital", (41, 7), (1, 0)), ("cubic1", (23, 6, 5), (1, 1, 0))])
@pytest.mark.parametrize("dtype,nb", [(np.complex128, 1), (np.complex128, 4), (np.complex64, 1), (np.complex64, 4)])
@pytest.mark.parametrize("kernel", [1, 2])
def test_generated_per_orbital_field_and_single_orbital_stencils(name, L, per, dtype, nb, kernel):
    """Generated kernels with a field per orbital row, and on a one-orbital
    stencil, where a complex64 site of one column is half a 16-byte chunk (the
    staged request then takes the direct kernel); against the oracle and the
    interpreted kernels."""
    lat, H, D = _extra_case(name, L, per, np.float64 if dtype == np.complex128 else np.float32)
    code = pv.PV_C128 if dtype == np.complex128 else pv.PV_C64
    pv.pv_lattice_set_tuning(lat, code, nb, {"kernel": kernel})
    x = W.gaussian_block(D, nb, W.generator(5, 2, nb), dtype)
    z = W.gaussian_block(D, nb, W.generator(5, 3, nb), dtype)
    ref = spmmv.spmmv(H, x.astype(np.complex128), 0.4, 0.2, -1.0, z.astype(np.complex128))
    tol = 1e-13 if dtype == np.complex128 else 2e-6
    outs = []
    for gen in (True, False):
        pv.pv_lattice_set_codegen(lat, gen)
        n0 = pv.pv_codegen_instances()
        y = dev(z.copy())
        pv.pv_spmmv(lat, dev(x), y, 0.4, 0.2, -1.0, z=y, dot_flags=7)
        out = host(y).astype(np.complex128)
        assert rel_err(out, ref) < tol, gen
        if gen:
            assert pv.pv_codegen_instances() >= n0 and pv.pv_codegen_instances() > 0
        outs.append(out)
    assert rel_err(outs[0], outs[1]) < tol
