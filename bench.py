"""Benchmark of the Chebyshev-SpMMV hot path on one MI355X.

Workload (one GPU): 3D topological insulator, 256 x 256 x 64 periodic cubic
lattice, 4 orbitals per site (D = 16,777,216 rows), t = 1, m = 2, uniform
disorder W = 2 (seeded), random-phase start block of nb columns.  One step is
one Chebyshev recurrence sweep w_{k+1} = 2 H~ w_k - w_{k-1} (a = 7, b = 0)
with the fused partial dot products <w_k,w_k>, <w_k,w_{k+1}> that give two
KPM moments, followed by their fixed-order reduction.

Prints ONE JSON line.  GLUP/s counts row-column updates (one row of H times
one column, the paper's lattice-site-update unit per orbital row).
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "GLUP/s & % HBM roofline, Chebyshev-SpMMV fwd vs fwd+adjoint, FP64 vs FP32"
HBM_PEAK_GBS = 8000.0
L_BENCH = (256, 256, 64)
WORKLOAD_INDEX = 2            # seeds of the 256x256x64 TI workload
A_SCALE, B_SHIFT = 7.0, 0.0


# Bytes per Chebyshev-step launch of the sweep kernel as built now that miss
# L2 (FETCH_SIZE / WRITE_SIZE counters scaled by the copy-kernel factors,
# profiles/*_counters.txt; the Infinity Cache serves part of them), with the
# launch shape the counters were taken with; other shapes and (dtype, nb)
# pairs without a counter run report null.
_STAGED = {"kernel": 2, "walk_planes": 0, "strip_rows": 0, "groups_per_xcd": 0, "tiles_per_group": 0, "slab_rows": 0,
           "workgroup_size": 0}
COUNTED_TRAFFIC = {
    ("c128", 32): [(dict(_STAGED, elems_per_lane=2, strip_rows=32, workgroup_size=512), 35_604_000_000),
                   (dict(_STAGED, elems_per_lane=2, strip_rows=64, workgroup_size=512), 35_564_000_000),
                   (dict(_STAGED, elems_per_lane=2, workgroup_size=512), 36_003_000_000)],
    ("c64", 16): [(dict(_STAGED, elems_per_lane=4, workgroup_size=512), 6_957_000_000)],
}


def counted_traffic(dtype: str, nb: int, shape: dict):
    for sh, nbytes in COUNTED_TRAFFIC.get((dtype, nb), []):
        if {**_STAGED, "elems_per_lane": 0, **sh} == {**_STAGED, "elems_per_lane": 0, **shape}:
            return nbytes
    return None


def bytes_per_step(n_rows: int, n_sites: int, nb: int, dtype: str) -> int:
    """Algorithmic HBM bytes of one Chebyshev sweep: read x (w_k), read z
    (w_{k-1}), write y (w_{k+1}), read the on-site field once per site."""
    e = 16 if dtype == "c128" else 8
    v = 8 if dtype == "c128" else 4
    return 3 * n_rows * nb * e + n_sites * v


TUNE_CACHE = os.path.join(tempfile.gettempdir(), "pvdtm_bench_tune.jsonl")


class Sweep:
    """State of one (dtype, nb) Chebyshev recurrence on the benchmark lattice.
    The launch shape comes from the library's autotuner (cached per device in
    a temporary file), as a user of the library would run it, unless a shape
    is pinned (fields of pv_tuning; the rest default)."""

    def __init__(self, pv, torch, lat, nb, dtype, dev, shape=None):
        self.pv, self.torch, self.lat, self.nb, self.dtype = pv, torch, lat, nb, dtype
        code = pv.PV_C128 if dtype == "c128" else pv.PV_C64
        if shape is None:
            self.shape, self.tune_ms = pv.pv_autotune(lat, nb, code, cache_path=TUNE_CACHE)
        else:
            self.shape = {**_STAGED, "elems_per_lane": 0, **shape}
            pv.pv_lattice_set_tuning(lat, code, nb, self.shape)
        import workloads as W
        self.w0 = W.random_phase_device(lat.n_rows, nb, 10 * WORKLOAD_INDEX + nb, dev,
                                        "complex128" if dtype == "c128" else "complex64")
        self.w1 = torch.empty_like(self.w0)
        # w1 = H~ w0 (first Chebyshev vector), then recurrences in place
        pv.pv_spmmv(lat, self.w0, self.w1, 1.0 / A_SCALE, B_SHIFT, 0.0, nb=nb)
        self.dots = torch.empty((nb, 4), dtype=torch.float64, device=dev)
        self.ws = None

    def step(self):
        pv = self.pv
        # w_{k+1} = 2 H~ w_k - w_{k-1}, written over w_{k-1}; dots of (w_k, w_{k+1})
        pv.pv_spmmv(self.lat, self.w1, self.w0, 2.0 / A_SCALE, B_SHIFT, -1.0, z=self.w0,
                    dot_flags=pv.PV_DOT_XX | pv.PV_DOT_XY, dots=self.dots, nb=self.nb)
        self.w0, self.w1 = self.w1, self.w0


def time_steps(torch, sw: Sweep, warmup: int, steps: int) -> float:
    for _ in range(warmup):
        sw.step()
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        sw.step()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps  # ms per step


def median_steps(torch, sw: Sweep, runs: int = 3, steps: int = 10) -> float:
    """ms per step of a variant: the median of `runs` timed runs of `steps`
    steps each (a one-off stall of a few tens of milliseconds, seen now and
    then in a short timed region, then does not decide the figure)."""
    return sorted(time_steps(torch, sw, 3, steps) for _ in range(runs))[runs // 2]


def copy_probe(pv, torch, dev, nbytes=4 << 30, reps=10) -> float:
    """Achievable bandwidth of a plain streaming copy (GB/s, read + write)."""
    src = torch.empty(nbytes // 8, dtype=torch.float64, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(2):
        pv.pv_stream_copy(src, dst)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        pv.pv_stream_copy(src, dst)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def triad_probe(pv, torch, dev, nbytes=4 << 30, reps=10) -> float:
    """Achievable bandwidth of a streaming triad y = x + z (GB/s, two reads +
    one write: the stream mix of a Chebyshev step without the stencil)."""
    x = torch.empty(nbytes // 8, dtype=torch.float64, device=dev).fill_(1.0)
    z = torch.empty_like(x).fill_(2.0)
    y = torch.empty_like(x)
    for _ in range(2):
        pv.pv_stream_triad(x, z, y)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        pv.pv_stream_triad(x, z, y)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del x, z, y
    return 3.0 * nbytes / (ms * 1e-3) / 1e9


def read_probe(pv, torch, dev, nbytes=8 << 30, reps=10) -> float:
    """Achievable bandwidth of a streaming read (GB/s, reads only)."""
    x = torch.empty(nbytes // 8, dtype=torch.float64, device=dev).fill_(1.0)
    sink = torch.empty(pv.PV_STREAM_READ_SINK_BYTES // 4, dtype=torch.int32, device=dev)
    for _ in range(2):
        pv.pv_stream_read(x, sink)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        pv.pv_stream_read(x, sink)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del x, sink
    return nbytes / (ms * 1e-3) / 1e9


def memcpy_probe(torch, dev, nbytes=4 << 30, reps=10) -> float:
    """Device-to-device copy through the runtime (torch's copy_ of contiguous
    tensors of one dtype: hipMemcpyAsync), GB/s read + write: a copy that is
    not this library's, as a cross-check of the copy probe."""
    src = torch.empty(nbytes // 8, dtype=torch.float64, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def torch_triad_probe(torch, dev, nbytes=4 << 30, reps=10) -> float:
    """y = x + z by PyTorch's own elementwise kernel (GB/s, two reads + one
    write): a triad that is not this library's, as a cross-check of the
    triad probe's ceiling."""
    x = torch.empty(nbytes // 8, dtype=torch.float64, device=dev).fill_(1.0)
    z = torch.empty_like(x).fill_(2.0)
    y = torch.empty_like(x)
    for _ in range(2):
        torch.add(x, z, out=y)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.add(x, z, out=y)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del x, z, y
    return 3.0 * nbytes / (ms * 1e-3) / 1e9


def cpu_baseline(nb: int, budget_s: float = 8.0) -> dict:
    """The oracle on a bounded sample of the same workload (the same x-y
    planes, 4 of the 64 z-layers): its C++/OpenMP Chebyshev step with fused
    dots over the explicit CSR matrix, on all the threads OpenMP is given
    (OMP_NUM_THREADS) and on one, each for about budget_s seconds."""
    import workloads as W
    from oracle import hamiltonian, lattice, models, omp_sweep
    L = (L_BENCH[0], L_BENCH[1], 4)
    olat = lattice.Lattice(L, (1, 1, 1), 4)
    V = W.uniform_potential(olat.n_sites, 2.0, W.generator(WORKLOAD_INDEX, W.STREAM_POTENTIAL))
    A = omp_sweep.Csr(hamiltonian.assemble(models.topological_insulator(1.0, 2.0), olat, V))
    g = W.generator(WORKLOAD_INDEX, W.STREAM_VECTORS, nb)
    r = W.random_phase_block(olat.n_rows, nb, g)
    n_all = omp_sweep.threads()

    def run(threads):
        omp_sweep.set_threads(threads)
        w0 = r.copy()
        w1, _ = omp_sweep.sweep(A, w0, 1.0 / A_SCALE, B_SHIFT, 0.0)
        sweeps, t0 = 0, time.perf_counter()
        while True:
            # w_{k+1} = 2 H~ w_k - w_{k-1} over w_{k-1}, with <w_k,w_k>, <w_k,w_{k+1}>
            omp_sweep.sweep(A, w1, 2.0 / A_SCALE, B_SHIFT, -1.0, z=w0, y=w0)
            w0, w1 = w1, w0
            sweeps += 1
            el = time.perf_counter() - t0
            if el > budget_s:
                return olat.n_rows * nb * sweeps / el / 1e9, sweeps, el
    try:
        all_glups, all_sweeps, all_s = run(n_all)
        one_glups, one_sweeps, one_s = run(1)
    finally:
        omp_sweep.set_threads(n_all)
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), model)
    except OSError:
        pass
    sample = f"TI {L[0]}x{L[1]}x{L[2]} periodic (4 of 64 z-layers), W=2, nb={nb}, complex128, Chebyshev sweeps + dots"
    return {"value": round(all_glups, 5), "unit": "GLUP/s", "cores": n_all, "kind": "oracle",
            "sample": f"{sample}: {all_sweeps} sweeps in {all_s:.1f} s, C++/OpenMP CSR oracle, {n_all} threads",
            "single_thread": {"value": round(one_glups, 5), "cores": 1,
                              "sample": f"{sample}: {one_sweeps} sweeps in {one_s:.1f} s, same code, 1 thread"},
            "host": f"{os.cpu_count()} logical CPUs visible, {model}"}


def _timed(torch, fn, reps=1):
    """Average ms of fn() over reps calls, timed with events on the current stream."""
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def fp32_step_error(pv, torch, lat, dev, nb, set_field):
    """The FP32 path's error at the benchmark size: one Chebyshev step with
    dots from the same complex64-representable x and z, complex64 vectors
    with the FP32 field against complex128 vectors with the FP64 field (the
    complex128 path equals the oracle to 1e-13 in the parity tests)."""
    import workloads as W
    x32 = W.random_phase_device(lat.n_rows, nb, 930 + nb, dev, "complex64")
    z32 = W.random_phase_device(lat.n_rows, nb, 931 + nb, dev, "complex64")
    flags = pv.PV_DOT_XX | pv.PV_DOT_XY
    set_field("c128")
    y64 = z32.to(torch.complex128)
    d64 = pv.pv_spmmv(lat, x32.to(torch.complex128), y64, 2.0 / A_SCALE, B_SHIFT, -1.0, z=y64, dot_flags=flags)
    set_field("c64")
    y32 = z32.clone()
    d32 = pv.pv_spmmv(lat, x32, y32, 2.0 / A_SCALE, B_SHIFT, -1.0, z=y32, dot_flags=flags)
    torch.cuda.synchronize()
    step = float(((y32.to(torch.complex128) - y64).abs().max() / y64.abs().max()).item())
    dots = float(((d32[:, :2] - d64[:, :2]).abs().max() / d64[:, 0].abs().max()).item())
    return {"step_max_rel": float(f"{step:.3g}"), "dots_max_rel": float(f"{dots:.3g}"),
            "note": f"one Chebyshev step at nb={nb} from the same complex64-representable input: complex64 vectors "
                    "and FP32 field vs complex128 and FP64 field; max |dy| / max |y|, and max |d(xx, xy)| / max xx"}


def with_hbm_fracs(obj):
    """Every result holding "GB/s" (or "approx_GB/s") also gets its fraction
    of the 8 TB/s HBM peak, "frac_hbm_peak"."""
    if isinstance(obj, dict):
        for key in ("GB/s", "approx_GB/s"):
            if isinstance(obj.get(key), (int, float)) and "frac_hbm_peak" not in obj:
                obj["frac_hbm_peak"] = round(obj[key] / HBM_PEAK_GBS, 4)
        for v in obj.values():
            with_hbm_fracs(v)
    elif isinstance(obj, list):
        for v in obj:
            with_hbm_fracs(v)
    return obj


def _median_timed(torch, fn, reps=1, runs=3):
    """Median over `runs` of _timed: a one-off stall of a few tens of
    milliseconds in one run does not decide the figure."""
    return sorted(_timed(torch, fn, reps) for _ in range(runs))[runs // 2]


def bench_kpm16(pv, torch, W, dev):
    """TI 16^3 periodic, W = 1, one random-phase column, M = 128 (a = 7):
    eager launches vs the same run replayed as a captured HIP graph."""
    st = pv.pv_model_stencil(pv.PV_MODEL_TI, [1.0, 2.0, 0.0, 0.0])
    lat = pv.Lattice((16, 16, 16), (1, 1, 1), st)
    lat.set_potential(torch.from_numpy(W.uniform_potential(lat.n_sites, 1.0, W.generator(0, W.STREAM_POTENTIAL))).to(dev))
    r = torch.from_numpy(W.random_phase_block(lat.n_rows, 1, W.generator(0, W.STREAM_VECTORS))).to(dev)
    mu = torch.empty((1, 128), dtype=torch.float64, device=dev)
    for _ in range(3):
        pv.pv_kpm_moments(lat, r, 128, 7.0, 0.0, mu=mu)
    ms_eager = _median_timed(torch, lambda: pv.pv_kpm_moments(lat, r, 128, 7.0, 0.0, mu=mu), 20)
    batch = pv.Batch([lat])
    for _ in range(3):
        pv.pv_batch_kpm_moments(batch, [r], 128, [7.0], [0.0])
    ms_graph = _median_timed(torch, lambda: pv.pv_batch_kpm_moments(batch, [r], 128, [7.0], [0.0]), 20)
    lups = lat.n_rows * 64
    return {"workload": "TI 16x16x16 periodic, W=1, nb=1, M=128 (64 sweeps), complex128",
            "us_per_kpm_eager": round(ms_eager * 1e3, 1), "us_per_kpm_graph": round(ms_graph * 1e3, 1),
            "GLUP/s_eager": round(lups / (ms_eager * 1e-3) / 1e9, 3),
            "GLUP/s_graph": round(lups / (ms_graph * 1e-3) / 1e9, 3), "captures_replays": batch.stats(),
            "note": "cache-resident (0.6 MB): launch-latency bound, no HBM roofline claim"}


def bench_random_block(pv, torch, lat, dev, nb=32):
    """Random start blocks generated on the device for the benchmark lattice
    (counter-based generator, n_rows x nb): write-only, 16 B per complex128
    element, against the copy probe's bound of one read and one write."""
    out = torch.empty((lat.n_rows, nb), dtype=torch.complex128, device=dev)
    res = {"workload": f"TI 256x256x64 start block, nb={nb}, complex128 ({out.numel() * 16 / 1e9:.1f} GB)"}
    for name, kind in (("phase", pv.PV_RANDOM_PHASE), ("z4", pv.PV_RANDOM_Z4)):
        pv.pv_random_block(lat, nb, 5, kind, out=out)
        ms = _median_timed(torch, lambda: pv.pv_random_block(lat, nb, 5, kind, out=out), 5)
        res[f"{name}_ms"] = round(ms, 3)
        res[f"{name}_GBs_written"] = round(out.numel() * 16 / (ms * 1e-3) / 1e9, 1)
    return res


def bench_chebtp_graphene(pv, torch, W, dev, steps=5):
    """Graphene two-site cells 1024 x 1024 (open x, periodic y), 8x8 dot array
    (radius 20, V0 = 0.1), Gaussian packet (width 50, E = 0.2), a = 3.06,
    b = 0.05, dt = 10, M = 64 sweeps per time step."""
    Li = Lj = 1024
    st = pv.pv_model_stencil(pv.PV_MODEL_GRAPHENE2, [1.0])
    lat = pv.Lattice((Li, Lj), (0, 1), st)
    lat.set_potential(torch.from_numpy(W.dot_array_potential(Li, Lj)).to(dev))
    psi = torch.from_numpy(W.gaussian_wave_packet(Li, Lj, i0=200, width=50, energy=0.2).reshape(-1, 1)).to(dev)
    pv.pv_cheb_propagate(lat, psi, 3.06, 0.05, 10.0, 64, 1)
    # median of three runs of `steps` time steps (one run is ~10 ms)
    runs = sorted(_timed(torch, lambda: pv.pv_cheb_propagate(lat, psi, 3.06, 0.05, 10.0, 64, steps)) / steps
                  for _ in range(3))
    ms = runs[1]
    norm = float(torch.linalg.vector_norm(psi).item())
    # the configured run: 200 steps from the initial packet, then 200 back
    psi0 = torch.from_numpy(W.gaussian_wave_packet(Li, Lj, i0=200, width=50, energy=0.2).reshape(-1, 1)).to(dev)
    psi = psi0.clone()
    ms200 = _timed(torch, lambda: pv.pv_cheb_propagate(lat, psi, 3.06, 0.05, 10.0, 64, 200))
    n200 = float(torch.linalg.vector_norm(psi).item())
    pv.pv_cheb_propagate(lat, psi, 3.06, 0.05, -10.0, 64, 200)
    back = float((torch.linalg.vector_norm(psi - psi0) / torch.linalg.vector_norm(psi0)).item())
    lups = lat.n_rows * 64
    by = lat.n_rows * (4 * 16) + lat.n_sites * 8   # x, z, acc in/out (+y) per sweep, field
    return {"workload": "graphene 1024x1024 cells x 2 sites, open x / periodic y, dot array, packet; "
                        f"runs of {steps} time steps of dt=10 (median of 3), M=64, complex128",
            "ms_per_time_step": round(ms, 4), "GLUP/s": round(lups / (ms * 1e-3) / 1e9, 3),
            "norm_after": round(norm, 12), "approx_GB/s": round(by * 64 / (ms * 1e-3) / 1e9, 1),
            "run_200_steps": {"ms": round(ms200, 2), "norm_minus_1": float(f"{n200 - 1.0:.3g}"),
                              "back_200_steps_rel_err": float(f"{back:.3g}"),
                              "note": "200 steps of dt=10 from the packet, then 200 steps of dt=-10"},
            "note": "working set ~170 MB: largely resident in the 256 MB Infinity Cache"}


def bench_filter(pv, torch, lat, dev, nb=32, K=8):
    """Chebyshev filter / propagation sweeps (accumulate epilogue) on the
    256x256x64 TI at nb = 32: Y = sum_k c_k T_k(H~) X."""
    import workloads as W
    X = W.random_phase_device(lat.n_rows, nb, 77, dev)
    Y = torch.empty_like(X)
    coef = np.linspace(1.0, 0.1, K + 1)
    pv.pv_cheb_series(lat, X, Y, A_SCALE, B_SHIFT, coef)
    ms = _median_timed(torch, lambda: pv.pv_cheb_series(lat, X, Y, A_SCALE, B_SHIFT, coef), 2) / K
    by = lat.n_rows * nb * 16 * 5 + lat.n_sites * 8
    return {"workload": f"TI 256x256x64, nb={nb}, complex128, series of degree {K} (filter step)",
            "ms_per_sweep": round(ms, 4), "GLUP/s": round(lat.n_rows * nb / (ms * 1e-3) / 1e9, 3),
            "GB/s": round(by / (ms * 1e-3) / 1e9, 1), "bytes_per_LUP": 80}


def bench_plain(pv, torch, lat, dev):
    """The plain stencil SpMMV y = alpha (H x - beta x) on the 256x256x64 TI
    (gamma = 0: y is written only), complex128, in the launch shape the
    lattice holds for that block width (the autotuner's, when the variants
    ran first): two vector streams and the field."""
    import workloads as W
    out = {}
    for nb in (4, 32):
        x = W.random_phase_device(lat.n_rows, nb, 78, dev)
        y = torch.empty_like(x)
        pv.pv_spmmv(lat, x, y, 1.0 / A_SCALE, B_SHIFT, 0.0, nb=nb)
        ms = _median_timed(torch, lambda: pv.pv_spmmv(lat, x, y, 1.0 / A_SCALE, B_SHIFT, 0.0, nb=nb), 20)
        by = lat.n_rows * nb * 16 * 2 + lat.n_sites * 8
        out[f"nb{nb}"] = {"ms_per_sweep": round(ms, 4), "GLUP/s": round(lat.n_rows * nb / (ms * 1e-3) / 1e9, 3),
                          "GB/s": round(by / (ms * 1e-3) / 1e9, 1),
                          "bytes_per_LUP": round(by / (lat.n_rows * nb), 3),
                          "shape": {k: v for k, v in pv.pv_lattice_get_tuning(lat, pv.PV_C128, nb).items() if v}}
        del x, y
        torch.cuda.empty_cache()
    out["workload"] = "TI 256x256x64, W=2, complex128, y = alpha (H - beta) x"
    return out


def bench_batch(pv, torch, W, dev, n=96, M=1024, nb=16):
    """96 TI disorder realisations, L ~ U{24..96}, W ~ U[0.5, 3], 16 random-phase
    columns, M = 1024: one graph-captured batched launch per step with
    complex64 vectors and FP64 moments, vs a per-instance complex128 loop over
    the same phases (drawn in complex128, rounded to complex64 for the batch);
    the FP32 path's error is max|dmu| per instance against that loop."""
    inst = W.batch_instances(n, W.generator(3, W.STREAM_SIZES))
    st = pv.pv_model_stencil(pv.PV_MODEL_TI, [1.0, 2.0, 0.0, 0.0])
    lats, Vs, rs = [], [], []
    for i, (L, Wd) in enumerate(inst):
        lat = pv.Lattice((L, L, L), (1, 1, 1), st)
        V = torch.from_numpy(W.uniform_potential(lat.n_sites, Wd, W.generator(3, W.STREAM_POTENTIAL, i))).to(dev)
        lats.append(lat)
        Vs.append(V)
    sites = sum(l.n_sites for l in lats)
    for lat, V in zip(lats, Vs):
        lat.set_potential(V.float())
    # start blocks from the library's counter-based generator: the complex64
    # block is the complex128 one rounded, so both runs start from the same phases
    rs = [pv.pv_random_block(l, nb, 300 + i, pv.PV_RANDOM_PHASE, pv.PV_C64, device=dev) for i, l in enumerate(lats)]
    batch = pv.Batch(lats)
    a = [7.0 + 0.5 * Wd for (_, Wd) in inst]
    # the batch's launch shape from its own autotuner (timed on its own steps)
    t0 = time.perf_counter()
    shape, tune_ms = pv.pv_batch_autotune(batch, rs, a, 0.0)
    tune_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    mu = pv.pv_batch_kpm_moments(batch, rs, M, a, 0.0)       # capture + first run
    torch.cuda.synchronize()
    first = time.perf_counter() - t0
    ms = _median_timed(torch, lambda: pv.pv_batch_kpm_moments(batch, rs, M, a, 0.0), 1)
    ok = bool(torch.isfinite(mu).all().item()) and float((mu[:, :, 0] - 1).abs().max().item()) < 1e-5
    mu64 = mu.cpu().numpy()
    lups = sum(l.n_rows for l in lats) * nb * (M // 2)
    b64 = sum(3 * l.n_rows * nb * 8 + l.n_sites * 4 for l in lats) * (M // 2)
    del rs
    torch.cuda.empty_cache()
    # per-instance complex128 loop (each instance its own launches), same phases
    for lat, V in zip(lats, Vs):
        lat.set_potential(V)
    mu128 = []

    def loop():
        mu128.clear()
        for i, (l, a_i) in enumerate(zip(lats, a)):
            r = pv.pv_random_block(l, nb, 300 + i, pv.PV_RANDOM_PHASE, pv.PV_C128, device=dev)
            mu128.append(pv.pv_kpm_moments(l, r, M, a_i, 0.0))
            del r
    ms_loop = _timed(torch, loop, 1)
    err = [float(np.abs(mu64[i] - m.cpu().numpy()).max()) for i, m in enumerate(mu128)]
    return {"workload": f"{n} TI realisations L~U{{24..96}} ({sites} sites), W~U[0.5,3], nb={nb}, M={M}",
            "batched_c64": {"ms_per_run": round(ms, 2), "GLUP/s": round(lups / (ms * 1e-3) / 1e9, 3),
                            "GB/s": round(b64 / (ms * 1e-3) / 1e9, 1), "first_call_s_incl_capture": round(first, 2),
                            "mu0_check": ok, "launches_per_run": M // 2 + 1, "graph_replays": batch.stats()[1],
                            "shape": {k: v for k, v in shape.items() if k in ("kernel", "elems_per_lane",
                                                                             "workgroup_size")},
                            "autotune_s": round(tune_s, 2), "autotune_ms_per_step": round(tune_ms, 3)},
            "loop_c128": {"M": M, "ms_per_run": round(ms_loop, 2),
                          "GLUP/s": round(lups / (ms_loop * 1e-3) / 1e9, 3),
                          "note": "phase draws on the device (pv_random_block) included in the timed loop"},
            "c64_vs_c128": {"max_abs_dmu": max(err), "median_abs_dmu": float(np.median(err)),
                            "max_abs_dmu_per_instance": [float(f"{e:.3g}") for e in err],
                            "note": "complex64 vectors, FP32 stencil, FP64 moments vs the complex128 run on the same "
                                    "phases, per instance over all 16 columns and 1024 moments"}}


def bench_adjoint(pv, torch, W, dev, ckpt=16):
    """TI 64^3 periodic, W = 1, nb = 8, M = 256: KPM forward vs the gradient
    (checkpointed forward + segment recompute + adjoint sweeps); graphene
    512 x 512 transmission gradient (50 steps, dt = 10, M = 64)."""
    st = pv.pv_model_stencil(pv.PV_MODEL_TI, [1.0, 2.0, 0.0, 0.0])
    lat = pv.Lattice((64, 64, 64), (1, 1, 1), st)
    V = torch.from_numpy(W.uniform_potential(lat.n_sites, 1.0, W.generator(4, W.STREAM_POTENTIAL))).to(dev)
    lat.set_potential(V)
    r = W.random_phase_device(lat.n_rows, 8, 400, dev)
    M = 256
    gbar = torch.from_numpy(W.generator(4, W.STREAM_COTANGENT).standard_normal((8, M))).to(dev)
    pv.pv_kpm_moments(lat, r, M, 7.0, 0.0)
    ms_f = _median_timed(torch, lambda: pv.pv_kpm_moments(lat, r, M, 7.0, 0.0), 2)
    pv.pv_kpm_moments_vjp(lat, r, M, 7.0, 0.0, gbar, ckpt)
    ms_b = _median_timed(torch, lambda: pv.pv_kpm_moments_vjp(lat, r, M, 7.0, 0.0, gbar, ckpt), 2)
    # the pair autograd runs: a forward that keeps its checkpoints, then the
    # recompute + adjoint from them
    _, work = pv.pv_kpm_moments_ckpt(lat, r, M, 7.0, 0.0, ckpt)
    ms_cf = _median_timed(torch, lambda: pv.pv_kpm_moments_ckpt(lat, r, M, 7.0, 0.0, ckpt), 2)
    pv.pv_kpm_moments_vjp_ckpt(lat, r, M, 7.0, 0.0, gbar, work, ckpt)
    ms_cb = _median_timed(torch, lambda: pv.pv_kpm_moments_vjp_ckpt(lat, r, M, 7.0, 0.0, gbar, work, ckpt), 2)
    del work
    # memory-rich variant: one segment (ckpt_every = M/2), every w_k kept by
    # the forward (M/2 + 6 vectors, 18 GB here), no recompute
    _, work = pv.pv_kpm_moments_ckpt(lat, r, M, 7.0, 0.0, M // 2)
    ms_af = _timed(torch, lambda: pv.pv_kpm_moments_ckpt(lat, r, M, 7.0, 0.0, M // 2), 2)
    pv.pv_kpm_moments_vjp_ckpt(lat, r, M, 7.0, 0.0, gbar, work, M // 2)
    ms_ab = _timed(torch, lambda: pv.pv_kpm_moments_vjp_ckpt(lat, r, M, 7.0, 0.0, gbar, work, M // 2), 2)
    del work
    torch.cuda.empty_cache()
    # central differences of the forward on 32 seeded sites
    g = pv.pv_kpm_moments_vjp(lat, r, M, 7.0, 0.0, gbar, ckpt).cpu().numpy()
    sites = W.sample_sites(lat.n_sites, 32, W.generator(4, W.STREAM_FD_SITES))
    fd = {}
    for h in (1e-6, 1e-4):
        worst = 0.0
        for m in sites:
            v0 = float(V[m].item())
            vals = []
            for sgn in (1, -1):
                V[m] = v0 + sgn * h
                vals.append(float((pv.pv_kpm_moments(lat, r, M, 7.0, 0.0) * gbar).sum().item()))
            V[m] = v0
            worst = max(worst, abs((vals[0] - vals[1]) / (2 * h) - g[m]))
        fd[f"h={h:g}"] = float(f"{worst / np.abs(g).max():.3g}")
    lups = lat.n_rows * 8 * (M // 2)
    # algorithmic bytes: a forward step 48 B per LUP (+ the field), the
    # checkpointed backward recomputes the forward once and runs adjoint
    # steps of 96 B per LUP
    fwd_bytes = bytes_per_step(lat.n_rows, lat.n_sites, 8, "c128") * (M // 2)
    fa_gbs = 4 * fwd_bytes / ((ms_cf + ms_cb) * 1e-3) / 1e9
    out = {"ti": {"workload": "TI 64^3, W=1, nb=8, M=256, checkpoint every 16, complex128",
                  "fwd_ms": round(ms_f, 3), "fwd_GLUP/s": round(lups / (ms_f * 1e-3) / 1e9, 3),
                  "fwd_GB/s": round(fwd_bytes / (ms_f * 1e-3) / 1e9, 1),
                  "fwd_frac_hbm_peak": round(fwd_bytes / (ms_f * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                  "fwd+adj_GB/s": round(fa_gbs, 1), "fwd+adj_frac_hbm_peak": round(fa_gbs / HBM_PEAK_GBS, 4),
                  "bytes_note": "fwd+adj bytes: forward 48 B/LUP, recompute 48, adjoint 96 (4x the forward's)",
                  "grad_ms": round(ms_b, 3), "grad_over_fwd": round(ms_b / ms_f, 2),
                  "fwd_ckpt_ms": round(ms_cf, 3), "adj_from_ckpt_ms": round(ms_cb, 3),
                  "fwd+adj_GLUP/s": round(lups / ((ms_cf + ms_cb) * 1e-3) / 1e9, 3),
                  "fwd+adj_over_fwd": round((ms_cf + ms_cb) / ms_f, 2),
                  "keep_all": {"fwd_ms": round(ms_af, 3), "adj_ms": round(ms_ab, 3),
                               "fwd+adj_GLUP/s": round(lups / ((ms_af + ms_ab) * 1e-3) / 1e9, 3),
                               "fwd+adj_over_fwd": round((ms_af + ms_ab) / ms_f, 2),
                               "note": "ckpt_every = M/2: the forward keeps every w_k, the adjoint recomputes none"},
                  "fd_max_rel_err": fd,
                  "fd_note": "gradient vs central differences of the forward on 32 seeded sites, max error relative "
                             "to max|grad|; at h=1e-6 the loss's rounding dominates",
                  "note": "GLUP/s counted on the forward's LUPs. fwd+adj: the forward keeping its checkpoints "
                          "(fwd_ckpt_ms) then recompute + adjoint from them (adj_from_ckpt_ms), as autograd runs "
                          "them; grad_ms: the one-call gradient (its own checkpointed forward + recompute + adjoint)"}}
    Li = Lj = 512
    g2 = pv.pv_model_stencil(pv.PV_MODEL_GRAPHENE2, [1.0])
    lg = pv.Lattice((Li, Lj), (0, 1), g2)
    Vg = torch.from_numpy(W.dot_array_potential(Li, Lj, radius=10, pitch=32, first_centre=(224, 144))).to(dev)
    psi0 = torch.from_numpy(W.gaussian_wave_packet(Li, Lj, i0=100, width=25, energy=0.2).reshape(-1, 1)).to(dev)
    region = torch.zeros(lg.n_rows, 1, dtype=torch.bool, device=dev)
    region.view(Lj, Li, 2)[:, 464:, :] = True

    grads = []

    def grad_T(keep_series=False):
        V = Vg.clone().requires_grad_(True)
        psiT = pv.cheb_propagate(V, psi0, lg, 3.06, 0.05, 10.0, 64, 50, keep_series)
        T = (psiT.abs() ** 2)[region].sum()
        T.backward()
        grads[:] = [V.grad]
        return T
    grad_T()
    gT = grads[0].cpu().numpy()

    def trans(Vv):
        lg.set_potential(Vv)
        p = psi0.clone()
        pv.pv_cheb_propagate(lg, p, 3.06, 0.05, 10.0, 64, 50)
        return float((p.abs() ** 2)[region].sum().item())
    fd_sites = list(W.sample_sites(lg.n_sites, 24, W.generator(4, W.STREAM_FD_SITES, 1))) + \
        list(np.argsort(-np.abs(gT))[:8])
    worst = 0.0
    for m in fd_sites:
        Vp, Vm = Vg.clone(), Vg.clone()
        Vp[m] += 1e-6
        Vm[m] -= 1e-6
        worst = max(worst, abs((trans(Vp) - trans(Vm)) / 2e-6 - gT[m]))
    lg.set_potential(Vg)
    fd_g = float(f"{worst / np.abs(gT).max():.3g}")
    ms_g = _timed(torch, grad_T, 1)
    # every step's Chebyshev vectors kept (50 * 64 vectors, 27 GB): no recompute
    grad_T(True)
    ms_gk = _timed(torch, lambda: grad_T(True), 1)
    torch.cuda.empty_cache()
    psi = psi0.clone()
    ms_gf = _timed(torch, lambda: pv.pv_cheb_propagate(lg, psi, 3.06, 0.05, 10.0, 64, 50), 1)
    out["graphene"] = {"workload": "graphene 512x512x2, 50 steps dt=10 M=64, dT/dV by autograd",
                       "fwd_ms": round(ms_gf, 2), "fwd+adj_ms": round(ms_g, 2),
                       "fwd+adj_keep_series_ms": round(ms_gk, 2),
                       "fwd_GLUP/s": round(lg.n_rows * 64 * 50 / (ms_gf * 1e-3) / 1e9, 3),
                       "fd_max_rel_err": {"h=1e-06": fd_g},
                       "fd_note": "dT/dV vs central differences on 32 sites (24 seeded, the 8 largest gradients)"}
    return out


def bench_weyl_spectral(pv, torch, W, dev, nk=64, M=256):
    """A(k, E) of a disordered Weyl semimetal along k_x (k_y = k_z = 0), the
    Fermi-arc setup of the paper's Weyl figure: 256 x 32 x 32 sites, periodic
    x, y, open z, box disorder of strength 2, test states on the z = 0
    surface; nk momenta x 2 orbitals as Bloch columns in blocks of 32, M
    moments each (complex128)."""
    import math
    st = pv.pv_model_stencil(pv.PV_MODEL_WEYL, [math.pi / 2])
    lat = pv.Lattice((256, 32, 32), (1, 1, 0), st)
    lat.set_potential(torch.from_numpy(W.uniform_potential(lat.n_sites, 2.0, W.generator(5, W.STREAM_POTENTIAL))).to(dev))
    kx = 2 * math.pi * np.arange(nk) / 256
    ks = np.array([[k, 0.0, 0.0] for k in kx for _ in (0, 1)])
    nu = [n for _ in kx for n in (0, 1)]
    a = 7.5
    blocks = [(ks[i:i + 32], nu[i:i + 32]) for i in range(0, len(nu), 32)]
    R = [pv.pv_bloch_block(lat, k, n, layer=(2, 0)) for k, n in blocks]
    pv.pv_kpm_moments(lat, R[0], M, a, 0.0)
    mus = []
    ms = _median_timed(torch, lambda: mus.extend(pv.pv_kpm_moments(lat, r, M, a, 0.0) for r in R), 1)
    mu = torch.cat(mus[-len(R):]).cpu().numpy()
    E = np.array([0.0])
    A0 = [float(pv.pv_kpm_spectral_function(mu[2 * i:2 * i + 2], E, a, 0.0, 32.0)[0]) for i in range(nk)]
    lups = lat.n_rows * 32 * (M // 2) * len(R)
    wbytes = bytes_per_step(lat.n_rows, lat.n_sites, 32, "c128") * (M // 2) * len(R)
    return {"workload": f"Weyl 256x32x32 (periodic x,y, open z), W=2, surface Bloch states, {nk} k_x x 2 orbitals, "
                        f"M={M}, complex128, blocks of 32",
            "ms_total": round(ms, 2), "GLUP/s": round(lups / (ms * 1e-3) / 1e9, 3),
            "GB/s": round(wbytes / (ms * 1e-3) / 1e9, 1),
            "A_E0_along_kx_first8": [round(v, 4) for v in A0[:8]]}


def _dsl_program(st: dict, extra=()) -> str:
    """DSL text (Sec. 3.2 format) of a stencil dict plus extra (offset, block)
    terms, with the per-site field as variable coefficient 0."""
    def num(z):
        z = complex(z)
        if z.imag == 0.0:
            return repr(z.real)
        if z.real == 0.0:
            return f"{z.imag!r}i"
        return f"{z.real!r}{z.imag:+}i"
    no = int(st["n_orb"])
    terms = list(zip([tuple(int(v) for v in o) for o in np.asarray(st["offsets"]).reshape(-1, 3)],
                     np.asarray(st["blocks"]).reshape(-1, no, no))) + list(extra)
    out = [f"dim {int(st['dim'])}", f"size {no}", "n_coeff_variable 1"]
    for off, B in terms:
        out.append("nn " + " ".join(str(v) for v in off))
        for k in range(no):
            out.append(f"l{k}; " + "; ".join(f"{q}|{num(B[k, q])}" for q in range(no) if B[k, q] != 0))
    out.append("nn 0 0 0")
    E = np.asarray(st["onsite"]).reshape(no, no)
    for k in range(no):
        ent = [f"{q}|{num(E[k, q])}" for q in range(no) if E[k, q] != 0] + [f"{k}|v|0"]
        out.append(f"l{k}; " + "; ".join(ent))
    return "\n".join(out) + "\n"


def bench_dsl(pv, torch, W, dev, nb=16):
    """Stencils given as DSL text, on the 256x256x64 lattice, Chebyshev step
    with dots, complex128: the TI program (recognised as the compiled TI
    family) and the TI plus next-nearest-neighbour hops -(t'/2) G1, t' = 0.1,
    along (+-1, 0, +-1), along (+-1, +-1, 0) and along (0, +-1, +-1) (no
    compiled family).  Those run on kernels generated from the stencil's
    pattern (staged: the third stages its side rows at z -+ 1 as well), each
    in the launch shape the autotuner picks, and on the interpreted generic
    kernels in their default shape (staged for the first two, direct for the
    third).  The TI program runs in the default and in the autotuned shape."""
    ti = pv.pv_model_stencil(pv.PV_MODEL_TI, [1.0, 2.0, 0.0, 0.0])
    G1 = np.diag([1.0, 1.0, -1.0, -1.0]).astype(np.complex128)
    h = -0.05 * G1
    xz = [((1, 0, 1), h), ((-1, 0, -1), h), ((1, 0, -1), h), ((-1, 0, 1), h)]
    xy = [((1, 1, 0), h), ((-1, -1, 0), h), ((1, -1, 0), h), ((-1, 1, 0), h)]
    yz = [((0, 1, 1), h), ((0, -1, -1), h), ((0, 1, -1), h), ((0, -1, 1), h)]
    out = {}
    for name, text in (("ti", _dsl_program(ti)), ("ti_nnn_xz", _dsl_program(ti, xz)),
                       ("ti_nnn_xy", _dsl_program(ti, xy)), ("ti_nnn_yz", _dsl_program(ti, yz))):
        st = pv.pv_dsl_stencil(text)
        lat = pv.Lattice(L_BENCH, (1, 1, 1), st)
        lat.set_potential(torch.from_numpy(W.uniform_potential(lat.n_sites, 2.0,
                                                               W.generator(WORKLOAD_INDEX, W.STREAM_POTENTIAL))).to(dev))
        w0 = W.random_phase_device(lat.n_rows, nb, 10 * WORKLOAD_INDEX + nb, dev)
        w1 = torch.empty_like(w0)
        dots = torch.empty((nb, 4), dtype=torch.float64, device=dev)
        state = [w0, w1]

        def step():
            pv.pv_spmmv(lat, state[1], state[0], 2.0 / A_SCALE, B_SHIFT, -1.0, z=state[0],
                        dot_flags=pv.PV_DOT_XX | pv.PV_DOT_XY, dots=dots, nb=nb)
            state.reverse()

        def timed():
            pv.pv_spmmv(lat, w0, w1, 1.0 / A_SCALE, B_SHIFT, 0.0, nb=nb)
            step()   # compiles a generated instance on first use
            # median of three timed runs: a one-off stall does not decide it
            ms = sorted(_timed(torch, step, 10) for _ in range(3))[1]
            b = bytes_per_step(lat.n_rows, lat.n_sites, nb, "c128")
            return {"ms_per_step": round(ms, 4), "GLUP/s": round(lat.n_rows * nb / (ms * 1e-3) / 1e9, 3),
                    "GB/s": round(b / (ms * 1e-3) / 1e9, 1)}

        generic = lat.family == 0
        entry = {"family": "generic" if generic else "compiled TI", "terms": int(len(st["offsets"]))}
        if generic:
            entry["kernels"] = "generated from the stencil's pattern"
            shape, _ = pv.pv_autotune(lat, nb, pv.PV_C128, cache_path=TUNE_CACHE)
            entry.update(timed())
            entry["shape"] = {k: v for k, v in shape.items() if v}
            pv.pv_lattice_set_codegen(lat, False)
            pv.pv_lattice_set_tuning(lat, pv.PV_C128, nb, None)
            entry["interpreted"] = timed()
        else:
            entry.update(timed())   # the default shape
            shape, _ = pv.pv_autotune(lat, nb, pv.PV_C128, cache_path=TUNE_CACHE)
            entry["autotuned"] = {**timed(), "shape": {k: v for k, v in shape.items() if v}}
        out[name] = entry
        del w0, w1, state
        torch.cuda.empty_cache()
    out["workload"] = f"TI 256x256x64 from DSL text, W=2, nb={nb}, complex128, Chebyshev step + dots"
    return out


def bench_fd(pv, torch, W, dev, half=0.05):
    """Interior eigenpairs near E = 0 of a TI slab like the paper's filter
    diagonalisation test cases: 240 x 240 x 6 sites, periodic x, y, open z
    (surface states in the bulk gap), W = 1, a = 6: trLanczosFD (block size 4)
    and ChebFD on the same window, complex128.  ChebFD takes a search space of
    about 2.5 times the pairs trLanczosFD finds (whole 32-column blocks) and a
    filter degree of 2.4 pi a / h for the window's half-width h: the Jackson
    damping then smears the window's edges over about 0.4 h.  ChebFD runs
    again with complex64 vectors (FP64 Gram and Rayleigh-Ritz) to a residual
    tolerance of 1e-4 a, its eigenvalues compared with the complex128 run's."""
    st = pv.pv_model_stencil(pv.PV_MODEL_TI, [1.0, 2.0, 0.0, 0.0])
    lat = pv.Lattice((240, 240, 6), (1, 1, 0), st)
    lat.set_potential(torch.from_numpy(W.uniform_potential(lat.n_sites, 1.0, W.generator(6, W.STREAM_POTENTIAL))).to(dev))
    a = 6.0
    V0 = torch.from_numpy(W.gaussian_block(lat.n_rows, 4, W.generator(6, W.STREAM_VECTORS))).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    th, res, _, it = pv.pv_trlanczos_fd(lat, V0, a, 0.0, -half, half, 400, 160, 1e-9 * a, max_restarts=40,
                                        raise_unconverged=False)
    torch.cuda.synchronize()
    t_tr = time.perf_counter() - t0
    out = {"workload": f"TI 240x240x6 (periodic x,y, open z), W=1, window |E| < {half}, complex128, tol 1e-9 a",
           "trlanczos": {"pairs": int(th.size), "restarts": it, "seconds": round(t_tr, 2),
                         "max_residual": float(res.max()) if th.size else None,
                         "theta_range": [float(th.min()), float(th.max())] if th.size else None}}
    print(f"# trlanczos: {json.dumps(out['trlanczos'])}", file=sys.stderr, flush=True)
    if th.size:
        nt = int(th.size)
        ns = -(-(5 * nt // 2) // 32) * 32
        X = torch.from_numpy(W.gaussian_block(lat.n_rows, ns, W.generator(6, W.STREAM_VECTORS, 1))).to(dev)
        t0 = time.perf_counter()
        degree = int(math.ceil(2.4 * math.pi * a / half))
        thf, resf, nconv, itf = pv.pv_chebfd(lat, X, 32, a, 0.0, -half, half, degree, nt, 1e-9 * a,
                                             max_iter=30, raise_on_fail=False)
        torch.cuda.synchronize()
        t_fd = time.perf_counter() - t0
        out["chebfd"] = {"search_vectors": ns, "degree": degree,
                         "converged": int(nconv), "targets": nt, "iterations": itf, "seconds": round(t_fd, 2),
                         "max_residual": float(resf[:nt].max()),
                         "max_abs_theta_diff_vs_trlanczos": float(np.abs(np.sort(thf[:nt]) - th).max())}
        out["chebfd_over_trlanczos_time"] = round(t_fd / t_tr, 2)
        # the same run with complex64 vectors (FP32 filter sweeps; Gram,
        # Rayleigh-Ritz and residuals in FP64), to a tolerance FP32 reaches
        X32 = torch.from_numpy(W.gaussian_block(lat.n_rows, ns, W.generator(6, W.STREAM_VECTORS, 1))
                               .astype(np.complex64)).to(dev)
        t0 = time.perf_counter()
        th32, res32, nconv32, it32 = pv.pv_chebfd(lat, X32, 32, a, 0.0, -half, half, degree, nt, 1e-4 * a,
                                                  max_iter=30, raise_on_fail=False)
        torch.cuda.synchronize()
        t32 = time.perf_counter() - t0
        out["chebfd_c64"] = {"converged": int(nconv32), "targets": nt, "iterations": it32, "seconds": round(t32, 2),
                             "tol": 1e-4 * a, "max_residual": float(res32[:nt].max()),
                             "max_abs_theta_diff_vs_c128": float(np.abs(np.sort(th32[:nt]) - np.sort(thf[:nt])).max()),
                             "note": "complex64 vectors, FP64 Gram / Rayleigh-Ritz / residuals"}
    out["note"] = ("the 256x256x64 periodic TI at W=2 (64 eigenvalues near E=0, degree 500) has an open bulk gap: a "
                   "KPM count finds 2.8 states with |E| < 0.5 and 11,882 with |E| < 0.7, so its 64 states nearest 0 "
                   "sit on a band edge inside the filter's resolution; the filter step at that size is the "
                   "filter_sweeps_ti256 workload, and the full interior run is this slab, the paper's kind of case")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--nb", type=int, default=32, help="block width of the headline line")
    ap.add_argument("--dtype", default="c128", choices=["c128", "c64"])
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-copy", action="store_true")
    ap.add_argument("--no-configs", action="store_true", help="skip the per-workload measurements")
    ap.add_argument("--no-fd", action="store_true", help="skip the interior-eigenpair comparison (about 35 s)")
    ap.add_argument("--shape", type=json.loads, default=None,
                    help="pin the headline launch shape (JSON object of pv_tuning fields) instead of autotuning")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build targets one GPU; --gpus {args.gpus} is not supported "
              "(multi-GPU sharding is described in the design notes, not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1708_09689_amd as pv
    import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    st = pv.pv_model_stencil(pv.PV_MODEL_TI, [1.0, 2.0, 0.0, 0.0])
    lat = pv.Lattice(L_BENCH, (1, 1, 1), st)
    V = W.uniform_potential(lat.n_sites, 2.0, W.generator(WORKLOAD_INDEX, W.STREAM_POTENTIAL))
    V64 = torch.from_numpy(V).to(dev)
    V32 = V64.float()

    def set_field(dtype):
        lat.set_potential(V64 if dtype == "c128" else V32)

    copy_gbs = None if args.no_copy else copy_probe(pv, torch, dev)
    triad_gbs = None if args.no_copy else triad_probe(pv, torch, dev)
    read_gbs = None if args.no_copy else read_probe(pv, torch, dev)
    memcpy_gbs = None if args.no_copy else memcpy_probe(torch, dev)
    torch_triad_gbs = None if args.no_copy else torch_triad_probe(torch, dev)

    # headline
    set_field(args.dtype)
    sw = Sweep(pv, torch, lat, args.nb, args.dtype, dev, shape=args.shape)
    ms = time_steps(torch, sw, args.warmup, args.steps)
    print(f"# headline {args.dtype} nb={args.nb}: {ms:.4f} ms/step, shape {sw.shape}", file=sys.stderr, flush=True)
    shape = sw.shape
    nbytes = bytes_per_step(lat.n_rows, lat.n_sites, args.nb, args.dtype)
    glups = lat.n_rows * args.nb / (ms * 1e-3) / 1e9
    achieved = nbytes / (ms * 1e-3) / 1e9
    del sw
    torch.cuda.empty_cache()

    variants = []
    if not args.no_variants:
        for dtype in ("c128", "c64"):
            set_field(dtype)
            for nb in (1, 4, 16, 32):
                s2 = Sweep(pv, torch, lat, nb, dtype, dev)
                m2 = median_steps(torch, s2)
                b2 = bytes_per_step(lat.n_rows, lat.n_sites, nb, dtype)
                variants.append({"dtype": dtype, "nb": nb, "shape": s2.shape, "ms_per_step": round(m2, 5),
                                 "GLUP/s": round(lat.n_rows * nb / (m2 * 1e-3) / 1e9, 3),
                                 "site_GLUP/s": round(lat.n_sites * nb / (m2 * 1e-3) / 1e9, 3),
                                 "GB/s": round(b2 / (m2 * 1e-3) / 1e9, 1),
                                 "frac_hbm_peak": round(b2 / (m2 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                 "bytes_per_LUP": round(b2 / (lat.n_rows * nb), 3)})
                print(f"# {dtype} nb={nb}: {m2:.4f} ms/step {variants[-1]['GB/s']} GB/s", file=sys.stderr, flush=True)
                del s2
                torch.cuda.empty_cache()
            # on-the-fly field (counter-based generator in the kernel): no field stream
            lat.set_random_potential(W.MASTER_SEED + WORKLOAD_INDEX, 2.0)
            for nb in (1, 4):
                s2 = Sweep(pv, torch, lat, nb, dtype, dev)
                m2 = median_steps(torch, s2)
                b2 = bytes_per_step(lat.n_rows, 0, nb, dtype)
                variants.append({"dtype": dtype, "nb": nb, "field": "generated in the kernel",
                                 "ms_per_step": round(m2, 5),
                                 "GLUP/s": round(lat.n_rows * nb / (m2 * 1e-3) / 1e9, 3),
                                 "GB/s": round(b2 / (m2 * 1e-3) / 1e9, 1),
                                 "frac_hbm_peak": round(b2 / (m2 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                 "bytes_per_LUP": round(b2 / (lat.n_rows * nb), 3)})
                print(f"# {dtype} nb={nb} generated field: {m2:.4f} ms/step {variants[-1]['GB/s']} GB/s",
                      file=sys.stderr, flush=True)
                del s2
                torch.cuda.empty_cache()

    configs = {}
    if not args.no_configs:
        set_field("c128")
        for name, fn in (("kpm_ti16", lambda: bench_kpm16(pv, torch, W, dev)),
                         ("filter_sweeps_ti256", lambda: bench_filter(pv, torch, lat, dev)),
                         ("plain_spmmv_ti256", lambda: bench_plain(pv, torch, lat, dev)),
                         ("chebtp_graphene1024", lambda: bench_chebtp_graphene(pv, torch, W, dev)),
                         ("batched_kpm_96", lambda: bench_batch(pv, torch, W, dev)),
                         ("adjoint", lambda: bench_adjoint(pv, torch, W, dev)),
                         ("weyl_spectral", lambda: bench_weyl_spectral(pv, torch, W, dev)),
                         ("dsl_stencils", lambda: bench_dsl(pv, torch, W, dev)),
                         ("random_start_block", lambda: bench_random_block(pv, torch, lat, dev))):
            t0 = time.perf_counter()
            configs[name] = fn()
            torch.cuda.empty_cache()
            print(f"# {name} done in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
        set_field(args.dtype)
    if not args.no_fd and not args.no_configs:
        t0 = time.perf_counter()
        configs["interior_eigenpairs"] = bench_fd(pv, torch, W, dev)
        print(f"# interior_eigenpairs done in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)

    cpu = None if args.no_cpu else cpu_baseline(args.nb)

    # the metric's comparisons in one place: FP64 vs FP32 vectors at the
    # headline block width, forward vs forward + adjoint
    parts = {"fp64": {"GLUP/s": round(glups, 3), "frac_hbm_peak": round(achieved / HBM_PEAK_GBS, 4)}}
    v32 = [v for v in variants if v["dtype"] == "c64" and v["nb"] == args.nb and "field" not in v]
    if v32:
        parts["fp32_vectors_fp64_dots"] = {"GLUP/s": v32[0]["GLUP/s"], "frac_hbm_peak": v32[0]["frac_hbm_peak"],
                                           "error_vs_fp64": fp32_step_error(pv, torch, lat, dev, args.nb, set_field)}
        set_field(args.dtype)
        torch.cuda.empty_cache()
    if "adjoint" in configs:
        ti = configs["adjoint"]["ti"]
        parts["forward_vs_forward_plus_adjoint"] = {"workload": ti["workload"], "fwd_GLUP/s": ti["fwd_GLUP/s"],
                                                    "fwd+adj_GLUP/s": ti["fwd+adj_GLUP/s"],
                                                    "fwd+adj_over_fwd": ti["fwd+adj_over_fwd"]}

    out = {
        "metric": METRIC,
        "value": round(glups, 3),
        "site_GLUP/s": round(lat.n_sites * args.nb / (ms * 1e-3) / 1e9, 3),
        "unit": "GLUP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.dtype == "c128" else "f32",
        "data": "synthetic",
        "config": {"workload": f"TI 256x256x64 periodic (D=16777216 rows), W=2, Chebyshev step + fused KPM dots, "
                               f"nb={args.nb}, {'complex128' if args.dtype == 'c128' else 'complex64 vectors, FP64 dots'}",
                   "lattice": list(L_BENCH), "n_orb": 4, "nb": args.nb, "rows": lat.n_rows,
                   "a": A_SCALE, "b": B_SHIFT, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": counted_traffic(args.dtype, args.nb, shape),
                     "traffic_GBs": (None if counted_traffic(args.dtype, args.nb, shape) is None else
                                     round(counted_traffic(args.dtype, args.nb, shape) / (ms * 1e-3) / 1e9, 1)),
                     "kernel": ("staged_kernel<PatTI>" if shape["kernel"] == 2 else "sweep_kernel<PatTI>")
                               + " (Chebyshev step, fused dots) + reduce_dots_kernel",
                     "launch_shape": shape,
                     "bytes_per_launch": nbytes},
        "copy_probe_GBs": None if copy_gbs is None else round(copy_gbs, 1),
        "frac_of_copy_probe": None if copy_gbs is None else round(achieved / copy_gbs, 4),
        "triad_probe_GBs": None if triad_gbs is None else round(triad_gbs, 1),
        "frac_of_triad_probe": None if triad_gbs is None else round(achieved / triad_gbs, 4),
        "read_probe_GBs": None if read_gbs is None else round(read_gbs, 1),
        "memcpy_d2d_GBs": None if memcpy_gbs is None else round(memcpy_gbs, 1),
        "torch_triad_GBs": None if torch_triad_gbs is None else round(torch_triad_gbs, 1),
        "metric_parts": parts,
        "variants": variants,
        "workloads": with_hbm_fracs(configs),
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
