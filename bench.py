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
import os
import sys
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


def bytes_per_step(n_rows: int, n_sites: int, nb: int, dtype: str) -> int:
    """Algorithmic HBM bytes of one Chebyshev sweep: read x (w_k), read z
    (w_{k-1}), write y (w_{k+1}), read the on-site field once per site."""
    e = 16 if dtype == "c128" else 8
    v = 8 if dtype == "c128" else 4
    return 3 * n_rows * nb * e + n_sites * v


class Sweep:
    """State of one (dtype, nb) Chebyshev recurrence on the benchmark lattice."""

    def __init__(self, pv, torch, lat, nb, dtype, dev):
        self.pv, self.torch, self.lat, self.nb, self.dtype = pv, torch, lat, nb, dtype
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


def cpu_baseline(nb: int, budget_s: float = 12.0) -> dict:
    """The oracle (scipy CSR SpMMV + numpy dots, one thread) on a bounded
    sample of the same workload: the same x-y planes, 4 of the 64 z-layers."""
    import workloads as W
    from oracle import hamiltonian, lattice, models, spmmv
    L = (L_BENCH[0], L_BENCH[1], 4)
    olat = lattice.Lattice(L, (1, 1, 1), 4)
    V = W.uniform_potential(olat.n_sites, 2.0, W.generator(WORKLOAD_INDEX, W.STREAM_POTENTIAL))
    H = hamiltonian.assemble(models.topological_insulator(1.0, 2.0), olat, V)
    g = W.generator(WORKLOAD_INDEX, W.STREAM_VECTORS, nb)
    w0 = W.random_phase_block(olat.n_rows, nb, g)
    w1 = spmmv.spmmv(H, w0, 1.0 / A_SCALE, B_SHIFT, 0.0)
    sweeps = 0
    t0 = time.perf_counter()
    while True:
        w2 = spmmv.spmmv(H, w1, 2.0 / A_SCALE, B_SHIFT, -1.0, w0)
        spmmv.block_dots(w1, w2)
        w0, w1 = w1, w2
        sweeps += 1
        el = time.perf_counter() - t0
        if el > budget_s:
            break
    glups = olat.n_rows * nb * sweeps / el / 1e9
    return {"value": round(glups, 5), "unit": "GLUP/s", "cores": 1, "kind": "oracle",
            "sample": f"TI {L[0]}x{L[1]}x{L[2]} periodic (4 of 64 z-layers), W=2, nb={nb}, complex128, "
                      f"{sweeps} Chebyshev sweeps + dots in {el:.1f} s, scipy CSR + numpy, 1 thread"}


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

    # headline
    set_field(args.dtype)
    sw = Sweep(pv, torch, lat, args.nb, args.dtype, dev)
    ms = time_steps(torch, sw, args.warmup, args.steps)
    print(f"# headline {args.dtype} nb={args.nb}: {ms:.4f} ms/step", file=sys.stderr, flush=True)
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
                m2 = time_steps(torch, s2, 3, 10)
                b2 = bytes_per_step(lat.n_rows, lat.n_sites, nb, dtype)
                variants.append({"dtype": dtype, "nb": nb, "ms_per_step": round(m2, 5),
                                 "GLUP/s": round(lat.n_rows * nb / (m2 * 1e-3) / 1e9, 3),
                                 "site_GLUP/s": round(lat.n_sites * nb / (m2 * 1e-3) / 1e9, 3),
                                 "GB/s": round(b2 / (m2 * 1e-3) / 1e9, 1),
                                 "frac_hbm_peak": round(b2 / (m2 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                 "bytes_per_LUP": round(b2 / (lat.n_rows * nb), 3)})
                print(f"# {dtype} nb={nb}: {m2:.4f} ms/step {variants[-1]['GB/s']} GB/s", file=sys.stderr, flush=True)
                del s2
                torch.cuda.empty_cache()

    cpu = None if args.no_cpu else cpu_baseline(args.nb)

    out = {
        "metric": METRIC,
        "value": round(glups, 3),
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
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "sweep_kernel<PatTI> + reduce_dots_kernel (per step)",
                     "bytes_per_launch": nbytes},
        "copy_probe_GBs": None if copy_gbs is None else round(copy_gbs, 1),
        "frac_of_copy_probe": None if copy_gbs is None else round(achieved / copy_gbs, 4),
        "variants": variants,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
