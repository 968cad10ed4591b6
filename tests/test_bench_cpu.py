"""Host-side checks of the benchmark script's bookkeeping (no GPU needed):
the counted-traffic lookup matches a launch shape whether it is given in
full (as the autotuner returns it) or with the defaults left out (as it is
pinned on the command line), and nothing else."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import paper_1708_09689_amd as pv  # noqa: E402


def full(shape):
    out = {k: 0 for k in pv.TUNING_FIELDS}
    out.update(shape)
    return out


def test_counted_traffic_matches_full_and_partial_shapes():
    assert bench.COUNTED_TRAFFIC
    for (dtype, nb), entries in bench.COUNTED_TRAFFIC.items():
        for shape, nbytes in entries:
            assert set(shape) <= set(pv.TUNING_FIELDS)
            partial = {k: v for k, v in shape.items() if v}
            assert bench.counted_traffic(dtype, nb, full(shape)) == nbytes
            assert bench.counted_traffic(dtype, nb, partial) == nbytes
            # the algorithmic bytes bound the counted ones from below
            assert nbytes >= bench.bytes_per_step(256 * 256 * 64 * 4, 256 * 256 * 64, nb, dtype)


def test_counted_traffic_is_null_for_other_shapes():
    (dtype, nb), entries = next(iter(bench.COUNTED_TRAFFIC.items()))
    shape = dict(entries[0][0])
    shape["groups_per_xcd"] = 17
    assert bench.counted_traffic(dtype, nb, full(shape)) is None
    assert bench.counted_traffic(dtype, nb + 1, full(entries[0][0])) is None


def test_bench_refuses_several_gpus():
    """One GPU only: --gpus above 1 exits with a message before touching a GPU."""
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert out.returncode != 0 and "one GPU" in out.stderr


def test_every_workload_rate_gets_its_hbm_fraction():
    import bench
    d = {"a": {"GB/s": 4000.0, "runs": [{"approx_GB/s": 2000}]}, "b": {"GB/s": None}, "c": {"ms": 1.0}}
    out = bench.with_hbm_fracs(d)
    assert out["a"]["frac_hbm_peak"] == 0.5
    assert out["a"]["runs"][0]["frac_hbm_peak"] == 0.25
    assert "frac_hbm_peak" not in out["b"] and "frac_hbm_peak" not in out["c"]
