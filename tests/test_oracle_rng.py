"""Pins of the oracle's counter-based field generator: published SplitMix64
output sequences, counter form (any window of the stream), and the
distribution of the field (range, mean, variance, uniformity, lag
correlation) for the box disorder of strength W."""

import json
import os

import numpy as np

from oracle import rng

GOLD = os.path.join(os.path.dirname(__file__), "golden", "splitmix64.json")


def test_published_output_sequences():
    g = json.load(open(GOLD))
    for v in g["vectors"]:
        out = rng.splitmix64(v["seed"], 0, 3)
        if "outputs_hex" in v:
            assert [f"{int(o):016x}" for o in out] == v["outputs_hex"]
        else:
            assert [str(int(o)) for o in out] == v["outputs_dec"]


def test_counter_windows_agree():
    full = rng.splitmix64(99, 0, 1000)
    assert np.array_equal(rng.splitmix64(99, 417, 50), full[417:467])


def test_field_distribution():
    W = 2.0
    n = 1 << 20
    V = rng.field(12345, W, n)
    assert V.min() >= -W / 2 and V.max() < W / 2
    assert abs(V.mean()) < 4 * W / np.sqrt(12 * n)
    assert abs(V.var() - W * W / 12) < 0.01 * W * W / 12
    hist, _ = np.histogram(V, bins=64, range=(-W / 2, W / 2))
    expect = n / 64
    chi2 = ((hist - expect) ** 2 / expect).sum()
    assert chi2 < 63 + 6 * np.sqrt(2 * 63)          # chi-square, 63 dof, ~6 sigma
    u = rng.uniform(12345, n)
    r = np.corrcoef(u[:-1], u[1:])[0, 1]
    assert abs(r) < 5 / np.sqrt(n)


def test_field_is_one_rounded_product():
    """V = W (u - 1/2) with u a multiple of 2^-53: u - 1/2 is exact, so V is
    exactly representable as the rounded product (both sides agree bitwise)."""
    u = rng.uniform(7, 4096)
    assert np.array_equal(u * 2.0 ** 53, np.floor(u * 2.0 ** 53))
    d = u - 0.5
    assert np.array_equal(d + 0.5, u)
