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


def _golden_outputs():
    g = json.load(open(GOLD))
    out = {}
    for v in g["vectors"]:
        out[v["seed"]] = ([int(h, 16) for h in v["outputs_hex"]] if "outputs_hex" in v
                          else [int(d) for d in v["outputs_dec"]])
    return out


def test_start_blocks_from_published_outputs():
    """Entries 0, 1, 2 of a 3-column block are the first three published
    outputs, mapped by the phase definitions (integers from the golden file,
    not from the oracle's generator)."""
    for seed, outs in _golden_outputs().items():
        z4 = rng.random_block(seed, 1, 3, rng.Z4)[0]
        ph = rng.random_block(seed, 1, 3, rng.PHASE)[0]
        for j, o in enumerate(outs):
            k = o >> 62
            assert z4[j] == (1j) ** k
            u = (o >> 11) / 2.0 ** 53
            assert abs(abs(ph[j]) - 1.0) < 1e-15
            assert abs((np.angle(ph[j]) / (2 * np.pi)) % 1.0 - u) < 1e-15


def test_start_block_counter_form():
    """A row window (row0) and sampled entries are the same values as the
    whole block: the entries depend on (seed, global index) only."""
    for kind in (rng.PHASE, rng.Z4):
        full = rng.random_block(31, 100, 4, kind)
        assert np.array_equal(rng.random_block(31, 63, 4, kind, row0=37), full[37:])
        r = np.array([0, 5, 99, 37]), np.array([3, 0, 2, 1])
        assert np.array_equal(rng.random_block_at(31, 4, kind, *r), full[r])
        # the same stream read with another block width keeps each index's value
        assert np.array_equal(rng.random_block(31, 200, 2, kind).reshape(-1), full.reshape(-1))


def test_start_block_distribution():
    """Unit modulus; uniform phases (chi-square over 32 bins), Z4 values
    equally likely; E[v] = E[v^2] = 0 for both kinds and E[v^4] = 1 for Z4
    only; columns uncorrelated."""
    n, nb = 1 << 20, 16
    ph = rng.random_block(2024, n // nb, nb, rng.PHASE)
    z4 = rng.random_block(2024, n // nb, nb, rng.Z4)
    assert np.abs(np.abs(ph) - 1).max() < 1e-15 and np.array_equal(np.abs(z4), np.ones_like(z4.real))
    tol = 5 / np.sqrt(n)
    for b in (ph, z4):
        assert abs(b.mean()) < tol and abs((b ** 2).mean()) < tol
        c = (b[:, 0].conj() * b[:, 1]).mean()
        assert abs(c) < 5 / np.sqrt(n // nb)
    assert abs((ph ** 4).mean()) < tol and np.allclose((z4 ** 4).mean(), 1.0)
    hist, _ = np.histogram(np.angle(ph).reshape(-1), bins=32, range=(-np.pi, np.pi))
    chi2 = ((hist - n / 32) ** 2 / (n / 32)).sum()
    assert chi2 < 31 + 6 * np.sqrt(2 * 31)
    counts = np.array([(z4 == v).sum() for v in (1, 1j, -1, -1j)])
    assert np.abs(counts - n / 4).max() < 6 * np.sqrt(n * 3 / 16)


def test_start_blocks_give_an_unbiased_trace():
    """The stochastic trace (Sec. 4.2): the column mean of <r_c, A r_c> is
    Tr A up to the sampling error sqrt(sum_{i != j} |A_ij|^2 / R)."""
    g = np.random.default_rng(3)
    D, R = 24, 4096
    A = g.standard_normal((D, D)) + 1j * g.standard_normal((D, D))
    A = A + A.conj().T
    off = np.sqrt((np.abs(A) ** 2).sum() - (np.abs(np.diag(A)) ** 2).sum())
    for kind in (rng.PHASE, rng.Z4):
        r = rng.random_block(77, D, R, kind)
        est = np.einsum("ic,ij,jc->c", r.conj(), A, r).real.mean()
        assert abs(est - np.trace(A).real) < 5 * off / np.sqrt(R)
        # a diagonal A gives the trace exactly, column by column
        Dg = np.diag(np.diag(A).real)
        assert np.allclose(np.einsum("ic,ij,jc->c", r.conj(), Dg, r).real, np.trace(Dg), rtol=1e-13)
