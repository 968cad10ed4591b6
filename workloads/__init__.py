"""Seeded synthetic input generators.

This module is shared by the CPU oracle (``oracle/``) and the HIP path
(``paper_1708_09689_amd``).  It produces inputs only -- random on-site
potentials, random-phase start vectors, the quantum-dot gate potential, the
Gaussian wave packet, the sizes of a batch of disorder realisations -- and
holds none of the method's arithmetic (no Hamiltonian application, no
Chebyshev recurrence, no moments).  Both sides receive the same arrays.

Layout conventions used by every generator:

* site index   ``s = x + Lx*(y + Ly*z)``                (x fastest)
* row index    ``r = s*n_orb + o``
* element      ``e = r*nb + c``   (the vector block is [rows][nb], column fastest)

Seeds: master ``S = 1708096890 + workload_index``; sub-streams
1 = potential, 2 = start vectors, 3 = batch sizes / disorder strengths,
4 = finite-difference sites, 5 = cotangents.
"""

from __future__ import annotations

import math

import numpy as np

MASTER_SEED = 1708096890
STREAM_POTENTIAL = 1
STREAM_VECTORS = 2
STREAM_SIZES = 3
STREAM_FD_SITES = 4
STREAM_COTANGENT = 5


def generator(workload: int, stream: int, extra: int = 0) -> np.random.Generator:
    """Independent, reproducible numpy generator for (workload, stream, extra)."""
    ss = np.random.SeedSequence([MASTER_SEED + int(workload), int(stream), int(extra)])
    return np.random.Generator(np.random.PCG64(ss))


def uniform_potential(n: int, W: float, gen: np.random.Generator) -> np.ndarray:
    """On-site disorder V ~ U[-W/2, W/2], float64, length n (box distribution
    of strength W, as used for the disordered TI and Weyl models)."""
    return (W * (gen.random(int(n)) - 0.5)).astype(np.float64)


def random_phase_block(n_rows: int, nb: int, gen: np.random.Generator,
                       dtype=np.complex128) -> np.ndarray:
    """Random-phase vectors r_i = exp(i*phi), phi ~ U[0, 2pi): shape [n_rows, nb]."""
    phi = 2.0 * math.pi * gen.random((int(n_rows), int(nb)))
    return np.exp(1j * phi).astype(dtype)


def z4_phase_block(n_rows: int, nb: int, gen: np.random.Generator,
                   dtype=np.complex128) -> np.ndarray:
    """Phases drawn from {1, i, -1, -i}: exactly representable, |r_i| = 1."""
    k = gen.integers(0, 4, size=(int(n_rows), int(nb)))
    re = np.array([1.0, 0.0, -1.0, 0.0])[k]
    im = np.array([0.0, 1.0, 0.0, -1.0])[k]
    return (re + 1j * im).astype(dtype)


def gaussian_block(n_rows: int, nb: int, gen: np.random.Generator,
                   dtype=np.complex128) -> np.ndarray:
    """Complex normal entries (real and imaginary parts N(0,1))."""
    v = gen.standard_normal((int(n_rows), int(nb))) + 1j * gen.standard_normal((int(n_rows), int(nb)))
    return v.astype(dtype)


def basis_block(n_rows: int, cols, dtype=np.complex128) -> np.ndarray:
    """Unit vectors: column c is e_{cols[c]}."""
    cols = list(cols)
    out = np.zeros((int(n_rows), len(cols)), dtype=dtype)
    for c, r in enumerate(cols):
        out[int(r), c] = 1.0
    return out


def dot_array_potential(Li: int, Lj: int, n_dots=(8, 8), radius: float = 20.0,
                        V0: float = 0.1, dV: float = 0.0, pitch: float = 64.0,
                        first_centre=(448.0, 288.0)) -> np.ndarray:
    """Gate potential of a square array of discs on a zero background.

    V(i, j) = sum_{l,k} V_k * [ |R_{l,k} - (i, j)| < radius ],
    V_k = V0 + dV * |k - K/2|, R_{l,k} = first_centre + pitch*(l, k),
    l = 0..n_dots[0]-1 along i, k = 0..n_dots[1]-1 along j.
    Returns float64 per site, site index s = i + Li*j.
    """
    ii = np.arange(Li, dtype=np.float64)[None, :]
    jj = np.arange(Lj, dtype=np.float64)[:, None]
    V = np.zeros((Lj, Li), dtype=np.float64)
    L, K = n_dots
    for l in range(L):
        for k in range(K):
            ci = first_centre[0] + pitch * l
            cj = first_centre[1] + pitch * k
            Vk = V0 + dV * abs(k - K / 2.0)
            inside = (ii - ci) ** 2 + (jj - cj) ** 2 < radius * radius
            V[inside] += Vk
    return V.reshape(-1)


def _honeycomb_f(k1: float, k2: float) -> complex:
    return 1.0 + np.exp(-1j * k1) + np.exp(-1j * k2)


def gaussian_wave_packet(Li: int, Lj: int, i0: float, width: float, energy: float,
                         t: float = 1.0) -> np.ndarray:
    """Gaussian wave packet on the two-site (A, B) honeycomb index grid.

    psi(i, j, o) = exp(-(i - i0)^2 / (4 width^2)) * exp(i (k1 i + k2 j)) * u_o,
    with k2 the lattice momentum of the j-periodic ribbon closest to the Dirac
    value -2pi/3, k1 > 2pi/3 chosen so that t*|1 + e^{-ik1} + e^{-ik2}| equals
    ``energy`` (upper band, moving towards +i), and u = (1, -conj(f)/|f|)/sqrt 2
    the upper-band spinor.  Normalised to unit 2-norm.  Returns complex128 of
    shape [Li*Lj*2] in the row layout (site*2 + o).
    """
    k2 = 2.0 * math.pi * round(-Lj / 3.0) / Lj
    target = energy / t
    lo, hi = 2.0 * math.pi / 3.0, 2.0 * math.pi / 3.0 + 1.0
    # |f| grows monotonically with k1 on this bracket, away from the Dirac point
    if not abs(_honeycomb_f(lo, k2)) < target < abs(_honeycomb_f(hi, k2)):
        raise ValueError("packet energy outside the bracketed branch")
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if abs(_honeycomb_f(mid, k2)) < target:
            lo = mid
        else:
            hi = mid
    k1 = 0.5 * (lo + hi)
    f = _honeycomb_f(k1, k2)
    uA = 1.0 / math.sqrt(2.0)
    uB = -np.conj(f) / abs(f) / math.sqrt(2.0)
    i = np.arange(Li, dtype=np.float64)[None, :]
    j = np.arange(Lj, dtype=np.float64)[:, None]
    env = np.exp(-((i - i0) ** 2) / (4.0 * width * width))
    phase = np.exp(1j * (k1 * i + k2 * j))
    amp = (env * phase).reshape(-1)
    psi = np.empty((Li * Lj, 2), dtype=np.complex128)
    psi[:, 0] = amp * uA
    psi[:, 1] = amp * uB
    psi = psi.reshape(-1)
    return psi / np.linalg.norm(psi)


def batch_instances(n: int, gen: np.random.Generator, L_range=(24, 96),
                    W_range=(0.5, 3.0)):
    """Sizes and disorder strengths of a batch of independent cubic lattices:
    L ~ U{L_range[0]..L_range[1]}, W ~ U[W_range]."""
    Ls = gen.integers(L_range[0], L_range[1] + 1, size=int(n))
    Ws = W_range[0] + (W_range[1] - W_range[0]) * gen.random(int(n))
    return [(int(L), float(W)) for L, W in zip(Ls, Ws)]


def sample_sites(n_sites: int, count: int, gen: np.random.Generator) -> np.ndarray:
    """Distinct sorted site indices, for sampled checks and finite differences."""
    count = min(int(count), int(n_sites))
    return np.sort(gen.choice(int(n_sites), size=count, replace=False)).astype(np.int64)


def random_phase_device(n_rows: int, nb: int, seed: int, device, dtype="complex128"):
    """Random-phase block generated on the device with torch's seeded
    generator (for large performance runs where host generation and upload
    would dominate; same distribution as random_phase_block, different
    stream).  Returns a contiguous torch tensor [n_rows, nb]."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(MASTER_SEED + seed))
    real = torch.float64 if dtype == "complex128" else torch.float32
    phi = torch.rand((int(n_rows), int(nb)), generator=g, device=device, dtype=real) * (2.0 * math.pi)
    return torch.polar(torch.ones_like(phi), phi).contiguous()
