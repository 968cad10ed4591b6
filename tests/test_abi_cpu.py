"""Host-side tests of the C ABI (no GPU needed): the library loads and exports
every declared symbol, model stencils equal the oracle's model terms,
descriptor validation, stencil-family selection, and the host-only helpers."""

import ctypes
import os
import re

import numpy as np
import pytest

import paper_1708_09689_amd as pv
from oracle import chebtp, kpm, models

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(pv.LIB_PATH):
        pytest.skip("libpvdtm.so not built")
    return pv.lib()


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "pvdtm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pv_[a-z0-9_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported(lib):
    syms = declared_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(lib, s), s
        assert s in pv.SIGNATURES, f"binding lacks {s}"


def test_version_and_status_strings(lib):
    assert lib.pv_version() >= 1
    assert lib.pv_status_string(0) == b"ok"


def oracle_descriptor(model):
    """Descriptor-convention blocks from the oracle model: (H x)[s] += A x[s - e]
    + A^H x[s + e] for every hop (e, A)."""
    out = {}
    for e, A in model.hops:
        out[tuple(-np.asarray(e))] = A
        out[tuple(np.asarray(e))] = A.conj().T
    return out, model.onsite


@pytest.mark.parametrize("code,model,params", [
    (pv.PV_MODEL_TI, models.topological_insulator(t=1.0, m=2.0), [1.0, 2.0, 0.0, 0.0]),
    (pv.PV_MODEL_TI, models.topological_insulator(t=0.7, m=1.3, delta1=0.2, delta2=-0.1), [0.7, 1.3, 0.2, -0.1]),
    (pv.PV_MODEL_GRAPHENE2, models.graphene_two_site(t=1.0), [1.0]),
    (pv.PV_MODEL_GRAPHENE4, models.graphene_four_site(t=1.0), [1.0]),
    (pv.PV_MODEL_WEYL, models.weyl_semimetal(), [np.pi / 2]),
])
def test_model_stencils_equal_oracle_terms(lib, code, model, params):
    st = pv.pv_model_stencil(code, params)
    ref, E0 = oracle_descriptor(model)
    assert st["n_orb"] == model.n_orb
    assert len(st["offsets"]) == len(ref)
    for off, B in zip(st["offsets"], st["blocks"]):
        assert np.abs(B - ref[tuple(off)]).max() < 1e-15
    assert np.abs(st["onsite"] - E0).max() < 1e-15


@pytest.mark.parametrize("code,params,L,family", [
    (pv.PV_MODEL_TI, [1.0, 2.0, 0, 0], (4, 4, 4), 1),
    (pv.PV_MODEL_TI, [1.0, 2.0, 0.3, 0], (4, 4, 4), 0),   # Delta1 breaks the compiled on-site structure
    (pv.PV_MODEL_GRAPHENE2, [1.0], (5, 4), 2),
    (pv.PV_MODEL_GRAPHENE4, [1.0], (5, 4), 3),
    (pv.PV_MODEL_WEYL, [np.pi / 2], (4, 3, 3), 4),
])
def test_family_selection(lib, code, params, L, family):
    lat = pv.Lattice(L, (1, 1, 1), pv.pv_model_stencil(code, params))
    assert lat.family == family
    assert lat.n_sites == int(np.prod(L))


def test_descriptor_validation(lib):
    st = pv.pv_model_stencil(pv.PV_MODEL_TI, [1.0, 2.0, 0, 0])
    bad = dict(st)
    bad["blocks"] = st["blocks"].copy()
    bad["blocks"][0, 0, 3] += 0.1j
    with pytest.raises(pv.PvError) as e:
        pv.Lattice((4, 4, 4), (1, 1, 1), bad)
    assert e.value.status == 3
    pv.Lattice((4, 4, 4), (1, 1, 1), bad, check_hermitian=False)  # accepted without the check
    # n_orb = 3 unsupported
    s3 = {"dim": 3, "n_orb": 3, "offsets": np.zeros((0, 3)), "blocks": np.zeros((0, 3, 3)),
          "onsite": np.eye(3), "pot_mode": 1}
    with pytest.raises(pv.PvError) as e:
        pv.Lattice((4, 4, 4), (1, 1, 1), s3)
    assert e.value.status == 2
    # offsets outside {-1,0,1}, zero offset, duplicates
    for offs in ([[2, 0, 0]], [[0, 0, 0]]):
        s = {"dim": 3, "n_orb": 1, "offsets": np.array(offs), "blocks": np.ones((1, 1, 1)),
             "onsite": np.zeros((1, 1)), "pot_mode": 1}
        with pytest.raises(pv.PvError):
            pv.Lattice((4, 4, 4), (1, 1, 1), s, check_hermitian=False)
    s = {"dim": 3, "n_orb": 1, "offsets": np.array([[1, 0, 0], [1, 0, 0]]), "blocks": np.ones((2, 1, 1)),
         "onsite": np.zeros((1, 1)), "pot_mode": 1}
    with pytest.raises(pv.PvError):
        pv.Lattice((4, 4, 4), (1, 1, 1), s, check_hermitian=False)
    # 2D lattice with L[2] != 1
    g = pv.pv_model_stencil(pv.PV_MODEL_GRAPHENE2, [1.0])
    with pytest.raises(pv.PvError):
        pv.Lattice((4, 4, 2), (1, 1, 1), g)


def test_x_row_length_limit(lib):
    """The sweeps address an x row with 32-bit offsets: a lattice whose x row
    of a PV_MAX_NB-wide complex128 block reaches 2^31 bytes is refused at
    creation (long ribbons), the longest row below that is accepted."""
    g = pv.pv_model_stencil(pv.PV_MODEL_GRAPHENE2, [1.0])
    limit = (1 << 31) // (2 * pv.PV_MAX_NB * 16)      # sites per row with n_orb = 2
    with pytest.raises(pv.PvError) as e:
        pv.Lattice((limit, 1), (0, 1), g)
    assert e.value.status == 2
    assert b"exceeds 2^31 bytes" in lib.pv_last_error()
    lat = pv.Lattice((limit - 1, 1), (0, 1), g)
    assert lat.n_sites == limit - 1
    ti = pv.pv_model_stencil(pv.PV_MODEL_TI, [1.0, 2.0, 0, 0])
    with pytest.raises(pv.PvError) as e:
        pv.Lattice(((1 << 31) // (4 * pv.PV_MAX_NB * 16), 1, 1), (1, 1, 1), ti)
    assert e.value.status == 2


def test_argument_errors_return_before_any_launch(lib):
    lat = pv.Lattice((4, 4, 4), (1, 1, 1), pv.pv_model_stencil(pv.PV_MODEL_TI, [1.0, 2.0, 0, 0]))
    one = np.ones(4)
    fake = ctypes.c_void_p(1 << 20)   # never dereferenced: validation fails first
    # nb not a power of two
    st = lib.pv_spmmv(lat.handle, 0, 3, fake, None, fake, pv._dptr(one), pv._dptr(one), pv._dptr(np.zeros(4)),
                      0, None, fake, 1 << 20, None)
    assert st == 2
    # x aliases y
    st = lib.pv_spmmv(lat.handle, 0, 1, fake, None, fake, pv._dptr(one), pv._dptr(one), pv._dptr(np.zeros(4)),
                      0, None, fake, 1 << 20, None)
    assert st == 1
    # odd M
    st = lib.pv_kpm_moments(lat.handle, 0, 1, 7, 7.0, 0.0, fake, fake, fake, 1 << 30, None)
    assert st == 1
    # workspace too small
    st = lib.pv_kpm_moments(lat.handle, 0, 1, 8, 7.0, 0.0, fake, fake, fake, 16, None)
    assert st == 4
    # a <= 0
    st = lib.pv_kpm_moments(lat.handle, 0, 1, 8, 0.0, 0.0, fake, fake, fake, 1 << 30, None)
    assert st == 1
    assert b"a > 0" in lib.pv_last_error()
    # misaligned complex128 pointer
    st = lib.pv_kpm_moments(lat.handle, 0, 1, 8, 7.0, 0.0, ctypes.c_void_p((1 << 20) + 8), fake, fake, 1 << 30, None)
    assert st == 1


def test_tp_coefficients_match_oracle(lib):
    for adt in (0.0, 3.3, 30.6, -12.0):
        c = pv.pv_cheb_tp_coefficients(1.0, adt, 80)
        ref = chebtp.tp_coefficients(1.0, adt, 80)
        assert np.abs(c - ref).max() < 1e-15


def test_kpm_dos_matches_oracle(lib):
    g = np.random.default_rng(3)
    mu = np.concatenate([[1.0], 0.3 * g.standard_normal(63) / np.arange(1, 64)])
    E = np.linspace(-6.9, 6.9, 101)
    rho = pv.pv_kpm_dos(mu, E, 7.0, 0.0)
    ref = kpm.dos(mu, E, 7.0, 0.0)
    assert np.abs(rho - ref).max() < 1e-13


@pytest.mark.parametrize("n", [1, 2, 5, 17, 48])
def test_host_jacobi_eigensolver(lib, n):
    g = np.random.default_rng(n)
    A = g.standard_normal((n, n)) + 1j * g.standard_normal((n, n))
    A = A + A.conj().T
    w, V = pv.pv_host_heev(A)
    ref = np.linalg.eigvalsh(A)
    assert np.abs(w - ref).max() < 1e-12 * max(1.0, np.abs(ref).max())
    assert np.abs(V.conj().T @ V - np.eye(n)).max() < 1e-12
    assert np.abs(A @ V - V * w[None, :]).max() < 1e-11 * max(1.0, np.abs(ref).max())


def test_host_jacobi_degenerate_pairs(lib):
    """Kramers-like doubly degenerate spectrum: eigenvalues exact, vectors orthonormal."""
    g = np.random.default_rng(7)
    Q, _ = np.linalg.qr(g.standard_normal((12, 12)) + 1j * g.standard_normal((12, 12)))
    d = np.repeat(np.linspace(-2, 2, 6), 2)
    A = Q @ np.diag(d) @ Q.conj().T
    w, V = pv.pv_host_heev(A)
    assert np.abs(w - np.sort(d)).max() < 1e-12
    assert np.abs(V.conj().T @ V - np.eye(12)).max() < 1e-12


def test_chebfd_filter_coefficients_match_oracle(lib):
    from oracle import chebfd
    for (l, r, a, b, K) in [(-0.8, 0.8, 7.0, 0.0, 300), (-1.0, 0.5, 6.0, 0.2, 50), (0.1, 0.3, 3.1, 0.0, 1)]:
        c = pv.pv_chebfd_filter_coefficients(l, r, a, b, K)
        assert np.abs(c - chebfd.filter_coefficients(l, r, a, b, K)).max() < 1e-15


def test_tuning_set_get_and_validation(lib):
    lat = pv.Lattice((6, 5, 4), (1, 1, 1), pv.pv_model_stencil(pv.PV_MODEL_TI, [1.0, 2.0, 0, 0]))
    assert pv.pv_lattice_get_tuning(lat, pv.PV_C128, 4) == {k: 0 for k in pv.TUNING_FIELDS}
    sh = {"kernel": 2, "elems_per_lane": 2, "strip_rows": 8, "walk_planes": 3, "groups_per_xcd": 40, "workgroup_size": 512}
    pv.pv_lattice_set_tuning(lat, pv.PV_C128, 4, sh)
    got = pv.pv_lattice_get_tuning(lat, pv.PV_C128, 4)
    assert all(got[k] == sh.get(k, 0) for k in pv.TUNING_FIELDS)
    assert pv.pv_lattice_get_tuning(lat, pv.PV_C128, 8)["kernel"] == 0      # per block width
    assert pv.pv_lattice_get_tuning(lat, pv.PV_C64, 4)["kernel"] == 0       # per dtype
    for bad, dt in [({"kernel": 3}, pv.PV_C128), ({"elems_per_lane": 4}, pv.PV_C128),
                    ({"elems_per_lane": 1}, pv.PV_C64), ({"groups_per_xcd": 257}, pv.PV_C128),
                    ({"tiles_per_group": 65}, pv.PV_C128), ({"walk_planes": -1}, pv.PV_C128),
                    ({"workgroup_size": 128}, pv.PV_C128), ({"workgroup_size": 1024}, pv.PV_C64)]:
        with pytest.raises(pv.PvError) as e:
            pv.pv_lattice_set_tuning(lat, dt, 4, bad)
        assert e.value.status == 1
    with pytest.raises(pv.PvError):
        pv.pv_lattice_set_tuning(lat, pv.PV_C128, 3, sh)                    # nb not a power of two
    pv.pv_lattice_set_tuning(lat, pv.PV_C128, 4, None)
    assert pv.pv_lattice_get_tuning(lat, pv.PV_C128, 4)["kernel"] == 0


def test_random_potential_validation(lib):
    st = pv.pv_model_stencil(pv.PV_MODEL_TI, [1.0, 2.0, 0, 0])
    lat = pv.Lattice((4, 4, 4), (1, 1, 1), st)
    lat.set_random_potential(2**64 - 1, 2.0)          # any 64-bit seed
    with pytest.raises(pv.PvError):
        lat.set_random_potential(1, float("nan"))
    s0 = dict(st)
    s0["pot_mode"] = pv.PV_POT_NONE
    lat0 = pv.Lattice((4, 4, 4), (1, 1, 1), s0)
    with pytest.raises(pv.PvError) as e:
        lat0.set_random_potential(1, 1.0)
    assert e.value.status == 1


def test_spectral_function_matches_oracle(lib):
    from oracle import spectral
    g = np.random.default_rng(5)
    mu = np.concatenate([np.full((3, 1), 0.5), 0.2 * g.standard_normal((3, 47)) / np.arange(1, 48)], axis=1)
    E = np.linspace(-6.5, 6.5, 77)
    A = pv.pv_kpm_spectral_function(mu, E, 7.0, 0.1, 2.0)
    assert np.abs(A - spectral.spectral_function(mu, E, 7.0, 0.1, 2.0)).max() < 1e-13


def test_trlanczos_filter_matches_oracle(lib):
    from oracle import trlanczos
    for (l, r, a, b, K) in [(0.9, 1.3, 7.0, 0.1, 150), (-0.2, 0.2, 6.0, 0.0, 40), (2.0, 2.5, 3.1, 0.05, 300)]:
        c, tau = pv.pv_trlanczos_filter(l, r, a, b, K)
        rc, rtau = trlanczos.delta_filter(l, r, a, b, K)
        assert np.abs(c - rc).max() < 1e-13 and abs(tau - rtau) < 1e-13


def test_gradient_split_entry_points_validate_before_any_launch(lib):
    """The checkpointing forwards and the adjoints that read their workspace
    reject bad arguments with a status before touching the device."""
    lat = pv.Lattice((4, 4, 4), (1, 1, 1), pv.pv_model_stencil(pv.PV_MODEL_TI, [1.0, 2.0, 0, 0]))
    fake = ctypes.c_void_p(1 << 20)   # never dereferenced: validation fails first
    other = ctypes.c_void_p(1 << 21)
    big = 1 << 40
    # KPM: odd M, interval 0, workspace too small, gbar NULL
    assert lib.pv_kpm_moments_ckpt(lat.handle, 0, 1, 7, 7.0, 0.0, fake, fake, 4, fake, big, None) == 1
    assert lib.pv_kpm_moments_ckpt(lat.handle, 0, 1, 8, 7.0, 0.0, fake, fake, 0, fake, big, None) == 1
    assert lib.pv_kpm_moments_ckpt(lat.handle, 0, 1, 8, 7.0, 0.0, fake, fake, 4, fake, 16, None) == 4
    need = lib.pv_kpm_vjp_workspace_size(lat.handle, 0, 1, 8, 4)
    assert need > 0
    # intervals from M/2 up all mean one segment: the same workspace
    assert lib.pv_kpm_vjp_workspace_size(lat.handle, 0, 1, 8, 1000) == need
    assert lib.pv_kpm_vjp_workspace_size(lat.handle, 0, 1, 8, 3) > need
    assert lib.pv_kpm_moments_vjp_ckpt(lat.handle, 0, 1, 8, 7.0, 0.0, fake, None, fake, 4, fake, big, None) == 1
    assert lib.pv_kpm_moments_vjp_ckpt(lat.handle, 0, 1, 8, 7.0, 0.0, fake, fake, fake, 4, fake, need - 1, None) == 4
    # propagation: psiT aliasing psi0, no steps, workspace sized without the kept series
    assert lib.pv_cheb_propagate_keep(lat.handle, 0, 1, 7.0, 0.0, 1.0, 8, 2, fake, fake, 0, other, big, None) == 1
    assert b"alias" in lib.pv_last_error()
    assert lib.pv_cheb_propagate_keep(lat.handle, 0, 1, 7.0, 0.0, 1.0, 8, 0, fake, other, 0, other, big, None) == 1
    base = lib.pv_cheb_propagate_keep_workspace_size(lat.handle, 0, 1, 8, 3, 0)
    full = lib.pv_cheb_propagate_keep_workspace_size(lat.handle, 0, 1, 8, 3, 1)
    assert base == lib.pv_cheb_propagate_vjp_workspace_size(lat.handle, 0, 1, 8, 3)
    vb = lat.n_rows * 16
    assert full - base >= 3 * 8 * vb
    assert lib.pv_cheb_propagate_keep(lat.handle, 0, 1, 7.0, 0.0, 1.0, 8, 3, fake, other, 1, other, base, None) == 4
    assert lib.pv_cheb_propagate_vjp_keep(lat.handle, 0, 1, 7.0, 0.0, 1.0, 8, 3, fake, fake, None, fake, 1, other,
                                          base, None) == 4


def test_noalloc_sweep_rejects_oversized_scratch_before_any_device_call(lib):
    """pv_spmmv_noalloc refuses a sweep whose scratch need exceeds the static
    array (PV_ERR_UNSUPPORTED), and bad arguments, before touching a device."""
    lat = pv.Lattice((512, 512, 512), (1, 1, 1), pv.pv_model_stencil(pv.PV_MODEL_TI, [1.0, 2.0, 0, 0]))
    assert lib.pv_spmmv_workspace_size(lat.handle, 0, 64) > pv.PV_NOALLOC_SCRATCH_BYTES
    one = np.ones(64)
    fake = ctypes.c_void_p(1 << 20)   # never dereferenced: validation fails first
    st = lib.pv_spmmv_noalloc(lat.handle, 0, 64, fake, None, ctypes.c_void_p(1 << 21), pv._dptr(one),
                              pv._dptr(one), pv._dptr(np.zeros(64)), 0, None, None)
    assert st == 2 and b"static" in lib.pv_last_error()
    st = lib.pv_spmmv_noalloc(lat.handle, 0, 3, fake, None, ctypes.c_void_p(1 << 21), pv._dptr(one),
                              pv._dptr(one), pv._dptr(np.zeros(64)), 0, None, None)
    assert st == 2   # nb not a power of two
    st = lib.pv_spmmv_noalloc(lat.handle, 0, 1, fake, None, fake, pv._dptr(one), pv._dptr(one),
                              pv._dptr(np.zeros(64)), 0, None, None)
    assert st == 1   # x aliases y


def test_library_built_from_these_sources(lib):
    """The loaded library carries the hash of the sources it was built from,
    and it is the tree's (the binding refuses a stale build, whose structures
    could differ from the ones it declares)."""
    from paper_1708_09689_amd import build
    assert lib.pv_source_hash().decode() == build.source_hash()


def test_dos_of_non_finite_moments_is_an_error(lib):
    """A NaN or Inf moment gives PV_ERR_NONFINITE (status 7), not a NaN
    density."""
    mu = np.zeros(16)
    mu[0] = 1.0
    for bad in (np.nan, np.inf):
        mu[5] = bad
        with pytest.raises(pv.PvError) as e:
            pv.pv_kpm_dos(mu, np.linspace(-1, 1, 5), 7.0, 0.0)
        assert e.value.status == 7
        assert b"not finite" in lib.pv_last_error()


def _pattern_fields(text):
    """Offsets, entry codes and flags of a generated pattern struct's text."""
    head = re.search(r"NO = (\d+), NT = (\d+), DIM = (\d+);", text)
    no, nt, dim = (int(v) for v in head.groups())
    flags = re.search(r"SIDE_HALO = (true|false), SIDE_W = (true|false);", text)
    halo = (flags.group(1) == "true", flags.group(2) == "true")
    offs = re.search(r"off\[\d+\]\[3\] = \{(.*)\};", text).group(1)
    offsets = [tuple(int(v) for v in m) for m in re.findall(r"\{(-?\d+), (-?\d+), (-?\d+)\}", offs)]
    codes = re.findall(r"\b(C[ZRIC])\b", text.split("code[")[1])
    kinds = np.array([{"CZ": 0, "CR": 1, "CI": 2, "CC": 3}[c] for c in codes]).reshape(nt + 1, no, no)
    return no, nt, dim, halo, offsets[:nt], kinds


def _entry_kind(z):
    return 0 if z == 0 else (1 if z.imag == 0 else (2 if z.real == 0 else 3))


@pytest.mark.parametrize("dim,per_hops,halo", [
    (3, [(1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0)], (True, False)),   # y with x steps: halo side rows
    (3, [(1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1)], (False, False)),
    (3, [(0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)], (False, True)),   # y with z steps: rows at w -+ 1
    (3, [(1, 1, 1), (-1, -1, -1)], (True, True)),
    (2, [(1, 1, 0), (-1, -1, 0)], (False, False)),
])
def test_generated_pattern_states_the_stencil_structure(lib, dim, per_hops, halo):
    """The pattern struct generated for a generic stencil lists its offsets in
    descriptor order and, per block entry, the zero / real / imaginary /
    complex kind of the value the lattice holds (on-site block last); on a 3D
    lattice the side-row halo flag is set exactly when an offset has both a y
    and an x step, the flag for side rows at w -+ 1 exactly when one has both
    a y and a z step."""
    g = np.random.default_rng(5)
    no = 2
    base = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0)] + ([(0, 0, 1), (0, 0, -1)] if dim == 3 else [])
    offsets, blocks = [], []
    for o in base + per_hops:
        if tuple(-v for v in o) in offsets:
            continue
        B = np.array([[1.0, 0.5j], [0.0, -0.3 + 0.2j]]) * g.choice([1.0, -0.5])
        offsets += [o, tuple(-v for v in o)]
        blocks += [B, B.conj().T]
    E0 = np.array([[0.2, 0.1 - 0.4j], [0.1 + 0.4j, -0.1]])
    st = {"dim": dim, "n_orb": no, "offsets": np.array(offsets), "blocks": np.array(blocks), "onsite": E0,
          "pot_mode": pv.PV_POT_SITE}
    L = (6, 5, 4) if dim == 3 else (6, 5)
    lat = pv.Lattice(L, (1, 1, 1), st)
    assert lat.family == 0
    assert pv.pv_lattice_get_codegen(lat)
    NO, NT, DIM, HALO, offs, kinds = _pattern_fields(pv.pv_lattice_codegen_source(lat))
    assert (NO, NT, DIM, HALO) == (no, len(offsets), dim, halo)
    assert offs == [tuple(o) for o in offsets]
    for t, B in enumerate(blocks + [E0]):
        for o in range(no):
            for q in range(no):
                assert kinds[t, o, q] == _entry_kind(B[o, q]), (t, o, q)
    pv.pv_lattice_set_codegen(lat, False)
    assert not pv.pv_lattice_get_codegen(lat)
    pv.pv_lattice_set_codegen(lat, True)
    assert pv.pv_lattice_get_codegen(lat)


def test_generated_pattern_availability(lib):
    """Built-in families have no generated pattern; a stencil whose block rows
    need more per-lane slots than a kernel holds (26 dense complex 4x4
    blocks: 104 slots) keeps the interpreted kernels; bad arguments fail."""
    ti = pv.Lattice((4, 4, 4), (1, 1, 1), pv.pv_model_stencil(pv.PV_MODEL_TI, [1.0, 2.0, 0.0, 0.0]))
    assert ti.family == 1 and not pv.pv_lattice_get_codegen(ti)
    with pytest.raises(pv.PvError, match="built-in family"):
        pv.pv_lattice_codegen_source(ti)
    g = np.random.default_rng(9)
    offsets, blocks = [], []
    for o in [(dx, dy, dz) for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1) if (dx, dy, dz) > (0, 0, 0)]:
        B = g.standard_normal((4, 4)) + 1j * g.standard_normal((4, 4))
        offsets += [o, tuple(-v for v in o)]
        blocks += [B, B.conj().T]
    st = {"dim": 3, "n_orb": 4, "offsets": np.array(offsets), "blocks": np.array(blocks),
          "onsite": np.eye(4, dtype=np.complex128), "pot_mode": pv.PV_POT_SITE}
    dense = pv.Lattice((3, 3, 3), (1, 1, 1), st)
    assert dense.family == 0 and not pv.pv_lattice_get_codegen(dense)
    with pytest.raises(pv.PvError, match="slots"):
        pv.pv_lattice_codegen_source(dense)
    assert lib.pv_lattice_set_codegen(ti.handle, 2) == 1
    assert lib.pv_lattice_get_codegen(None, None) == 1


def test_batch_autotune_workspace_covers_every_candidate_shape(lib):
    """The autotune workspace holds the timed runs under every shape it tries
    (block counts differ between shapes) whatever shape the batch holds."""
    g = np.random.default_rng(5)
    offsets, blocks = [], []
    for o in [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1)]:
        B = g.standard_normal((2, 2)) + 1j * g.standard_normal((2, 2))
        offsets += [o, tuple(-v for v in o)]
        blocks += [B, B.conj().T]
    st = {"dim": 3, "n_orb": 2, "offsets": np.array(offsets), "blocks": np.array(blocks),
          "onsite": np.eye(2, dtype=np.complex128), "pot_mode": pv.PV_POT_NONE}
    sizes = [(6, 5, 4), (7, 6, 5), (8, 4, 6)]
    ti = pv.pv_model_stencil(pv.PV_MODEL_TI, [1.0, 2.0, 0.0, 0.0])
    for stencil in (st, ti):
        lats = [pv.Lattice(L, (1, 1, 1), stencil) for L in sizes]
        batch = pv.Batch(lats)
        for dt, elems in ((pv.PV_C128, (1, 2)), (pv.PV_C64, (2, 4))):
            for nb in (1, 8):
                need = lib.pv_batch_autotune_workspace_size(batch.handle, dt, nb)
                mu_bytes = len(lats) * nb * 16 * 8
                shapes = [{"kernel": 1}] + [{"kernel": 2, "elems_per_lane": e, "workgroup_size": wg}
                                            for wg in (0, 512) for e in elems]
                for t in shapes:
                    pv.pv_batch_set_tuning(batch, dt, nb, t)
                    assert lib.pv_batch_autotune_workspace_size(batch.handle, dt, nb) == need
                    assert lib.pv_batch_kpm_workspace_size(batch.handle, dt, nb, 16) + mu_bytes <= need
                pv.pv_batch_set_tuning(batch, dt, nb, None)


def test_random_block_argument_errors_before_any_launch(lib):
    lat = pv.Lattice((4, 4, 4), (1, 1, 1), pv.pv_model_stencil(pv.PV_MODEL_TI, [1.0, 2.0, 0, 0]))
    fake = ctypes.c_void_p(1 << 20)   # never dereferenced: validation fails first
    cases = [
        ((lat.handle, 0, 3, 1, 0, 0, fake, None), 2, b"power of two"),        # nb
        ((lat.handle, 0, 4, 1, 2, 0, fake, None), 1, b"kind"),                # unknown kind
        ((lat.handle, 0, 4, 1, 0, -1, fake, None), 1, b"row0"),               # negative row0
        ((lat.handle, 0, 64, 1, 0, (1 << 63) // 64, fake, None), 1, b"row0"),  # index overflow
        ((lat.handle, 0, 4, 1, 0, 0, ctypes.c_void_p((1 << 20) + 8), None), 1, b"out"),   # misaligned
        ((lat.handle, 0, 4, 1, 0, 0, None, None), 1, b"out"),                 # NULL
        ((lat.handle, 2, 4, 1, 0, 0, fake, None), 1, b"dtype"),
        ((None, 0, 4, 1, 0, 0, fake, None), 1, b"NULL"),
    ]
    for args, status, text in cases:
        assert lib.pv_random_block(*args) == status
        assert text in lib.pv_last_error()


def test_vector_from_func_argument_errors_before_any_callback(lib):
    lat = pv.Lattice((4, 4, 4), (1, 1, 1), pv.pv_model_stencil(pv.PV_MODEL_TI, [1.0, 2.0, 0, 0]))
    calls = []
    f = pv.PV_VECTOR_FUNC(lambda r, k, parm, seed: calls.append(k) or 0.0)
    fp = ctypes.cast(f, ctypes.c_void_p)
    fake = ctypes.c_void_p(1 << 20)
    cases = [
        ((lat.handle, 0, 3, fp, None, None, 1, fake, None), 2, b"power of two"),
        ((lat.handle, 0, 4, None, None, None, 1, fake, None), 1, b"fnc"),
        ((lat.handle, 0, 4, fp, None, None, 1, ctypes.c_void_p((1 << 20) + 8), None), 1, b"out"),
        ((lat.handle, 5, 4, fp, None, None, 1, fake, None), 1, b"dtype"),
        ((None, 0, 4, fp, None, None, 1, fake, None), 1, b"NULL"),
    ]
    for args, status, text in cases:
        assert lib.pv_vector_from_func(*args) == status
        assert text in lib.pv_last_error()
    # no device: refused before the callback is called
    assert lib.pv_vector_from_func(lat.handle, 0, 4, fp, None, None, 1, fake, None) == 8
    assert calls == []
