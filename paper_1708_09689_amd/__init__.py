"""Python binding of libpvdtm (MI355X matrix-free Chebyshev / stencil library).

Argument marshalling only: every function here forwards to the C ABI declared
in ``include/pvdtm.h`` under the same name.  Torch tensors provide device
memory and the current HIP stream (``tensor.data_ptr()`` and
``torch.cuda.current_stream().cuda_stream``); no computation runs in Python or
in torch.  If the HIP library is not built, every call raises.

Vector blocks are torch complex tensors (complex128 or complex64) with
``numel == n_rows * nb``, row-major [rows][nb] (any shape with that memory
layout, e.g. [Lz, Ly, Lx, n_orb, nb]).
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libpvdtm.so")

PV_C128, PV_C64 = 0, 1
PV_F64, PV_F32 = 0, 1
PV_POT_NONE, PV_POT_SITE, PV_POT_ORBITAL = 0, 1, 2
PV_CHECK_HERMITIAN = 1
PV_DOT_XX, PV_DOT_XY, PV_DOT_YY = 1, 2, 4
PV_MAX_TERMS, PV_MAX_ORB, PV_MAX_NB = 26, 4, 64
PV_MODEL_TI, PV_MODEL_GRAPHENE2, PV_MODEL_GRAPHENE4, PV_MODEL_WEYL = 0, 1, 2, 3
PV_RANDOM_PHASE, PV_RANDOM_Z4 = 0, 1
FAMILY_NAMES = {0: "generic", 1: "ti", 2: "graphene2", 3: "graphene4", 4: "weyl"}

STATUS_NAMES = {0: "PV_OK", 1: "PV_ERR_INVALID_ARG", 2: "PV_ERR_UNSUPPORTED", 3: "PV_ERR_NOT_HERMITIAN",
                4: "PV_ERR_WORKSPACE", 5: "PV_ERR_OOM", 6: "PV_ERR_HIP", 7: "PV_ERR_NONFINITE",
                8: "PV_ERR_NO_DEVICE", 9: "PV_ERR_NOT_CONVERGED"}

# exported symbols of include/pvdtm.h with (restype, argtypes)
_vp, _sz, _i64, _d, _i, _u = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int64, ctypes.c_double, ctypes.c_int, ctypes.c_uint
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


class pv_lattice_desc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("L", ctypes.c_int64 * 3), ("n_orb", ctypes.c_int),
                ("periodic", ctypes.c_int * 3), ("n_terms", ctypes.c_int), ("offsets", _ip),
                ("blocks", _dp), ("onsite", _dp), ("pot_mode", ctypes.c_int), ("flags", ctypes.c_uint)]


class pv_tuning(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int) for n in ("kernel", "elems_per_lane", "walk_planes", "strip_rows",
                                            "groups_per_xcd", "tiles_per_group", "slab_rows", "workgroup_size")]


TUNING_FIELDS = [f[0] for f in pv_tuning._fields_]

SIGNATURES = {
    "pv_last_error": (ctypes.c_char_p, []),
    "pv_status_string": (ctypes.c_char_p, [_i]),
    "pv_version": (_i, []),
    "pv_source_hash": (ctypes.c_char_p, []),
    "pv_model_stencil": (_i, [_i, _dp, _ip, _ip, _ip, _ip, _dp, _dp, _ip]),
    "pv_lattice_create": (_i, [ctypes.POINTER(pv_lattice_desc), ctypes.POINTER(_vp)]),
    "pv_lattice_destroy": (None, [_vp]),
    "pv_lattice_info": (_i, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64), _ip]),
    "pv_lattice_set_potential": (_i, [_vp, _vp, _i]),
    "pv_lattice_set_random_potential": (_i, [_vp, ctypes.c_uint64, _d]),
    "pv_spmmv_workspace_size": (_sz, [_vp, _i, _i]),
    "pv_spmmv": (_i, [_vp, _i, _i, _vp, _vp, _vp, _dp, _dp, _dp, _u, _vp, _vp, _sz, _vp]),
    "pv_spmmv_noalloc": (_i, [_vp, _i, _i, _vp, _vp, _vp, _dp, _dp, _dp, _u, _vp, _vp]),
    "pv_kpm_workspace_size": (_sz, [_vp, _i, _i, _i]),
    "pv_kpm_moments": (_i, [_vp, _i, _i, _i, _d, _d, _vp, _vp, _vp, _sz, _vp]),
    "pv_kpm_dos": (_i, [_i, _dp, _d, _d, _i, _dp, _dp]),
    "pv_cheb_series_workspace_size": (_sz, [_vp, _i, _i]),
    "pv_cheb_series": (_i, [_vp, _i, _i, _d, _d, _i, _dp, _vp, _vp, _vp, _sz, _vp]),
    "pv_cheb_propagate_workspace_size": (_sz, [_vp, _i, _i]),
    "pv_cheb_propagate": (_i, [_vp, _i, _i, _d, _d, _d, _i, _i, _vp, _vp, _sz, _vp]),
    "pv_cheb_tp_coefficients": (_i, [_d, _d, _i, _dp]),
    "pv_gram_workspace_size": (_sz, [_i64, _i, _i]),
    "pv_gram": (_i, [_i, _i64, _i, _i, _vp, _vp, _vp, _vp, _sz, _vp]),
    "pv_block_rotate": (_i, [_i, _i64, _i, _i, _vp, _vp, _i, _vp, _vp]),
    "pv_stream_copy": (_i, [_vp, _vp, _sz, _vp]),
    "pv_stream_triad": (_i, [_vp, _vp, _vp, _sz, _vp]),
    "pv_stream_read": (_i, [_vp, _sz, _vp, _vp]),
    "pv_chebfd_workspace_size": (_sz, [_vp, _i, _i, _i]),
    "pv_chebfd": (_i, [_vp, _i, _i, _i, _d, _d, _d, _d, _i, _i, _d, _i, _vp, _dp, _dp, _ip, _ip, _vp, _sz, _vp]),
    "pv_chebfd_filter_coefficients": (_i, [_d, _d, _d, _d, _i, _dp]),
    "pv_host_heev": (_i, [_i, _dp, _dp, _dp]),
    "pv_batch_create": (_i, [_i, ctypes.POINTER(_vp), ctypes.POINTER(_vp)]),
    "pv_batch_destroy": (None, [_vp]),
    "pv_batch_kpm_workspace_size": (_sz, [_vp, _i, _i, _i]),
    "pv_batch_kpm_moments": (_i, [_vp, _i, _i, _i, _dp, _dp, ctypes.POINTER(_vp), _vp, _vp, _sz, _vp]),
    "pv_batch_stats": (_i, [_vp, _ip, _ip]),
    "pv_batch_set_tuning": (_i, [_vp, _i, _i, ctypes.POINTER(pv_tuning)]),
    "pv_batch_get_tuning": (_i, [_vp, _i, _i, ctypes.POINTER(pv_tuning)]),
    "pv_batch_autotune_workspace_size": (_sz, [_vp, _i, _i]),
    "pv_batch_autotune": (_i, [_vp, _i, _i, _dp, _dp, ctypes.POINTER(_vp), _vp, _sz, _vp, ctypes.POINTER(pv_tuning),
                               _dp]),
    "pv_kpm_vjp_workspace_size": (_sz, [_vp, _i, _i, _i, _i]),
    "pv_kpm_moments_vjp": (_i, [_vp, _i, _i, _i, _d, _d, _vp, _vp, _vp, _i, _vp, _sz, _vp]),
    "pv_kpm_moments_ckpt": (_i, [_vp, _i, _i, _i, _d, _d, _vp, _vp, _i, _vp, _sz, _vp]),
    "pv_kpm_moments_vjp_ckpt": (_i, [_vp, _i, _i, _i, _d, _d, _vp, _vp, _vp, _i, _vp, _sz, _vp]),
    "pv_cheb_propagate_vjp_workspace_size": (_sz, [_vp, _i, _i, _i, _i]),
    "pv_cheb_propagate_vjp": (_i, [_vp, _i, _i, _d, _d, _d, _i, _i, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "pv_cheb_propagate_keep_workspace_size": (_sz, [_vp, _i, _i, _i, _i, _i]),
    "pv_cheb_propagate_keep": (_i, [_vp, _i, _i, _d, _d, _d, _i, _i, _vp, _vp, _i, _vp, _sz, _vp]),
    "pv_cheb_propagate_vjp_keep": (_i, [_vp, _i, _i, _d, _d, _d, _i, _i, _vp, _vp, _vp, _vp, _i, _vp, _sz, _vp]),
    "pv_bloch_block": (_i, [_vp, _i, _i, _dp, _ip, _i, _i64, _vp, _vp]),
    "pv_random_block": (_i, [_vp, _i, _i, ctypes.c_uint64, _i, _i64, _vp, _vp]),
    "pv_vector_from_func": (_i, [_vp, _i, _i, _vp, _vp, _vp, ctypes.c_uint64, _vp, _vp]),
    "pv_kpm_spectral_function": (_i, [_i, _i, _dp, _d, _d, _d, _i, _dp, _dp]),
    "pv_dsl_stencil": (_i, [ctypes.c_char_p, _dp, _i, _ip, _ip, _ip, _ip, _dp, _dp, _ip, _ip]),
    "pv_trlanczos_filter": (_i, [_d, _d, _d, _d, _i, _dp, _dp]),
    "pv_trlanczos_workspace_size": (_sz, [_vp, _i, _i, _i]),
    "pv_trlanczos_fd": (_i, [_vp, _i, _d, _d, _d, _d, _i, _i, _i, _d, _i, _vp, _i, _vp, _dp, _dp, _ip, _ip, _vp,
                             _sz, _vp]),
    "pv_lattice_set_tuning": (_i, [_vp, _i, _i, ctypes.POINTER(pv_tuning)]),
    "pv_lattice_get_tuning": (_i, [_vp, _i, _i, ctypes.POINTER(pv_tuning)]),
    "pv_lattice_set_codegen": (_i, [_vp, _i]),
    "pv_lattice_get_codegen": (_i, [_vp, _ip]),
    "pv_lattice_codegen_source": (_i, [_vp, ctypes.c_char_p, _sz, ctypes.POINTER(_sz)]),
    "pv_codegen_instances": (_i, []),
    "pv_autotune_workspace_size": (_sz, [_vp, _i, _i]),
    "pv_autotune": (_i, [_vp, _i, _i, ctypes.c_char_p, _vp, _sz, _vp, ctypes.POINTER(pv_tuning), _dp]),
}

_lib = None


class PvError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def lib():
    """Load libpvdtm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_1708_09689_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name, None)
            if f is None:
                raise RuntimeError(f"{LIB_PATH} lacks {name}: it was built from other sources; rebuild with "
                                   "`python -m paper_1708_09689_amd.build`")
            f.restype = res
            f.argtypes = args
        # the structures this module declares (pv_tuning, pv_lattice_desc)
        # must have the library's layout: refuse a library built from other
        # sources than the ones shipped beside this module
        from . import build as _build
        if os.path.isdir(_build.CSRC):
            want, have = _build.source_hash(), L.pv_source_hash().decode()
            if have != want:
                raise RuntimeError(f"{LIB_PATH} was built from other sources (hash {have}, sources {want}): "
                                   "rebuild with `python -m paper_1708_09689_amd.build`")
        _lib = L
    return _lib


def _check(status):
    if status != 0:
        raise PvError(status, lib().pv_last_error().decode())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


# ----------------------------------------------------------------- torch plumbing

def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.complex128:
        return PV_C128
    if t.dtype == torch.complex64:
        return PV_C64
    raise TypeError(f"vector blocks must be complex128 or complex64, got {t.dtype}")


def _vec(t, name, rows, nb, dtype=None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != rows * nb:
        raise ValueError(f"{name} has {t.numel()} elements, expected rows*nb = {rows * nb}")
    if dtype is not None and _dtype_code(t) != dtype:
        raise TypeError(f"{name} dtype differs from the other blocks")
    return ctypes.c_void_p(t.data_ptr())


def _workspace(nbytes, device):
    torch = _torch()
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


# ----------------------------------------------------------------- model / lattice

def pv_model_stencil(model: int, params=None) -> dict:
    p = np.zeros(4) if params is None else np.asarray(params, dtype=np.float64).copy()
    if params is None:
        p = None
    dim, n_orb, n_terms, pot = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    offs = np.zeros(PV_MAX_TERMS * 3, dtype=np.int32)
    blocks = np.zeros(PV_MAX_TERMS * PV_MAX_ORB * PV_MAX_ORB * 2)
    onsite = np.zeros(PV_MAX_ORB * PV_MAX_ORB * 2)
    _check(lib().pv_model_stencil(model, None if p is None else _dptr(p), ctypes.byref(dim), ctypes.byref(n_orb),
                                  ctypes.byref(n_terms), offs.ctypes.data_as(_ip), _dptr(blocks), _dptr(onsite),
                                  ctypes.byref(pot)))
    no, nt = n_orb.value, n_terms.value
    b = blocks[: nt * no * no * 2].reshape(nt, no, no, 2)
    e = onsite[: no * no * 2].reshape(no, no, 2)
    return {"dim": dim.value, "n_orb": no, "offsets": offs[: 3 * nt].reshape(nt, 3).copy(),
            "blocks": b[..., 0] + 1j * b[..., 1], "onsite": e[..., 0] + 1j * e[..., 1], "pot_mode": pot.value}


def pv_trlanczos_filter(lam_l, lam_r, a, b, K):
    coef = np.zeros(K + 1)
    tau = ctypes.c_double()
    _check(lib().pv_trlanczos_filter(lam_l, lam_r, a, b, K, _dptr(coef), ctypes.byref(tau)))
    return coef, tau.value


def pv_trlanczos_fd(lat, V0, a, b, lam_l, lam_r, degree, m, tol, max_restarts=60, n_out=0, raise_unconverged=True):
    """Eigenpairs in [lam_l, lam_r] by filtered thick-restart block Lanczos;
    V0: device start block [n_rows, nbl].  Returns (theta, res, X or None, restarts)."""
    torch = _torch()
    dt = _dtype_code(V0)
    nbl = V0.numel() // lat.n_rows
    ws = _workspace(lib().pv_trlanczos_workspace_size(lat.handle, dt, nbl, m), V0.device)
    th, rs = np.zeros(m), np.zeros(m)
    nf, nr = ctypes.c_int(), ctypes.c_int()
    X = None
    if n_out:
        X = torch.empty((lat.n_rows, n_out), dtype=V0.dtype, device=V0.device)
    st = lib().pv_trlanczos_fd(lat.handle, dt, a, b, lam_l, lam_r, degree, nbl, m, tol, max_restarts,
                               _vec(V0, "V0", lat.n_rows, nbl), n_out,
                               None if X is None else ctypes.c_void_p(X.data_ptr()), _dptr(th), _dptr(rs),
                               ctypes.byref(nf), ctypes.byref(nr), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                               _stream())
    if st != 0 and (raise_unconverged or st != 9):
        _check(st)
    n = nf.value
    return th[:n].copy(), rs[:n].copy(), X, nr.value


def pv_dsl_stencil(text: str, coeff_const=None) -> dict:
    """Parse a DSL program (Sec. 3.2) into a stencil dict (as pv_model_stencil),
    plus "field": 0 none, 1 variable (array), 2 random (on the fly)."""
    cc = None if coeff_const is None else np.ascontiguousarray(np.asarray(coeff_const, dtype=np.float64))
    dim, n_orb, n_terms, pot, fk = (ctypes.c_int() for _ in range(5))
    offs = np.zeros(PV_MAX_TERMS * 3, dtype=np.int32)
    blocks = np.zeros(PV_MAX_TERMS * PV_MAX_ORB * PV_MAX_ORB * 2)
    onsite = np.zeros(PV_MAX_ORB * PV_MAX_ORB * 2)
    _check(lib().pv_dsl_stencil(text.encode(), None if cc is None else _dptr(cc), 0 if cc is None else cc.size,
                                ctypes.byref(dim), ctypes.byref(n_orb), ctypes.byref(n_terms),
                                offs.ctypes.data_as(_ip), _dptr(blocks), _dptr(onsite), ctypes.byref(pot),
                                ctypes.byref(fk)))
    no, nt = n_orb.value, n_terms.value
    b = blocks[: nt * no * no * 2].reshape(nt, no, no, 2)
    e = onsite[: no * no * 2].reshape(no, no, 2)
    return {"dim": dim.value, "n_orb": no, "offsets": offs[: 3 * nt].reshape(nt, 3).copy(),
            "blocks": b[..., 0] + 1j * b[..., 1], "onsite": e[..., 0] + 1j * e[..., 1], "pot_mode": pot.value,
            "field": fk.value}


class Lattice:
    """Owns a pv_lattice handle (pv_lattice_create / pv_lattice_destroy)."""

    def __init__(self, L, periodic, stencil: dict, check_hermitian: bool = True):
        L = list(L) + [1] * (3 - len(L))
        periodic = list(periodic) + [1] * (3 - len(periodic))
        no = int(stencil["n_orb"])
        offs = np.ascontiguousarray(np.asarray(stencil["offsets"], dtype=np.int32).reshape(-1))
        B = np.asarray(stencil["blocks"], dtype=np.complex128).reshape(-1, no, no)
        E = np.asarray(stencil["onsite"], dtype=np.complex128).reshape(no, no)
        self._blocks = np.ascontiguousarray(np.stack([B.real, B.imag], axis=-1).reshape(-1))
        self._onsite = np.ascontiguousarray(np.stack([E.real, E.imag], axis=-1).reshape(-1))
        self._offs = offs
        d = pv_lattice_desc()
        d.dim = int(stencil["dim"])
        d.L = (ctypes.c_int64 * 3)(*[int(v) for v in L])
        d.n_orb = no
        d.periodic = (ctypes.c_int * 3)(*[1 if p else 0 for p in periodic])
        d.n_terms = B.shape[0]
        d.offsets = offs.ctypes.data_as(_ip)
        d.blocks = self._blocks.ctypes.data_as(_dp)
        d.onsite = self._onsite.ctypes.data_as(_dp)
        d.pot_mode = int(stencil.get("pot_mode", PV_POT_SITE))
        d.flags = PV_CHECK_HERMITIAN if check_hermitian else 0
        h = ctypes.c_void_p()
        _check(lib().pv_lattice_create(ctypes.byref(d), ctypes.byref(h)))
        self.handle = h
        ns, nr, fam = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int()
        _check(lib().pv_lattice_info(h, ctypes.byref(ns), ctypes.byref(nr), ctypes.byref(fam)))
        self.n_sites, self.n_rows, self.family = ns.value, nr.value, fam.value
        self.n_orb = no
        self.L = tuple(L)
        self.periodic = tuple(periodic)
        self.pot_mode = d.pot_mode
        self._V = None

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.pv_lattice_destroy(h)
            self.handle = None

    def set_potential(self, V):
        """pv_lattice_set_potential: V is a device float64/float32 tensor (kept alive here) or None."""
        torch = _torch()
        if V is None:
            _check(lib().pv_lattice_set_potential(self.handle, None, PV_F64))
            self._V = None
            return
        if not V.is_cuda or not V.is_contiguous():
            raise ValueError("V must be a contiguous device tensor")
        n = self.n_sites if self.pot_mode == PV_POT_SITE else self.n_rows
        if V.numel() != n:
            raise ValueError(f"V has {V.numel()} entries, expected {n}")
        rt = {torch.float64: PV_F64, torch.float32: PV_F32}.get(V.dtype)
        if rt is None:
            raise TypeError("V must be float64 or float32")
        _check(lib().pv_lattice_set_potential(self.handle, ctypes.c_void_p(V.data_ptr()), rt))
        self._V = V

    def set_random_potential(self, seed: int, W: float):
        """pv_lattice_set_random_potential: on-the-fly field W (u_i - 1/2) from
        the counter-based generator seeded with `seed` (no array is stored)."""
        _check(lib().pv_lattice_set_random_potential(self.handle, int(seed) & ((1 << 64) - 1), float(W)))
        self._V = None


def pv_lattice_create(L, periodic, stencil, check_hermitian=True) -> Lattice:
    return Lattice(L, periodic, stencil, check_hermitian)


# ----------------------------------------------------------------- sweeps and algorithms

def pv_spmmv(lat: Lattice, x, y, alpha, beta, gamma, z=None, dot_flags: int = 0, dots=None, nb=None):
    """y = alpha (H x - beta x) + gamma z per column; optional FP64 dots [nb][4]."""
    torch = _torch()
    nb = nb if nb is not None else x.numel() // lat.n_rows
    dt = _dtype_code(x)
    a = np.broadcast_to(np.asarray(alpha, dtype=np.float64), (nb,)).copy()
    b = np.broadcast_to(np.asarray(beta, dtype=np.float64), (nb,)).copy()
    g = np.broadcast_to(np.asarray(gamma, dtype=np.float64), (nb,)).copy()
    if dot_flags and dots is None:
        dots = torch.empty((nb, 4), dtype=torch.float64, device=x.device)
    ws = _workspace(lib().pv_spmmv_workspace_size(lat.handle, dt, nb), x.device)
    _check(lib().pv_spmmv(lat.handle, dt, nb, _vec(x, "x", lat.n_rows, nb), _vec(z, "z", lat.n_rows, nb, dt),
                          _vec(y, "y", lat.n_rows, nb, dt), _dptr(a), _dptr(b), _dptr(g), dot_flags,
                          None if dots is None else ctypes.c_void_p(dots.data_ptr()),
                          ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return dots


PV_NOALLOC_SCRATCH_BYTES = 64 << 20


def pv_spmmv_noalloc(lat: Lattice, x, y, alpha, beta, gamma, z=None, dot_flags: int = 0, dots=None, nb=None):
    """pv_spmmv with the library's static scratch instead of a workspace (the
    library allocates nothing; dots, when requested, is the caller's [nb][4]
    FP64 device tensor)."""
    nb = nb if nb is not None else x.numel() // lat.n_rows
    dt = _dtype_code(x)
    a = np.broadcast_to(np.asarray(alpha, dtype=np.float64), (nb,)).copy()
    b = np.broadcast_to(np.asarray(beta, dtype=np.float64), (nb,)).copy()
    g = np.broadcast_to(np.asarray(gamma, dtype=np.float64), (nb,)).copy()
    _check(lib().pv_spmmv_noalloc(lat.handle, dt, nb, _vec(x, "x", lat.n_rows, nb),
                                  _vec(z, "z", lat.n_rows, nb, dt), _vec(y, "y", lat.n_rows, nb, dt), _dptr(a),
                                  _dptr(b), _dptr(g), dot_flags,
                                  None if dots is None else ctypes.c_void_p(dots.data_ptr()), _stream()))
    return dots


def pv_kpm_moments(lat: Lattice, r, M: int, a: float, b: float, mu=None, nb=None):
    """mu[c][n] = Re <r_c, T_n(H~) r_c> / D (device FP64 [nb][M])."""
    torch = _torch()
    nb = nb if nb is not None else r.numel() // lat.n_rows
    dt = _dtype_code(r)
    if mu is None:
        mu = torch.empty((nb, M), dtype=torch.float64, device=r.device)
    ws = _workspace(lib().pv_kpm_workspace_size(lat.handle, dt, nb, M), r.device)
    _check(lib().pv_kpm_moments(lat.handle, dt, nb, M, a, b, _vec(r, "r", lat.n_rows, nb),
                                ctypes.c_void_p(mu.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                _stream()))
    return mu


def pv_kpm_dos(mu, E, a: float, b: float):
    mu = np.ascontiguousarray(np.asarray(mu, dtype=np.float64))
    E = np.ascontiguousarray(np.asarray(E, dtype=np.float64))
    rho = np.zeros_like(E)
    _check(lib().pv_kpm_dos(mu.size, _dptr(mu), a, b, E.size, _dptr(E), _dptr(rho)))
    return rho


def _coef_array(coef):
    c = np.asarray(coef, dtype=np.complex128).reshape(-1)
    return np.ascontiguousarray(np.stack([c.real, c.imag], axis=-1).reshape(-1))


def pv_cheb_series(lat: Lattice, X, Y, a: float, b: float, coef, nb=None):
    """Y = sum_k coef[k] T_k(H~) X."""
    nb = nb if nb is not None else X.numel() // lat.n_rows
    dt = _dtype_code(X)
    c = _coef_array(coef)
    ws = _workspace(lib().pv_cheb_series_workspace_size(lat.handle, dt, nb), X.device)
    _check(lib().pv_cheb_series(lat.handle, dt, nb, a, b, c.size // 2 - 1, _dptr(c), _vec(X, "X", lat.n_rows, nb),
                                _vec(Y, "Y", lat.n_rows, nb, dt), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                _stream()))
    return Y


def pv_cheb_propagate(lat: Lattice, psi, a: float, b: float, dt: float, M: int, nsteps: int, nb=None):
    """psi <- U(dt)^nsteps psi in place (Chebyshev propagator)."""
    nb = nb if nb is not None else psi.numel() // lat.n_rows
    dtc = _dtype_code(psi)
    ws = _workspace(lib().pv_cheb_propagate_workspace_size(lat.handle, dtc, nb), psi.device)
    _check(lib().pv_cheb_propagate(lat.handle, dtc, nb, a, b, dt, M, nsteps, _vec(psi, "psi", lat.n_rows, nb),
                                   ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return psi


def pv_cheb_tp_coefficients(a: float, dt: float, M: int) -> np.ndarray:
    out = np.zeros(2 * (M + 1))
    _check(lib().pv_cheb_tp_coefficients(a, dt, M, _dptr(out)))
    return out[0::2] + 1j * out[1::2]


def pv_gram(X, Y, G=None, rows=None):
    """G = X^H Y (device complex128 [nx][ny]) for X [rows][nx], Y [rows][ny]."""
    torch = _torch()
    rows = rows if rows is not None else X.shape[0]
    nx, ny = X.numel() // rows, Y.numel() // rows
    dt = _dtype_code(X)
    if G is None:
        G = torch.empty((nx, ny), dtype=torch.complex128, device=X.device)
    ws = _workspace(lib().pv_gram_workspace_size(rows, nx, ny), X.device)
    _check(lib().pv_gram(dt, rows, nx, ny, _vec(X, "X", rows, nx), _vec(Y, "Y", rows, ny, dt),
                         ctypes.c_void_p(G.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return G


def pv_block_rotate(X, Q, Y, rows=None, accumulate=False):
    """Y = X Q (+ Y when accumulate), Q device complex128 [nx][ny]."""
    rows = rows if rows is not None else X.shape[0]
    nx, ny = X.numel() // rows, Y.numel() // rows
    dt = _dtype_code(X)
    _check(lib().pv_block_rotate(dt, rows, nx, ny, _vec(X, "X", rows, nx), ctypes.c_void_p(Q.data_ptr()),
                                 1 if accumulate else 0, _vec(Y, "Y", rows, ny, dt), _stream()))
    return Y


def pv_stream_copy(src, dst):
    n = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < n:
        raise ValueError("dst too small")
    _check(lib().pv_stream_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), n, _stream()))
    return dst


def pv_stream_triad(x, z, y):
    """y = x + z over float64 tensors of equal size (bandwidth reference)."""
    import torch
    for t in (x, z, y):
        if t.dtype != torch.float64 or not t.is_contiguous():
            raise ValueError("triad takes contiguous float64 tensors")
    if not (x.numel() == z.numel() == y.numel()):
        raise ValueError("triad operands differ in size")
    n = x.numel() * 8
    _check(lib().pv_stream_triad(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(z.data_ptr()),
                                 ctypes.c_void_p(y.data_ptr()), n, _stream()))
    return y


PV_STREAM_READ_SINK_BYTES = 65536


def pv_stream_read(x, sink):
    """Reads every byte of the contiguous device tensor x once (bandwidth
    reference); sink: a device tensor of at least PV_STREAM_READ_SINK_BYTES
    that receives a checksum per wave."""
    if not x.is_contiguous() or sink.numel() * sink.element_size() < PV_STREAM_READ_SINK_BYTES:
        raise ValueError("read probe takes a contiguous tensor and a sink of PV_STREAM_READ_SINK_BYTES")
    n = x.numel() * x.element_size()
    _check(lib().pv_stream_read(ctypes.c_void_p(x.data_ptr()), n, ctypes.c_void_p(sink.data_ptr()), _stream()))
    return sink


def pv_bloch_block(lat, k, orbital, layer=None, dtype=PV_C128, out=None, device="cuda"):
    """Bloch start columns exp(i k_c . r) on orbital[c] (optionally one layer:
    (axis, index)); k: [nb][3]; returns the device block [n_rows, nb]."""
    torch = _torch()
    k = np.ascontiguousarray(np.asarray(k, dtype=np.float64).reshape(-1, 3))
    orb = np.ascontiguousarray(np.asarray(orbital, dtype=np.int32).reshape(-1))
    nb = k.shape[0]
    if orb.size != nb:
        raise ValueError("k and orbital need the same number of columns")
    if out is None:
        out = torch.empty((lat.n_rows, nb), dtype=torch.complex128 if dtype == PV_C128 else torch.complex64,
                          device=device)
    axis, index = (-1, 0) if layer is None else layer
    _check(lib().pv_bloch_block(lat.handle, dtype, nb, _dptr(k), orb.ctypes.data_as(_ip), axis, index,
                                _vec(out, "out", lat.n_rows, nb, dtype), _stream()))
    return out


def pv_random_block(lat, nb: int, seed: int, kind=PV_RANDOM_PHASE, dtype=PV_C128, row0: int = 0, out=None,
                    device="cuda"):
    """Random start block [n_rows, nb] from the counter-based generator:
    entry (r, c) is a function of (seed, (row0 + r) * nb + c) only."""
    torch = _torch()
    if out is None:
        out = torch.empty((lat.n_rows, nb), dtype=torch.complex128 if dtype == PV_C128 else torch.complex64,
                          device=device)
    _check(lib().pv_random_block(lat.handle, dtype, nb, seed & 0xFFFFFFFFFFFFFFFF, kind, row0,
                                 _vec(out, "out", lat.n_rows, nb, dtype), _stream()))
    return out


PV_VECTOR_FUNC = ctypes.CFUNCTYPE(ctypes.c_double, ctypes.POINTER(ctypes.c_int64), ctypes.c_int, ctypes.c_void_p,
                                  ctypes.c_void_p)


def pv_vector_from_func(lat, nb: int, fnc, fnc_im=None, seed: int = 0, dtype=PV_C128, out=None, device="cuda"):
    """Block [n_rows, nb] from host callbacks fnc(r, k, parm, seed) -> real
    part (and fnc_im for the imaginary part), r = (x, y, z, orbital), as
    the C interface calls them (ctypes arguments; parm is NULL here)."""
    torch = _torch()
    if out is None:
        out = torch.empty((lat.n_rows, nb), dtype=torch.complex128 if dtype == PV_C128 else torch.complex64,
                          device=device)
    cf = PV_VECTOR_FUNC(fnc)
    ci = PV_VECTOR_FUNC(fnc_im) if fnc_im is not None else None
    _check(lib().pv_vector_from_func(lat.handle, dtype, nb, ctypes.cast(cf, _vp),
                                     None if ci is None else ctypes.cast(ci, _vp), None,
                                     seed & 0xFFFFFFFFFFFFFFFF, _vec(out, "out", lat.n_rows, nb, dtype), _stream()))
    return out


def pv_kpm_spectral_function(mu, E, a: float, b: float, norm: float) -> np.ndarray:
    """A(E) = norm * sum_c rho_c(E) from host moments mu [nb][M]."""
    mu = np.ascontiguousarray(np.asarray(mu, dtype=np.float64))
    if mu.ndim == 1:
        mu = mu[None, :]
    E = np.ascontiguousarray(np.asarray(E, dtype=np.float64))
    A = np.zeros(E.size)
    _check(lib().pv_kpm_spectral_function(mu.shape[0], mu.shape[1], _dptr(mu), a, b, norm, E.size, _dptr(E),
                                          _dptr(A)))
    return A


def pv_lattice_set_tuning(lat, dtype: int, nb: int, tuning=None):
    """Launch shape for (dtype, nb): dict with keys of TUNING_FIELDS (missing = 0), None = defaults."""
    if tuning is None:
        _check(lib().pv_lattice_set_tuning(lat.handle, dtype, nb, None))
        return
    bad = set(tuning) - set(TUNING_FIELDS)
    if bad:
        raise ValueError(f"unknown tuning fields {sorted(bad)}")
    t = pv_tuning(**{k: int(v) for k, v in tuning.items()})
    _check(lib().pv_lattice_set_tuning(lat.handle, dtype, nb, ctypes.byref(t)))


def pv_lattice_get_tuning(lat, dtype: int, nb: int) -> dict:
    t = pv_tuning()
    _check(lib().pv_lattice_get_tuning(lat.handle, dtype, nb, ctypes.byref(t)))
    return {k: getattr(t, k) for k in TUNING_FIELDS}


def pv_lattice_set_codegen(lat, enable: bool):
    """Generated kernels (True, the default) or the interpreted generic ones
    (False) for the sweeps of a generic-stencil lattice."""
    _check(lib().pv_lattice_set_codegen(lat.handle, 1 if enable else 0))


def pv_lattice_get_codegen(lat) -> bool:
    """True when sweeps of the lattice take kernels generated from its stencil."""
    v = ctypes.c_int()
    _check(lib().pv_lattice_get_codegen(lat.handle, ctypes.byref(v)))
    return bool(v.value)


def pv_codegen_instances() -> int:
    """Generated kernel instances loaded in this process."""
    return int(lib().pv_codegen_instances())


def pv_lattice_codegen_source(lat) -> str:
    """C++ text of the pattern struct the generated kernels are compiled for."""
    n = ctypes.c_size_t()
    _check(lib().pv_lattice_codegen_source(lat.handle, None, 0, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value)
    _check(lib().pv_lattice_codegen_source(lat.handle, buf, n.value, ctypes.byref(n)))
    return buf.value.decode()


def pv_autotune(lat, nb: int, dtype: int = PV_C128, cache_path=None, device="cuda"):
    """Time candidate launch shapes of one Chebyshev step and apply the fastest;
    returns (shape dict, ms per step; 0.0 when taken from the cache)."""
    ws = _workspace(lib().pv_autotune_workspace_size(lat.handle, dtype, nb), device)
    t = pv_tuning()
    ms = ctypes.c_double()
    path = None if cache_path is None else os.fsencode(cache_path)
    _check(lib().pv_autotune(lat.handle, dtype, nb, path, ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(),
                             ctypes.byref(t), ctypes.byref(ms)))
    return {k: getattr(t, k) for k in TUNING_FIELDS}, ms.value


def pv_chebfd_filter_coefficients(lam_l, lam_r, a, b, K):
    out = np.zeros(K + 1)
    _check(lib().pv_chebfd_filter_coefficients(lam_l, lam_r, a, b, K, _dptr(out)))
    return out


def pv_host_heev(A):
    A = np.ascontiguousarray(np.asarray(A, dtype=np.complex128))
    n = A.shape[0]
    a = np.ascontiguousarray(np.stack([A.real, A.imag], axis=-1).reshape(-1))
    w = np.zeros(n)
    V = np.zeros(2 * n * n)
    _check(lib().pv_host_heev(n, _dptr(a), _dptr(w), _dptr(V)))
    return w, (V[0::2] + 1j * V[1::2]).reshape(n, n)


def pv_chebfd(lat: Lattice, X, bw: int, a: float, b: float, lam_l: float, lam_r: float, degree: int,
              n_target: int, tol: float, max_iter: int = 20, raise_on_fail: bool = True):
    """Chebyshev filter diagonalisation.  X: device block [nblk, rows, bw]
    (start vectors in, Ritz vectors out).  Returns (theta, res, n_conv, iters)."""
    nblk = X.numel() // (lat.n_rows * bw)
    dt = _dtype_code(X)
    ns = bw * nblk
    theta, res = np.zeros(ns), np.zeros(ns)
    nc, it = ctypes.c_int(), ctypes.c_int()
    ws = _workspace(lib().pv_chebfd_workspace_size(lat.handle, dt, bw, nblk), X.device)
    st = lib().pv_chebfd(lat.handle, dt, bw, nblk, a, b, lam_l, lam_r, degree, n_target, tol, max_iter,
                         _vec(X, "X", lat.n_rows, ns), _dptr(theta), _dptr(res), ctypes.byref(nc),
                         ctypes.byref(it), ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream())
    if st != 0 and (raise_on_fail or st != 9):
        _check(st)
    return theta, res, nc.value, it.value


class Batch:
    """pv_batch_create / pv_batch_destroy over a list of Lattice objects (kept alive here)."""

    def __init__(self, lattices):
        self.lattices = list(lattices)
        arr = (_vp * len(self.lattices))(*[l.handle.value for l in self.lattices])
        h = ctypes.c_void_p()
        _check(lib().pv_batch_create(len(self.lattices), arr, ctypes.byref(h)))
        self.handle = h
        self._ws = None

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.pv_batch_destroy(h)
            self.handle = None

    def stats(self):
        c, r = ctypes.c_int(), ctypes.c_int()
        _check(lib().pv_batch_stats(self.handle, ctypes.byref(c), ctypes.byref(r)))
        return c.value, r.value


def pv_batch_kpm_moments(batch: Batch, rs, M: int, a, b, mu=None, nb=None):
    """Moments of every instance: rs list of device blocks; returns mu [n][nb][M].
    The workspace is cached on the Batch object (the captured graph refers to it)."""
    torch = _torch()
    n = len(batch.lattices)
    nb = nb if nb is not None else rs[0].numel() // batch.lattices[0].n_rows
    dt = _dtype_code(rs[0])
    for l, r in zip(batch.lattices, rs):
        _vec(r, "r", l.n_rows, nb, dt)
    if mu is None:
        mu = torch.empty((n, nb, M), dtype=torch.float64, device=rs[0].device)
    need = lib().pv_batch_kpm_workspace_size(batch.handle, dt, nb, M)
    if batch._ws is None or batch._ws.numel() < need:
        batch._ws = _workspace(need, rs[0].device)
    av = np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), (n,)))
    bv = np.ascontiguousarray(np.broadcast_to(np.asarray(b, dtype=np.float64), (n,)))
    ptrs = (_vp * n)(*[r.data_ptr() for r in rs])
    _check(lib().pv_batch_kpm_moments(batch.handle, dt, nb, M, _dptr(av), _dptr(bv), ptrs,
                                      ctypes.c_void_p(mu.data_ptr()), ctypes.c_void_p(batch._ws.data_ptr()),
                                      batch._ws.numel(), _stream()))
    return mu


def pv_batch_set_tuning(batch: Batch, dtype: int, nb: int, tuning=None):
    """Launch shape of the batch for (dtype, nb): dict of TUNING_FIELDS (only
    kernel, elems_per_lane and workgroup_size count), None = the default."""
    if tuning is None:
        _check(lib().pv_batch_set_tuning(batch.handle, dtype, nb, None))
        return
    bad = set(tuning) - set(TUNING_FIELDS)
    if bad:
        raise ValueError(f"unknown tuning fields {sorted(bad)}")
    t = pv_tuning(**{k: int(v) for k, v in tuning.items()})
    _check(lib().pv_batch_set_tuning(batch.handle, dtype, nb, ctypes.byref(t)))


def pv_batch_get_tuning(batch: Batch, dtype: int, nb: int) -> dict:
    t = pv_tuning()
    _check(lib().pv_batch_get_tuning(batch.handle, dtype, nb, ctypes.byref(t)))
    return {k: getattr(t, k) for k in TUNING_FIELDS}


def pv_batch_autotune(batch: Batch, rs, a, b, nb=None):
    """Time the batch's candidate launch shapes on its own captured steps and
    keep the fastest; returns (shape dict, ms per batched step)."""
    n = len(batch.lattices)
    nb = nb if nb is not None else rs[0].numel() // batch.lattices[0].n_rows
    dt = _dtype_code(rs[0])
    for l, r in zip(batch.lattices, rs):
        _vec(r, "r", l.n_rows, nb, dt)
    ws = _workspace(lib().pv_batch_autotune_workspace_size(batch.handle, dt, nb), rs[0].device)
    av = np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), (n,)))
    bv = np.ascontiguousarray(np.broadcast_to(np.asarray(b, dtype=np.float64), (n,)))
    ptrs = (_vp * n)(*[r.data_ptr() for r in rs])
    t = pv_tuning()
    ms = ctypes.c_double()
    _check(lib().pv_batch_autotune(batch.handle, dt, nb, _dptr(av), _dptr(bv), ptrs, ctypes.c_void_p(ws.data_ptr()),
                                   ws.numel(), _stream(), ctypes.byref(t), ctypes.byref(ms)))
    return {k: getattr(t, k) for k in TUNING_FIELDS}, ms.value


def _grad_len(lat: Lattice) -> int:
    return lat.n_rows if lat.pot_mode == PV_POT_ORBITAL else lat.n_sites


def pv_kpm_moments_vjp(lat: Lattice, r, M: int, a: float, b: float, gbar, ckpt_every: int = 16, gradV=None, nb=None):
    """dL/dV for L = sum gbar * mu (gbar device [nb][M] float64)."""
    torch = _torch()
    nb = nb if nb is not None else r.numel() // lat.n_rows
    dt = _dtype_code(r)
    if gradV is None:
        gradV = torch.empty(_grad_len(lat), dtype=torch.float64, device=r.device)
    gbar = gbar.contiguous()
    ws = _workspace(lib().pv_kpm_vjp_workspace_size(lat.handle, dt, nb, M, ckpt_every), r.device)
    _check(lib().pv_kpm_moments_vjp(lat.handle, dt, nb, M, a, b, _vec(r, "r", lat.n_rows, nb),
                                    ctypes.c_void_p(gbar.data_ptr()), ctypes.c_void_p(gradV.data_ptr()), ckpt_every,
                                    ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return gradV


def pv_kpm_moments_ckpt(lat: Lattice, r, M: int, a: float, b: float, ckpt_every: int = 16, nb=None):
    """(mu, work): the moments of pv_kpm_moments plus a workspace holding the
    forward checkpoints, for pv_kpm_moments_vjp_ckpt."""
    torch = _torch()
    nb = nb if nb is not None else r.numel() // lat.n_rows
    dt = _dtype_code(r)
    mu = torch.empty((nb, M), dtype=torch.float64, device=r.device)
    ws = _workspace(lib().pv_kpm_vjp_workspace_size(lat.handle, dt, nb, M, ckpt_every), r.device)
    _check(lib().pv_kpm_moments_ckpt(lat.handle, dt, nb, M, a, b, _vec(r, "r", lat.n_rows, nb),
                                     ctypes.c_void_p(mu.data_ptr()), ckpt_every,
                                     ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return mu, ws


def pv_kpm_moments_vjp_ckpt(lat: Lattice, r, M: int, a: float, b: float, gbar, work, ckpt_every: int = 16,
                            gradV=None, nb=None):
    """dL/dV for L = sum gbar * mu from the checkpoints of pv_kpm_moments_ckpt (same arguments)."""
    torch = _torch()
    nb = nb if nb is not None else r.numel() // lat.n_rows
    dt = _dtype_code(r)
    if gradV is None:
        gradV = torch.empty(_grad_len(lat), dtype=torch.float64, device=r.device)
    gbar = gbar.contiguous()
    _check(lib().pv_kpm_moments_vjp_ckpt(lat.handle, dt, nb, M, a, b, _vec(r, "r", lat.n_rows, nb),
                                         ctypes.c_void_p(gbar.data_ptr()), ctypes.c_void_p(gradV.data_ptr()),
                                         ckpt_every, ctypes.c_void_p(work.data_ptr()), work.numel(), _stream()))
    return gradV


def pv_cheb_propagate_vjp(lat: Lattice, psi0, psibar, a, b, dt, M, nsteps, want_psi0bar=True, nb=None):
    """(dL/dV, cotangent of psi0) for psi_T = U^nsteps psi0 and cotangent psibar of psi_T."""
    torch = _torch()
    nb = nb if nb is not None else psi0.numel() // lat.n_rows
    dtc = _dtype_code(psi0)
    gradV = torch.empty(_grad_len(lat), dtype=torch.float64, device=psi0.device)
    psi0bar = torch.empty_like(psi0) if want_psi0bar else None
    psibar = psibar.contiguous()
    ws = _workspace(lib().pv_cheb_propagate_vjp_workspace_size(lat.handle, dtc, nb, M, nsteps), psi0.device)
    _check(lib().pv_cheb_propagate_vjp(lat.handle, dtc, nb, a, b, dt, M, nsteps, _vec(psi0, "psi0", lat.n_rows, nb),
                                       _vec(psibar, "psibar", lat.n_rows, nb, dtc),
                                       None if psi0bar is None else ctypes.c_void_p(psi0bar.data_ptr()),
                                       ctypes.c_void_p(gradV.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                                       ws.numel(), _stream()))
    return gradV, psi0bar


def pv_cheb_propagate_keep(lat: Lattice, psi0, a, b, dt, M, nsteps, keep_series=False, nb=None):
    """(psi_T, work): psi_T = U^nsteps psi0 (psi0 unchanged) plus a workspace
    holding the intermediate states (and with keep_series every step's
    Chebyshev vectors), for pv_cheb_propagate_vjp_keep."""
    torch = _torch()
    nb = nb if nb is not None else psi0.numel() // lat.n_rows
    dtc = _dtype_code(psi0)
    psiT = torch.empty_like(psi0)
    ks = int(bool(keep_series))
    ws = _workspace(lib().pv_cheb_propagate_keep_workspace_size(lat.handle, dtc, nb, M, nsteps, ks), psi0.device)
    _check(lib().pv_cheb_propagate_keep(lat.handle, dtc, nb, a, b, dt, M, nsteps, _vec(psi0, "psi0", lat.n_rows, nb),
                                        _vec(psiT, "psiT", lat.n_rows, nb, dtc), ks, ctypes.c_void_p(ws.data_ptr()),
                                        ws.numel(), _stream()))
    return psiT, ws


def pv_cheb_propagate_vjp_keep(lat: Lattice, psi0, psibar, a, b, dt, M, nsteps, work, keep_series=False,
                               want_psi0bar=True, nb=None):
    """pv_cheb_propagate_vjp from the states kept by pv_cheb_propagate_keep (same arguments)."""
    torch = _torch()
    nb = nb if nb is not None else psi0.numel() // lat.n_rows
    dtc = _dtype_code(psi0)
    gradV = torch.empty(_grad_len(lat), dtype=torch.float64, device=psi0.device)
    psi0bar = torch.empty_like(psi0) if want_psi0bar else None
    psibar = psibar.contiguous()
    _check(lib().pv_cheb_propagate_vjp_keep(lat.handle, dtc, nb, a, b, dt, M, nsteps,
                                            _vec(psi0, "psi0", lat.n_rows, nb),
                                            _vec(psibar, "psibar", lat.n_rows, nb, dtc),
                                            None if psi0bar is None else ctypes.c_void_p(psi0bar.data_ptr()),
                                            ctypes.c_void_p(gradV.data_ptr()), int(bool(keep_series)),
                                            ctypes.c_void_p(work.data_ptr()), work.numel(), _stream()))
    return gradV, psi0bar


def _autograd():
    torch = _torch()

    class KPMMoments(torch.autograd.Function):
        """mu = KPM moments of the lattice with on-site field V (differentiable in V)."""

        @staticmethod
        def forward(ctx, V, lat, r, M, a, b, ckpt_every):
            lat.set_potential(V.detach())
            # the forward keeps its checkpoint pairs for the backward
            mu, work = pv_kpm_moments_ckpt(lat, r, M, a, b, ckpt_every)
            ctx.lat, ctx.r, ctx.M, ctx.a, ctx.b, ctx.ck, ctx.work = lat, r, M, a, b, ckpt_every, work
            ctx.V = V.detach()
            return mu

        @staticmethod
        def backward(ctx, gbar):
            ctx.lat.set_potential(ctx.V)
            g = pv_kpm_moments_vjp_ckpt(ctx.lat, ctx.r, ctx.M, ctx.a, ctx.b, gbar.to(torch.float64), ctx.work, ctx.ck)
            return g.to(ctx.V.dtype), None, None, None, None, None, None

    class Propagate(torch.autograd.Function):
        """psi_T = U(dt)^nsteps psi0 for the lattice with field V (differentiable in V and psi0)."""

        @staticmethod
        def forward(ctx, V, psi0, lat, a, b, dt, M, nsteps, keep_series):
            lat.set_potential(V.detach())
            ctx.lat, ctx.a, ctx.b, ctx.dt, ctx.M, ctx.n, ctx.ks = lat, a, b, dt, M, nsteps, keep_series
            ctx.V = V.detach()
            ctx.psi0 = psi0.detach().contiguous()
            if nsteps < 1:
                ctx.work = None
                return ctx.psi0.clone()
            # the forward keeps its intermediate states for the backward
            psi, ctx.work = pv_cheb_propagate_keep(lat, ctx.psi0, a, b, dt, M, nsteps, keep_series)
            return psi

        @staticmethod
        def backward(ctx, psibar):
            if ctx.work is None:
                return torch.zeros_like(ctx.V), psibar, None, None, None, None, None, None, None
            ctx.lat.set_potential(ctx.V)
            g, p0 = pv_cheb_propagate_vjp_keep(ctx.lat, ctx.psi0, psibar, ctx.a, ctx.b, ctx.dt, ctx.M, ctx.n,
                                               ctx.work, ctx.ks)
            return g.to(ctx.V.dtype), p0, None, None, None, None, None, None, None

    return KPMMoments, Propagate


def kpm_moments(V, lat: Lattice, r, M: int, a: float, b: float, ckpt_every: int = 16):
    """Differentiable KPM moments mu(V) (torch.autograd.Function around
    pv_kpm_moments_ckpt / pv_kpm_moments_vjp_ckpt: the forward keeps its
    checkpoints for the backward)."""
    return _autograd()[0].apply(V, lat, r, M, a, b, ckpt_every)


def cheb_propagate(V, psi0, lat: Lattice, a: float, b: float, dt: float, M: int, nsteps: int,
                   keep_series: bool = False):
    """Differentiable Chebyshev propagation psi_T(V, psi0).  The forward keeps
    its time-step states for the backward; with keep_series also every
    step's Chebyshev vectors (nsteps * M more vectors), and the backward
    recomputes none."""
    return _autograd()[1].apply(V, psi0, lat, a, b, dt, M, nsteps, bool(keep_series))
