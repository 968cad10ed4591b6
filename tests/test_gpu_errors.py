"""Error paths that need a device: forced allocation failures of the
lattice's device tables (PV_ERR_OOM, through the PV_TEST_FAIL_DEVICE_ALLOC
hook) leave the lattice usable, and non-finite start blocks of the
interior-eigenvalue solvers give PV_ERR_NONFINITE instead of NaN results.
Every kernel runs normally; only host-side checks fail."""

import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1708_09689_amd as pv  # noqa: E402
from oracle import spmmv  # noqa: E402
import workloads as W  # noqa: E402

from gpu_common import Case, dev, host, rel_err  # noqa: E402


@pytest.fixture
def fail_alloc():
    def set_(v):
        if v is None:
            os.environ.pop("PV_TEST_FAIL_DEVICE_ALLOC", None)
        else:
            os.environ["PV_TEST_FAIL_DEVICE_ALLOC"] = v
    yield set_
    os.environ.pop("PV_TEST_FAIL_DEVICE_ALLOC", None)


@pytest.mark.parametrize("which,msg", [("all", b"coefficient upload"), ("1", b"coefficient upload"),
                                       ("3", b"zero row")])
def test_forced_allocation_failure_then_recovery(fail_alloc, which, msg):
    c = Case("ti", (6, 5, 4), (1, 1, 1), Wd=1.0, seed=31)     # fresh lattice: no device tables yet
    x = c.block(2, seed=1)
    y = torch.empty((c.D, 2), dtype=torch.complex128, device="cuda")
    fail_alloc(which)
    with pytest.raises(pv.PvError) as e:
        pv.pv_spmmv(c.lat, dev(x), y, 0.5, 0.1, 0.0)
    assert e.value.status == 5
    assert msg in pv.lib().pv_last_error()
    fail_alloc(None)
    pv.pv_spmmv(c.lat, dev(x), y, 0.5, 0.1, 0.0)
    assert rel_err(host(y), spmmv.spmmv(c.H, x, 0.5, 0.1, 0.0)) < 1e-13


def test_forced_failure_of_generic_offsets(fail_alloc):
    no = 2
    g = np.random.default_rng(5)
    offsets, blocks = [], []
    for o in [(1, 0, 0), (0, 1, 1)]:
        B = g.standard_normal((no, no)) + 1j * g.standard_normal((no, no))
        offsets += [o, tuple(-v for v in o)]
        blocks += [B, B.conj().T]
    st = {"dim": 3, "n_orb": no, "offsets": np.array(offsets), "blocks": np.array(blocks),
          "onsite": np.eye(no), "pot_mode": pv.PV_POT_NONE}
    lat = pv.Lattice((5, 4, 3), (1, 1, 1), st)
    x = torch.ones((lat.n_rows, 1), dtype=torch.complex128, device="cuda")
    y = torch.empty_like(x)
    fail_alloc("2")
    with pytest.raises(pv.PvError) as e:
        pv.pv_spmmv(lat, x, y, 1.0, 0.0, 0.0)
    assert e.value.status == 5 and b"offset upload" in pv.lib().pv_last_error()
    fail_alloc(None)
    pv.pv_spmmv(lat, x, y, 1.0, 0.0, 0.0)
    assert torch.isfinite(y).all()


def test_chebfd_and_trlanczos_non_finite_start_block():
    c = Case("ti", (5, 4, 4), (1, 1, 1), Wd=1.0, seed=32)
    X = W.random_phase_block(c.D, 32, W.generator(7, 2)).reshape(c.D, 2, 16).transpose(1, 0, 2).copy()
    X[1, 7, 3] = np.nan
    with pytest.raises(pv.PvError) as e:
        pv.pv_chebfd(c.lat, dev(X), 16, 7.0, 0.0, -0.5, 0.5, 50, 4, 1e-9, max_iter=2)
    assert e.value.status == 7
    V0 = W.gaussian_block(c.D, 4, W.generator(7, 3))
    V0[3, 1] = np.inf
    with pytest.raises(pv.PvError) as e:
        pv.pv_trlanczos_fd(c.lat, dev(V0), 7.0, 0.0, -0.5, 0.5, 60, 32, 1e-9, max_restarts=2)
    assert e.value.status == 7
