"""GPU parity of trLanczosFD (filtered thick-restart block Lanczos) against
the dense eigendecomposition of the oracle's H: exactly the eigenvalues
inside the window (1e-10 a), residuals below tol, Ritz vectors checked with
the oracle's H (||H u - theta u|| <= 10 tol, orthonormal to 1e-10); the
same eigenvalues as ChebFD; complex64 vectors to a stated 1e-4 a."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1708_09689_amd as pv  # noqa: E402
import workloads as W  # noqa: E402

from gpu_common import Case, dev, host  # noqa: E402


def window_case(centre, half):
    c = Case("ti", (6, 6, 6), (1, 1, 1), Wd=2.0, seed=9)
    ev = np.linalg.eigvalsh(c.H.toarray())
    return c, ev[np.abs(ev - centre) < half]


@pytest.mark.parametrize("centre,half,nbl", [(1.2, 0.06, 2), (-1.5, 0.1, 4), (1.2, 0.06, 4)])
def test_trlanczos_finds_window_eigenpairs(centre, half, nbl):
    c, inside = window_case(centre, half)
    V0 = dev(W.gaussian_block(c.D, nbl, W.generator(9, W.STREAM_VECTORS, nbl)))
    m = (2 * inside.size + 12 + nbl - 1) // nbl * nbl
    th, res, X, it = pv.pv_trlanczos_fd(c.lat, V0, 7.0, 0.0, centre - half, centre + half, 160, m, 1e-9,
                                        n_out=64)
    assert th.size == inside.size
    assert np.abs(th - inside).max() < 1e-10 * 7.0
    assert res.max() <= 1e-9
    U = host(X)[:, : th.size]
    R = c.H @ U - U * th[None, :]
    assert np.linalg.norm(R, axis=0).max() <= 1e-8
    assert np.abs(U.conj().T @ U - np.eye(th.size)).max() < 1e-10


def test_trlanczos_agrees_with_chebfd():
    centre, half = 1.2, 0.06
    c, inside = window_case(centre, half)
    V0 = dev(W.gaussian_block(c.D, 2, W.generator(10, W.STREAM_VECTORS)))
    th, res, _, _ = pv.pv_trlanczos_fd(c.lat, V0, 7.0, 0.0, centre - half, centre + half, 160, 48, 1e-9)
    X = dev(W.gaussian_block(c.D, 64, W.generator(11, W.STREAM_VECTORS)))
    thf, resf, nconv, _ = pv.pv_chebfd(c.lat, X, 32, 7.0, 0.0, centre - half, centre + half, 600, inside.size,
                                       1e-9, max_iter=40)
    thf = np.sort(thf[: inside.size])
    assert np.abs(th - thf).max() < 1e-10 * 7.0


def test_trlanczos_c64_stated_error():
    centre, half = 1.2, 0.06
    c = Case("ti", (6, 6, 6), (1, 1, 1), Wd=2.0, seed=9, vdtype=np.float32)
    Hq = c.H  # field differs from the float32 copy by < 1e-7
    ev = np.linalg.eigvalsh(Hq.toarray())
    inside = ev[np.abs(ev - centre) < half]
    V0 = dev(W.gaussian_block(c.D, 2, W.generator(9, W.STREAM_VECTORS), np.complex64))
    th, res, _, _ = pv.pv_trlanczos_fd(c.lat, V0, 7.0, 0.0, centre - half, centre + half, 160, 48, 1e-4)
    assert th.size == inside.size
    assert np.abs(th - inside).max() < 1e-4 * 7.0
