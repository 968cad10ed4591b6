"""The C ABI from a plain C99 program (tests/c_client/kpm_dos.c, built with
gcc against include/pvdtm.h and the in-tree library, no C++ or Python in the
client): on the CPU it must compile, link and report argument errors and the
missing device; on the GPU its KPM moments (on-the-fly field, device-made
random-phase columns) must equal the oracle's to 1e-12 and its DOS the
oracle's reconstruction of the same moments to 1e-10 relative."""

import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "c_client", "kpm_dos.c")
LIBDIR = os.path.join(ROOT, "paper_1708_09689_amd", "lib")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def _build(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    if not os.path.exists(os.path.join(LIBDIR, "libpvdtm.so")):
        pytest.fail("libpvdtm.so is not built")
    exe = str(tmp_path / "kpm_dos")
    cmd = [cc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"), SRC,
           "-L", LIBDIR, "-lpvdtm", "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
           f"-Wl,-rpath,{LIBDIR}", f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}", "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=120)
    return exe


def test_c_client_builds_and_reports_no_device(tmp_path):
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present: the GPU test runs the client")
    exe = _build(tmp_path)
    p = subprocess.run([exe, "6", "5", "4", "2", "16", "7", "1.0", "9"], capture_output=True, text=True, timeout=60)
    assert p.returncode == 0, p.stderr
    assert p.stdout.startswith("no-device ")


@pytest.mark.gpu
def test_c_client_kpm_matches_oracle(tmp_path):
    from oracle import hamiltonian, kpm, lattice, models, rng
    exe = _build(tmp_path)
    L, nb, M, fseed, W, vseed = (9, 6, 5), 4, 64, 7, 1.0, 9
    print(f"c client: L={L} nb={nb} M={M}", flush=True)
    p = subprocess.run([exe, *map(str, L), str(nb), str(M), str(fseed), repr(W), str(vseed)],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 0, p.stderr
    mu = np.zeros((nb, M))
    E, rho = [], []
    for line in p.stdout.splitlines():
        f = line.split()
        if f[0] == "mu":
            mu[int(f[1]), int(f[2])] = float(f[3])
        elif f[0] == "dos":
            E.append(float(f[1]))
            rho.append(float(f[2]))
    ol = lattice.Lattice(L, (1, 1, 1), 4)
    H = hamiltonian.assemble(models.topological_insulator(1.0, 2.0), ol, rng.field(fseed, W, ol.n_sites))
    r = rng.random_block(vseed, ol.n_rows, nb, rng.PHASE)
    ref = kpm.moments_direct(H, r, M, 7.0, 0.0)
    assert np.abs(mu - ref).max() < 1e-12
    ref_rho = kpm.dos(ref.mean(axis=0), np.array(E), 7.0, 0.0)
    assert np.abs(np.array(rho) - ref_rho).max() < 1e-10 * np.abs(ref_rho).max()
