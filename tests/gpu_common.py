"""Shared helpers of the GPU parity tests (seeded inputs -> device tensors,
oracle matrices for the same lattices)."""

import numpy as np
import torch

import paper_1708_09689_amd as pv
import workloads as W
from oracle import hamiltonian, lattice, models

DEV = torch.device("cuda:0")

MODELS = {
    "ti": (pv.PV_MODEL_TI, [1.0, 2.0, 0.0, 0.0], lambda: models.topological_insulator(1.0, 2.0)),
    "ti_delta": (pv.PV_MODEL_TI, [1.0, 1.5, 0.3, -0.2], lambda: models.topological_insulator(1.0, 1.5, 0.3, -0.2)),
    "graphene2": (pv.PV_MODEL_GRAPHENE2, [1.0], lambda: models.graphene_two_site(1.0)),
    "graphene4": (pv.PV_MODEL_GRAPHENE4, [1.0], lambda: models.graphene_four_site(1.0)),
    "weyl": (pv.PV_MODEL_WEYL, [np.pi / 2], lambda: models.weyl_semimetal()),
}


class Case:
    """A lattice on both sides: the library handle and the oracle's sparse H."""

    def __init__(self, name, L, periodic, Wd=1.0, seed=0, vdtype=np.float64, with_field=True):
        code, params, mk = MODELS[name]
        self.model = mk()
        self.stencil = pv.pv_model_stencil(code, params)
        self.lat = pv.Lattice(L, periodic, self.stencil)
        self.olat = lattice.Lattice(L, periodic, self.model.n_orb)
        n_field = self.olat.n_sites if self.model.pot == "site" else self.olat.n_rows
        self.V = W.uniform_potential(n_field, Wd, W.generator(seed, W.STREAM_POTENTIAL)) if with_field else None
        if self.V is not None:
            self.Vd = torch.from_numpy(self.V.astype(vdtype)).to(DEV)
            self.lat.set_potential(self.Vd)
        self.H = hamiltonian.assemble(self.model, self.olat, self.V)
        self.D = self.olat.n_rows

    def block(self, nb, seed=1, kind="gauss", dtype=np.complex128):
        g = W.generator(seed, W.STREAM_VECTORS, nb)
        if kind == "phase":
            return W.random_phase_block(self.D, nb, g, dtype)
        return W.gaussian_block(self.D, nb, g, dtype)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel_err(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


# Launch shapes of the parity cases: 1 the direct kernel, 2 the staged kernel,
# 3 the staged kernel with 512 lanes per workgroup (a tile twice as long).
SHAPE_KINDS = [1, 2, 3]


def shape(kind):
    return {"kernel": 2, "workgroup_size": 512} if kind == 3 else {"kernel": kind}
