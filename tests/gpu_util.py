"""Helpers shared by the GPU tests: move canonical numpy arrays through the C ABI."""
import numpy as np

import oracle
from paper_1710_07041_amd import synth

BC = (1, 1, 1, -1)
REL_TOL_APPLY = {"f64": 1e-12, "f32": 1e-5, "f16": 5e-3}  # per-apply error bounds of the method's targets
REL_TOL_SAP = {"f64": 1e-11, "f32": 1e-4, "f16": 5e-2}


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to("cuda")


def to_host(t):
    return t.cpu().numpy()


class Lattice:
    """A gauge field resident on the GPU plus its oracle clover (for small volumes)."""

    def __init__(self, dims, eps, csw=1.0, seed=0, oracle_clover=True):
        from paper_1710_07041_amd import ddsap
        self.dims = tuple(dims)
        self.V = synth.volume(dims)
        self.csw = csw
        self.U = synth.random_su3_links(dims, eps, seed=seed)
        self.ctx = ddsap.Context(dims, BC)
        self.ctx.set_gauge(self.U, csw)
        self.C = oracle.clover_field(dims, self.U, csw) if oracle_clover else None

    def apply(self, psi, m0, prec, nrhs=None):
        """GPU D on canonical spinor(s) psi (V,4,3) or (n,V,4,3); returns canonical FP64."""
        import torch
        single = nrhs is None
        n = 1 if single else nrhs
        x = to_dev(psi)
        xb = self.ctx.empty_blocked(prec, n)
        yb = self.ctx.empty_blocked(prec, n)
        self.ctx.pack(x, xb, prec, n)
        self.ctx.apply_D(m0, xb, yb, prec, n)
        y = torch.empty_like(x)
        self.ctx.unpack(yb, y, prec, n)
        self.ctx.synchronize()
        return to_host(y)
