"""Helpers shared by the GPU tests: move canonical numpy arrays through the C ABI."""
import numpy as np

import oracle
from paper_1710_07041_amd import synth

BC = (1, 1, 1, -1)
REL_TOL_APPLY = {"f64": 1e-12, "f32": 1e-5, "f16": 5e-3}  # per-apply error bounds of the method's targets
# Smoother parity (whole-lattice relative error, largest per-site error over
# the RMS site norm) against the oracle's SAP: about three times the largest
# error measured on MI355X over every SAP test (8^4, 4x4x8x24, 4^4, 16^4 and
# 32^3x64; one to twelve cycles; one to four right-hand sides):
#   f64  5.1e-16 / 1.1e-15    f32 1.9e-7 / 5.2e-7    f16 7.7e-4 / 2.7e-3
#   f32h (FP16 fields under the FP32 smoother, compressed links, against the
#        exact fields' SAP) 1.4e-4 / 2.8e-4
#   f32h-rounded (all link entries read, against the SAP of the FP16-rounded
#        fields: the rest is FP32 arithmetic plus the odd FP16 rounding that
#        falls the other way on the device-built clover) 3.5e-6 / 1.3e-4
#   even-odd smoother: f64 4.6e-16 / 8.5e-16, f32 1.8e-7 / 3.7e-7, f16 3.4e-4 / 9.6e-4
REL_TOL_SAP = {"f64": 2e-15, "f32": 6e-7, "f16": 2.5e-3, "f32h": 5e-4, "f32h-rounded": 1e-5,
               "eo-f64": 2e-15, "eo-f32": 6e-7, "eo-f16": 1e-3}
SITE_TOL_SAP = {"f64": 4e-15, "f32": 2e-6, "f16": 8e-3, "f32h": 1e-3, "f32h-rounded": 4e-4,
                "eo-f64": 4e-15, "eo-f32": 1.5e-6, "eo-f16": 3e-3}


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def site_err(a, b):
    """Largest per-site error, max_x |a(x) - b(x)|, over the root-mean-square
    site norm of b: an O(1) error on a single site shows as O(1) here however
    large the lattice, where the whole-lattice norm of rel() dilutes it."""
    d = np.sqrt(np.sum(np.abs(np.asarray(a) - np.asarray(b)) ** 2, axis=(-2, -1)))
    r = np.sqrt(np.mean(np.sum(np.abs(np.asarray(b)) ** 2, axis=(-2, -1))))
    return float(d.max() / r)


def check_sap(out, ref, key, tag=""):
    """The smoother's parity bar: whole-lattice relative error and largest
    per-site error against the oracle, both within the tolerance of `key`
    (the measured errors are printed as SAPERR lines)."""
    r, s = rel(out, ref), site_err(out, ref)
    print(f"SAPERR {key} {tag} rel={r:.3e} site={s:.3e}", flush=True)
    assert r <= REL_TOL_SAP[key], (key, tag, r)
    assert s <= SITE_TOL_SAP[key], (key, tag, s)


def round_fp16(z):
    """Each real part rounded as the library stores FP16 fields: to FP32, then
    to FP16, both to nearest even."""
    f = lambda a: a.astype(np.float32).astype(np.float16).astype(np.float64)
    return f(z.real) + 1j * f(z.imag)


def gpu_sap(ctx, eta, m0, ncy, nmr, prec, nrhs=None):
    """dd_sap on canonical spinor(s) eta through pack / sap / unpack; canonical FP64 out."""
    import torch
    n = 1 if nrhs is None else nrhs
    x = to_dev(eta)
    eb = ctx.empty_blocked(prec, n)
    pb = ctx.empty_blocked(prec, n)
    ctx.pack(x, eb, prec, n)
    ctx.sap(m0, eb, pb, ncy, nmr, prec, n)
    y = torch.empty_like(x)
    ctx.unpack(pb, y, prec, n)
    ctx.synchronize()
    return to_host(y)


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to("cuda")


def to_host(t):
    return t.cpu().numpy()


class Lattice:
    """A gauge field resident on the GPU plus its oracle clover (for small volumes)."""

    def __init__(self, dims, eps, csw=1.0, seed=0, oracle_clover=True, bcs=BC):
        from paper_1710_07041_amd import ddsap
        self.dims = tuple(dims)
        self.V = synth.volume(dims)
        self.csw = csw
        self.bcs = tuple(bcs)
        self.U = synth.random_su3_links(dims, eps, seed=seed)
        self.ctx = ddsap.Context(dims, self.bcs)
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
