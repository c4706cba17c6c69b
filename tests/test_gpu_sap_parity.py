"""SAP parity on a lattice with four Schwarz blocks in every direction, at the
production cycle count.

With two blocks in a direction, the forward and the backward neighbour block
are the same block, so a swapped face or neighbour offset would go unseen;
16^4 has four blocks per direction, so every face of a block has a distinct
neighbour.  ncy = 12 is the smoother's default: with FP32/FP16 storage every
block is then visited twelve times, eleven of them with the residual carried
from the previous visit.  Each comparison is element by element against the
oracle's SAP, both as a whole-lattice relative norm and as the largest
per-site error (which a single wrong site cannot hide in).
"""
import numpy as np
import pytest

import oracle
from gpu_util import BC, Lattice, check_sap, gpu_sap, round_fp16
from paper_1710_07041_amd import synth

pytestmark = pytest.mark.gpu

NMR = 4
M0 = -0.25


@pytest.fixture(scope="module")
def lat16():
    """16^4, eps = 0.5, csw = 1, seed 4: 256 blocks, four per direction."""
    return Lattice((16, 16, 16, 16), eps=0.5, csw=1.0, seed=4)


@pytest.fixture(scope="module")
def eta16(lat16):
    return synth.gaussian_spinor(lat16.dims, seed=21)


_refs = {}


def oracle_sap(lat, eta, ncy, rounded=False):
    key = (lat.dims, ncy, rounded)
    if key not in _refs:
        U, C = (round_fp16(lat.U), round_fp16(lat.C)) if rounded else (lat.U, lat.C)
        _refs[key] = oracle.sap(lat.dims, (4, 4, 4, 4), U, C, M0, eta, ncy, NMR, BC)
    return _refs[key]


@pytest.mark.parametrize("ncy", [4, 12])
@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_sap_16x4(lat16, eta16, prec, ncy):
    ref = oracle_sap(lat16, eta16, ncy)
    out = gpu_sap(lat16.ctx, eta16, M0, ncy, NMR, prec)
    check_sap(out, ref, prec, f"16^4 ncy={ncy}")


@pytest.mark.parametrize("ncy", [4, 12])
def test_sap_16x4_half_fields(lat16, eta16, ncy):
    """FP16 links and clover under the FP32 smoother: all nine link entries
    read, the result is the oracle's SAP on the FP16-rounded fields up to FP32
    rounding; with gauge compression (the default) it is compared with the
    exact fields' SAP at the FP16-field tolerance."""
    ref = oracle_sap(lat16, eta16, ncy)
    ref16 = oracle_sap(lat16, eta16, ncy, rounded=True)
    try:
        lat16.ctx.set_sap_half_fields(True)
        lat16.ctx.set_link_compression(False)
        out = gpu_sap(lat16.ctx, eta16, M0, ncy, NMR, "f32")
        check_sap(out, ref16, "f32h-rounded", f"16^4 ncy={ncy}")
        lat16.ctx.set_link_compression(True)
        out = gpu_sap(lat16.ctx, eta16, M0, ncy, NMR, "f32")
        check_sap(out, ref, "f32h", f"16^4 ncy={ncy}")
    finally:
        lat16.ctx.set_sap_half_fields(False)
        lat16.ctx.set_link_compression(True)


@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_sap_16x4_batch_of_masses(lat16, prec):
    """Four right-hand sides with their own masses in one launch at ncy = 12,
    each against the oracle and bitwise against its solo call."""
    n = 4
    etas = synth.gaussian_spinor(lat16.dims, nrhs=n, seed=22)
    m0 = np.array([-0.38, -0.3, -0.2, 0.1])
    out = gpu_sap(lat16.ctx, etas, m0, 12, NMR, prec, nrhs=n)
    for r in range(n):
        ref = oracle.sap(lat16.dims, (4, 4, 4, 4), lat16.U, lat16.C, m0[r], etas[r], 12, NMR, BC)
        check_sap(out[r], ref, prec, f"16^4 ncy=12 batch m0={m0[r]}")
        assert np.array_equal(out[r], gpu_sap(lat16.ctx, etas[r], m0[r], 12, NMR, prec))
