"""Fermion boundary signs in every direction, not only in t.

Every other GPU test runs with periodic x, y and z and an antiperiodic t,
so a sign applied in the wrong direction (or only in t) on one of the
paths would pass them.  Here the operator (every form: one right-hand side,
lane-shared FP64, the block-wise FP32 form with cooperative face hops, FP16),
the block operator, the smoother and a full solve run with antiperiodic x
and z (and y), on lattices where a direction is one block (the sign applies
inside the block) and several blocks (across a face), against the oracle
with the same boundary conditions."""
import numpy as np
import pytest

import oracle
from gpu_util import REL_TOL_APPLY, Lattice, check_sap, gpu_sap, rel
from paper_1710_07041_amd import synth

pytestmark = pytest.mark.gpu

CASES = [((4, 4, 4, 4), (-1, 1, -1, 1)), ((8, 8, 8, 8), (-1, -1, -1, -1)), ((16, 8, 16, 8), (-1, 1, -1, -1)),
         ((4, 8, 16, 8), (-1, -1, 1, -1))]


@pytest.fixture(scope="module", params=CASES, ids=lambda c: "x".join(map(str, c[0])) + "_bc" + "".join(
    "+" if b > 0 else "-" for b in c[1]))
def lat(request):
    dims, bcs = request.param
    return Lattice(dims, eps=0.5, seed=7, bcs=bcs)


@pytest.mark.parametrize("n", [1, 2, 4])
@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_operator(lat, prec, n):
    psi = synth.gaussian_spinor(lat.dims, nrhs=n, seed=3)
    m0 = np.linspace(-0.3, 0.1, n)
    out = lat.apply(psi, m0, prec, nrhs=n)
    for r in range(n):
        ref = oracle.apply_D(lat.dims, lat.U, lat.C, m0[r], psi[r], lat.bcs)
        assert rel(out[r], ref) <= REL_TOL_APPLY[prec], (prec, n, r)


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_block_operator(lat, prec):
    """D_BB on the first and last block: the sign applies to an in-block hop
    only where the block spans the direction."""
    import torch
    from dense_ref import block_sites
    from gpu_util import to_dev, to_host
    psi = synth.gaussian_spinor(lat.dims, seed=5)
    nblk = lat.V // 256
    xb, yb = lat.ctx.empty_blocked(prec), lat.ctx.empty_blocked(prec)
    lat.ctx.pack(to_dev(psi), xb, prec)
    lat.ctx.pack(to_dev(np.zeros_like(psi)), yb, prec)
    blocks = sorted({0, nblk - 1})
    for bid in blocks:
        lat.ctx.apply_D_block(-0.25, bid, xb, yb, prec)
    y = torch.empty_like(to_dev(psi))
    lat.ctx.unpack(yb, y, prec)
    lat.ctx.synchronize()
    y = to_host(y)
    for bid in blocks:
        ref = oracle.apply_DBB(lat.dims, (4, 4, 4, 4), lat.U, lat.C, -0.25, bid, psi, lat.bcs)
        sites, _ = block_sites(lat.dims, (4, 4, 4, 4), bid)
        assert rel(y[sites], ref[sites]) <= REL_TOL_APPLY[prec], bid


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_smoother(lat, prec):
    eta = synth.gaussian_spinor(lat.dims, seed=9)
    ref = oracle.sap(lat.dims, (4, 4, 4, 4), lat.U, lat.C, -0.25, eta, 3, 4, lat.bcs)
    out = gpu_sap(lat.ctx, eta, -0.25, 3, 4, prec)
    check_sap(out, ref, prec, f"{lat.dims} bcs={lat.bcs}")


def test_solve(lat):
    from gpu_util import to_dev, to_host
    from paper_1710_07041_amd import ddsap
    import torch
    b = synth.gaussian_spinor(lat.dims, seed=11)
    bd = to_dev(b)
    xd = torch.zeros_like(bd)
    p = ddsap.default_params()
    p.sap_prec = ddsap.PREC["f16"]
    st, info = lat.ctx.solve(-0.2, bd, xd, 1, p, raise_on_fail=False)
    assert st == 0 and info[0]["status"] == 0
    x = to_host(xd)
    r = b - oracle.apply_D(lat.dims, lat.U, lat.C, -0.2, x, lat.bcs)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-10
