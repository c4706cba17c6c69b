"""dd_sap_noalloc against dd_sap: the same smoother with its scratch in the
library's fixed device array instead of an allocation.  Two calls in a row
on one GPU (the second on a smaller input, which must not see the first
one's leftovers), each compared bitwise with dd_sap on the same input, and
an input whose scratch exceeds the fixed array rejected with an error."""
import numpy as np
import pytest

from gpu_util import BC, Lattice, check_sap, to_dev, to_host
import oracle
from paper_1710_07041_amd import synth

pytestmark = pytest.mark.gpu


def run(ctx, eta, m0, ncy, nmr, prec, nrhs, noalloc):
    import torch
    x = to_dev(eta)
    eb, pb = ctx.empty_blocked(prec, nrhs), ctx.empty_blocked(prec, nrhs)
    ctx.pack(x, eb, prec, nrhs)
    pb.fill_(7)  # psi is overwritten, whatever it held
    if noalloc:
        ctx.sap_noalloc(m0, eb, pb, ncy, nmr, prec, nrhs)
    else:
        ctx.sap(m0, eb, pb, ncy, nmr, prec, nrhs)
    y = torch.empty_like(x)
    ctx.unpack(pb, y, prec, nrhs)
    ctx.synchronize()
    return to_host(y)


def test_noalloc_equals_sap_two_calls():
    from paper_1710_07041_amd import ddsap
    big = Lattice((16, 16, 16, 16), eps=0.5, seed=4, oracle_clover=False)
    small = Lattice((8, 8, 8, 8), eps=0.3, seed=0)
    # first call: 16^4, three right-hand sides in FP32, twelve cycles
    eta = synth.gaussian_spinor(big.dims, nrhs=3, seed=61)
    m0 = np.array([-0.3, -0.25, -0.2])
    a = run(big.ctx, eta, m0, 12, 4, "f32", 3, noalloc=True)
    b = run(big.ctx, eta, m0, 12, 4, "f32", 3, noalloc=False)
    assert np.array_equal(a, b)
    # second call: a smaller input (8^4, one right-hand side, FP16 storage)
    eta2 = synth.gaussian_spinor(small.dims, seed=62)
    a2 = run(small.ctx, eta2, -0.2, 4, 4, "f16", 1, noalloc=True)
    b2 = run(small.ctx, eta2, -0.2, 4, 4, "f16", 1, noalloc=False)
    assert np.array_equal(a2, b2)
    # and against the oracle, at the FP16 smoother's tolerance
    ref = oracle.sap(small.dims, (4, 4, 4, 4), small.U, small.C, -0.2, eta2, 4, 4, BC)
    check_sap(a2, ref, "f16", "8^4 noalloc")
    # zero cycles clear psi without hipMemsetAsync
    z = run(small.ctx, eta2, -0.2, 0, 4, "f64", 1, noalloc=True)
    assert np.max(np.abs(z)) == 0
    # 16 FP64 right-hand sides on 16^4 need 2 x 201 MB of scratch: rejected
    import torch
    eb = big.ctx.empty_blocked("f64", 16)
    pb = big.ctx.empty_blocked("f64", 16)
    st = big.ctx.sap_noalloc(np.full(16, -0.2), eb, pb, 1, 4, "f64", 16, raise_on_fail=False)
    assert st == ddsap.DD_INVALID_ARG
    assert "scratch" in big.ctx.last_error()
    big.ctx.close()
    small.ctx.close()
