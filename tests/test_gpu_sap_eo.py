"""GPU parity of the even-odd preconditioned smoother (dd_sap_eo) against the
oracle's even-odd SAP, and of SAP-FGMRES solves that use it, through the C ABI."""
import numpy as np
import pytest

import oracle
from gpu_util import BC, Lattice, check_sap, to_dev, to_host
from paper_1710_07041_amd import synth
from test_gpu_solver import gpu_solve

pytestmark = pytest.mark.gpu


def gpu_sap_eo(lat, eta, m0, ncy, nmr, prec, nrhs=None):
    import torch
    n = 1 if nrhs is None else nrhs
    x = to_dev(eta)
    eb = lat.ctx.empty_blocked(prec, n)
    pb = lat.ctx.empty_blocked(prec, n)
    lat.ctx.pack(x, eb, prec, n)
    lat.ctx.sap(m0, eb, pb, ncy, nmr, prec, n, eo=True)
    y = torch.empty_like(x)
    lat.ctx.unpack(pb, y, prec, n)
    lat.ctx.synchronize()
    return to_host(y)


@pytest.fixture(scope="module", params=[(8, 8, 8, 8), (4, 4, 8, 24), (4, 4, 4, 4)], ids=lambda d: "x".join(map(str, d)))
def lat(request):
    return Lattice(request.param, eps=0.4, seed=2)


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
@pytest.mark.parametrize("ncy,nmr", [(1, 4), (3, 2), (2, 0)])
def test_sap_eo_matches_oracle(lat, prec, ncy, nmr):
    """nmr = 0 still reconstructs the odd sites: delta_o = A_oo^-1 rho_o."""
    eta = synth.gaussian_spinor(lat.dims, seed=3)
    m0 = -0.2
    ref = oracle.sap(lat.dims, (4, 4, 4, 4), lat.U, lat.C, m0, eta, ncy, nmr, BC, eo=True)
    out = gpu_sap_eo(lat, eta, m0, ncy, nmr, prec)
    check_sap(out, ref, "eo-" + prec, f"{'x'.join(map(str, lat.dims))} ncy={ncy} nmr={nmr}")


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_sap_eo_multi_rhs(lat, prec):
    """Each right-hand side with its own mass (its own A_oo factor); FP64 batch = solo bitwise."""
    n = 3
    eta = synth.gaussian_spinor(lat.dims, nrhs=n, seed=5)
    m0 = np.array([-0.3, -0.1, 0.2])
    out = gpu_sap_eo(lat, eta, m0, 2, 4, prec, nrhs=n)
    for r in range(n):
        ref = oracle.sap(lat.dims, (4, 4, 4, 4), lat.U, lat.C, m0[r], eta[r], 2, 4, BC, eo=True)
        check_sap(out[r], ref, "eo-" + prec, f"{'x'.join(map(str, lat.dims))} multi-rhs r={r}")
        if prec == "f64":
            assert np.array_equal(out[r], gpu_sap_eo(lat, eta[r], m0[r], 2, 4, prec))


@pytest.fixture(scope="module")
def c1():
    return Lattice((8, 8, 8, 8), eps=0.3, csw=1.0, seed=0)


@pytest.mark.parametrize("sap_prec", ["f64", "f32", "f16"])
def test_solve_eo_residual_against_oracle(c1, sap_prec):
    b = synth.gaussian_spinor(c1.dims, seed=0)
    m0 = -0.2
    st, info, x = gpu_solve(c1, b, m0, sap_prec, sap_eo=1)
    assert st == 0 and info[0]["status"] == 0
    r = b - oracle.apply_D(c1.dims, c1.U, c1.C, m0, x, BC)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-10
    _, info_plain, _ = gpu_solve(c1, b, m0, sap_prec)
    assert info[0]["iterations"] <= info_plain[0]["iterations"]


def test_solve_eo_multi_rhs_point_sources(c1):
    b = synth.point_sources(c1.dims)
    st, info, x = gpu_solve(c1, b, -0.2, "f32", nrhs=12, sap_eo=1)
    assert st == 0
    for r in range(12):
        res = b[r] - oracle.apply_D(c1.dims, c1.U, c1.C, -0.2, x[r], BC)
        assert np.linalg.norm(res) / np.linalg.norm(b[r]) <= 1e-10
