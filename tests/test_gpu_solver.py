"""GPU parity of the Schwarz smoother and of SAP-FGMRES solves, through the C ABI.

SAP is an iteration, so the GPU result is compared with the oracle's SAP at a
precision-dependent tolerance; a solve is correct when the oracle's own FP64
operator gives relative residual <= 1e-10 for the GPU solution.
"""
import numpy as np
import pytest

import oracle
import gpu_util
from gpu_util import BC, REL_TOL_SAP, Lattice, check_sap, rel, round_fp16, to_dev, to_host
from paper_1710_07041_amd import synth

pytestmark = pytest.mark.gpu


def gpu_sap(lat, eta, m0, ncy, nmr, prec, nrhs=None):
    return gpu_util.gpu_sap(lat.ctx, eta, m0, ncy, nmr, prec, nrhs)


@pytest.fixture(scope="module", params=[(8, 8, 8, 8), (4, 4, 8, 24), (4, 4, 4, 4)], ids=lambda d: "x".join(map(str, d)))
def lat(request):
    return Lattice(request.param, eps=0.4, seed=2)


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
@pytest.mark.parametrize("ncy,nmr", [(1, 4), (3, 2), (2, 0), (4, 4)])
def test_sap_matches_oracle(lat, prec, ncy, nmr):
    """(4, 4) is the production setting: with FP32/FP16 storage every block
    is visited four times, three of them with the carried residual."""
    eta = synth.gaussian_spinor(lat.dims, seed=3)
    m0 = -0.2
    ref = oracle.sap(lat.dims, (4, 4, 4, 4), lat.U, lat.C, m0, eta, ncy, nmr, BC)
    out = gpu_sap(lat, eta, m0, ncy, nmr, prec)
    if nmr == 0:
        assert np.max(np.abs(out)) == 0
    else:
        check_sap(out, ref, prec, f"{'x'.join(map(str, lat.dims))} ncy={ncy} nmr={nmr}")


def test_sap_zero_cycles_is_zero(lat):
    out = gpu_sap(lat, synth.gaussian_spinor(lat.dims, seed=4), 0.0, 0, 4, "f32")
    assert np.max(np.abs(out)) == 0


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_sap_multi_rhs(lat, prec):
    """Three right-hand sides with their own masses, then each alone: the
    context's smoother scratch (faces, carried residual) is reused across
    calls of different width."""
    n = 3
    eta = synth.gaussian_spinor(lat.dims, nrhs=n, seed=5)
    m0 = np.array([-0.3, -0.1, 0.2])
    out = gpu_sap(lat, eta, m0, 2, 4, prec, nrhs=n)
    for r in range(n):
        ref = oracle.sap(lat.dims, (4, 4, 4, 4), lat.U, lat.C, m0[r], eta[r], 2, 4, BC)
        check_sap(out[r], ref, prec, f"{'x'.join(map(str, lat.dims))} multi-rhs r={r}")
        # each right-hand side runs the same instruction sequence alone
        assert np.array_equal(out[r], gpu_sap(lat, eta[r], m0[r], 2, 4, prec))


@pytest.mark.parametrize("ncy,nmr", [(1, 4), (4, 4)])
def test_sap_half_fields_is_sap_on_rounded_fields(lat, ncy, nmr):
    """FP16 links and clover under the FP32 smoother.  With all nine link
    entries read, the result is the oracle's SAP on the FP16-rounded fields
    to 2e-5, while the rounding itself moves SAP by about 1e-4; with gauge
    compression the third row is rebuilt from the rounded rows, and the
    result stays within 1e-3 of the exact SAP.  A batch of right-hand sides
    gives each one's result bitwise."""
    eta = synth.gaussian_spinor(lat.dims, seed=3)
    m0 = -0.2
    ref = oracle.sap(lat.dims, (4, 4, 4, 4), lat.U, lat.C, m0, eta, ncy, nmr, BC)
    ref16 = oracle.sap(lat.dims, (4, 4, 4, 4), round_fp16(lat.U), round_fp16(lat.C), m0, eta, ncy, nmr, BC)
    assert rel(ref16, ref) >= 5e-5  # the pin below tells FP16 fields from FP32 ones
    try:
        lat.ctx.set_sap_half_fields(True)
        assert lat.ctx.sap_half_fields
        lat.ctx.set_link_compression(False)
        check_sap(gpu_sap(lat, eta, m0, ncy, nmr, "f32"), ref16, "f32h-rounded", f"{'x'.join(map(str, lat.dims))} ncy={ncy}")
        lat.ctx.set_link_compression(True)
        check_sap(gpu_sap(lat, eta, m0, ncy, nmr, "f32"), ref, "f32h", f"{'x'.join(map(str, lat.dims))} ncy={ncy}")
        etas = synth.gaussian_spinor(lat.dims, nrhs=2, seed=6)
        m0s = np.array([-0.3, 0.1])
        batch = gpu_sap(lat, etas, m0s, ncy, nmr, "f32", nrhs=2)
        for r in range(2):
            assert np.array_equal(batch[r], gpu_sap(lat, etas[r], m0s[r], ncy, nmr, "f32"))
    finally:
        lat.ctx.set_sap_half_fields(False)
        lat.ctx.set_link_compression(True)
    check_sap(gpu_sap(lat, eta, m0, ncy, nmr, "f32"), ref, "f32", f"{'x'.join(map(str, lat.dims))} ncy={ncy} after")


def gpu_solve(lat, b, m0, sap_prec, nrhs=None, **kw):
    from paper_1710_07041_amd import ddsap
    import torch
    n = 1 if nrhs is None else nrhs
    bd = to_dev(b)
    xd = torch.zeros_like(bd)
    p = ddsap.default_params()
    p.sap_prec = ddsap.PREC[sap_prec]
    for k, v in kw.items():
        setattr(p, k, v)
    st, info = lat.ctx.solve(m0, bd, xd, n, p, raise_on_fail=False)
    return st, info, to_host(xd)


@pytest.fixture(scope="module")
def c1():
    """8^4, eps = 0.3, csw = 1, m0 = -0.2, Gaussian right-hand side, seed 0."""
    return Lattice((8, 8, 8, 8), eps=0.3, csw=1.0, seed=0)


@pytest.mark.parametrize("sap_prec", ["f64", "f32", "f16"])
def test_solve_c1_residual_against_oracle(c1, sap_prec):
    b = synth.gaussian_spinor(c1.dims, seed=0)
    m0 = -0.2
    st, info, x = gpu_solve(c1, b, m0, sap_prec)
    assert st == 0 and info[0]["status"] == 0
    r = b - oracle.apply_D(c1.dims, c1.U, c1.C, m0, x, BC)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-10
    assert info[0]["rel_residual"] <= 1e-10


def test_solve_half_fields_residual_against_oracle(c1):
    """FP16 fields under the FP32 smoother change the preconditioner only:
    the solve still reaches the FP64 true residual, checked by the oracle."""
    b = synth.gaussian_spinor(c1.dims, seed=0)
    m0 = -0.2
    c1.ctx.set_sap_half_fields(True)
    try:
        st, info, x = gpu_solve(c1, b, m0, "f32")
    finally:
        c1.ctx.set_sap_half_fields(False)
    assert st == 0 and info[0]["status"] == 0
    r = b - oracle.apply_D(c1.dims, c1.U, c1.C, m0, x, BC)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-10


def test_solve_mixed_vs_fp64_agree(c1):
    b = synth.gaussian_spinor(c1.dims, seed=7)
    _, _, x64 = gpu_solve(c1, b, -0.2, "f64")
    _, _, x32 = gpu_solve(c1, b, -0.2, "f32")
    assert rel(x32, x64) <= 1e-7


def test_solve_multi_rhs_equals_solo(c1):
    n = 4
    b = synth.gaussian_spinor(c1.dims, nrhs=n, seed=8)
    m0 = np.array([-0.2, -0.1, 0.0, 0.15])
    st, info, x = gpu_solve(c1, b, m0, "f32", nrhs=n)
    assert st == 0
    for r in range(n):
        res = b[r] - oracle.apply_D(c1.dims, c1.U, c1.C, m0[r], x[r], BC)
        assert np.linalg.norm(res) / np.linalg.norm(b[r]) <= 1e-10
        _, _, xs = gpu_solve(c1, b[r], m0[r], "f32")
        assert rel(x[r], xs) <= 1e-8


@pytest.mark.parametrize("sap_prec", ["f32", "f16"])
def test_solve_point_sources(c1, sap_prec):
    """The twelve spin-colour point sources, fused.  With the FP16 smoother
    the first basis vectors are concentrated on a few sites (the largest
    entry close to the 2-norm), the far end of the FP16 copy's range."""
    b = synth.point_sources(c1.dims)
    st, info, x = gpu_solve(c1, b, -0.2, sap_prec, nrhs=12)
    assert st == 0
    for r in range(12):
        res = b[r] - oracle.apply_D(c1.dims, c1.U, c1.C, -0.2, x[r], BC)
        assert np.linalg.norm(res) / np.linalg.norm(b[r]) <= 1e-10


def test_solve_error_paths(c1):
    from paper_1710_07041_amd import ddsap
    b = synth.gaussian_spinor(c1.dims, seed=1)
    bad = b.copy()
    bad[5, 0, 0] = np.inf
    st, info, _ = gpu_solve(c1, bad, -0.2, "f32")
    assert st == ddsap.DD_NAN
    st, info, _ = gpu_solve(c1, b, -0.2, "f32", max_restarts=1, m=2)
    assert st == ddsap.DD_NOT_CONVERGED and info[0]["status"] == ddsap.DD_NOT_CONVERGED
    assert info[0]["iterations"] == 2
    st, info, x = gpu_solve(c1, np.zeros_like(b), -0.2, "f32")
    assert st == 0 and np.max(np.abs(x)) == 0


def test_solve_warm_start(c1):
    from paper_1710_07041_amd import ddsap
    import torch
    b = synth.gaussian_spinor(c1.dims, seed=2)
    _, _, x = gpu_solve(c1, b, -0.2, "f32")
    bd, xd = to_dev(b), to_dev(x)
    st, info = c1.ctx.solve(-0.2, bd, xd, 1, ddsap.default_params())
    assert st == 0 and info[0]["iterations"] == 0


@pytest.mark.parametrize("n", [1, 2])
def test_solve_initial_guess_with_one_nonzero_entry(c1, n):
    """A solve that starts from zero takes r = b without applying the
    operator; an initial guess with a single nonzero entry (in one of the
    right-hand sides of a fused batch) must not be taken for zero: the
    result then differs from b's solution by that guess unless D x0 enters
    the first residual."""
    from paper_1710_07041_amd import ddsap
    b = synth.gaussian_spinor(c1.dims, nrhs=n, seed=12)
    x0 = np.zeros_like(b)
    x0[n - 1, 77, 2, 1] = 0.25 - 0.5j
    bd, xd = to_dev(b), to_dev(x0)
    m0 = np.full(n, -0.2)
    st, info = c1.ctx.solve(m0, bd, xd, n, ddsap.default_params())
    assert st == 0
    x = xd.cpu().numpy()
    for r in range(n):
        res = b[r] - oracle.apply_D(c1.dims, c1.U, c1.C, -0.2, x[r], BC)
        assert np.linalg.norm(res) / np.linalg.norm(b[r]) <= 1e-10, r


def test_fp16_range_fallback_to_fp32(c1):
    """The FP16 smoother's range safeguard: with every FP16 smoother output
    poisoned by an infinity (the host-side test hook), the FP16 path can
    never converge, so a converged solve shows that the engine dropped the
    broken column and continued with the FP32 smoother.  The oracle checks
    the result."""
    b = synth.gaussian_spinor(c1.dims, seed=0)
    m0 = -0.2
    c1.ctx.debug_poison_half_smoother(-1)
    try:
        st, info, x = gpu_solve(c1, b, m0, "f16")
    finally:
        c1.ctx.debug_poison_half_smoother(0)
    assert st == 0 and info[0]["status"] == 0, info
    r = b - oracle.apply_D(c1.dims, c1.U, c1.C, m0, x, BC)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-10
    # one poisoned call: the same fallback, then a normal FP32 finish
    c1.ctx.debug_poison_half_smoother(1)
    try:
        st1, info1, x1 = gpu_solve(c1, b, m0, "f16")
    finally:
        c1.ctx.debug_poison_half_smoother(0)
    assert st1 == 0
    assert np.linalg.norm(b - oracle.apply_D(c1.dims, c1.U, c1.C, m0, x1, BC)) / np.linalg.norm(b) <= 1e-10


def test_breakdown_on_singular_system():
    """A singular system whose right-hand side lies in the null space: the
    free field (unit links, csw irrelevant: the clover term vanishes) with
    periodic boundaries in all four directions and m0 = 0 has D u = m0 u = 0
    for every constant spinor u, and the constant b = e_(spin 0, colour 0)
    is orthogonal to the range of the normal operator D.  Unpreconditioned
    FGMRES finds D v_1 = 0 exactly (dyadic entries, exact arithmetic), the
    Krylov space closes on a singular projection and the solve reports
    DD_BREAKDOWN with x left at the initial guess.  With m0 = 1/2 the same b
    is an eigenvector: one step, x = 2 b."""
    import torch
    from paper_1710_07041_amd import ddsap
    dims = (8, 8, 8, 8)
    V = synth.volume(dims)
    ctx = ddsap.Context(dims, (1, 1, 1, 1))
    ctx.set_gauge(synth.unit_links(dims), 1.0)
    b = np.zeros((V, 4, 3), dtype=np.complex128)
    b[:, 0, 0] = 1.0
    bd = to_dev(b)[None]
    p = ddsap.default_params()
    p.ncy = 0
    p.sap_prec = ddsap.DD_F64
    xd = torch.zeros_like(bd)
    st, info = ctx.solve(0.0, bd, xd, 1, p, raise_on_fail=False)
    assert st == ddsap.DD_BREAKDOWN and info[0]["status"] == ddsap.DD_BREAKDOWN, info
    assert np.max(np.abs(to_host(xd))) == 0
    xd.zero_()
    st, info = ctx.solve(0.5, bd, xd, 1, p, raise_on_fail=False)
    assert st == ddsap.DD_OK and info[0]["iterations"] == 1, info
    assert np.allclose(to_host(xd)[0], 2 * b, rtol=0, atol=1e-14)
    ctx.close()
