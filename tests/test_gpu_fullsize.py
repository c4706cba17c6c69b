"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times: operator outputs on sampled sites computed one by one by the oracle
(clover formed on the fly), the Schwarz smoother at its production setting
against the oracle's SAP element by element, and the solves' true residuals
evaluated with the oracle's own FP64 operator over the whole lattice."""
import numpy as np
import pytest

import oracle
from gpu_util import BC, REL_TOL_APPLY, check_sap, gpu_sap, rel, round_fp16, to_dev, to_host
from paper_1710_07041_amd import synth

pytestmark = pytest.mark.gpu


def sample_sites(dims, n, seed):
    """Random sites plus every lattice corner (all boundary wraps) and a set of
    sites on Schwarz-block faces."""
    V = synth.volume(dims)
    rng = np.random.default_rng(seed)
    sites = set(int(s) for s in rng.integers(0, V, size=n))
    for corner in np.ndindex(2, 2, 2, 2):
        c = [0 if k == 0 else dims[m] - 1 for m, k in enumerate(corner)]
        sites.add(c[0] + dims[0] * (c[1] + dims[1] * (c[2] + dims[2] * c[3])))
    for _ in range(64):
        c = [int(rng.integers(0, d)) for d in dims]
        m = int(rng.integers(0, 4))
        c[m] = 4 * int(rng.integers(0, dims[m] // 4)) + int(rng.choice([0, 3]))
        sites.add(c[0] + dims[0] * (c[1] + dims[1] * (c[2] + dims[2] * c[3])))
    return np.array(sorted(sites), dtype=np.int64)


class Field:
    def __init__(self, dims, eps, seed):
        from paper_1710_07041_amd import ddsap
        self.dims, self.V = dims, synth.volume(dims)
        self.U = synth.random_su3_links(dims, eps, seed=seed)
        self.ctx = ddsap.Context(dims, BC)
        self.ctx.set_gauge(self.U, 1.0)

    def apply(self, psi, m0, prec):
        import torch
        x = to_dev(psi)
        xb, yb = self.ctx.empty_blocked(prec), self.ctx.empty_blocked(prec)
        self.ctx.pack(x, xb, prec)
        self.ctx.apply_D(m0, xb, yb, prec)
        y = torch.empty_like(x)
        self.ctx.unpack(yb, y, prec)
        self.ctx.synchronize()
        return to_host(y)


@pytest.fixture(scope="module")
def c2():
    """32^3x64, eps = 0.5, csw = 1, seed 0 -- the benchmark workload."""
    return Field((32, 32, 32, 64), 0.5, 0)


@pytest.fixture(scope="module")
def c2_clover(c2):
    return oracle.clover_field(c2.dims, c2.U, 1.0)


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_c2_operator_sampled(c2, prec):
    psi = synth.gaussian_spinor(c2.dims, seed=5)
    m0 = -0.35
    out = c2.apply(psi, m0, prec)
    sites = sample_sites(c2.dims, 1500, seed=1)
    ref = oracle.apply_D_sites(c2.dims, c2.U, 1.0, m0, psi, sites, BC)
    err = np.linalg.norm(out[sites] - ref) / np.linalg.norm(ref)
    assert err <= REL_TOL_APPLY[prec]


def test_c2_mixed_solve_oracle_residual(c2, c2_clover):
    """The benchmark's step: FP32 SAP, FGMRES(20) FP64, tol 1e-10; the residual
    is recomputed with the oracle operator on the whole 32^3x64 lattice."""
    import torch
    from paper_1710_07041_amd import ddsap
    b = synth.gaussian_spinor(c2.dims, seed=0)
    bd = to_dev(b)[None]
    xd = torch.zeros_like(bd)
    st, info = c2.ctx.solve(-0.35, bd, xd, 1, ddsap.default_params())
    assert st == ddsap.DD_OK
    x = to_host(xd)[0]
    r = b - oracle.apply_D(c2.dims, c2.U, c2_clover, -0.35, x, BC)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-10


def test_c2_mixed_solve_eo_oracle_residual(c2, c2_clover):
    """The same solve with the even-odd preconditioned smoother (dd_sap_eo)."""
    import torch
    from paper_1710_07041_amd import ddsap
    b = synth.gaussian_spinor(c2.dims, seed=0)
    bd = to_dev(b)[None]
    xd = torch.zeros_like(bd)
    p = ddsap.default_params()
    p.sap_eo = 1
    st, info = c2.ctx.solve(-0.35, bd, xd, 1, p)
    assert st == ddsap.DD_OK
    x = to_host(xd)[0]
    r = b - oracle.apply_D(c2.dims, c2.U, c2_clover, -0.35, x, BC)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-10


def test_c2_mixed_solve_half_fields_oracle_residual(c2, c2_clover):
    """The same solve with FP16 links and clover under the FP32 smoother."""
    import torch
    from paper_1710_07041_amd import ddsap
    b = synth.gaussian_spinor(c2.dims, seed=0)
    bd = to_dev(b)[None]
    xd = torch.zeros_like(bd)
    c2.ctx.set_sap_half_fields(True)
    try:
        st, info = c2.ctx.solve(-0.35, bd, xd, 1, ddsap.default_params())
    finally:
        c2.ctx.set_sap_half_fields(False)
    assert st == ddsap.DD_OK
    x = to_host(xd)[0]
    r = b - oracle.apply_D(c2.dims, c2.U, c2_clover, -0.35, x, BC)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-10


def test_c4_point_sources_oracle_residual(c2, c2_clover):
    """Twelve spin-colour point sources solved fused; each residual <= 1e-10 by the oracle."""
    import torch
    from paper_1710_07041_amd import ddsap
    b = synth.point_sources(c2.dims)
    bd = to_dev(b)
    xd = torch.zeros_like(bd)
    st, info = c2.ctx.solve(np.full(12, -0.35), bd, xd, 12, ddsap.default_params())
    assert st == ddsap.DD_OK
    x = to_host(xd)
    for r in range(12):
        res = b[r] - oracle.apply_D(c2.dims, c2.U, c2_clover, -0.35, x[r], BC)
        assert np.linalg.norm(res) / np.linalg.norm(b[r]) <= 1e-10


@pytest.fixture(scope="module")
def c2_sap_refs(c2, c2_clover):
    """The oracle's SAP at the production setting (ncy = 12, nmr = 4, 4^4
    blocks, m0 = -0.35) on the exact fields and on the FP16-rounded ones."""
    eta = synth.gaussian_spinor(c2.dims, seed=31)
    ref = oracle.sap(c2.dims, (4, 4, 4, 4), c2.U, c2_clover, -0.35, eta, 12, 4, BC)
    ref16 = oracle.sap(c2.dims, (4, 4, 4, 4), round_fp16(c2.U), round_fp16(c2_clover), -0.35, eta, 12, 4, BC)
    return eta, ref, ref16


@pytest.mark.timeout(900)
@pytest.mark.parametrize("mode", ["f32", "f16", "f32h"])
def test_c2_sap_parity_production(c2, c2_sap_refs, mode):
    """The smoother exactly as the 32^3x64 solve runs it (twelve cycles of four
    MR steps, gauge compression on), against the oracle element by element.
    f32h: FP16 links and clover under the FP32 smoother -- with compression
    against the exact fields' SAP, and with all nine link entries read against
    the SAP of the FP16-rounded fields."""
    eta, ref, ref16 = c2_sap_refs
    prec = "f16" if mode == "f16" else "f32"
    try:
        c2.ctx.set_sap_half_fields(mode == "f32h")
        out = gpu_sap(c2.ctx, eta, -0.35, 12, 4, prec)
        check_sap(out, ref, mode, "32^3x64 ncy=12")
        if mode == "f32h":
            c2.ctx.set_link_compression(False)
            out = gpu_sap(c2.ctx, eta, -0.35, 12, 4, prec)
            check_sap(out, ref16, "f32h-rounded", "32^3x64 ncy=12")
    finally:
        c2.ctx.set_sap_half_fields(False)
        c2.ctx.set_link_compression(True)


@pytest.fixture(scope="module")
def c3():
    """48^3x96, eps = 0.6, csw = 1, seed 0 -- the largest workload."""
    f = Field((48, 48, 48, 96), 0.6, 0)
    yield f
    f.ctx.close()


def test_c3_operator_sampled(c3):
    """48^3x96, eps = 0.6: operator in FP16 storage and FP64 on sampled sites."""
    psi = synth.gaussian_spinor(c3.dims, seed=7)
    sites = sample_sites(c3.dims, 800, seed=2)
    ref = oracle.apply_D_sites(c3.dims, c3.U, 1.0, -0.38, psi, sites, BC)
    for prec in ("f16", "f64"):
        out = c3.apply(psi, -0.38, prec)
        err = np.linalg.norm(out[sites] - ref) / np.linalg.norm(ref)
        assert err <= REL_TOL_APPLY[prec], prec


@pytest.mark.timeout(1200)
def test_c3_solves_oracle_residual(c3):
    """The 48^3x96 workload as the benchmark times it: FP16-storage SAP (FP32
    arithmetic, ten cycles) inside FP64 FGMRES(20), and the FP64 GPU path
    beside it; both
    solutions' true residuals are recomputed by the oracle over all
    10,616,832 sites (clover formed site by site, in chunks) and must be
    <= 1e-10."""
    import torch
    from paper_1710_07041_amd import ddsap
    b = synth.gaussian_spinor(c3.dims, seed=0)
    bd = to_dev(b)[None]
    xs = []
    for sap in ("f16", "f64"):
        xd = torch.zeros_like(bd)
        p = ddsap.default_params()
        p.sap_prec = ddsap.PREC[sap]
        p.ncy = 10  # the benchmark's setting for this lattice
        st, info = c3.ctx.solve(-0.38, bd, xd, 1, p)
        assert st == ddsap.DD_OK and info[0]["rel_residual"] <= 1e-10, (sap, info)
        print(f"C3SOLVE {sap}: {info[0]['iterations']} iterations, GPU residual {info[0]['rel_residual']:.3e}",
              flush=True)
        xs.append(to_host(xd)[0])
        del xd
    del bd
    torch.cuda.empty_cache()
    res = oracle.rel_residuals(c3.dims, c3.U, 1.0, -0.38, b, np.stack(xs), BC)
    print(f"C3SOLVE oracle residuals f16={res[0]:.3e} f64={res[1]:.3e}", flush=True)
    assert np.all(res <= 1e-10), res
    # the two paths solve the same system: their solutions agree within the
    # conditioning times the tolerance
    assert rel(xs[0], xs[1]) <= 1e-7
