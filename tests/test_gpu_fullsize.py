"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times: operator outputs on sampled sites computed one by one by the oracle
(clover formed on the fly), and the solve's true residual evaluated with the
oracle's own FP64 operator over the whole lattice."""
import numpy as np
import pytest

import oracle
from gpu_util import BC, REL_TOL_APPLY, to_dev, to_host
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


def test_c3_operator_sampled():
    """48^3x96, eps = 0.6: operator in FP16 storage and FP64 on sampled sites."""
    f = Field((48, 48, 48, 96), 0.6, 0)
    psi = synth.gaussian_spinor(f.dims, seed=7)
    sites = sample_sites(f.dims, 800, seed=2)
    ref = oracle.apply_D_sites(f.dims, f.U, 1.0, -0.38, psi, sites, BC)
    for prec in ("f16", "f64"):
        out = f.apply(psi, -0.38, prec)
        err = np.linalg.norm(out[sites] - ref) / np.linalg.norm(ref)
        assert err <= REL_TOL_APPLY[prec], prec
    f.ctx.close()
