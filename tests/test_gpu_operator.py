"""GPU parity of the operator, the block operator and the layout transform, through
the C ABI, element by element against the FP64 oracle."""
import numpy as np
import pytest

import oracle
from gpu_util import BC, REL_TOL_APPLY, Lattice, rel, to_dev, to_host
from paper_1710_07041_amd import synth

pytestmark = pytest.mark.gpu

# lattices: one block spanning everything (every hop wraps inside the block),
# mixed one/two/four blocks per direction, a 12-block lattice whose block
# count is not a multiple of the eight XCDs (ragged workgroup remap), and
# four blocks in x, y and z (forward and backward neighbour blocks distinct)
SHAPES = [(4, 4, 4, 4), (8, 4, 16, 8), (4, 4, 8, 24), (8, 8, 8, 8), (16, 16, 16, 8)]


@pytest.fixture(scope="module", params=SHAPES, ids=lambda d: "x".join(map(str, d)))
def lat(request):
    return Lattice(request.param, eps=0.5, seed=1)


def test_pack_unpack_roundtrip_bitexact(lat):
    import torch
    for nrhs in (1, 3):
        psi = synth.gaussian_spinor(lat.dims, nrhs=nrhs, seed=2)
        x = to_dev(psi)
        b = lat.ctx.empty_blocked("f64", nrhs)
        lat.ctx.pack(x, b, "f64", nrhs)
        y = torch.zeros_like(x)
        lat.ctx.unpack(b, y, "f64", nrhs)
        lat.ctx.synchronize()
        assert np.array_equal(to_host(y), psi)


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_apply_D_single(lat, prec):
    psi = synth.gaussian_spinor(lat.dims, seed=3)
    m0 = -0.2
    ref = oracle.apply_D(lat.dims, lat.U, lat.C, m0, psi, BC)
    out = lat.apply(psi, m0, prec)
    assert rel(out, ref) <= REL_TOL_APPLY[prec]


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 8, 12])
@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_apply_D_multi_rhs_own_masses(lat, prec, n):
    """Full and partial lane groups of right-hand sides, each with its own mass."""
    psi = synth.gaussian_spinor(lat.dims, nrhs=n, seed=4)
    m0 = np.linspace(-0.38, 0.1, n)
    out = lat.apply(psi, m0, prec, nrhs=n)
    for r in range(n):
        ref = oracle.apply_D(lat.dims, lat.U, lat.C, m0[r], psi[r], BC)
        assert rel(out[r], ref) <= REL_TOL_APPLY[prec]


def test_apply_D_f64_batch_equals_single(lat):
    """A right-hand side gives the same result alone and inside a batch, to
    FP64 rounding: a single right-hand side runs the form that stages the
    block in LDS, a batch of four the form in which lanes share sites, and
    the two may round a fused multiply-add differently in the last bit."""
    n = 4
    psi = synth.gaussian_spinor(lat.dims, nrhs=n, seed=5)
    m0 = np.array([-0.3, -0.2, 0.0, 0.2])
    batch = lat.apply(psi, m0, "f64", nrhs=n)
    for r in range(n):
        assert rel(batch[r], lat.apply(psi[r], m0[r], "f64")) <= 1e-15


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_apply_D_block(lat, prec):
    import torch
    psi = synth.gaussian_spinor(lat.dims, seed=6)
    nblk = lat.V // 256
    x = to_dev(psi)
    xb = lat.ctx.empty_blocked(prec)
    yb = lat.ctx.empty_blocked(prec)
    lat.ctx.pack(x, xb, prec)
    sentinel = to_dev(np.full_like(psi, 7.0 + 3.0j))
    lat.ctx.pack(sentinel, yb, prec)
    blocks = sorted({0, nblk // 2, nblk - 1})
    m0 = -0.25
    for bid in blocks:
        lat.ctx.apply_D_block(m0, bid, xb, yb, prec)
    y = torch.empty_like(x)
    lat.ctx.unpack(yb, y, prec)
    lat.ctx.synchronize()
    y = to_host(y)
    from dense_ref import block_sites
    touched = np.zeros(lat.V, bool)
    for bid in blocks:
        ref = oracle.apply_DBB(lat.dims, (4, 4, 4, 4), lat.U, lat.C, m0, bid, psi, BC)
        sites, _ = block_sites(lat.dims, (4, 4, 4, 4), bid)
        touched[sites] = True
        assert rel(y[sites], ref[sites]) <= REL_TOL_APPLY[prec]
    assert np.all(y[~touched] == 7.0 + 3.0j)


def test_explicit_clover_roundtrip():
    """dd_set_clover with the oracle's clover (chiral halves) reproduces the operator."""
    dims = (8, 4, 4, 8)
    lat = Lattice(dims, eps=0.4, seed=9)
    C = lat.C
    halves = np.stack([C[:, 0:6, 0:6], C[:, 6:12, 6:12]], axis=1)
    assert np.max(np.abs(C[:, 0:6, 6:12])) < 1e-15
    psi = synth.gaussian_spinor(dims, seed=1)
    before = lat.apply(psi, 0.1, "f64")
    lat.ctx.set_clover(2.0 * halves)  # a different clover: D changes by the extra C
    after = lat.apply(psi, 0.1, "f64")
    ref = oracle.apply_D(dims, lat.U, 2.0 * C, 0.1, psi, BC)
    assert rel(after, ref) <= 1e-12
    assert rel(before, oracle.apply_D(dims, lat.U, C, 0.1, psi, BC)) <= 1e-12


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_link_compression_matches_full_links(lat, prec):
    """The synthetic links are SU(3), so the context reads two rows per link and
    rebuilds the third; the result equals the one with all nine entries read
    up to rounding, and both match the oracle."""
    assert lat.ctx.link_compression
    psi = synth.gaussian_spinor(lat.dims, seed=7)
    m0 = -0.25
    on = lat.apply(psi, m0, prec)
    lat.ctx.set_link_compression(False)
    try:
        assert not lat.ctx.link_compression
        off = lat.apply(psi, m0, prec)
    finally:
        lat.ctx.set_link_compression(True)
    tol = {"f64": 1e-13, "f32": 1e-6, "f16": 2e-3}[prec]
    assert rel(on, off) <= tol
    ref = oracle.apply_D(lat.dims, lat.U, lat.C, m0, psi, BC)
    assert rel(off, ref) <= REL_TOL_APPLY[prec]


def test_link_compression_needs_su3():
    """A field that is not SU(3) keeps all nine entries per link; asking for
    compression is an error, and the operator still matches the oracle."""
    from paper_1710_07041_amd import ddsap
    dims = (8, 4, 4, 8)
    U = synth.random_su3_links(dims, 0.4, seed=3)
    U[5, 2] *= 1.001  # one link off the group
    ctx = ddsap.Context(dims, BC)
    ctx.set_gauge(U, 1.0)
    assert not ctx.link_compression
    with pytest.raises(ddsap.DDError) as e:
        ctx.set_link_compression(True)
    assert e.value.status == ddsap.DD_INVALID_ARG
    import torch
    psi = synth.gaussian_spinor(dims, seed=8)
    x = to_dev(psi)
    xb = ctx.empty_blocked("f64")
    yb = ctx.empty_blocked("f64")
    ctx.pack(x, xb, "f64")
    ctx.apply_D(-0.2, xb, yb, "f64")
    y = torch.empty_like(x)
    ctx.unpack(yb, y, "f64")
    ctx.synchronize()
    C = oracle.clover_field(dims, U, 1.0)
    assert rel(to_host(y), oracle.apply_D(dims, U, C, -0.2, psi, BC)) <= REL_TOL_APPLY["f64"]


def test_free_field_plane_wave_gpu():
    """Unit links: the GPU operator reproduces the closed form directly."""
    from dense_ref import gammas
    dims = (8, 4, 4, 8)
    lat = Lattice(dims, eps=0.0, seed=0)
    V = lat.V
    idx = np.arange(V)
    coords = [(idx // int(np.prod(dims[:m]))) % dims[m] for m in range(4)]
    p = [2 * np.pi * 3 / 8, 2 * np.pi / 4, 0.0, (2 * np.pi * 5 + np.pi) / 8]
    u = np.arange(12).reshape(4, 3) * (0.1 + 0.3j) + 1.0
    psi = np.exp(1j * sum(p[m] * coords[m] for m in range(4)))[:, None, None] * u[None]
    m0 = -0.3
    g = gammas()
    K = (m0 + sum(1 - np.cos(q) for q in p)) * np.eye(4) + 1j * sum(g[m] * np.sin(p[m]) for m in range(4))
    expect = np.exp(1j * sum(p[m] * coords[m] for m in range(4)))[:, None, None] * (K @ u)[None]
    assert rel(lat.apply(psi, m0, "f64"), expect) <= 1e-13


def test_error_paths():
    from paper_1710_07041_amd import ddsap
    with pytest.raises(ddsap.DDError) as e:
        ddsap.Context((12, 4, 4, 4))  # three blocks in x: no red-black colouring
    assert e.value.status == ddsap.DD_INVALID_ARG
    with pytest.raises(ddsap.DDError) as e:
        ddsap.Context((6, 4, 4, 4))
    assert e.value.status == ddsap.DD_INVALID_ARG
    ctx = ddsap.Context((4, 4, 4, 8))
    xb = ctx.empty_blocked("f64")
    yb = ctx.empty_blocked("f64")
    with pytest.raises(ddsap.DDError) as e:
        ctx.apply_D(0.0, xb, yb, "f64")
    assert e.value.status == ddsap.DD_NO_FIELD
    U = synth.random_su3_links((4, 4, 4, 8), 0.3, seed=0)
    bad = U.copy()
    bad[3, 1, 0, 0] = np.nan
    with pytest.raises(ddsap.DDError) as e:
        ctx.set_gauge(bad, 1.0)
    assert e.value.status == ddsap.DD_NAN
    ctx.set_gauge(U, 1.0)
    with pytest.raises(ddsap.DDError) as e:
        ctx.apply_D_block(0.0, 2, xb, yb, "f64")  # only blocks 0, 1 exist
    assert e.value.status == ddsap.DD_INVALID_ARG
    with pytest.raises(ddsap.DDError) as e:
        ctx.apply_D(0.0, xb, xb, "f64")  # in place is not allowed
    assert e.value.status == ddsap.DD_INVALID_ARG
