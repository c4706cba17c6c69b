"""Pins of the oracle's Wilson-clover operator against mathematics it must obey.

None of these retypes the oracle's formulas: they check closed forms (free
field, uniform abelian flux), invariants (gamma5-hermiticity, gauge
covariance, clover symmetries) and an independent sparse-matrix assembly.
"""
import numpy as np
import pytest

import oracle
from dense_ref import (block_sites, clover_dense, component_index, dirac_sparse, gamma5, gammas)
from paper_1710_07041_amd import synth

BC = (1, 1, 1, -1)


def rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b))


def g5_apply(psi):
    out = psi.copy()
    out[..., 2:, :] *= -1
    return out


def test_gamma_basis_algebra():
    g = gammas()
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T)
        for nu in range(4):
            assert np.allclose(g[mu] @ g[nu] + g[nu] @ g[mu], 2 * (mu == nu) * np.eye(4))
    assert np.allclose(gamma5(), np.diag([1, 1, -1, -1]))


@pytest.mark.parametrize("dims", [(4, 6, 2, 8), (2, 2, 2, 2)])
@pytest.mark.parametrize("m0", [-0.2, 0.3])
def test_free_field_plane_waves(dims, m0):
    """Unit links: D e^{ip.x} u = [m0 + sum(1 - cos p) + i sum gamma_mu sin p_mu] e^{ip.x} u,
    p_mu = (2 pi n_mu + theta_mu)/L_mu with theta = pi in the antiperiodic direction.
    The clover term vanishes.  L = 2 directions check that both hops accumulate."""
    V = synth.volume(dims)
    U = synth.unit_links(dims)
    C = oracle.clover_field(dims, U, 1.0)
    assert np.max(np.abs(C)) == 0.0
    g = gammas()
    rng = np.random.default_rng(5)
    idx = np.arange(V)
    coords = [(idx // int(np.prod(dims[:m]))) % dims[m] for m in range(4)]
    for trial in range(4):
        n = [rng.integers(0, d) for d in dims]
        p = [(2 * np.pi * n[m] + (np.pi if BC[m] < 0 else 0.0)) / dims[m] for m in range(4)]
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        phase = np.exp(1j * sum(p[m] * coords[m] for m in range(4)))
        psi = phase[:, None, None] * u[None]
        out = oracle.apply_D(dims, U, C, m0, psi, BC)
        K = (m0 + sum(1 - np.cos(p[m]) for m in range(4))) * np.eye(4) + 1j * sum(g[m] * np.sin(p[m]) for m in range(4))
        expect = phase[:, None, None] * (K @ u)[None]
        assert rel(out, expect) < 1e-13


def test_free_field_spectrum_closed_form():
    """Spectrum of the free operator on 2^4 (antiperiodic t): m0 + sum(1-cos p) +- i sqrt(sum sin^2 p),
    each with multiplicity 6 per momentum."""
    dims, m0 = (2, 2, 2, 2), 0.1
    U = synth.unit_links(dims)
    C = oracle.clover_field(dims, U, 1.0)
    V = synth.volume(dims)
    N = 12 * V
    Dm = np.empty((N, N), dtype=np.complex128)
    for k in range(N):
        e = np.zeros(N, dtype=np.complex128)
        e[k] = 1
        Dm[:, k] = oracle.apply_D(dims, U, C, m0, e.reshape(V, 4, 3), BC).ravel()
    ev = np.linalg.eigvals(Dm)
    expect = []
    for n in np.ndindex(*dims):
        p = [(2 * np.pi * n[m] + (np.pi if BC[m] < 0 else 0.0)) / dims[m] for m in range(4)]
        a = m0 + sum(1 - np.cos(q) for q in p)
        b = np.sqrt(sum(np.sin(q) ** 2 for q in p))
        expect += [a + 1j * b] * 6 + [a - 1j * b] * 6
    expect = np.array(expect)
    key = lambda z: np.lexsort((np.round(z.imag, 9), np.round(z.real, 9)))
    assert np.max(np.abs(np.sort_complex(ev)[key(np.sort_complex(ev))] - np.sort_complex(expect)[key(np.sort_complex(expect))])) < 1e-12


def test_abelian_flux_clover_closed_form():
    """Uniform flux B in the (x,y) plane: C(x) = -(csw/2) sin B sigma_12 (x) diag(1,-1,0),
    sigma_12 = i gamma_x gamma_y; spectrum of (4+m0)+C: 4+m0 +- (csw/2) sin B (x4 each), 4+m0 (x4)."""
    dims, csw, m0 = (6, 4, 2, 2), 1.3, -0.1
    U, B = synth.abelian_flux_links(dims, k=1)
    C = oracle.clover_field(dims, U, csw)
    g = gammas()
    sigma12 = 1j * g[0] @ g[1]
    expect = -(csw / 2) * np.sin(B) * np.kron(sigma12, np.diag([1, -1, 0]))
    assert np.max(np.abs(C - expect[None])) < 1e-13
    ev = np.sort(np.linalg.eigvalsh(C[0] + (4 + m0) * np.eye(12)))
    h = (csw / 2) * np.sin(B)
    assert np.allclose(ev, np.sort([4 + m0 - h] * 4 + [4 + m0] * 4 + [4 + m0 + h] * 4), atol=1e-13)


@pytest.fixture(scope="module")
def rand_field():
    dims = (4, 4, 2, 6)
    U = synth.random_su3_links(dims, eps=0.6, seed=3)
    return dims, U


def test_links_are_su3(rand_field):
    dims, U = rand_field
    I3 = np.eye(3)
    assert np.max(np.abs(np.einsum("xmab,xmcb->xmac", U, U.conj()) - I3)) < 1e-13
    assert np.max(np.abs(np.linalg.det(U) - 1)) < 1e-13


def test_su3_third_row_is_conjugate_cross_product(rand_field):
    """The identity behind gauge compression: for U in SU(3) the third row is
    the complex conjugate of the cross product of the first two.  A general
    unitary matrix (determinant a phase) breaks it by that phase."""
    dims, U = rand_field
    row2 = np.conj(np.cross(U[..., 0, :], U[..., 1, :]))
    assert np.max(np.abs(row2 - U[..., 2, :])) < 1e-13
    W = U * np.exp(1j * 0.3 / 3)  # det W = exp(0.3 i)
    assert np.max(np.abs(np.conj(np.cross(W[..., 0, :], W[..., 1, :])) - W[..., 2, :])) > 0.1


def test_clover_symmetries(rand_field):
    """C(x) Hermitian, commutes with gamma5, and is traceless (spin trace of sigma vanishes)."""
    dims, U = rand_field
    C = oracle.clover_field(dims, U, 1.0)
    G5 = np.kron(gamma5(), np.eye(3))
    assert np.max(np.abs(C - np.conj(np.swapaxes(C, 1, 2)))) < 1e-14
    assert np.max(np.abs(C @ G5 - G5 @ C)) < 1e-14
    assert np.max(np.abs(np.trace(C, axis1=1, axis2=2))) < 1e-14
    assert np.max(np.abs(C)) > 0.05  # a random field has a nonzero clover


def test_clover_site_matches_field(rand_field):
    dims, U = rand_field
    C = oracle.clover_field(dims, U, 0.7)
    for s in (0, 17, synth.volume(dims) - 1):
        assert np.array_equal(oracle.clover_site(dims, U, 0.7, s), C[s])


def test_clover_matches_independent_assembly(rand_field):
    dims, U = rand_field
    C = oracle.clover_field(dims, U, 1.0)
    assert np.max(np.abs(C - clover_dense(dims, U, 1.0))) < 1e-14


def test_gamma5_hermiticity(rand_field):
    """<phi, D psi> = <g5 D g5 phi, psi>."""
    dims, U = rand_field
    C = oracle.clover_field(dims, U, 1.0)
    phi = synth.gaussian_spinor(dims, seed=1)
    psi = synth.gaussian_spinor(dims, seed=2)
    m0 = -0.3
    lhs = np.vdot(phi, oracle.apply_D(dims, U, C, m0, psi, BC))
    rhs = np.vdot(g5_apply(oracle.apply_D(dims, U, C, m0, g5_apply(phi), BC)), psi)
    assert abs(lhs - rhs) / abs(lhs) < 1e-13


def test_gauge_covariance(rand_field):
    """U^W_mu(x) = W(x) U_mu(x) W(x+mu)^+ : D[U^W](W psi) = W (D[U] psi) and C[U^W] = W C W^+."""
    dims, U = rand_field
    V = synth.volume(dims)
    W = synth.random_gauge_transform(dims, seed=11)
    idx = np.arange(V)
    Ug = np.empty_like(U)
    for mu in range(4):
        stride = int(np.prod(dims[:mu]))
        c = (idx // stride) % dims[mu]
        xp = idx + np.where(c == dims[mu] - 1, -(dims[mu] - 1) * stride, stride)
        Ug[:, mu] = W @ U[:, mu] @ np.conj(np.swapaxes(W[xp], 1, 2))
    csw, m0 = 1.0, -0.25
    C = oracle.clover_field(dims, U, csw)
    Cg = oracle.clover_field(dims, Ug, csw)
    W12 = np.einsum("st,xab->xsatb", np.eye(4), W).reshape(V, 12, 12)
    assert np.max(np.abs(Cg - W12 @ C @ np.conj(np.swapaxes(W12, 1, 2)))) < 1e-13
    psi = synth.gaussian_spinor(dims, seed=4)
    Wpsi = np.einsum("xab,xsb->xsa", W, psi)
    lhs = oracle.apply_D(dims, Ug, Cg, m0, Wpsi, BC)
    rhs = np.einsum("xab,xsb->xsa", W, oracle.apply_D(dims, U, C, m0, psi, BC))
    assert rel(lhs, rhs) < 1e-13


def test_wrong_transport_breaks_covariance(rand_field):
    """Sanity of the covariance pin itself: using U_mu(x) instead of U_mu(x-mu)^+ on the
    backward hop (a plausible indexing mistake) is not covariant."""
    dims, U = rand_field
    V = synth.volume(dims)
    W = synth.random_gauge_transform(dims, seed=11)
    g = gammas()
    from dense_ref import neighbours
    fwd, bwd, wf, wb = neighbours(dims)

    def bad_D(Ux, psi):
        out = 4.0 * psi
        for mu in range(4):
            out = out - 0.5 * np.einsum("st,xab,xtb->xsa", np.eye(4) - g[mu], Ux[:, mu], psi[fwd[mu]])
            out = out - 0.5 * np.einsum("st,xab,xtb->xsa", np.eye(4) + g[mu], Ux[:, mu], psi[bwd[mu]])
        return out

    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[:, mu] = W @ U[:, mu] @ np.conj(np.swapaxes(W[fwd[mu]], 1, 2))
    psi = synth.gaussian_spinor(dims, seed=4)
    Wpsi = np.einsum("xab,xsb->xsa", W, psi)
    assert rel(bad_D(Ug, Wpsi), np.einsum("xab,xsb->xsa", W, bad_D(U, psi))) > 1e-2


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 2, 2, 4)])
def test_dense_assembly_matches(dims):
    """The oracle applied to every unit vector equals the independent sparse assembly."""
    V = synth.volume(dims)
    U = synth.random_su3_links(dims, eps=0.5, seed=7)
    C = oracle.clover_field(dims, U, 1.0)
    m0 = -0.2
    M = dirac_sparse(dims, U, C, m0, BC).toarray()
    N = 12 * V
    E = np.eye(N, dtype=np.complex128)
    cols = np.stack([oracle.apply_D(dims, U, C, m0, E[:, k].reshape(V, 4, 3), BC).ravel() for k in range(N)], axis=1)
    assert np.max(np.abs(cols - M)) < 1e-14
    # gamma5-hermiticity at the matrix level: the spectrum is closed under conjugation
    ev = np.linalg.eigvals(M)
    d = np.abs(ev[:, None] - np.conj(ev)[None, :]).min(axis=1)
    assert d.max() < 1e-10


def test_apply_D_sites_matches_field(rand_field):
    dims, U = rand_field
    C = oracle.clover_field(dims, U, 1.0)
    psi = synth.gaussian_spinor(dims, seed=9)
    full = oracle.apply_D(dims, U, C, 0.1, psi, BC)
    sites = np.array([0, 5, 31, synth.volume(dims) - 1])
    part = oracle.apply_D_sites(dims, U, 1.0, 0.1, psi, sites, BC)
    assert np.array_equal(part, full[sites])


def test_apply_D_sites_multi_and_chunked_residual(rand_field):
    """Several vectors at once equal the whole-lattice operator on each
    (bitwise); the chunked residual equals ||b - D x|| / ||b|| formed from the
    whole-lattice operator, and tells a perturbed solution apart."""
    dims, U = rand_field
    C = oracle.clover_field(dims, U, 1.0)
    V = synth.volume(dims)
    xs = synth.gaussian_spinor(dims, nrhs=3, seed=11)
    sites = np.array([0, 7, 33, V // 2, V - 1])
    part = oracle.apply_D_sites_multi(dims, U, 1.0, -0.2, xs, sites, BC)
    for k in range(3):
        assert np.array_equal(part[k], oracle.apply_D(dims, U, C, -0.2, xs[k], BC)[sites])
    b = synth.gaussian_spinor(dims, seed=12)
    res = oracle.rel_residuals(dims, U, 1.0, -0.2, b, xs, BC, chunk=V // 3 + 1)
    for k in range(3):
        ref = np.linalg.norm(b - oracle.apply_D(dims, U, C, -0.2, xs[k], BC)) / np.linalg.norm(b)
        assert abs(res[k] - ref) <= 1e-14 * ref
    # D x = b exactly for x = D^-1 b would give 0; a solution that is exact up
    # to one site's perturbation gives that site's hop-weighted error
    x = xs[0].copy()
    bx = oracle.apply_D(dims, U, C, -0.2, x, BC)
    x[5, 1, 2] += 1e-6
    r = oracle.rel_residuals(dims, U, 1.0, -0.2, bx, x[None], BC, chunk=V // 2)[0]
    assert 1e-8 < r * np.linalg.norm(bx) < 1e-5


def test_DBB_is_restriction():
    """For psi supported on B: (D psi)_B = D_BB psi_B; off the block D_BB is zero."""
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    U = synth.random_su3_links(dims, eps=0.5, seed=1)
    C = oracle.clover_field(dims, U, 1.0)
    psi = synth.gaussian_spinor(dims, seed=3)
    for bid in (0, 5, 15):
        sites, _ = block_sites(dims, block, bid)
        masked = np.zeros_like(psi)
        masked[sites] = psi[sites]
        full = oracle.apply_D(dims, U, C, -0.1, masked, BC)
        blk = oracle.apply_DBB(dims, block, U, C, -0.1, bid, psi, BC)
        assert rel(blk[sites], full[sites]) < 1e-15
        off = np.ones(synth.volume(dims), bool)
        off[sites] = False
        assert np.max(np.abs(blk[off])) == 0


def test_DBB_whole_lattice_equals_D():
    """One block spanning the lattice keeps the wrap hops (with their boundary sign): D_BB = D."""
    dims = (4, 4, 2, 4)
    U = synth.random_su3_links(dims, eps=0.5, seed=2)
    C = oracle.clover_field(dims, U, 1.0)
    psi = synth.gaussian_spinor(dims, seed=3)
    a = oracle.apply_DBB(dims, dims, U, C, 0.05, 0, psi, BC)
    b = oracle.apply_D(dims, U, C, 0.05, psi, BC)
    assert rel(a, b) < 1e-15


def test_DBB_gamma5_hermitian_and_dense():
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    U = synth.random_su3_links(dims, eps=0.5, seed=1)
    C = oracle.clover_field(dims, U, 1.0)
    M = dirac_sparse(dims, U, C, -0.1, BC)
    sites, _ = block_sites(dims, block, 6)
    ci = component_index(sites)
    Mbb = M[ci][:, ci].toarray()
    phi = synth.gaussian_spinor(dims, seed=5)
    out = oracle.apply_DBB(dims, block, U, C, -0.1, 6, phi, BC)
    assert rel(out[sites].ravel(), Mbb @ phi[sites].ravel()) < 1e-14
    psi = synth.gaussian_spinor(dims, seed=6)
    lhs = np.vdot(phi[sites], oracle.apply_DBB(dims, block, U, C, -0.1, 6, psi, BC)[sites])
    rhs = np.vdot(g5_apply(oracle.apply_DBB(dims, block, U, C, -0.1, 6, g5_apply(phi), BC))[sites], psi[sites])
    assert abs(lhs - rhs) / abs(lhs) < 1e-13


def test_invalid_blocking_rejected():
    dims = (6, 4, 4, 4)
    U = synth.unit_links(dims)
    C = np.zeros((synth.volume(dims), 12, 12), complex)
    psi = np.zeros((synth.volume(dims), 4, 3), complex)
    with pytest.raises(ValueError):
        oracle.apply_DBB(dims, (2, 2, 2, 2), U, C, 0.0, 0, psi)  # 3 blocks in x: odd
    with pytest.raises(ValueError):
        oracle.apply_DBB(dims, (4, 2, 2, 2), U, C, 0.0, 0, psi)  # 4 does not divide 6
