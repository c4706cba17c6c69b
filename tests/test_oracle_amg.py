"""Pins of the oracle's two-level coarse correction (oracle/amg.py) against
things other than itself: an independently assembled dense operator
(dense_ref), the algebra the construction must satisfy (orthonormal and
chirality-preserving interpolation, Galerkin orthogonality, gamma_5
symmetry and locality of the coarse operator), closed-form limits (a
full-rank interpolation makes the coarse correction an exact solve; with
exact block solves the two-grid error propagator factorises into the
smoother's and the coarse correction's) and library routines (a complete
GMRES equals numpy.linalg.solve)."""
import numpy as np
import pytest

import oracle
from oracle import amg
from dense_ref import block_sites, component_index, dirac_sparse
from paper_1710_07041_amd import synth

BC = (1, 1, 1, -1)


def rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b))


def dense_P(dims, block, P):
    """The interpolation as an explicit (12 V, nc) matrix, column by column."""
    nc = int(np.prod(P.shape[:3]))
    cols = []
    for k in range(nc):
        e = np.zeros(nc, complex)
        e[k] = 1.0
        cols.append(amg.prolong(dims, block, P, e).ravel())
    return np.stack(cols, axis=1)


@pytest.fixture(scope="module")
def small():
    """4^4 lattice, 2^4 blocks (16 aggregates pairs), N = 3 random test vectors."""
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    U = synth.random_su3_links(dims, eps=0.4, seed=0)
    C = oracle.clover_field(dims, U, 1.0)
    vs = synth.gaussian_spinor(dims, nrhs=3, seed=40)
    P = amg.interpolation(dims, block, vs)
    return dims, block, U, C, vs, P


def test_interpolation_orthonormal_chiral_and_spans_the_test_vectors(small):
    dims, block, U, C, vs, P = small
    Pd = dense_P(dims, block, P)
    assert np.abs(Pd.conj().T @ Pd - np.eye(Pd.shape[1])).max() < 1e-14
    # every test vector lies in the range of P (P P^+ is the projector onto it)
    for v in vs:
        assert rel(Pd @ (Pd.conj().T @ v.ravel()), v.ravel()) < 1e-13
    # gamma_5 P = P Gamma_5: a coarse vector on chiral half 0 prolongs to spins 0-1 only
    xc = np.zeros(P.shape[:3], complex)
    xc[:, 0] = np.random.default_rng(1).standard_normal(xc[:, 0].shape)
    f = amg.prolong(dims, block, P, xc)
    assert np.abs(f[:, 2:]).max() == 0 and np.abs(f[:, :2]).max() > 0
    # restriction is the adjoint of prolongation
    eta = synth.gaussian_spinor(dims, seed=41)
    assert rel(amg.restrict(dims, block, P, eta).ravel(), Pd.conj().T @ eta.ravel()) < 1e-14


def test_interpolation_is_gram_schmidt_of_the_pieces(small):
    """On one aggregate, P's columns are the QR factor of the restricted test
    vectors with positive real diagonal (the Gram-Schmidt convention)."""
    dims, block, U, C, vs, P = small
    sites, _ = block_sites(dims, block, 5)
    A = np.stack([v[sites][:, 2:4, :].reshape(-1) for v in vs], axis=1)  # chiral half 1 of block 5
    Q, R = np.linalg.qr(A)
    ph = np.diag(R) / np.abs(np.diag(R))
    Q = Q * ph[None, :]
    got = np.stack([P[5, 1, i].reshape(len(sites), 2, 3).reshape(-1) for i in range(3)], axis=1)
    assert np.abs(got - Q).max() < 1e-13


def test_galerkin_operator_against_dense_assembly(small):
    """D_c = P^+ D P with D from the independent sparse assembly."""
    dims, block, U, C, vs, P = small
    Dc = amg.coarse_operator(dims, block, U, C, P, BC)
    M = dirac_sparse(dims, U, C, 0.0, BC).toarray()
    Pd = dense_P(dims, block, P)
    assert rel(Dc, Pd.conj().T @ M @ Pd) < 1e-13
    # the mass enters as m0 times the identity (P^+ P = 1)
    M1 = dirac_sparse(dims, U, C, 0.3, BC).toarray()
    assert rel(Dc + 0.3 * np.eye(Dc.shape[0]), Pd.conj().T @ M1 @ Pd) < 1e-13


def test_coarse_operator_gamma5_symmetry_and_locality():
    """Gamma_5 D_c Gamma_5 = D_c^+ (D is gamma_5-hermitian and P keeps
    chirality), and D_c couples only aggregates of the same or neighbouring
    blocks (8^4 with 2^4 blocks: four blocks per direction)."""
    dims, block = (8, 8, 8, 8), (2, 2, 2, 2)
    U = synth.random_su3_links(dims, eps=0.4, seed=3)
    C = oracle.clover_field(dims, U, 1.0)
    N = 2
    P = amg.interpolation(dims, block, synth.gaussian_spinor(dims, nrhs=N, seed=42))
    Dc = amg.coarse_operator(dims, block, U, C, P, BC)
    nblk = P.shape[0]
    g5 = np.tile(np.repeat([1.0, -1.0], N), nblk)
    assert np.abs(g5[:, None] * Dc * g5[None, :] - Dc.conj().T).max() < 1e-13
    nb = [dims[m] // block[m] for m in range(4)]

    def coords(b):
        c = []
        for m in range(4):
            c.append(b % nb[m])
            b //= nb[m]
        return c

    for b in range(nblk):
        for b2 in range(nblk):
            d = [min((coords(b)[m] - coords(b2)[m]) % nb[m], (coords(b2)[m] - coords(b)[m]) % nb[m]) for m in range(4)]
            blk = Dc[b * 2 * N:(b + 1) * 2 * N, b2 * 2 * N:(b2 + 1) * 2 * N]
            if sum(d) > 1:
                assert np.abs(blk).max() == 0
            elif sum(d) == 1:
                assert np.abs(blk).max() > 0


def test_coarse_gmres_minimal_residual():
    """All steps: the exact solve (numpy.linalg.solve); fewer: the residual is
    orthogonal to A K_k (the minimal-residual condition) and falls with k."""
    rng = np.random.default_rng(5)
    n = 40
    A = 3 * np.eye(n) + 0.3 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x = amg.coarse_gmres(A, 0.5, b, n)
    assert rel(x, np.linalg.solve(A + 0.5 * np.eye(n), b)) < 1e-12
    prev = np.inf
    for k in (2, 5, 10):
        xk = amg.coarse_gmres(A, 0.5, b, k)
        r = b - (A + 0.5 * np.eye(n)) @ xk
        K = np.stack([np.linalg.matrix_power(A + 0.5 * np.eye(n), j) @ b for j in range(k)], axis=1)
        assert np.abs(((A + 0.5 * np.eye(n)) @ K).conj().T @ r).max() < 1e-10 * np.linalg.norm(b) * np.abs(K).max()
        assert np.linalg.norm(r) < prev
        prev = np.linalg.norm(r)


def test_exact_coarse_correction_is_galerkin_orthogonal(small):
    """With the coarse system solved exactly, the fine residual after the
    coarse correction has no component in the range of P."""
    dims, block, U, C, vs, P = small
    Dc = amg.coarse_operator(dims, block, U, C, P, BC)
    m0 = 0.1
    tl = amg.TwoLevel(dims, block, U, C, P, Dc, m0, k=Dc.shape[0], nu=0, nmr=4, bc=BC)
    eta = synth.gaussian_spinor(dims, seed=43)
    psi0 = tl.coarse_correction(eta)
    r = eta - oracle.apply_D(dims, U, C, m0, psi0, BC)
    assert np.abs(amg.restrict(dims, block, P, r)).max() < 1e-12 * np.linalg.norm(eta)


def test_full_rank_interpolation_solves_exactly():
    """2^4 lattice as one 2^4 block: with 96 independent test vectors each
    chiral aggregate (16 sites x 6 components) is spanned, P is unitary and
    the two-grid preconditioner returns D^-1 eta (post-smoothing then meets a
    zero residual)."""
    dims, block = (2, 2, 2, 2), (2, 2, 2, 2)
    U = synth.random_su3_links(dims, eps=0.4, seed=7)
    C = oracle.clover_field(dims, U, 1.0)
    P = amg.interpolation(dims, block, synth.gaussian_spinor(dims, nrhs=96, seed=44))
    Dc = amg.coarse_operator(dims, block, U, C, P, BC)
    m0 = -0.1
    tl = amg.TwoLevel(dims, block, U, C, P, Dc, m0, k=Dc.shape[0], nu=2, nmr=4, bc=BC)
    eta = synth.gaussian_spinor(dims, seed=45)
    M = dirac_sparse(dims, U, C, m0, BC).toarray()
    assert rel(tl(eta).ravel(), np.linalg.solve(M, eta.ravel())) < 1e-11


def test_two_grid_error_propagator_factorises():
    """With exact block solves (many MR steps) SAP is linear, M_nu =
    (I - E^nu) D^-1 with E = (I - K1 D)(I - K0 D), and the two-grid
    preconditioner B = P D_c^-1 P^+ + M_nu (I - D P D_c^-1 P^+) satisfies
    I - B D = (I - M_nu D)(I - P D_c^-1 P^+ D)."""
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    U = synth.random_su3_links(dims, eps=0.4, seed=0)
    C = oracle.clover_field(dims, U, 1.0)
    m0 = 0.1
    P = amg.interpolation(dims, block, synth.gaussian_spinor(dims, nrhs=4, seed=46))
    Dc = amg.coarse_operator(dims, block, U, C, P, BC)
    nu = 2
    tl = amg.TwoLevel(dims, block, U, C, P, Dc, m0, k=Dc.shape[0], nu=nu, nmr=60, bc=BC)
    M = dirac_sparse(dims, U, C, m0, BC).toarray()
    N = M.shape[0]
    I = np.eye(N)
    K = [np.zeros((N, N), complex), np.zeros((N, N), complex)]
    for bid in range(16):
        sites, col = block_sites(dims, block, bid)
        ci = component_index(sites)
        K[col][np.ix_(ci, ci)] = np.linalg.inv(M[np.ix_(ci, ci)])
    E = (I - K[1] @ M) @ (I - K[0] @ M)
    Pd = dense_P(dims, block, P)
    Cc = Pd @ np.linalg.solve(Dc + m0 * np.eye(Dc.shape[0]), Pd.conj().T)
    Ms = (I - np.linalg.matrix_power(E, nu)) @ np.linalg.inv(M)
    B = Cc + Ms @ (I - M @ Cc)
    eta = synth.gaussian_spinor(dims, seed=47)
    assert rel(tl(eta).ravel(), B @ eta.ravel()) < 1e-10
    assert np.abs((I - B @ M) - (I - Ms @ M) @ (I - Cc @ M)).max() < 1e-10


def test_setup_inverse_iteration_lowers_the_rayleigh_quotient():
    """Inverse iteration with the smoother amplifies the low modes of D: after
    the setup every test vector has a smaller |D v|/|v| than it started with,
    and the adaptive round lowers it further on average."""
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    U = synth.random_su3_links(dims, eps=0.3, seed=0)
    C = oracle.clover_field(dims, U, 1.0)
    m0 = -0.2
    v0 = synth.gaussian_spinor(dims, nrhs=4, seed=48)
    q = lambda v: np.linalg.norm(oracle.apply_D(dims, U, C, m0, v, BC)) / np.linalg.norm(v)
    vs, P, Dc = amg.setup(dims, block, U, C, m0, v0, n_inv=2, ncy=4, nmr=4, n_adapt=0)
    for a, b in zip(v0, vs):
        assert q(b) < 0.5 * q(a)
    vs2, _, _ = amg.setup(dims, block, U, C, m0, v0, n_inv=2, ncy=4, nmr=4, n_adapt=1, k=8, nu=2)
    assert np.mean([q(v) for v in vs2]) < np.mean([q(v) for v in vs])


def test_two_level_fgmres_solves_the_8x4_workload():
    """FGMRES(20) with the two-grid preconditioner reaches 1e-10 on the 8^4
    workload (eps 0.3, m0 = -0.2), checked with the plain operator."""
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    U = synth.random_su3_links(dims, eps=0.3, seed=0)
    C = oracle.clover_field(dims, U, 1.0)
    m0 = -0.2
    _, P, Dc = amg.setup(dims, block, U, C, m0, synth.gaussian_spinor(dims, nrhs=4, seed=49), n_inv=2)
    tl = amg.TwoLevel(dims, block, U, C, P, Dc, m0, k=16, nu=2, nmr=4, bc=BC)
    b = synth.gaussian_spinor(dims, seed=0)
    x, info = oracle.fgmres(dims, block, U, C, m0, b, m=20, tol=1e-10, precond=tl)
    assert info["status"] == 0
    assert np.linalg.norm(b - oracle.apply_D(dims, U, C, m0, x, BC)) / np.linalg.norm(b) <= 1e-10
