"""Pins of the oracle's MR, SAP and FGMRES against textbook algorithms written
separately on explicit matrices, exact limits and special cases."""
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from dense_ref import block_sites, component_index, dirac_sparse, gammas
from paper_1710_07041_amd import synth

BC = (1, 1, 1, -1)


def rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b))


@pytest.fixture(scope="module")
def small():
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    U = synth.random_su3_links(dims, eps=0.4, seed=0)
    C = oracle.clover_field(dims, U, 1.0)
    m0 = 0.1
    M = dirac_sparse(dims, U, C, m0, BC).toarray()
    return dims, block, U, C, m0, M


def textbook_mr(A, b, steps):
    """Minimal residual iteration x_{k+1} = x_k + alpha r_k, alpha = (Ar, r)/(Ar, Ar)."""
    x = np.zeros_like(b)
    r = b.copy()
    norms = [np.linalg.norm(r)]
    for _ in range(steps):
        p = A @ r
        alpha = np.vdot(p, r) / np.vdot(p, p)
        x = x + alpha * r
        r = r - alpha * p
        norms.append(np.linalg.norm(r))
    return x, r, norms


def test_mr_matches_textbook(small):
    dims, block, U, C, m0, M = small
    rho = synth.gaussian_spinor(dims, seed=1)
    for bid in (0, 9):
        sites, _ = block_sites(dims, block, bid)
        ci = component_index(sites)
        Abb = M[np.ix_(ci, ci)]
        delta, r, steps = oracle.mr_block(dims, block, U, C, m0, bid, rho, 6, BC)
        assert steps == 6
        xt, rt, norms = textbook_mr(Abb, rho[sites].ravel(), 6)
        assert rel(delta[sites].ravel(), xt) < 1e-13
        assert rel(r[sites].ravel(), rt) < 1e-12
        assert all(b <= a * (1 + 1e-14) for a, b in zip(norms, norms[1:]))


def test_mr_zero_rhs_stops():
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    U = synth.unit_links(dims)
    C = oracle.clover_field(dims, U, 1.0)
    rho = np.zeros((synth.volume(dims), 4, 3), complex)
    delta, r, steps = oracle.mr_block(dims, block, U, C, 0.0, 3, rho, 4, BC)
    assert steps == 0 and np.max(np.abs(delta)) == 0


def test_mr_free_field_eigenvector_one_step():
    """A plane wave built on an eigenvector of sum gamma_mu sin p_mu is an eigenvector of D;
    one MR step then has alpha = 1/lambda and leaves a zero residual."""
    dims = (4, 4, 4, 4)
    U = synth.unit_links(dims)
    C = oracle.clover_field(dims, U, 1.0)
    m0 = 0.2
    V = synth.volume(dims)
    idx = np.arange(V)
    coords = [(idx // 4 ** m) % 4 for m in range(4)]
    p = [2 * np.pi / 4, 0.0, 2 * np.pi * 3 / 4, np.pi / 4]  # t antiperiodic: (2 pi 0 + pi)/4
    K = sum(gammas()[m] * np.sin(p[m]) for m in range(4))
    w, Wv = np.linalg.eigh(K)
    u = np.outer(Wv[:, -1], [1.0, 0.5j, -0.25])
    psi = np.exp(1j * sum(p[m] * coords[m] for m in range(4)))[:, None, None] * u[None]
    delta, r, steps = oracle.mr_block(dims, dims, U, C, m0, 0, psi, 1, BC)
    lam = m0 + sum(1 - np.cos(q) for q in p) + 1j * w[-1]
    assert np.linalg.norm(r) / np.linalg.norm(psi) < 1e-13
    assert rel(delta, psi / lam) < 1e-13


def sap_exact_cycle_matrices(dims, block, M):
    """K_c = sum_{B of colour c} I_B D_BB^-1 I_B^T (dense)."""
    N = M.shape[0]
    nblk = int(np.prod([dims[m] // block[m] for m in range(4)]))
    K = [np.zeros((N, N), complex), np.zeros((N, N), complex)]
    for bid in range(nblk):
        sites, col = block_sites(dims, block, bid)
        ci = component_index(sites)
        K[col][np.ix_(ci, ci)] = np.linalg.inv(M[np.ix_(ci, ci)])
    return K


def test_sap_exact_block_limit(small):
    """With exact block solves one SAP cycle is M1 = K0 + K1 - K1 D K0 and after k cycles
    psi_k = (I - E^k) D^-1 eta with E = (I - K1 D)(I - K0 D).  Many MR steps reach that limit."""
    dims, block, U, C, m0, M = small
    K0, K1 = sap_exact_cycle_matrices(dims, block, M)
    N = M.shape[0]
    I = np.eye(N)
    eta = synth.gaussian_spinor(dims, seed=2)
    e = eta.ravel()
    M1 = K0 + K1 - K1 @ M @ K0
    psi1 = oracle.sap(dims, block, U, C, m0, eta, 1, 60, BC)
    assert rel(psi1.ravel(), M1 @ e) < 1e-10
    E = (I - K1 @ M) @ (I - K0 @ M)
    psi3 = oracle.sap(dims, block, U, C, m0, eta, 3, 60, BC)
    expect = (I - np.linalg.matrix_power(E, 3)) @ np.linalg.solve(M, e)
    assert rel(psi3.ravel(), expect) < 1e-10


def test_sap_single_block_is_global_mr(small):
    """One block = the whole lattice: SAP(ncy=1) is nmr global MR steps (colour 1 is empty)."""
    dims, block, U, C, m0, M = small
    eta = synth.gaussian_spinor(dims, seed=3)
    psi = oracle.sap(dims, dims, U, C, m0, eta, 1, 5, BC)
    xt, _, _ = textbook_mr(M, eta.ravel(), 5)
    assert rel(psi.ravel(), xt) < 1e-13


def test_sap_homogeneous(small):
    dims, block, U, C, m0, M = small
    eta = synth.gaussian_spinor(dims, seed=4)
    s = 0.3 - 1.7j
    a = oracle.sap(dims, block, U, C, m0, s * eta, 2, 4, BC)
    b = oracle.sap(dims, block, U, C, m0, eta, 2, 4, BC)
    assert rel(a, s * b) < 1e-14


def test_sap_not_linear(small):
    """SAP-MR is not a linear map (alpha depends on the input): the outer solver must be flexible."""
    dims, block, U, C, m0, M = small
    a = synth.gaussian_spinor(dims, seed=5)
    b = synth.gaussian_spinor(dims, seed=6)
    sa = oracle.sap(dims, block, U, C, m0, a, 1, 2, BC)
    sb = oracle.sap(dims, block, U, C, m0, b, 1, 2, BC)
    sab = oracle.sap(dims, block, U, C, m0, a + b, 1, 2, BC)
    assert rel(sab, sa + sb) > 1e-6


_ORDER_SCRIPT = r"""
import sys, numpy as np
sys.path.insert(0, %r)
import oracle
from paper_1710_07041_amd import synth
dims, block = (8, 4, 4, 4), (2, 2, 2, 2)
U = synth.random_su3_links(dims, eps=0.4, seed=0)
C = oracle.clover_field(dims, U, 1.0)
eta = synth.gaussian_spinor(dims, seed=8)
psi = oracle.sap(dims, block, U, C, -0.1, eta, 2, 4)
sys.stdout.write(psi.tobytes().hex()[:0] + str(hash(psi.tobytes())))
"""


def test_sap_order_independent_bitwise():
    """Blocks of one colour are processed by a dynamic thread schedule; one thread and many
    threads (different block orders) must give bitwise identical results."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    outs = []
    for nt in ("1", "5"):
        env = dict(os.environ, OMP_NUM_THREADS=nt, PYTHONHASHSEED="0")
        r = subprocess.run([sys.executable, "-c", _ORDER_SCRIPT % root], env=env, capture_output=True, text=True,
                           check=True)
        outs.append(r.stdout.strip())
    assert outs[0] == outs[1]


def textbook_gmres(A, b, m, cycles):
    """Restarted GMRES(m) with Householder-free Arnoldi (MGS) and a least-squares solve."""
    x = np.zeros_like(b)
    for _ in range(cycles):
        r = b - A @ x
        beta = np.linalg.norm(r)
        Q = np.zeros((len(b), m + 1), complex)
        H = np.zeros((m + 1, m), complex)
        Q[:, 0] = r / beta
        k = m
        for j in range(m):
            w = A @ Q[:, j]
            for i in range(j + 1):
                H[i, j] = np.vdot(Q[:, i], w)
                w = w - H[i, j] * Q[:, i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] == 0:
                k = j + 1
                break
            Q[:, j + 1] = w / H[j + 1, j]
        e1 = np.zeros(k + 1, complex)
        e1[0] = beta
        y = np.linalg.lstsq(H[: k + 1, :k], e1, rcond=None)[0]
        x = x + Q[:, :k] @ y
    return x


def test_fgmres_identity_is_gmres(small):
    dims, block, U, C, m0, M = small
    b = synth.gaussian_spinor(dims, seed=7)
    x, info = oracle.fgmres(dims, block, U, C, m0, b, m=6, tol=1e-30, max_restarts=3, ncy=0, bc=BC)
    assert info["iterations"] == 18 and info["status"] == 1
    xt = textbook_gmres(M, b.ravel(), 6, 3)
    assert rel(x.ravel(), xt) < 1e-10


def test_fgmres_exact_preconditioner_one_step(small):
    dims, block, U, C, m0, M = small
    V = synth.volume(dims)
    Minv = np.linalg.inv(M)
    b = synth.gaussian_spinor(dims, seed=8)
    x, info = oracle.fgmres(dims, block, U, C, m0, b, m=10, tol=1e-10, ncy=0,
                            precond=lambda v: (Minv @ v.ravel()).reshape(V, 4, 3), bc=BC)
    assert info["status"] == 0 and info["iterations"] == 1 and info["rel_residual"] < 1e-10


def test_fgmres_happy_breakdown_free_field():
    dims = (4, 4, 4, 4)
    U = synth.unit_links(dims)
    C = oracle.clover_field(dims, U, 1.0)
    m0 = 0.2
    V = synth.volume(dims)
    idx = np.arange(V)
    coords = [(idx // 4 ** m) % 4 for m in range(4)]
    p = [0.0, 2 * np.pi / 4, 0.0, 3 * np.pi / 4]
    K = sum(gammas()[m] * np.sin(p[m]) for m in range(4))
    w, Wv = np.linalg.eigh(K)
    u = np.outer(Wv[:, 0], [0.3, 1.0, -1j])
    b = np.exp(1j * sum(p[m] * coords[m] for m in range(4)))[:, None, None] * u[None]
    lam = m0 + sum(1 - np.cos(q) for q in p) + 1j * w[0]
    x, info = oracle.fgmres(dims, dims, U, C, m0, b, m=10, tol=1e-12, ncy=0, bc=BC)
    assert info["iterations"] == 1 and info["status"] == 0
    assert rel(x, b / lam) < 1e-13


def test_fgmres_sap_solve_matches_dense(small):
    dims, block, U, C, m0, M = small
    b = synth.gaussian_spinor(dims, seed=9)
    x, info = oracle.fgmres(dims, block, U, C, m0, b, m=20, tol=1e-10, ncy=4, nmr=4, bc=BC)
    assert info["status"] == 0 and info["rel_residual"] <= 1e-10
    xs = np.linalg.solve(M, b.ravel())
    cond = np.linalg.cond(M)
    assert rel(x.ravel(), xs) <= cond * 1e-10
    # the reported residual is the true residual of the independent matrix
    assert np.linalg.norm(b.ravel() - M @ x.ravel()) / np.linalg.norm(b) <= 1e-10


def test_fgmres_warm_start_and_zero_rhs(small):
    dims, block, U, C, m0, M = small
    b = synth.gaussian_spinor(dims, seed=10)
    x0 = np.linalg.solve(M, b.ravel()).reshape(b.shape)
    x, info = oracle.fgmres(dims, block, U, C, m0, b, x0=x0, ncy=4, bc=BC)
    assert info["iterations"] == 0 and info["status"] == 0
    z, info = oracle.fgmres(dims, block, U, C, m0, np.zeros_like(b), ncy=4, bc=BC)
    assert info["status"] == 0 and np.max(np.abs(z)) == 0


def test_fgmres_max_restarts_not_converged(small):
    dims, block, U, C, m0, M = small
    b = synth.gaussian_spinor(dims, seed=11)
    x, info = oracle.fgmres(dims, block, U, C, m0, b, m=2, tol=1e-14, max_restarts=1, ncy=0, bc=BC)
    assert info["status"] == 1 and info["iterations"] == 2 and info["rel_residual"] > 1e-14


def test_gauge_covariance_of_solution():
    """x[U^W, W b] = W x[U, b]."""
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    U = synth.random_su3_links(dims, eps=0.4, seed=1)
    V = synth.volume(dims)
    W = synth.random_gauge_transform(dims, seed=2)
    from dense_ref import neighbours
    fwd = neighbours(dims)[0]
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[:, mu] = W @ U[:, mu] @ np.conj(np.swapaxes(W[fwd[mu]], 1, 2))
    C, Cg = oracle.clover_field(dims, U, 1.0), oracle.clover_field(dims, Ug, 1.0)
    b = synth.gaussian_spinor(dims, seed=3)
    x, i1 = oracle.fgmres(dims, block, U, C, 0.05, b, tol=1e-12, bc=BC)
    xg, i2 = oracle.fgmres(dims, block, Ug, Cg, 0.05, np.einsum("xab,xsb->xsa", W, b), tol=1e-12, bc=BC)
    assert i1["status"] == 0 and i2["status"] == 0
    assert rel(xg, np.einsum("xab,xsb->xsa", W, x)) < 1e-10
