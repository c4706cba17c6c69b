"""Pins of the oracle's even-odd preconditioned block solve and the SAP built
on it, against the Schur complement formed from an independently assembled
dense matrix, the textbook MR iteration on it, and exact-solve limits."""
import numpy as np
import pytest

import oracle
from dense_ref import block_sites, component_index, dirac_sparse
from paper_1710_07041_amd import synth
from test_oracle_solvers import sap_exact_cycle_matrices, textbook_mr

BC = (1, 1, 1, -1)


def rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b))


def parity(dims, sites):
    s = np.asarray(sites)
    c = [(s // int(np.prod(dims[:m]))) % dims[m] for m in range(4)]
    return (c[0] + c[1] + c[2] + c[3]) % 2


def eo_split(dims, sites):
    """Component indices (into the block's own 12*len(sites) vector) of the even and odd sites."""
    p = parity(dims, sites)
    ev = np.concatenate([12 * k + np.arange(12) for k in np.flatnonzero(p == 0)])
    od = np.concatenate([12 * k + np.arange(12) for k in np.flatnonzero(p == 1)])
    return ev, od


def dense_eo_block_solve(A, rho, ev, od, nmr):
    """Schur complement on the even sites, nmr textbook MR steps, odd reconstruction."""
    Aee, Aeo, Aoe, Aoo = A[np.ix_(ev, ev)], A[np.ix_(ev, od)], A[np.ix_(od, ev)], A[np.ix_(od, od)]
    Aoo_inv = np.linalg.inv(Aoo)
    S = Aee - Aeo @ Aoo_inv @ Aoe
    rhat = rho[ev] - Aeo @ (Aoo_inv @ rho[od])
    xe, re, norms = textbook_mr(S, rhat, nmr)
    x = np.zeros_like(rho)
    x[ev] = xe
    x[od] = Aoo_inv @ (rho[od] - Aoe @ xe)
    r = np.zeros_like(rho)
    r[ev] = re
    return x, r, norms


@pytest.fixture(scope="module", params=[(2, 2, 2, 2), (4, 4, 4, 4)])
def setup(request):
    dims = (4, 4, 4, 8)
    block = request.param
    U = synth.random_su3_links(dims, eps=0.4, seed=4)
    C = oracle.clover_field(dims, U, 1.0)
    m0 = -0.1
    M = dirac_sparse(dims, U, C, m0, BC).tocsr()
    return dims, block, U, C, m0, M


def test_eo_block_matches_textbook_schur(setup):
    dims, block, U, C, m0, M = setup
    rho = synth.gaussian_spinor(dims, seed=5)
    nblk = int(np.prod([dims[m] // block[m] for m in range(4)]))
    for bid in (0, nblk - 1):
        sites, _ = block_sites(dims, block, bid)
        ci = component_index(sites)
        A = M[ci][:, ci].toarray()
        ev, od = eo_split(dims, sites)
        x, r, norms = dense_eo_block_solve(A, rho[sites].ravel(), ev, od, 4)
        delta, r_or, steps = oracle.mr_block_eo(dims, block, U, C, m0, bid, rho, 4, BC)
        assert steps == 4
        assert rel(delta[sites].ravel(), x) < 1e-12
        assert rel(r_or[sites].ravel(), r) < 1e-11
        assert all(b <= a * (1 + 1e-14) for a, b in zip(norms, norms[1:]))
        # nothing outside the block is written
        mask = np.ones(synth.volume(dims), bool)
        mask[sites] = False
        assert np.max(np.abs(delta[mask])) == 0


def test_eo_block_exact_limit(setup):
    """Enough MR steps on the Schur complement solve the block system exactly."""
    dims, block, U, C, m0, M = setup
    rho = synth.gaussian_spinor(dims, seed=6)
    sites, _ = block_sites(dims, block, 1)
    ci = component_index(sites)
    A = M[ci][:, ci].toarray()
    delta, _, _ = oracle.mr_block_eo(dims, block, U, C, m0, 1, rho, 80, BC)
    assert rel(delta[sites].ravel(), np.linalg.solve(A, rho[sites].ravel())) < 1e-10


def test_eo_beats_plain_mr_per_step(setup):
    """Same number of steps: the block residual of the even-odd solve is smaller."""
    dims, block, U, C, m0, M = setup
    rho = synth.gaussian_spinor(dims, seed=7)
    sites, _ = block_sites(dims, block, 1)
    ci = component_index(sites)
    A = M[ci][:, ci].toarray()
    b = rho[sites].ravel()
    d_eo, _, _ = oracle.mr_block_eo(dims, block, U, C, m0, 1, rho, 4, BC)
    d_mr, _, _ = oracle.mr_block(dims, block, U, C, m0, 1, rho, 4, BC)
    res_eo = np.linalg.norm(b - A @ d_eo[sites].ravel())
    res_mr = np.linalg.norm(b - A @ d_mr[sites].ravel())
    assert res_eo < res_mr


def test_sap_eo_exact_block_limit(setup):
    """With exact block solves the even-odd SAP is the same multiplicative Schwarz cycle:
    M1 = K0 + K1 - K1 D K0."""
    dims, block, U, C, m0, M = setup
    Md = M.toarray()
    K0, K1 = sap_exact_cycle_matrices(dims, block, Md)
    eta = synth.gaussian_spinor(dims, seed=8)
    psi1 = oracle.sap(dims, block, U, C, m0, eta, 1, 80, BC, eo=True)
    assert rel(psi1.ravel(), (K0 + K1 - K1 @ Md @ K0) @ eta.ravel()) < 1e-9


def test_sap_eo_single_block_is_global_eo_mr():
    """One block = the whole lattice: one cycle is the even-odd solve of D itself."""
    dims = (4, 4, 4, 4)
    U = synth.random_su3_links(dims, eps=0.4, seed=9)
    C = oracle.clover_field(dims, U, 1.0)
    m0 = 0.05
    A = dirac_sparse(dims, U, C, m0, BC).toarray()
    eta = synth.gaussian_spinor(dims, seed=10)
    sites = np.arange(synth.volume(dims))
    ev, od = eo_split(dims, sites)
    x, _, _ = dense_eo_block_solve(A, eta.ravel(), ev, od, 5)
    psi = oracle.sap(dims, dims, U, C, m0, eta, 1, 5, BC, eo=True)
    assert rel(psi.ravel(), x) < 1e-12


def test_fgmres_with_sap_eo_solves():
    # the 4^4 blocking of the setup fixture (one blocking is enough here)
    dims, block = (4, 4, 4, 8), (4, 4, 4, 4)
    U = synth.random_su3_links(dims, eps=0.4, seed=4)
    C = oracle.clover_field(dims, U, 1.0)
    m0 = -0.1
    M = dirac_sparse(dims, U, C, m0, BC).tocsr()
    b = synth.gaussian_spinor(dims, seed=11)
    x, info = oracle.fgmres(dims, block, U, C, m0, b, m=10, tol=1e-10,
                            precond=lambda v: oracle.sap(dims, block, U, C, m0, v, 4, 4, BC, eo=True))
    assert info["status"] == 0
    assert rel(M @ x.ravel(), b.ravel()) <= 1e-10
    _, info_mr = oracle.fgmres(dims, block, U, C, m0, b, m=10, tol=1e-10, ncy=4, nmr=4)
    assert info["iterations"] <= info_mr["iterations"]
