"""GPU parity of the two-level coarse correction against the oracle
(oracle/amg.py), stage by stage, through the C ABI:

* setup: the interpolation built on the device from the same starting
  vectors (FP64 setup smoother) against the oracle's setup;
* coarse operator: the device's nine blocks per block row, assembled into
  the dense D_c, against P^+ D P formed by the oracle from the device's P;
  the Galerkin identity on random coarse vectors at 16^4 (four blocks per
  direction, so every neighbour is distinct);
* restriction and prolongation in FP64 and FP32;
* the coarse solve (k GMRES steps) against the least-residual vector of the
  Krylov space, on the FP16-rounded coarse operator the device applies;
* the two-grid preconditioner against the oracle's, in FP64 and FP32;
* SAP-FGMRES solves with the two-grid preconditioner, residual checked by
  the oracle's operator.
"""
import numpy as np
import pytest

import oracle
from gpu_util import BC, Lattice, rel, to_dev, to_host
from oracle import amg
from paper_1710_07041_amd import synth

pytestmark = pytest.mark.gpu

N = 4
M0 = -0.2


def dense_from_blocks(dims, A):
    """The dense coarse matrix from the device's blocks A[b][d][k'][k]."""
    nb = [d // 4 for d in dims]
    nblk, N2 = A.shape[0], A.shape[2]
    D = np.zeros((nblk * N2, nblk * N2), complex)
    for b in range(nblk):
        c, t = [], b
        for m in range(4):
            c.append(t % nb[m])
            t //= nb[m]
        for d in range(9):
            if d == 0:
                src = b
            else:
                mu, back = (d - 1) // 2, (d - 1) % 2
                cc = list(c)
                cc[mu] = (cc[mu] + (-1 if back else 1)) % nb[mu]
                src = cc[0] + nb[0] * (cc[1] + nb[1] * (cc[2] + nb[2] * cc[3]))
            D[b * N2:(b + 1) * N2, src * N2:(src + 1) * N2] += A[b, d].T
    return D


def f16(z):
    """The device's copy of D_c for the coarse solve: each real part rounded
    to FP32, then to FP16, both to nearest even."""
    r = lambda a: a.astype(np.float32).astype(np.float16).astype(np.float64)
    return r(z.real) + 1j * r(z.imag)


@pytest.fixture(scope="module")
def c1():
    """8^4, eps = 0.3, csw = 1, seed 0, with an FP64-smoother setup of N = 4
    test vectors from seeded Gaussian starting vectors."""
    lat = Lattice((8, 8, 8, 8), eps=0.3, csw=1.0, seed=0)
    from paper_1710_07041_amd import ddsap
    v0 = synth.gaussian_spinor(lat.dims, nrhs=N, seed=70)
    p = ddsap.default_amg_params()
    p.nvec, p.setup_iters, p.setup_ncy, p.setup_nmr, p.setup_prec, p.adapt = N, 2, 4, 4, ddsap.DD_F64, 0
    p.coarse_k, p.post_ncy, p.post_nmr = 8, 2, 4
    lat.ctx.amg_setup(M0, to_dev(v0), p)
    lat.v0, lat.amgp = v0, p
    lat.P = lat.ctx.amg_interpolation()  # (nblocks, 2, N, 6, 256)
    lat.Ad = lat.ctx.amg_coarse_operator()  # (nblocks, 9, 2N, 2N): [b][d][k'][k]
    return lat


def oracle_P(P_dev):
    """Device interpolation [b][c][i][comp][site] in the oracle's layout."""
    return np.ascontiguousarray(np.swapaxes(P_dev, -1, -2))


def test_setup_interpolation_matches_oracle(c1):
    _, P_ref, _ = amg.setup(c1.dims, (4, 4, 4, 4), c1.U, c1.C, M0, c1.v0, n_inv=2, ncy=4, nmr=4, n_adapt=0)
    P = oracle_P(c1.P)
    assert np.abs(P - P_ref).max() < 1e-12
    # orthonormal on every aggregate
    G = np.einsum("bcisk,bcjsk->bcij", np.conj(P), P)
    assert np.abs(G - np.eye(N)[None, None]).max() < 1e-13


def test_coarse_operator_is_galerkin(c1):
    P = oracle_P(c1.P)
    Dc_ref = amg.coarse_operator(c1.dims, (4, 4, 4, 4), c1.U, c1.C, P, BC)
    Dc = dense_from_blocks(c1.dims, c1.Ad)
    assert rel(Dc, Dc_ref) < 1e-13


@pytest.mark.parametrize("prec,tol", [("f64", 1e-14), ("f32", 2e-6)])
def test_restrict_prolong(c1, prec, tol):
    import torch
    P = oracle_P(c1.P)
    nc = c1.ctx.amg_coarse_size()
    eta = synth.gaussian_spinor(c1.dims, nrhs=2, seed=71)
    x = to_dev(eta)
    xb = c1.ctx.empty_blocked(prec, 2)
    c1.ctx.pack(x, xb, prec, 2)
    xc = torch.empty((2, nc), dtype=torch.complex128, device="cuda")
    c1.ctx.amg_restrict(xb, xc, prec, 2)
    got = to_host(xc)
    for r in range(2):
        assert rel(got[r], amg.restrict(c1.dims, (4, 4, 4, 4), P, eta[r]).reshape(-1)) < tol
    yc = np.random.default_rng(72).standard_normal((2, nc)) + 1j * np.random.default_rng(73).standard_normal((2, nc))
    yb = c1.ctx.empty_blocked(prec, 2)
    c1.ctx.amg_prolong(to_dev(yc), yb, prec, 2)
    y = torch.empty_like(x)
    c1.ctx.unpack(yb, y, prec, 2)
    c1.ctx.synchronize()
    fine = to_host(y)
    for r in range(2):
        assert rel(fine[r], amg.prolong(c1.dims, (4, 4, 4, 4), P, yc[r])) < tol


def test_coarse_solve_is_the_krylov_minimiser(c1):
    """k = 8 GMRES steps on (D_c + m0) x = b for two right-hand sides with
    their own masses; the device applies the FP16 copy of D_c."""
    import torch
    # the device rounds every block to FP16 and sums neighbours that coincide
    # (two blocks per direction) in FP64
    Dc = dense_from_blocks(c1.dims, f16(c1.Ad))
    nc = Dc.shape[0]
    rng = np.random.default_rng(74)
    b = rng.standard_normal((2, nc)) + 1j * rng.standard_normal((2, nc))
    m0 = np.array([-0.2, 0.1])
    xc = torch.empty((2, nc), dtype=torch.complex128, device="cuda")
    c1.ctx.amg_coarse_solve(m0, to_dev(b), xc, 8, 2)
    yc = torch.empty_like(xc)
    c1.ctx.amg_coarse_apply(m0, to_dev(b), yc, 2)
    c1.ctx.synchronize()
    x, y = to_host(xc), to_host(yc)
    for r in range(2):
        assert rel(y[r], (Dc + m0[r] * np.eye(nc)) @ b[r]) < 1e-13
        ref = amg.coarse_gmres(Dc, m0[r], b[r], 8)
        assert rel(x[r], ref) < 1e-10
    # every step: the exact coarse solution
    full = torch.empty_like(xc)
    c1.ctx.amg_coarse_solve(m0, to_dev(b), full, 32, 2)
    c1.ctx.synchronize()
    if nc <= 32:
        for r in range(2):
            assert rel(to_host(full)[r], np.linalg.solve(Dc + m0[r] * np.eye(nc), b[r])) < 1e-10


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 2e-5)])
def test_two_grid_preconditioner(c1, prec, tol):
    import torch
    P = oracle_P(c1.P)
    Dc = dense_from_blocks(c1.dims, f16(c1.Ad))
    tl = amg.TwoLevel(c1.dims, (4, 4, 4, 4), c1.U, c1.C, P, Dc, M0, k=8, nu=2, nmr=4, bc=BC)
    eta = synth.gaussian_spinor(c1.dims, seed=75)
    x = to_dev(eta)
    eb, pb = c1.ctx.empty_blocked(prec), c1.ctx.empty_blocked(prec)
    c1.ctx.pack(x, eb, prec)
    c1.ctx.amg_precondition(M0, eb, pb, prec)
    y = torch.empty_like(x)
    c1.ctx.unpack(pb, y, prec)
    c1.ctx.synchronize()
    assert rel(to_host(y), tl(eta)) < tol


@pytest.mark.parametrize("sap_prec", ["f64", "f32"])
def test_amg_solve_residual_against_oracle(c1, sap_prec):
    from test_gpu_solver import gpu_solve
    b = synth.gaussian_spinor(c1.dims, seed=0)
    st, info, x = gpu_solve(c1, b, M0, sap_prec, amg=1)
    assert st == 0 and info[0]["status"] == 0, info
    r = b - oracle.apply_D(c1.dims, c1.U, c1.C, M0, x, BC)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-10
    print(f"AMGSOLVE 8^4 {sap_prec}: {info[0]['iterations']} iterations", flush=True)


def test_amg_solve_multi_rhs_equals_solo(c1):
    from test_gpu_solver import gpu_solve
    n = 3
    b = synth.gaussian_spinor(c1.dims, nrhs=n, seed=76)
    m0 = np.array([-0.2, -0.1, 0.1])
    st, info, x = gpu_solve(c1, b, m0, "f32", nrhs=n, amg=1)
    assert st == 0
    for r in range(n):
        res = b[r] - oracle.apply_D(c1.dims, c1.U, c1.C, m0[r], x[r], BC)
        assert np.linalg.norm(res) / np.linalg.norm(b[r]) <= 1e-10
        _, _, xs = gpu_solve(c1, b[r], m0[r], "f32", amg=1)
        assert rel(x[r], xs) <= 1e-8


def test_galerkin_identity_16x4():
    """16^4 (four blocks per direction): D_c x_c = P^+ D P x_c for random
    coarse vectors, the right side formed by the oracle from the device's P;
    FP32 setup smoother, one adaptive round."""
    import torch
    from paper_1710_07041_amd import ddsap
    lat = Lattice((16, 16, 16, 16), eps=0.5, csw=1.0, seed=4)
    p = ddsap.default_amg_params()
    p.nvec, p.setup_iters, p.adapt, p.coarse_k = 6, 2, 1, 12
    lat.ctx.amg_setup(-0.25, to_dev(synth.gaussian_spinor(lat.dims, nrhs=6, seed=77)), p)
    P = oracle_P(lat.ctx.amg_interpolation())
    G = np.einsum("bcisk,bcjsk->bcij", np.conj(P), P)
    assert np.abs(G - np.eye(6)[None, None]).max() < 1e-13
    nc = lat.ctx.amg_coarse_size()
    xc = np.random.default_rng(78).standard_normal(nc) + 1j * np.random.default_rng(79).standard_normal(nc)
    yc = torch.empty((1, nc), dtype=torch.complex128, device="cuda")
    lat.ctx.amg_coarse_apply(-0.25, to_dev(xc)[None], yc, 1)
    lat.ctx.synchronize()
    fine = oracle.apply_D(lat.dims, lat.U, lat.C, -0.25, amg.prolong(lat.dims, (4, 4, 4, 4), P, xc), BC)
    ref = amg.restrict(lat.dims, (4, 4, 4, 4), P, fine).reshape(-1)
    assert rel(to_host(yc)[0], ref) < 2e-3  # the device applies the FP16 copy of D_c
    lat.ctx.close()


def test_amg_errors(c1):
    from paper_1710_07041_amd import ddsap
    lat = Lattice((8, 8, 8, 8), eps=0.3, seed=1, oracle_clover=False)
    from test_gpu_solver import gpu_solve
    st, info, _ = gpu_solve(lat, synth.gaussian_spinor(lat.dims, seed=1), M0, "f32", amg=1)
    assert st == ddsap.DD_INVALID_ARG  # no setup yet
    p = ddsap.default_amg_params()
    p.nvec = 0
    with pytest.raises(ddsap.DDError):
        lat.ctx.amg_setup(M0, to_dev(synth.gaussian_spinor(lat.dims, nrhs=1, seed=2)), p)
    lat.ctx.close()
