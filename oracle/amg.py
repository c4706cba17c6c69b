"""Two-level adaptive-aggregation coarse correction (the multigrid level of
DD-alpha-AMG) in plain FP64 numpy on top of the C oracle.

TEST INFRASTRUCTURE ONLY: the slow, obviously correct definition that the GPU
path's setup, coarse operator, restriction, prolongation, coarse solve and
two-grid preconditioner are checked against.  Only the tests, the smoke check
and the benchmark's CPU-baseline leg may import this module.

The paper solves the Dirac equation with DD-alpha-AMG (Sec. 1), whose
fine-grid smoother is the Schwarz method of Sec. 2.1/3.1 and whose coarse grid
it names in Sec. 5; it prints no formula of the multigrid part.  The method
followed here is the published one: A. Frommer, K. Kahl, S. Krieg, B. Leder,
M. Rottmann, "Adaptive aggregation-based domain decomposition multigrid for
the lattice Wilson-Dirac operator", SIAM J. Sci. Comput. 36 (2014) A1581,
restated in this module's own terms:

* aggregates: every Schwarz block split into its two chiral halves (spins
  0-1 and spins 2-3), so that the interpolation commutes with gamma_5;
* interpolation P: N test vectors, each restricted to every aggregate, the N
  pieces of an aggregate orthonormalised among themselves (Gram-Schmidt in
  the order of the vectors), so that P^+ P = 1;
* test vectors: N given starting vectors, each improved by n_inv steps of
  inverse iteration with the SAP smoother as approximate inverse
  (v <- SAP(v), then v <- v/|v|), then by n_adapt adaptive rounds in which
  the current two-grid method takes the smoother's place;
* coarse operator: the Galerkin product D_c = P^+ D P, a nearest-neighbour
  operator on the lattice of blocks with 2N unknowns per block; since
  P^+ P = 1, D_c(m0) = D_c(0) + m0;
* coarse solve: k steps of GMRES from zero -- by definition the vector of
  the Krylov space K_k(D_c, b_c) with the smallest residual norm;
* two-grid preconditioner (coarse correction, then post-smoothing):
  psi_0 = P x_c with x_c the coarse solve of D_c x_c = P^+ eta, and
  psi = psi_0 + SAP_nu(eta - D psi_0).

Array conventions: spinors canonical (V, 4, 3) complex128; test vectors
(N, V, 4, 3); blocks numbered like oracle.c (bx fastest), sites inside a
block lexicographically (x fastest).  P is returned as (nblocks, 2, N, Vb, 6)
with Vb the sites of a block and the last axis (spin - 2c) * 3 + colour of
chiral half c.  Coarse vectors are (nblocks, 2, N) complex128, flattened to
index (block * 2 + c) * N + i where a matrix needs one index.
"""
from __future__ import annotations

import numpy as np

import oracle


def block_site_table(dims, block):
    """(nblocks, Vb) global site indices: row b lists block b's sites in
    lexicographic order inside the block."""
    dims, block = tuple(int(d) for d in dims), tuple(int(b) for b in block)
    nb = [dims[m] // block[m] for m in range(4)]
    nblk = int(np.prod(nb))
    Vb = int(np.prod(block))
    tab = np.empty((nblk, Vb), dtype=np.int64)
    for bid in range(nblk):
        bc, t = [], bid
        for m in range(4):
            bc.append(t % nb[m])
            t //= nb[m]
        for k in range(Vb):
            c, kk = [], k
            for m in range(4):
                c.append(bc[m] * block[m] + kk % block[m])
                kk //= block[m]
            tab[bid, k] = c[0] + dims[0] * (c[1] + dims[1] * (c[2] + dims[2] * c[3]))
    return tab


def _aggregate_pieces(vs, tab):
    """(nblocks, 2, N, Vb, 6): the N vectors restricted to each aggregate."""
    N = vs.shape[0]
    x = vs[:, tab]  # (N, nblocks, Vb, 4, 3)
    x = x.reshape(N, tab.shape[0], tab.shape[1], 2, 6)  # chiral half c: spins 2c, 2c+1
    return np.ascontiguousarray(np.transpose(x, (1, 3, 0, 2, 4)))


def interpolation(dims, block, vs):
    """P from test vectors vs (N, V, 4, 3): on each aggregate, modified
    Gram-Schmidt over the N restricted pieces in their order."""
    vs = np.asarray(vs, dtype=np.complex128)
    tab = block_site_table(dims, block)
    P = _aggregate_pieces(vs, tab)
    nblk, _, N = P.shape[:3]
    for b in range(nblk):
        for c in range(2):
            for i in range(N):
                w = P[b, c, i].copy()
                for j in range(i):
                    w -= np.vdot(P[b, c, j], w) * P[b, c, j]
                P[b, c, i] = w / np.linalg.norm(w)
    return P


def prolong(dims, block, P, xc):
    """P x_c: the fine spinor whose aggregate (b, c) holds sum_i x_c[b, c, i] P[b, c, i]."""
    tab = block_site_table(dims, block)
    V = int(np.prod(dims))
    out = np.zeros((V, 4, 3), dtype=np.complex128)
    pieces = np.einsum("bcisk,bci->bcsk", P, np.asarray(xc).reshape(P.shape[:3]))  # (nblocks, 2, Vb, 6)
    sp = np.transpose(pieces, (0, 2, 1, 3)).reshape(tab.shape[0], tab.shape[1], 4, 3)
    out[tab.reshape(-1)] = sp.reshape(-1, 4, 3)
    return out


def restrict(dims, block, P, eta):
    """P^+ eta as (nblocks, 2, N)."""
    tab = block_site_table(dims, block)
    e = _aggregate_pieces(np.asarray(eta, dtype=np.complex128)[None], tab)[:, :, 0]  # (nblocks, 2, Vb, 6)
    return np.einsum("bcisk,bcsk->bci", np.conj(P), e)


def coarse_operator(dims, block, U, C, P, bc=oracle.DEFAULT_BC):
    """D_c = P^+ D P at m0 = 0 as a dense (nc, nc) matrix, nc = nblocks * 2N,
    column by column: D applied to each column of P."""
    nblk, _, N = P.shape[:3]
    nc = nblk * 2 * N
    Dc = np.zeros((nc, nc), dtype=np.complex128)
    for col in range(nc):
        e = np.zeros(nc, dtype=np.complex128)
        e[col] = 1.0
        y = oracle.apply_D(dims, U, C, 0.0, prolong(dims, block, P, e), bc)
        Dc[:, col] = restrict(dims, block, P, y).reshape(nc)
    return Dc


def coarse_gmres(Dc, m0, bc_vec, k):
    """k steps of GMRES from zero on (D_c + m0) x = b: the x in
    K_k = span{b, A b, ..., A^(k-1) b} with the least residual norm, formed
    from an orthonormal basis of K_k (Arnoldi, modified Gram-Schmidt) and a
    least-squares solve.  If the space closes before k steps, the basis stops
    there (the minimiser is then the exact solution)."""
    A = Dc + m0 * np.eye(Dc.shape[0])
    b = np.asarray(bc_vec, dtype=np.complex128).reshape(-1)
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return np.zeros_like(b)
    Q = [b / nb]
    for j in range(k - 1):
        w = A @ Q[-1]
        for q in Q:
            w = w - np.vdot(q, w) * q
        nw = np.linalg.norm(w)
        if nw <= 1e-14 * nb:
            break
        Q.append(w / nw)
    Qm = np.stack(Q, axis=1)
    y, *_ = np.linalg.lstsq(A @ Qm, b, rcond=None)
    return Qm @ y


class TwoLevel:
    """The two-grid preconditioner for one mass, with everything it needs."""

    def __init__(self, dims, block, U, C, P, Dc, m0, k, nu, nmr, bc=oracle.DEFAULT_BC):
        self.dims, self.block, self.U, self.C, self.P, self.Dc = dims, block, U, C, P, Dc
        self.m0, self.k, self.nu, self.nmr, self.bc = m0, k, nu, nmr, bc

    def coarse_correction(self, eta):
        xc = coarse_gmres(self.Dc, self.m0, restrict(self.dims, self.block, self.P, eta), self.k)
        return prolong(self.dims, self.block, self.P, xc)

    def __call__(self, eta):
        psi0 = self.coarse_correction(eta)
        r = np.asarray(eta).reshape(psi0.shape) - oracle.apply_D(self.dims, self.U, self.C, self.m0, psi0, self.bc)
        if self.nu == 0:
            return psi0
        return psi0 + oracle.sap(self.dims, self.block, self.U, self.C, self.m0, r, self.nu, self.nmr, self.bc)


def setup(dims, block, U, C, m0, v0, n_inv=2, ncy=4, nmr=4, n_adapt=0, k=20, nu=2, bc=oracle.DEFAULT_BC):
    """Test vectors from the starting vectors v0 (N, V, 4, 3), then P and D_c.
    Returns (vs, P, Dc)."""
    vs = np.array(v0, dtype=np.complex128, copy=True)
    for _ in range(n_inv):
        for i in range(vs.shape[0]):
            v = oracle.sap(dims, block, U, C, m0, vs[i], ncy, nmr, bc)
            vs[i] = v / np.linalg.norm(v)
    P = interpolation(dims, block, vs)
    Dc = coarse_operator(dims, block, U, C, P, bc)
    for _ in range(n_adapt):
        tl = TwoLevel(dims, block, U, C, P, Dc, m0, k, nu, nmr, bc)
        for i in range(vs.shape[0]):
            v = tl(vs[i])
            vs[i] = v / np.linalg.norm(v)
        P = interpolation(dims, block, vs)
        Dc = coarse_operator(dims, block, U, C, P, bc)
    return vs, P, Dc
