"""Independent matrix assembly of the Wilson-clover operator (numpy / scipy).

Used only as a cross-check of the C oracle.  It builds D as an explicit sparse
matrix from shifted index grids (np.roll) and Kronecker-structured spin
factors, and the clover term from whole-field array products, so that it shares
neither code nor loop structure with oracle.c.  Matrix index of the component
(site, spin, colour) is ``site*12 + spin*3 + colour``.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

SIGMA = np.array(
    [
        [[0, 1], [1, 0]],
        [[0, -1j], [1j, 0]],
        [[1, 0], [0, -1]],
    ],
    dtype=np.complex128,
)


def gammas() -> np.ndarray:
    """Chiral-basis Euclidean gamma matrices gamma_x, gamma_y, gamma_z, gamma_t."""
    g = np.zeros((4, 4, 4), dtype=np.complex128)
    z = np.zeros((2, 2))
    for k in range(3):
        g[k] = np.block([[z, -1j * SIGMA[k]], [1j * SIGMA[k], z]])
    g[3] = np.block([[z, np.eye(2)], [np.eye(2), z]])
    return g


def gamma5() -> np.ndarray:
    g = gammas()
    return g[0] @ g[1] @ g[2] @ g[3]


def _grid(dims):
    Lx, Ly, Lz, Lt = dims
    return np.arange(Lx * Ly * Lz * Lt).reshape(Lt, Lz, Ly, Lx)


def neighbours(dims):
    """fwd[mu], bwd[mu] index arrays and wrap masks (forward: x_mu == L-1)."""
    g = _grid(dims)
    V = g.size
    fwd, bwd, wf, wb = [], [], [], []
    for mu in range(4):
        ax = 3 - mu
        fwd.append(np.roll(g, -1, axis=ax).reshape(V))
        bwd.append(np.roll(g, +1, axis=ax).reshape(V))
        coord = np.indices(g.shape)[ax].reshape(V)
        wf.append(coord == dims[mu] - 1)
        wb.append(coord == 0)
    return fwd, bwd, wf, wb


def _mm(a, b):
    return np.einsum("...ij,...jk->...ik", a, b)


def _dag(a):
    return np.conj(np.swapaxes(a, -1, -2))


def clover_dense(dims, U, csw):
    """C(x) as (V, 12, 12) from whole-field plaquette products."""
    V = int(np.prod(dims))
    fwd, bwd, _, _ = neighbours(dims)
    g = gammas()
    C = np.zeros((V, 12, 12), dtype=np.complex128)

    def Q(mu, nu):
        Um, Un = U[:, mu], U[:, nu]
        sh = lambda a, idx: a[idx]
        p_m, p_n, m_m, m_n = fwd[mu], fwd[nu], bwd[mu], bwd[nu]
        leaf1 = _mm(_mm(_mm(Um, sh(Un, p_m)), _dag(sh(Um, p_n))), _dag(Un))
        leaf2 = _mm(_mm(_mm(Un, _dag(sh(Um, p_n[m_m]))), _dag(sh(Un, m_m))), sh(Um, m_m))
        leaf3 = _mm(_mm(_mm(_dag(sh(Um, m_m)), _dag(sh(Un, m_n[m_m]))), sh(Um, m_n[m_m])), sh(Un, m_n))
        leaf4 = _mm(_mm(_mm(_dag(sh(Un, m_n)), sh(Um, m_n)), sh(Un, p_m[m_n])), _dag(Um))
        return leaf1 + leaf2 + leaf3 + leaf4

    for mu in range(4):
        for nu in range(4):
            if mu == nu:
                continue
            F = Q(mu, nu) - Q(nu, mu)
            G = g[mu] @ g[nu]
            C += -(csw / 32.0) * np.einsum("st,xab->xsatb", G, F).reshape(V, 12, 12)
    return C


def dirac_sparse(dims, U, C, m0, bc=(1, 1, 1, -1)):
    """Sparse CSR matrix of the Wilson-clover operator."""
    V = int(np.prod(dims))
    N = 12 * V
    fwd, bwd, wf, wb = neighbours(dims)
    g = gammas()
    eye4 = np.eye(4)
    rows, cols, vals = [], [], []
    x = np.arange(V)
    s_idx, a_idx, t_idx, b_idx = np.meshgrid(np.arange(4), np.arange(3), np.arange(4), np.arange(3), indexing="ij")

    def add_block(xs, ys, spin, colour_blocks):
        # entries (x, s, a) <- (y, t, b): spin[s, t] * colour_blocks[x][a, b]
        val = spin[None, s_idx, t_idx] * colour_blocks[:, a_idx, b_idx]
        r = xs[:, None, None, None, None] * 12 + s_idx * 3 + a_idx
        c = ys[:, None, None, None, None] * 12 + t_idx * 3 + b_idx
        rows.append(r.ravel())
        cols.append(c.ravel())
        vals.append(val.ravel())

    # diagonal: (4 + m0) + C(x)
    diag = C.copy()
    diag[:, np.arange(12), np.arange(12)] += 4.0 + m0
    r = x[:, None, None] * 12 + np.arange(12)[None, :, None]
    c = x[:, None, None] * 12 + np.arange(12)[None, None, :]
    rows.append(np.broadcast_to(r, diag.shape).ravel())
    cols.append(np.broadcast_to(c, diag.shape).ravel())
    vals.append(diag.ravel())
    for mu in range(4):
        sf = np.where(wf[mu], bc[mu], 1.0)
        sb = np.where(wb[mu], bc[mu], 1.0)
        add_block(x, fwd[mu], -0.5 * (eye4 - g[mu]), U[:, mu] * sf[:, None, None])
        add_block(x, bwd[mu], -0.5 * (eye4 + g[mu]), _dag(U[bwd[mu], mu]) * sb[:, None, None])
    M = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))
    return M.tocsr()


def block_sites(dims, block, block_id):
    """Global site indices of a block, in the block's own lexicographic order."""
    nb = [dims[m] // block[m] for m in range(4)]
    bc = []
    i = block_id
    for m in range(4):
        bc.append(i % nb[m])
        i //= nb[m]
    loc = np.indices(tuple(reversed(block))).reshape(4, -1)[::-1]  # x fastest
    glob = [bc[m] * block[m] + loc[m] for m in range(4)]
    Lx, Ly, Lz, _ = dims
    return glob[0] + Lx * (glob[1] + Ly * (glob[2] + Lz * glob[3])), sum(bc) % 2


def component_index(sites):
    return (np.asarray(sites)[:, None] * 12 + np.arange(12)[None, :]).ravel()
