"""Seeded synthetic inputs shared by the GPU path, the oracle and the tests.

This module draws random numbers and shapes them into gauge links, sources and
gauge transformations.  It holds none of the solver's arithmetic (no Dirac
operator, no clover term, no Schwarz or Krylov step), so that both sides of a
parity comparison can consume the very same host arrays.

Canonical host layouts (complex128 numpy arrays):

* lattice site index ``x + Lx*(y + Ly*(z + Lz*t))`` (x fastest);
* gauge field ``U[site, mu, a, b]`` with ``mu`` in the order x, y, z, t;
* spinor ``psi[site, spin, colour]`` (12 complex numbers per site), or
  ``psi[rhs, site, spin, colour]`` for several right-hand sides.

Gauge links follow the recipe of the synthetic workloads: ``U = exp(i eps H)``
with ``H = sum_a h_a lambda_a / 2``, ``h_a ~ N(0, 1)`` i.i.d. over the eight
Gell-Mann matrices, exponentiated in float64 by the Cayley-Hamilton closed
form (the Hermitian eigendecomposition for the rare near-degenerate
spectra).  Draw order: for every site (lexicographic), for every direction, the
eight ``h_a``; right-hand sides are drawn afterwards from their own generator
stream (real part, then imaginary part, each ``N(0, 1)``).
"""
from __future__ import annotations

import os

import numpy as np

__all__ = [
    "gell_mann",
    "volume",
    "random_su3_links",
    "unit_links",
    "gaussian_spinor",
    "point_sources",
    "random_gauge_transform",
    "abelian_flux_links",
]


def volume(dims) -> int:
    dims = tuple(int(d) for d in dims)
    if len(dims) != 4 or min(dims) < 1:
        raise ValueError(f"dims must be four positive extents, got {dims}")
    return int(np.prod(dims))


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, shape (8, 3, 3), complex128."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0, 0, 1] = lam[0, 1, 0] = 1
    lam[1, 0, 1], lam[1, 1, 0] = -1j, 1j
    lam[2, 0, 0], lam[2, 1, 1] = 1, -1
    lam[3, 0, 2] = lam[3, 2, 0] = 1
    lam[4, 0, 2], lam[4, 2, 0] = -1j, 1j
    lam[5, 1, 2] = lam[5, 2, 1] = 1
    lam[6, 1, 2], lam[6, 2, 1] = -1j, 1j
    lam[7] = np.diag([1, 1, -2]) / np.sqrt(3)
    return lam


def _exp_i_hermitian_eigh(H: np.ndarray, eps: float) -> np.ndarray:
    """exp(i eps H) for a stack of Hermitian 3x3 matrices (eigendecomposition)."""
    w, W = np.linalg.eigh(H)
    phase = np.exp(1j * eps * w)
    return (W * phase[..., None, :]) @ np.conj(np.swapaxes(W, -1, -2))


def _exp_i_hermitian(H: np.ndarray, eps: float, fallback: bool = True):
    """exp(i Q), Q = eps H traceless Hermitian 3x3, by the Cayley-Hamilton closed
    form of Morningstar & Peardon, Phys. Rev. D 69 (2004) 054501:
    exp(iQ) = f0 + f1 Q + f2 Q^2 with f_j from c0 = det Q, c1 = tr Q^2 / 2.
    Stacks whose spectrum is close to degenerate fall back to the
    eigendecomposition; with fallback=False they are left for the caller, and
    (U, mask of those entries) is returned.  Only elementwise numpy runs here
    unless the fallback is taken."""
    shape = H.shape[:-2]
    Q = eps * H.reshape(-1, 9)
    q = [[np.ascontiguousarray(Q[:, 3 * i + j]) for j in range(3)] for i in range(3)]
    q2 = [[q[i][0] * q[0][k] + q[i][1] * q[1][k] + q[i][2] * q[2][k] for k in range(3)] for i in range(3)]
    c0 = np.real(q[0][0] * (q[1][1] * q[2][2] - q[1][2] * q[2][1])
                 - q[0][1] * (q[1][0] * q[2][2] - q[1][2] * q[2][0])
                 + q[0][2] * (q[1][0] * q[2][1] - q[1][1] * q[2][0]))
    c1 = 0.5 * np.real(q2[0][0] + q2[1][1] + q2[2][2])
    sign = np.where(c0 < 0, -1.0, 1.0)
    c0 = np.abs(c0)
    c0max = 2.0 * (c1 / 3.0) ** 1.5
    ratio = np.clip(np.divide(c0, c0max, out=np.zeros_like(c0), where=c0max > 0), -1.0, 1.0)
    theta = np.arccos(ratio)
    u = np.sqrt(c1 / 3.0) * np.cos(theta / 3.0)
    w = np.sqrt(c1) * np.sin(theta / 3.0)
    xi0 = np.where(np.abs(w) > 1e-4, np.sin(w) / np.where(w == 0, 1.0, w), 1.0 - w * w / 6.0)
    e2iu = np.exp(2j * u)
    emiu = np.exp(-1j * u)
    cw = np.cos(w)
    h0 = (u * u - w * w) * e2iu + emiu * (8 * u * u * cw + 2j * u * (3 * u * u + w * w) * xi0)
    h1 = 2 * u * e2iu - emiu * (2 * u * cw - 1j * (3 * u * u - w * w) * xi0)
    h2 = e2iu - emiu * (cw + 3j * u * xi0)
    den = 9 * u * u - w * w
    bad = np.abs(den) < 1e-6 * np.maximum(c1, 1e-300)
    den = np.where(bad, 1.0, den)
    f0, f1, f2 = h0 / den, h1 / den, h2 / den
    # det Q < 0: exp(iQ) = [exp(-i(-Q))]^+ with f_j(-c0) = (-1)^j conj(f_j(c0))
    neg = sign < 0
    f0 = np.where(neg, np.conj(f0), f0)
    f1 = np.where(neg, -np.conj(f1), f1)
    f2 = np.where(neg, np.conj(f2), f2)
    U = np.empty((Q.shape[0], 9), dtype=np.complex128)
    for i in range(3):
        for j in range(3):
            e = f1 * q[i][j] + f2 * q2[i][j]
            if i == j:
                e += f0
            U[:, 3 * i + j] = e
    U = U.reshape(shape + (3, 3))
    if not fallback:
        return U, bad.reshape(shape)
    if np.any(bad):
        U[bad.reshape(shape)] = _exp_i_hermitian_eigh(H[bad.reshape(shape)], eps)
    return U


def random_su3_links(dims, eps: float, seed: int = 0, chunk: int = 1 << 20) -> np.ndarray:
    """Random SU(3) gauge field ``U = exp(i eps H)``, shape (V, 4, 3, 3).

    ``eps`` controls the distance from the unit (free) field; ``eps = 0``
    gives unit links.  The eight normals per link are consumed site-major,
    then direction, then generator index.
    """
    from concurrent.futures import ThreadPoolExecutor

    V = volume(dims)
    rng = np.random.default_rng(seed)
    lam = gell_mann() / 2.0
    U = np.empty((V * 4, 3, 3), dtype=np.complex128)
    nlinks = V * 4

    def fill(start, H):
        Uc, bad = _exp_i_hermitian(H, eps, fallback=False)
        U[start:start + len(H)] = Uc
        return start, H, bad

    def finish(job):
        # the rare eigendecomposition fallback runs here, on the calling
        # thread, like every BLAS/LAPACK call of this function
        start, H, bad = job.result()
        if np.any(bad):
            U[start:start + len(H)][bad] = _exp_i_hermitian_eigh(H[bad], eps)

    # the normals and H (a matrix product) are formed in order on this
    # thread; the closed-form exponentials (elementwise numpy, which releases
    # the GIL) run on a few worker threads
    workers = max(1, min(8, len(os.sched_getaffinity(0))))
    with ThreadPoolExecutor(workers) as ex:
        jobs = []
        for start in range(0, nlinks, chunk):
            stop = min(nlinks, start + chunk)
            h = rng.standard_normal((stop - start, 8))
            H = (h.astype(np.complex128) @ lam.reshape(8, 9)).reshape(-1, 3, 3)
            jobs.append(ex.submit(fill, start, H))
            if len(jobs) >= 2 * workers:
                finish(jobs.pop(0))
        for j in jobs:
            finish(j)
    return U.reshape(V, 4, 3, 3)


def unit_links(dims) -> np.ndarray:
    V = volume(dims)
    U = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    U[:, :, 0, 0] = U[:, :, 1, 1] = U[:, :, 2, 2] = 1.0
    return U


def gaussian_spinor(dims, nrhs: int | None = None, seed: int = 0) -> np.ndarray:
    """Gaussian complex spinor(s): real and imaginary parts i.i.d. N(0, 1).

    Returns shape (V, 4, 3) when ``nrhs`` is None, else (nrhs, V, 4, 3).
    """
    V = volume(dims)
    rng = np.random.default_rng(seed)
    n = 1 if nrhs is None else int(nrhs)
    re = rng.standard_normal((n, V, 4, 3))
    im = rng.standard_normal((n, V, 4, 3))
    out = re + 1j * im
    return out[0] if nrhs is None else out


def point_sources(dims, origin=(0, 0, 0, 0)) -> np.ndarray:
    """The twelve unit point sources delta_{x,origin} e_{spin,colour}.

    Shape (12, V, 4, 3); right-hand side ``k`` has spin ``k // 3`` and colour
    ``k % 3``.
    """
    dims = tuple(int(d) for d in dims)
    V = volume(dims)
    x, y, z, t = (int(o) % d for o, d in zip(origin, dims))
    site = x + dims[0] * (y + dims[1] * (z + dims[2] * t))
    out = np.zeros((12, V, 4, 3), dtype=np.complex128)
    for k in range(12):
        out[k, site, k // 3, k % 3] = 1.0
    return out


def random_gauge_transform(dims, seed: int = 0, eps: float = 2.0) -> np.ndarray:
    """Random SU(3) matrix per site, shape (V, 3, 3)."""
    V = volume(dims)
    rng = np.random.default_rng(seed)
    lam = gell_mann() / 2.0
    h = rng.standard_normal((V, 8))
    H = np.einsum("na,aij->nij", h, lam)
    return _exp_i_hermitian(H, eps)


def abelian_flux_links(dims, k: int = 1) -> tuple[np.ndarray, float]:
    """Uniform abelian magnetic flux in the (x, y) plane embedded in SU(3).

    The U(1) phase ``u`` enters as ``diag(u, conj(u), 1)``.  With
    ``B = 2 pi k / (Lx Ly)`` the x-links are ``exp(-i B y)`` and the y-links
    on the last y slice are ``exp(i B Ly x)``; every other link is the unit
    matrix.  Every elementary (x, y) plaquette
    U_x(n) U_y(n+x) U_x(n+y)^+ U_y(n)^+ then carries the phase ``exp(+i B)``.
    Returns ``(U, B)``.
    """
    dims = tuple(int(d) for d in dims)
    Lx, Ly, Lz, Lt = dims
    V = volume(dims)
    B = 2.0 * np.pi * k / (Lx * Ly)
    U = unit_links(dims)
    idx = np.arange(V)
    xs = idx % Lx
    ys = (idx // Lx) % Ly
    ux = np.exp(-1j * B * ys)
    U[:, 0, 0, 0] = ux
    U[:, 0, 1, 1] = ux.conj()
    last = ys == Ly - 1
    uy = np.exp(1j * B * Ly * xs[last])
    U[last, 1, 0, 0] = uy
    U[last, 1, 1, 1] = uy.conj()
    return U, B
