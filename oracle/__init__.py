"""ctypes front end of the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: the slow, obviously correct definition of the
Wilson-clover operator, block MR, red-black SAP and FGMRES that the GPU path is
checked against.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the GPU library never does.

All arrays are numpy complex128 in the canonical layouts documented in
oracle.h (spinor ``[V, 4, 3]``, gauge ``[V, 4, 3, 3]``, clover ``[V, 12, 12]``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "oracle.c"
_HDR = _HERE / "oracle.h"
_LIB = _HERE / "liboracle.so"

# -fcx-fortran-rules: textbook complex multiply/divide (no C99 Annex G
# inf/nan recovery calls); IEEE double arithmetic is otherwise untouched.
CFLAGS = ["-O2", "-std=c99", "-fopenmp", "-fcx-fortran-rules", "-Wall", "-shared", "-fPIC"]


def build(force: bool = False) -> Path:
    """Compile liboracle.so with gcc if it is missing or older than its sources."""
    stale = (not _LIB.exists()) or any(p.stat().st_mtime > _LIB.stat().st_mtime for p in (_SRC, _HDR))
    if force or stale:
        tmp = _LIB.with_suffix(".so.tmp%d" % os.getpid())
        subprocess.run(["gcc", *CFLAGS, str(_SRC), "-o", str(tmp), "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


class OrInfo(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int),
        ("restarts", ctypes.c_int),
        ("precond_calls", ctypes.c_int),
        ("status", ctypes.c_int),
        ("rel_residual", ctypes.c_double),
    ]


PRECOND_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(str(_LIB))
        vp, ip, d, l_, i_ = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.c_double, ctypes.c_long, ctypes.c_int
        L.or_clover_field.argtypes = [ip, vp, d, vp]
        L.or_clover_site.argtypes = [ip, vp, d, l_, vp]
        L.or_apply_D.argtypes = [ip, ip, vp, vp, d, vp, vp]
        L.or_apply_D_sites.argtypes = [ip, ip, vp, d, d, vp, vp, l_, vp]
        L.or_apply_D_sites_nv.argtypes = [ip, ip, vp, d, d, vp, l_, vp, l_, vp]
        L.or_apply_DBB.argtypes = [ip, ip, ip, vp, vp, d, l_, vp, vp]
        L.or_apply_DBB.restype = i_
        L.or_mr_block.argtypes = [ip, ip, ip, vp, vp, d, l_, i_, vp, vp, vp]
        L.or_mr_block.restype = i_
        L.or_sap.argtypes = [ip, ip, ip, vp, vp, d, vp, vp, i_, i_]
        L.or_sap.restype = i_
        L.or_mr_block_eo.argtypes = [ip, ip, ip, vp, vp, d, l_, i_, vp, vp, vp]
        L.or_mr_block_eo.restype = i_
        L.or_sap_eo.argtypes = [ip, ip, ip, vp, vp, d, vp, vp, i_, i_]
        L.or_sap_eo.restype = i_
        L.or_fgmres.argtypes = [ip, ip, ip, vp, vp, d, vp, vp, i_, d, i_, i_, i_, PRECOND_FN, vp,
                                ctypes.POINTER(OrInfo)]
        L.or_fgmres.restype = i_
        L.or_num_threads.restype = i_
        _lib = L
    return _lib


def _ivec(v):
    v = [int(a) for a in v]
    if len(v) != 4:
        raise ValueError("expected four integers")
    return (ctypes.c_int * 4)(*v)


def _c(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    if shape is not None and a.shape != tuple(shape):
        a = a.reshape(shape)
    return a


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


DEFAULT_BC = (1, 1, 1, -1)


def num_threads() -> int:
    return int(lib().or_num_threads())


def clover_field(dims, U, csw):
    V = int(np.prod(dims))
    U = _c(U, (V, 4, 3, 3))
    C = np.empty((V, 12, 12), dtype=np.complex128)
    lib().or_clover_field(_ivec(dims), _p(U), float(csw), _p(C))
    return C


def clover_site(dims, U, csw, site):
    V = int(np.prod(dims))
    U = _c(U, (V, 4, 3, 3))
    C = np.empty((12, 12), dtype=np.complex128)
    lib().or_clover_site(_ivec(dims), _p(U), float(csw), int(site), _p(C))
    return C


def apply_D(dims, U, C, m0, psi, bc=DEFAULT_BC):
    V = int(np.prod(dims))
    U, C, psi = _c(U, (V, 4, 3, 3)), _c(C, (V, 12, 12)), _c(psi, (V, 4, 3))
    out = np.empty_like(psi)
    lib().or_apply_D(_ivec(dims), _ivec(bc), _p(U), _p(C), float(m0), _p(psi), _p(out))
    return out


def apply_D_sites(dims, U, csw, m0, psi, sites, bc=DEFAULT_BC):
    V = int(np.prod(dims))
    U, psi = _c(U, (V, 4, 3, 3)), _c(psi, (V, 4, 3))
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    out = np.empty((len(sites), 4, 3), dtype=np.complex128)
    lib().or_apply_D_sites(_ivec(dims), _ivec(bc), _p(U), float(csw), float(m0), _p(psi), _p(sites),
                           len(sites), _p(out))
    return out


def apply_D_sites_multi(dims, U, csw, m0, psis, sites, bc=DEFAULT_BC):
    """(D psi_v)(x) for several vectors psis (n, V, 4, 3) at the listed sites;
    returns (n, len(sites), 4, 3).  The clover term is formed once per site."""
    V = int(np.prod(dims))
    U = _c(U, (V, 4, 3, 3))
    psis = np.ascontiguousarray(psis, dtype=np.complex128)
    nvec = psis.size // (V * 12)
    psis = psis.reshape(nvec, V, 4, 3)
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    out = np.empty((nvec, len(sites), 4, 3), dtype=np.complex128)
    lib().or_apply_D_sites_nv(_ivec(dims), _ivec(bc), _p(U), float(csw), float(m0), _p(psis), nvec, _p(sites),
                              len(sites), _p(out))
    return out


def rel_residuals(dims, U, csw, m0, b, xs, bc=DEFAULT_BC, chunk=1 << 20):
    """||b - D x|| / ||b|| for each x in xs (n, V, 4, 3), evaluated over the
    whole lattice in chunks of sites with the clover term formed on the fly
    (no field-sized clover array)."""
    V = int(np.prod(dims))
    b = _c(b, (V, 4, 3))
    xs = np.ascontiguousarray(xs, dtype=np.complex128).reshape(-1, V, 4, 3)
    acc = np.zeros(xs.shape[0])
    for start in range(0, V, chunk):
        sites = np.arange(start, min(V, start + chunk), dtype=np.int64)
        dx = apply_D_sites_multi(dims, U, csw, m0, xs, sites, bc)
        acc += np.sum(np.abs(b[sites][None] - dx) ** 2, axis=(1, 2, 3))
    return np.sqrt(acc) / np.linalg.norm(b)


def apply_DBB(dims, block, U, C, m0, block_id, psi, bc=DEFAULT_BC):
    """D_BB on block ``block_id``; returns a whole-lattice array, zero off the block."""
    V = int(np.prod(dims))
    U, C, psi = _c(U, (V, 4, 3, 3)), _c(C, (V, 12, 12)), _c(psi, (V, 4, 3))
    out = np.zeros_like(psi)
    rc = lib().or_apply_DBB(_ivec(dims), _ivec(block), _ivec(bc), _p(U), _p(C), float(m0), int(block_id),
                            _p(psi), _p(out))
    if rc != 0:
        raise ValueError("invalid blocking or block id")
    return out


def mr_block(dims, block, U, C, m0, block_id, rho, nmr, bc=DEFAULT_BC):
    """Algorithm M on one block; returns (delta, r, steps) as whole-lattice arrays."""
    V = int(np.prod(dims))
    U, C, rho = _c(U, (V, 4, 3, 3)), _c(C, (V, 12, 12)), _c(rho, (V, 4, 3))
    delta = np.zeros_like(rho)
    r = np.zeros_like(rho)
    steps = lib().or_mr_block(_ivec(dims), _ivec(block), _ivec(bc), _p(U), _p(C), float(m0), int(block_id),
                              int(nmr), _p(rho), _p(delta), _p(r))
    if steps < 0:
        raise ValueError("invalid blocking or block id")
    return delta, r, steps


def mr_block_eo(dims, block, U, C, m0, block_id, rho, nmr, bc=DEFAULT_BC):
    """Even-odd preconditioned block solve; returns (delta, r_schur, steps)."""
    V = int(np.prod(dims))
    U, C, rho = _c(U, (V, 4, 3, 3)), _c(C, (V, 12, 12)), _c(rho, (V, 4, 3))
    delta = np.zeros_like(rho)
    r = np.zeros_like(rho)
    steps = lib().or_mr_block_eo(_ivec(dims), _ivec(block), _ivec(bc), _p(U), _p(C), float(m0), int(block_id),
                                 int(nmr), _p(rho), _p(delta), _p(r))
    if steps < 0:
        raise ValueError("invalid blocking or block id")
    return delta, r, steps


def sap(dims, block, U, C, m0, eta, ncy, nmr, bc=DEFAULT_BC, eo=False):
    """Algorithm S; ``eo`` selects the even-odd preconditioned block solve."""
    V = int(np.prod(dims))
    U, C, eta = _c(U, (V, 4, 3, 3)), _c(C, (V, 12, 12)), _c(eta, (V, 4, 3))
    psi = np.zeros_like(eta)
    fn = lib().or_sap_eo if eo else lib().or_sap
    rc = fn(_ivec(dims), _ivec(block), _ivec(bc), _p(U), _p(C), float(m0), _p(eta), _p(psi), int(ncy), int(nmr))
    if rc != 0:
        raise ValueError("invalid blocking or parameters")
    return psi


def fgmres(dims, block, U, C, m0, b, m=20, tol=1e-10, max_restarts=100, ncy=4, nmr=4, x0=None,
           precond=None, bc=DEFAULT_BC):
    """Algorithm G.  ``precond`` (optional) is a Python callable mapping a
    canonical spinor to a canonical spinor; otherwise SAP(ncy, nmr) is used,
    or the identity when ``ncy == 0``.  Returns (x, info_dict)."""
    V = int(np.prod(dims))
    U, C, b = _c(U, (V, 4, 3, 3)), _c(C, (V, 12, 12)), _c(b, (V, 4, 3))
    x = np.zeros_like(b) if x0 is None else _c(x0, (V, 4, 3)).copy()
    info = OrInfo()
    if precond is not None:
        n = V * 12

        def _cb(pin, pout, _user):
            src = np.ctypeslib.as_array(ctypes.cast(pin, ctypes.POINTER(ctypes.c_double)), shape=(2 * n,))
            dst = np.ctypeslib.as_array(ctypes.cast(pout, ctypes.POINTER(ctypes.c_double)), shape=(2 * n,))
            vin = src.view(np.complex128).reshape(V, 4, 3).copy()
            res = np.ascontiguousarray(precond(vin), dtype=np.complex128).reshape(-1)
            dst[:] = res.view(np.float64)

        cb = PRECOND_FN(_cb)
    else:
        cb = PRECOND_FN()
    lib().or_fgmres(_ivec(dims), _ivec(block), _ivec(bc), _p(U), _p(C), float(m0), _p(b), _p(x), int(m),
                    float(tol), int(max_restarts), int(ncy), int(nmr), cb, None, ctypes.byref(info))
    return x, {
        "iterations": info.iterations,
        "restarts": info.restarts,
        "precond_calls": info.precond_calls,
        "status": info.status,
        "rel_residual": info.rel_residual,
    }
