"""Thin ctypes binding of libddsap.so (C ABI declared in include/ddsap.h).

Argument marshalling only: every step of the operator, the Schwarz smoother
and the solver runs in the library's HIP kernels.  Device buffers are torch
tensors on the GPU (PyTorch serves only for device memory and streams).  If the
shared library is missing this module raises ImportError: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os
from pathlib import Path

import numpy as np

_PKG = Path(__file__).resolve().parent
LIB_PATH = Path(os.environ.get("DDSAP_LIB", _PKG / "libddsap.so"))

# torch ships its own HIP runtime under the same soname (libamdhip64.so.7).
# Loading torch first makes this library bind to that one runtime instead of
# pulling a second copy (and a second HSA runtime) into the process.
import torch  # noqa: E402,F401

if not LIB_PATH.exists():
    raise ImportError(f"libddsap.so not found at {LIB_PATH}; build it with paper_1710_07041_amd/build.py "
                      "(or __graft_entry__.build())")

_lib = ctypes.CDLL(str(LIB_PATH))

DD_OK, DD_INVALID_ARG, DD_OOM, DD_HIP_ERROR, DD_NOT_CONVERGED, DD_BREAKDOWN, DD_NAN, DD_NO_FIELD = range(8)
STATUS_NAMES = ["DD_OK", "DD_INVALID_ARG", "DD_OOM", "DD_HIP_ERROR", "DD_NOT_CONVERGED", "DD_BREAKDOWN", "DD_NAN",
                "DD_NO_FIELD"]
DD_F64, DD_F32, DD_F16 = 0, 1, 2
PREC = {"f64": DD_F64, "f32": DD_F32, "f16": DD_F16}
DD_MAX_RHS = 16

EXPORTS = [
    "dd_abi_version", "dd_default_params", "dd_create", "dd_destroy", "dd_last_error", "dd_synchronize",
    "dd_set_gauge", "dd_set_link_compression", "dd_link_compression", "dd_set_sap_half_fields", "dd_sap_half_fields", "dd_set_clover", "dd_spinor_bytes", "dd_pack_spinor", "dd_unpack_spinor", "dd_apply_D",
    "dd_apply_D_block", "dd_sap", "dd_sap_eo", "dd_sap_noalloc", "dd_solve", "dd_amg_default_params",
    "dd_amg_setup", "dd_amg_coarse_size", "dd_amg_interpolation", "dd_amg_coarse_operator", "dd_amg_restrict",
    "dd_amg_prolong", "dd_amg_coarse_apply", "dd_amg_coarse_solve", "dd_amg_precondition", "dd_debug_poison_half_smoother", "dd_profile_enable",
    "dd_profile_read", "dd_stream_copy",
    "dd_server_default_config", "dd_server_create", "dd_server_add_field", "dd_server_field_info",
    "dd_server_submit", "dd_server_poll", "dd_server_wait", "dd_server_get_stats", "dd_server_last_error",
    "dd_server_destroy",
]


class dd_params(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int), ("tol", ctypes.c_double), ("max_restarts", ctypes.c_int),
                ("ncy", ctypes.c_int), ("nmr", ctypes.c_int), ("sap_prec", ctypes.c_int), ("sap_eo", ctypes.c_int),
                ("amg", ctypes.c_int)]


class dd_amg_params(ctypes.Structure):
    _fields_ = [("nvec", ctypes.c_int), ("setup_iters", ctypes.c_int), ("setup_ncy", ctypes.c_int),
                ("setup_nmr", ctypes.c_int), ("setup_prec", ctypes.c_int), ("adapt", ctypes.c_int),
                ("coarse_k", ctypes.c_int), ("post_ncy", ctypes.c_int), ("post_nmr", ctypes.c_int)]


class dd_solve_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iterations", ctypes.c_int), ("restarts", ctypes.c_int),
                ("sap_calls", ctypes.c_int), ("rel_residual", ctypes.c_double)]


class dd_kernel_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_long), ("total_ms", ctypes.c_double),
                ("bytes", ctypes.c_double), ("flops", ctypes.c_double)]


class dd_server_config(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_width", ctypes.c_int), ("m", ctypes.c_int),
                ("tol", ctypes.c_double), ("max_restarts", ctypes.c_int), ("ncy", ctypes.c_int),
                ("nmr", ctypes.c_int), ("sap_prec", ctypes.c_int), ("use_graphs", ctypes.c_int),
                ("sap_eo", ctypes.c_int), ("sap_half_fields", ctypes.c_int)]


class dd_server_stats(ctypes.Structure):
    _fields_ = [("requests_done", ctypes.c_long), ("rhs_done", ctypes.c_long), ("iterations", ctypes.c_long),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
                ("wall_s", ctypes.c_double), ("rhs_per_s", ctypes.c_double), ("busy_s", ctypes.c_double),
                ("workspace_bytes", ctypes.c_size_t)]


_vp, _ip, _d, _i, _l, _sz = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.c_double, ctypes.c_int, \
    ctypes.c_long, ctypes.c_size_t
_dp = ctypes.POINTER(ctypes.c_double)
_sigs = {
    "dd_abi_version": ([], _i),
    "dd_default_params": ([ctypes.POINTER(dd_params)], None),
    "dd_create": ([_ip, _ip, _ip, _vp, ctypes.POINTER(_vp)], _i),
    "dd_destroy": ([_vp], _i),
    "dd_last_error": ([_vp], ctypes.c_char_p),
    "dd_synchronize": ([_vp], _i),
    "dd_set_gauge": ([_vp, _vp, _d], _i),
    "dd_set_clover": ([_vp, _vp], _i),
    "dd_set_link_compression": ([_vp, _i], _i),
    "dd_link_compression": ([_vp], _i),
    "dd_set_sap_half_fields": ([_vp, _i], _i),
    "dd_sap_half_fields": ([_vp], _i),
    "dd_spinor_bytes": ([_vp, _i, _i], _sz),
    "dd_pack_spinor": ([_vp, _vp, _vp, _i, _i], _i),
    "dd_unpack_spinor": ([_vp, _vp, _vp, _i, _i], _i),
    "dd_apply_D": ([_vp, _dp, _vp, _vp, _i, _i], _i),
    "dd_apply_D_block": ([_vp, _d, _l, _vp, _vp, _i], _i),
    "dd_sap": ([_vp, _dp, _vp, _vp, _i, _i, _i, _i], _i),
    "dd_sap_eo": ([_vp, _dp, _vp, _vp, _i, _i, _i, _i], _i),
    "dd_sap_noalloc": ([_vp, _dp, _vp, _vp, _i, _i, _i, _i], _i),
    "dd_solve": ([_vp, _dp, _vp, _vp, _i, ctypes.POINTER(dd_params), ctypes.POINTER(dd_solve_info)], _i),
    "dd_debug_poison_half_smoother": ([_vp, _i], _i),
    "dd_amg_default_params": ([ctypes.POINTER(dd_amg_params)], None),
    "dd_amg_setup": ([_vp, _d, _vp, ctypes.POINTER(dd_amg_params)], _i),
    "dd_amg_coarse_size": ([_vp], ctypes.c_size_t),
    "dd_amg_interpolation": ([_vp, _vp], _i),
    "dd_amg_coarse_operator": ([_vp, _vp], _i),
    "dd_amg_restrict": ([_vp, _vp, _vp, _i, _i], _i),
    "dd_amg_prolong": ([_vp, _vp, _vp, _i, _i], _i),
    "dd_amg_coarse_apply": ([_vp, _dp, _vp, _vp, _i], _i),
    "dd_amg_coarse_solve": ([_vp, _dp, _vp, _vp, _i, _i], _i),
    "dd_amg_precondition": ([_vp, _dp, _vp, _vp, _i, _i], _i),
    "dd_profile_enable": ([_vp, _i], _i),
    "dd_stream_copy": ([_vp, _vp, _sz, _vp], _i),
    "dd_server_default_config": ([ctypes.POINTER(dd_server_config)], None),
    "dd_server_create": ([ctypes.POINTER(dd_server_config), ctypes.POINTER(_vp)], _i),
    "dd_server_add_field": ([_vp, _ip, _ip, _vp, _d, _i, _ip], _i),
    "dd_server_field_info": ([_vp, _i, _ip, ctypes.POINTER(_sz)], _i),
    "dd_server_submit": ([_vp, _i, _i, _dp, _vp, _vp, ctypes.POINTER(_l)], _i),
    "dd_server_poll": ([_vp, _l, _ip, ctypes.POINTER(dd_solve_info), _dp], _i),
    "dd_server_wait": ([_vp, _l, ctypes.POINTER(dd_solve_info), _dp], _i),
    "dd_server_get_stats": ([_vp, ctypes.POINTER(dd_server_stats)], _i),
    "dd_server_last_error": ([_vp], ctypes.c_char_p),
    "dd_server_destroy": ([_vp], _i),
    "dd_profile_read": ([_vp, ctypes.POINTER(dd_kernel_stat), _i], _i),
}
for _name, (_args, _res) in _sigs.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res


class DDError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else status}: {msg}")
        self.status = status


def abi_version() -> int:
    return _lib.dd_abi_version()


def default_params() -> dd_params:
    p = dd_params()
    _lib.dd_default_params(ctypes.byref(p))
    return p


def _ptr(t) -> int:
    """Device or host address of a torch tensor / numpy array."""
    if hasattr(t, "data_ptr"):
        return t.data_ptr()
    return t.ctypes.data


def _masses(m0, nrhs):
    a = np.broadcast_to(np.asarray(m0, dtype=np.float64), (nrhs,)).copy()
    return a, a.ctypes.data_as(_dp)


class Context:
    """One lattice on the current HIP device (wraps dd_ctx)."""

    def __init__(self, dims, bcs=(1, 1, 1, -1), stream=None, block=(4, 4, 4, 4)):
        import torch
        self.dims = tuple(int(d) for d in dims)
        self.volume = int(np.prod(self.dims))
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self._h = _vp()
        blk = None if block is None else (ctypes.c_int * 4)(*block)
        st = _lib.dd_create((ctypes.c_int * 4)(*self.dims), blk, (ctypes.c_int * 4)(*bcs), _vp(stream),
                            ctypes.byref(self._h))
        if st != DD_OK:
            raise DDError(st, _lib.dd_last_error(None).decode())

    # -- plumbing ---------------------------------------------------------
    def _check(self, st):
        if st != DD_OK:
            raise DDError(st, _lib.dd_last_error(self._h).decode())
        return st

    def close(self):
        if self._h:
            _lib.dd_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def synchronize(self):
        self._check(_lib.dd_synchronize(self._h))

    # -- C ABI, one method per entry point ------------------------------------
    def set_gauge(self, U, csw):
        """U: host complex128 array (V, 4, 3, 3) in canonical order."""
        U = np.ascontiguousarray(U, dtype=np.complex128)
        if U.size != self.volume * 36:
            raise ValueError("gauge field has the wrong size")
        self._check(_lib.dd_set_gauge(self._h, _vp(U.ctypes.data), float(csw)))

    def set_link_compression(self, enable):
        """dd_set_link_compression: read two rows per link and rebuild the
        third (SU(3) fields only)."""
        self._check(_lib.dd_set_link_compression(self._h, 1 if enable else 0))

    @property
    def link_compression(self) -> bool:
        return _lib.dd_link_compression(self._h) == 1

    def set_sap_half_fields(self, enable):
        """dd_set_sap_half_fields: the plain FP32 smoother reads FP16 links
        and clover."""
        self._check(_lib.dd_set_sap_half_fields(self._h, 1 if enable else 0))

    @property
    def sap_half_fields(self) -> bool:
        return _lib.dd_sap_half_fields(self._h) == 1

    def set_clover(self, C):
        """C: host complex128 array (V, 2, 6, 6): the two chiral 6x6 halves."""
        C = np.ascontiguousarray(C, dtype=np.complex128)
        if C.size != self.volume * 72:
            raise ValueError("clover field has the wrong size")
        self._check(_lib.dd_set_clover(self._h, _vp(C.ctypes.data)))

    def spinor_bytes(self, prec, nrhs=1) -> int:
        return int(_lib.dd_spinor_bytes(self._h, PREC.get(prec, prec), int(nrhs)))

    def empty_blocked(self, prec, nrhs=1):
        import torch
        return torch.empty(self.spinor_bytes(prec, nrhs), dtype=torch.uint8, device="cuda")

    def pack(self, canon, blocked, prec, nrhs=1):
        self._check(_lib.dd_pack_spinor(self._h, _vp(_ptr(canon)), _vp(_ptr(blocked)), PREC.get(prec, prec),
                                        int(nrhs)))

    def unpack(self, blocked, canon, prec, nrhs=1):
        self._check(_lib.dd_unpack_spinor(self._h, _vp(_ptr(blocked)), _vp(_ptr(canon)), PREC.get(prec, prec),
                                          int(nrhs)))

    def apply_D(self, m0, x, y, prec, nrhs=1):
        _, mp = _masses(m0, nrhs)
        self._check(_lib.dd_apply_D(self._h, mp, _vp(_ptr(x)), _vp(_ptr(y)), PREC.get(prec, prec), int(nrhs)))

    def apply_D_block(self, m0, block_id, x, y, prec):
        self._check(_lib.dd_apply_D_block(self._h, float(m0), int(block_id), _vp(_ptr(x)), _vp(_ptr(y)),
                                          PREC.get(prec, prec)))

    def sap(self, m0, eta, psi, ncy, nmr, prec, nrhs=1, eo=False):
        """dd_sap, or dd_sap_eo (even-odd block solves) when eo is set."""
        _, mp = _masses(m0, nrhs)
        fn = _lib.dd_sap_eo if eo else _lib.dd_sap
        self._check(fn(self._h, mp, _vp(_ptr(eta)), _vp(_ptr(psi)), int(ncy), int(nmr), PREC.get(prec, prec),
                       int(nrhs)))

    def sap_noalloc(self, m0, eta, psi, ncy, nmr, prec, nrhs=1, raise_on_fail=True):
        """dd_sap_noalloc: dd_sap with its scratch in the library's fixed device
        array (no allocation).  Returns the status when raise_on_fail is off."""
        _, mp = _masses(m0, nrhs)
        st = _lib.dd_sap_noalloc(self._h, mp, _vp(_ptr(eta)), _vp(_ptr(psi)), int(ncy), int(nmr),
                                 PREC.get(prec, prec), int(nrhs))
        if raise_on_fail:
            self._check(st)
        return st

    def last_error(self) -> str:
        return _lib.dd_last_error(self._h).decode()

    def solve(self, m0, b, x, nrhs=1, params: dd_params | None = None, raise_on_fail=True):
        """b, x: canonical complex128 device tensors (nrhs, V, 4, 3); x holds x0."""
        _, mp = _masses(m0, nrhs)
        infos = (dd_solve_info * nrhs)()
        p = params if params is not None else default_params()
        st = _lib.dd_solve(self._h, mp, _vp(_ptr(b)), _vp(_ptr(x)), int(nrhs), ctypes.byref(p), infos)
        out = [{k: getattr(i, k) for k, _ in dd_solve_info._fields_} for i in infos]
        if raise_on_fail and st not in (DD_OK,):
            raise DDError(st, _lib.dd_last_error(self._h).decode())
        return st, out

    # -- two-level coarse correction --------------------------------------
    def amg_setup(self, m0, v0, params=None):
        """v0: canonical complex128 device tensor (nvec, V, 4, 3) of starting vectors."""
        p = params if params is not None else default_amg_params()
        self._check(_lib.dd_amg_setup(self._h, float(m0), _vp(_ptr(v0)), ctypes.byref(p)))
        self._amg_nvec = p.nvec

    def amg_coarse_size(self) -> int:
        return int(_lib.dd_amg_coarse_size(self._h))

    def amg_interpolation(self):
        """P as numpy complex128 (nblocks, 2, nvec, 6, 256): [block][chirality][vector][component][site]."""
        n = self._amg_nvec
        nb = self.volume // 256
        out = np.empty((nb, 2, n, 6, 256), dtype=np.complex128)
        self._check(_lib.dd_amg_interpolation(self._h, _vp(out.ctypes.data)))
        return out

    def amg_coarse_operator(self):
        """D_c as numpy complex128 (nblocks, 9, 2 nvec, 2 nvec): [block][d][column k'][row k]."""
        n2 = 2 * self._amg_nvec
        nb = self.volume // 256
        out = np.empty((nb, 9, n2, n2), dtype=np.complex128)
        self._check(_lib.dd_amg_coarse_operator(self._h, _vp(out.ctypes.data)))
        return out

    def amg_restrict(self, x, xc, prec, nrhs=1):
        self._check(_lib.dd_amg_restrict(self._h, _vp(_ptr(x)), _vp(_ptr(xc)), PREC.get(prec, prec), int(nrhs)))

    def amg_prolong(self, xc, x, prec, nrhs=1):
        self._check(_lib.dd_amg_prolong(self._h, _vp(_ptr(xc)), _vp(_ptr(x)), PREC.get(prec, prec), int(nrhs)))

    def amg_coarse_apply(self, m0, xc, yc, nrhs=1):
        _, mp = _masses(m0, nrhs)
        self._check(_lib.dd_amg_coarse_apply(self._h, mp, _vp(_ptr(xc)), _vp(_ptr(yc)), int(nrhs)))

    def amg_coarse_solve(self, m0, bc, xc, k, nrhs=1):
        _, mp = _masses(m0, nrhs)
        self._check(_lib.dd_amg_coarse_solve(self._h, mp, _vp(_ptr(bc)), _vp(_ptr(xc)), int(k), int(nrhs)))

    def amg_precondition(self, m0, eta, psi, prec, nrhs=1):
        _, mp = _masses(m0, nrhs)
        self._check(_lib.dd_amg_precondition(self._h, mp, _vp(_ptr(eta)), _vp(_ptr(psi)), PREC.get(prec, prec),
                                             int(nrhs)))

    def debug_poison_half_smoother(self, count):
        """Test hook: the next `count` FP16 smoother outputs of solve() (all for
        count < 0) get a non-finite entry, which must trigger the FP32 fallback."""
        self._check(_lib.dd_debug_poison_half_smoother(self._h, int(count)))

    def profile_enable(self, on=True):
        self._check(_lib.dd_profile_enable(self._h, 1 if on else 0))

    def profile_read(self):
        """{kernel class: {launches, total_ms, bytes, flops}} (synchronises)."""
        buf = (dd_kernel_stat * 64)()
        n = _lib.dd_profile_read(self._h, buf, 64)
        if n < 0:
            raise DDError(DD_HIP_ERROR, _lib.dd_last_error(self._h).decode())
        return {buf[i].name.decode(): {"launches": buf[i].launches, "total_ms": buf[i].total_ms,
                                       "bytes": buf[i].bytes, "flops": buf[i].flops} for i in range(n)}


def stream_copy(src, dst, nbytes, stream=None):
    """dd_stream_copy on torch's current stream (or the given one)."""
    import torch
    st = torch.cuda.current_stream().cuda_stream if stream is None else stream
    s = _lib.dd_stream_copy(_vp(_ptr(src)), _vp(_ptr(dst)), int(nbytes), _vp(st))
    if s != DD_OK:
        raise DDError(s, "dd_stream_copy failed")


def default_amg_params() -> dd_amg_params:
    p = dd_amg_params()
    _lib.dd_amg_default_params(ctypes.byref(p))
    return p


def default_server_config() -> dd_server_config:
    c = dd_server_config()
    _lib.dd_server_default_config(ctypes.byref(c))
    return c


class Server:
    """Continuous-batching solve server over resident gauge fields (wraps dd_server)."""

    def __init__(self, config: dd_server_config | None = None, **kw):
        c = config if config is not None else default_server_config()
        for k, v in kw.items():
            setattr(c, k, PREC.get(v, v) if k == "sap_prec" else v)
        self._h = _vp()
        st = _lib.dd_server_create(ctypes.byref(c), ctypes.byref(self._h))
        if st != DD_OK:
            raise DDError(st, "dd_server_create failed")
        self._live = {}
        self._vol = {}

    def _check(self, st):
        if st != DD_OK:
            raise DDError(st, _lib.dd_server_last_error(self._h).decode())
        return st

    def add_field(self, dims, U, csw, bcs=(1, 1, 1, -1), width=0) -> int:
        U = np.ascontiguousarray(U, dtype=np.complex128)
        fid = ctypes.c_int()
        self._check(_lib.dd_server_add_field(self._h, (ctypes.c_int * 4)(*dims), (ctypes.c_int * 4)(*bcs),
                                             _vp(U.ctypes.data), float(csw), int(width), ctypes.byref(fid)))
        self._vol[fid.value] = int(np.prod(dims))
        return fid.value

    def field_info(self, fid):
        w, b = ctypes.c_int(), ctypes.c_size_t()
        self._check(_lib.dd_server_field_info(self._h, int(fid), ctypes.byref(w), ctypes.byref(b)))
        return w.value, b.value

    def submit(self, fid, m0, b, x) -> int:
        """b, x: canonical complex128 device tensors (nrhs, V, 4, 3); kept alive until waited for."""
        nrhs = int(b.shape[0])
        m, mp = _masses(m0, nrhs)
        # the server's streams are not ordered after the caller's: make b and
        # x (e.g. a pending zero fill) ready before handing them over
        torch.cuda.current_stream().synchronize()
        rid = ctypes.c_long()
        self._check(_lib.dd_server_submit(self._h, int(fid), nrhs, mp, _vp(_ptr(b)), _vp(_ptr(x)),
                                          ctypes.byref(rid)))
        self._live[rid.value] = (b, x, nrhs)
        return rid.value

    def poll(self, rid):
        nrhs = self._live[rid][2]
        done = ctypes.c_int()
        infos = (dd_solve_info * nrhs)()
        lat = ctypes.c_double()
        st = _lib.dd_server_poll(self._h, int(rid), ctypes.byref(done), infos, ctypes.byref(lat))
        if not done.value:
            return False, None, None, None
        self._live.pop(rid, None)
        return True, st, [{k: getattr(i, k) for k, _ in dd_solve_info._fields_} for i in infos], lat.value

    def wait(self, rid):
        nrhs = self._live[rid][2]
        infos = (dd_solve_info * nrhs)()
        lat = ctypes.c_double()
        st = _lib.dd_server_wait(self._h, int(rid), infos, ctypes.byref(lat))
        self._live.pop(rid, None)
        return st, [{k: getattr(i, k) for k, _ in dd_solve_info._fields_} for i in infos], lat.value

    def stats(self):
        s = dd_server_stats()
        self._check(_lib.dd_server_get_stats(self._h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in dd_server_stats._fields_}

    def close(self):
        if self._h:
            _lib.dd_server_destroy(self._h)
            self._h = _vp()
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
