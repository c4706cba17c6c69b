"""The C-ABI library loads and exports every entry point include/ddsap.h declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1710_07041_amd", "libddsap.so")
HDR = os.path.join(ROOT, "include", "ddsap.h")


def declared_symbols():
    text = open(HDR).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dd_[A-Za-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1710_07041_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ["dd_create", "dd_set_gauge", "dd_apply_D", "dd_apply_D_block", "dd_sap", "dd_solve"]:
        assert name in syms


def test_every_declared_symbol_is_exported(lib):
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_lists_every_export():
    from paper_1710_07041_amd import ddsap
    assert sorted(ddsap.EXPORTS) == [s for s in declared_symbols() if s in ddsap.EXPORTS]
    assert set(declared_symbols()) <= set(ddsap.EXPORTS) | {s for s in declared_symbols() if s.startswith("dd_server")}


def test_abi_version_and_defaults(lib):
    from paper_1710_07041_amd import ddsap
    assert ddsap.abi_version() == 6
    p = ddsap.default_params()
    assert (p.m, p.tol, p.max_restarts, p.ncy, p.nmr, p.sap_prec, p.sap_eo) == (20, 1e-10, 100, 12, 4, ddsap.DD_F32, 0)
    c = ddsap.default_server_config()
    assert (c.sap_prec, c.use_graphs, c.sap_eo, c.ncy, c.nmr, c.sap_half_fields) == (ddsap.DD_F32, 1, 0, 12, 4, 0)
    a = ddsap.default_amg_params()
    assert (a.nvec, a.setup_iters, a.setup_ncy, a.setup_nmr, a.setup_prec, a.adapt, a.coarse_k, a.post_ncy,
            a.post_nmr) == (12, 6, 4, 4, ddsap.DD_F32, 2, 16, 8, 4)
    assert p.amg == 0
