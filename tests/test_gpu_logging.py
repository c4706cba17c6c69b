"""DDSAP_LOG: the library prints nothing by default; with DDSAP_LOG=1 a solve
writes its summary and a failed call its message to stderr.  Each case runs
in a fresh process (the level is read once per process)."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SCRIPT = r"""
import sys
sys.path.insert(0, ROOT)
import numpy as np
import torch
from paper_1710_07041_amd import ddsap, synth
dims = (8, 8, 8, 8)
ctx = ddsap.Context(dims, (1, 1, 1, -1))
ctx.set_gauge(synth.random_su3_links(dims, 0.3, seed=0), 1.0)
b = torch.from_numpy(synth.gaussian_spinor(dims, seed=1)[None]).to("cuda")
x = torch.zeros_like(b)
st, info = ctx.solve(-0.2, b, x, 1)
assert st == 0
p = ddsap.default_params()
p.m = 0
st, _ = ctx.solve(-0.2, b, x, 1, p, raise_on_fail=False)
assert st == ddsap.DD_INVALID_ARG
print("ok")
""".replace("ROOT", repr(ROOT))


def run(level):
    env = dict(os.environ)
    env.pop("DDSAP_LOG", None)
    if level is not None:
        env["DDSAP_LOG"] = str(level)
    return subprocess.run([sys.executable, "-c", SCRIPT], capture_output=True, text=True, env=env, timeout=300)


def test_silent_by_default():
    p = run(None)
    assert p.returncode == 0, p.stderr
    assert "[ddsap]" not in p.stderr


def test_log_level_one():
    p = run(1)
    assert p.returncode == 0, p.stderr
    lines = [ln for ln in p.stderr.splitlines() if ln.startswith("[ddsap]")]
    assert any("dd_solve: 1 right-hand side(s), status 0" in ln for ln in lines), lines
    assert any("rhs 0: status 0" in ln and "iterations" in ln for ln in lines), lines
    assert any(ln.startswith("[ddsap] error 1:") and "dd_solve" in ln for ln in lines), lines
