"""GPU tests of the continuous-batching server: requests on several resident
fields, more right-hand sides than slots (so later ones are admitted while
earlier ones run), every result checked against the oracle residual and
against the same solve done alone."""
import time

import numpy as np
import pytest

import oracle
from gpu_util import BC, rel, to_dev, to_host
from paper_1710_07041_amd import synth

pytestmark = pytest.mark.gpu

FIELDS = [((8, 8, 8, 8), 0.3, 11), ((4, 4, 8, 8), 0.4, 12)]


@pytest.fixture(scope="module")
def fields():
    out = []
    for dims, eps, seed in FIELDS:
        U = synth.random_su3_links(dims, eps, seed=seed)
        out.append((dims, U, oracle.clover_field(dims, U, 1.0)))
    return out


def solo(dims, U, m0, b, sap="f32", eo=0, half=0):
    import torch
    from paper_1710_07041_amd import ddsap
    ctx = ddsap.Context(dims, BC)
    ctx.set_gauge(U, 1.0)
    ctx.set_sap_half_fields(bool(half))
    bd = to_dev(b)
    xd = torch.zeros_like(bd)
    p = ddsap.default_params()
    p.sap_prec = ddsap.PREC[sap]
    p.sap_eo = eo
    st, info = ctx.solve(m0, bd, xd, b.shape[0], p)
    ctx.close()
    return to_host(xd)


def make_requests(fields, n, seed=0):
    rng = np.random.default_rng(seed)
    reqs = []
    for k in range(n):
        fi = int(rng.integers(0, len(fields)))
        dims = fields[fi][0]
        nrhs = int(rng.integers(1, 4))
        m0 = rng.uniform(-0.3, -0.1, size=nrhs)
        b = synth.gaussian_spinor(dims, nrhs=nrhs, seed=100 + k)
        reqs.append((fi, m0, b))
    return reqs


@pytest.mark.parametrize("graphs,eo,half,sap", [(1, 0, 0, "f32"), (0, 0, 0, "f32"), (1, 1, 0, "f32"),
                                                  (1, 0, 1, "f32"), (1, 0, 0, "f16"), (1, 0, 0, "f64")],
                         ids=["graphs", "nographs", "graphs-evenodd", "graphs-halffields", "graphs-fp16",
                              "graphs-fp64"])
def test_serve_mix_equals_alone(fields, graphs, eo, half, sap):
    import torch
    from paper_1710_07041_amd import ddsap
    srv = ddsap.Server(max_width=3, use_graphs=graphs, hbm_budget_bytes=8 << 30, sap_eo=eo, sap_half_fields=half,
                       sap_prec=sap)
    fids = [srv.add_field(dims, U, 1.0, BC) for dims, U, _ in fields]
    for f in fids:
        assert srv.field_info(f)[0] == 3
    reqs = make_requests(fields, 7)
    handles = []
    for k, (fi, m0, b) in enumerate(reqs):
        bd = to_dev(b)
        xd = torch.zeros_like(bd)
        handles.append((srv.submit(fids[fi], m0, bd, xd), xd))
        if k == 3:
            time.sleep(0.05)  # later requests arrive while the first ones run
    results = []
    for (rid, xd) in handles:
        st, info, lat = srv.wait(rid)
        assert st == ddsap.DD_OK, info
        assert lat > 0
        results.append(to_host(xd))
    stats = srv.stats()
    srv.close()
    assert stats["requests_done"] == len(reqs)
    assert stats["rhs_done"] == sum(b.shape[0] for _, _, b in reqs)
    assert stats["p99_ms"] >= stats["p50_ms"] > 0
    for (fi, m0, b), x in zip(reqs, results):
        dims, U, C = fields[fi]
        for r in range(b.shape[0]):
            res = b[r] - oracle.apply_D(dims, U, C, m0[r], x[r], BC)
            assert np.linalg.norm(res) / np.linalg.norm(b[r]) <= 1e-10
        xs = solo(dims, U, m0, b, sap=sap, eo=eo, half=half)
        assert rel(x, xs) <= 1e-8


def test_serve_budget_and_errors(fields):
    from paper_1710_07041_amd import ddsap
    dims, U, _ = fields[0]
    srv = ddsap.Server(max_width=4, hbm_budget_bytes=1 << 20)  # 1 MiB: no slot fits
    with pytest.raises(ddsap.DDError) as e:
        srv.add_field(dims, U, 1.0, BC)
    assert e.value.status == ddsap.DD_OOM
    srv.close()
    srv = ddsap.Server(max_width=16, hbm_budget_bytes=64 << 20)  # budget caps the slot pool
    fid = srv.add_field(dims, U, 1.0, BC)
    w, nbytes = srv.field_info(fid)
    assert 1 <= w < 16 and nbytes <= 64 << 20
    srv.close()
