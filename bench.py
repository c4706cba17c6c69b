#!/usr/bin/env python3
"""Benchmark: Dslash GB/s against the HBM roofline and time-to-1e-10 of the
SAP-preconditioned FGMRES solve (mixed precision vs FP64) on one MI355X.

Default workload: the 48^3x96 lattice (eps = 0.6, csw = 1, m0 = -0.38), one
Gaussian right-hand side, the red-black SAP smoother (4^4 blocks, 4 MR steps,
10 cycles: the fastest count of a scan on this lattice) with FP16
link/clover/spinor storage and FP32 arithmetic inside
FP64 FGMRES(20), tolerance 1e-10; the FP64 GPU path (the same algorithm with
an FP64 smoother) is timed alongside.  One step = one complete solve: FP64
outer iteration (operator, CGS2 orthogonalisation, reductions, true-residual
restarts) with the smoother -- every stage of the hot path.  Inputs (gauge
field, clover, right-hand side) are resident in HBM before the timed region
starts.

The JSON line reports
  value            algorithmic GB/s of the FP64 Wilson-clover operator launches
                   inside the timed solves (HIP events on the launch stream);
  roofline         the kernel class that dominates the step time, priced with
                   the method's algorithmic count (10,584 flops per site and
                   SAP cycle: four MR steps of 2,184 and a block residual of
                   1,848), the kernel's own count beside it;
  roofline_dslash  the operator itself, against 8 TB/s HBM and against the
                   measured device-copy bandwidth;
  time_to_solution mixed vs the FP64 GPU path (median and min of the repeats);
  cpu_baseline     the FP64 CPU oracle on bounded samples: its operator (same
                   unit as value), one SAP cycle, and a full 8^4 solve.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_VEC_TFLOPS = 78.6         # MI355X vector FP64
# MI355X vector FP32: 256 CU x 4 SIMD x 32 FMA lanes x 2 flop x 2.4 GHz.
# The kernels are built without packed FP32 instructions; on gfx950 a plain
# (VOP2 or VOP3) FP32 FMA, add or multiply still issues once every two cycles
# per wavefront of 64 (measured: 2.3-2.5 cycles per wave instruction per SIMD
# with sixteen independent chains), so this published peak is also theirs.
# DPP moves and mixed-precision FMAs issue every four cycles.
FP32_VEC_TFLOPS = 256 * 4 * 32 * 2 * 2.4e9 / 1e12

WORKLOADS = {
    # name: dims, eps, m0, csw, smoother precision, nrhs, source
    "c2": dict(dims=(32, 32, 32, 64), eps=0.5, m0=-0.35, csw=1.0, sap="f32", nrhs=1, source="gaussian",
               text="32^3x64, random SU(3) eps=0.5, csw=1.0, m0=-0.35, 1 Gaussian RHS, SAP FP32 4^4 blocks "
                    "nmr=4 ncy=12, FGMRES(20) FP64, tol 1e-10"),
    "c1": dict(dims=(8, 8, 8, 8), eps=0.3, m0=-0.2, csw=1.0, sap="f32", nrhs=1, source="gaussian",
               text="8^4, eps=0.3, csw=1.0, m0=-0.2, 1 Gaussian RHS, 4^4 blocks, FGMRES(20), tol 1e-10"),
    "c3": dict(dims=(48, 48, 48, 96), eps=0.6, m0=-0.38, csw=1.0, sap="f16", nrhs=1, source="gaussian", ncy=10,
               text="48^3x96, eps=0.6, m0=-0.38, SAP FP16 storage / FP32 arithmetic, 4^4 blocks nmr=4 ncy=10, "
                    "FGMRES(20) FP64, tol 1e-10"),
    "c4": dict(dims=(32, 32, 32, 64), eps=0.5, m0=-0.35, csw=1.0, sap="f32", nrhs=12, source="point",
               text="32^3x64, 12 point-source RHS (spin x colour), fused multi-RHS SAP FP32, FGMRES(20) FP64 "
                    "per RHS, tol 1e-10"),
}


def log(msg):
    sys.stderr.write(f"[bench] {msg}\n")
    sys.stderr.flush()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--fp64-steps", type=int, default=3, help="FP64-smoother solves timed alongside")
    ap.add_argument("--eo-steps", type=int, default=1,
                    help="solves with the even-odd preconditioned smoother (mixed and FP64) timed alongside")
    ap.add_argument("--amg-steps", type=int, default=2,
                    help="solves with the two-level preconditioner (coarse correction + SAP post-smoothing, after "
                         "a separately timed setup) alongside; 0 skips")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=8.0, help="budget of the oracle operator sample")
    ap.add_argument("--cpu-full", action="store_true",
                    help="also time the oracle operator on the workload lattice, one SAP cycle there and the full "
                         "32^3x64 solve (minutes of host time)")
    ap.add_argument("--serve", action="store_true", help="run the continuous-batching serving workload instead")
    ap.add_argument("--serve-requests", type=int, default=200, help="requests per serving phase")
    ap.add_argument("--serve-budget-gb", type=int, default=200, help="HBM budget of the slot workspaces")
    ap.add_argument("--serve-inflight", type=int, default=16,
                    help="requests outstanding in the saturated phase (36 slots hold about six requests)")
    ap.add_argument("--serve-hold-gb", type=int, default=48,
                    help="device memory for the right-hand sides and solutions of requests in flight")
    ap.add_argument("--serve-fp64-requests", type=int, default=48, help="requests of the FP64-path comparison")
    ap.add_argument("--serve-prec", default="f32", choices=["f32", "f16"],
                    help="storage precision of the serving smoother (FP32 arithmetic either way)")
    ap.add_argument("--no-standalone", action="store_true")
    ap.add_argument("--standalone-only", default="",
                    help="only time the operator alone for these cases (e.g. f64x1,f32x12) on the workload lattice, "
                         "print them as one JSON line and stop (for counter runs of single operator forms)")
    ap.add_argument("--no-sequential", action="store_true",
                    help="multi-RHS workloads: skip the one-at-a-time solves (e.g. for counter runs that should "
                         "see only fused launches)")
    ap.add_argument("--sap-half-fields", action="store_true",
                    help="the FP32 smoother reads FP16 links and clover (dd_set_sap_half_fields)")
    ap.add_argument("--ncy-scan", default="",
                    help="comma-separated SAP cycle counts: time one mixed solve at each (e.g. 2,3,4,6)")
    return ap.parse_args()


def cpu_baseline(seconds, workload=None, full=False):
    """The FP64 oracle on bounded samples, on every host core it is given:
    its operator on the 16^3x32 lattice (the paper's single-chip lattice, the
    workloads' field recipe) in the metric's unit, one SAP cycle (nmr = 4) on
    the same lattice, and the full 8^4 solve (FGMRES(20) with 12 SAP cycles
    per preconditioner call, tol 1e-10).  With full: the operator and one SAP
    cycle on the workload's own lattice, and the complete 32^3x64 solve."""
    import oracle
    from paper_1710_07041_amd import synth
    dims = (16, 16, 16, 32)
    U = synth.random_su3_links(dims, 0.5, seed=0)
    C = oracle.clover_field(dims, U, 1.0)
    psi = synth.gaussian_spinor(dims, seed=1)
    V = synth.volume(dims)
    t0 = time.perf_counter()
    n = 0
    times = []
    while True:
        t1 = time.perf_counter()
        oracle.apply_D(dims, U, C, -0.35, psi)
        times.append(time.perf_counter() - t1)
        n += 1
        if time.perf_counter() - t0 >= seconds and n >= 3:
            break
    dt = float(np.median(times))
    sap = []
    for _ in range(3):
        t1 = time.perf_counter()
        oracle.sap(dims, (4, 4, 4, 4), U, C, -0.35, psi, 1, 4)
        sap.append(time.perf_counter() - t1)
    sap_s = float(np.median(sap))
    # the 8^4 workload, solved completely
    d1 = (8, 8, 8, 8)
    U1 = synth.random_su3_links(d1, 0.3, seed=0)
    C1 = oracle.clover_field(d1, U1, 1.0)
    b1 = synth.gaussian_spinor(d1, seed=0)
    t1 = time.perf_counter()
    _, info1 = oracle.fgmres(d1, (4, 4, 4, 4), U1, C1, -0.2, b1, m=20, tol=1e-10, ncy=12, nmr=4)
    c1_s = time.perf_counter() - t1
    out = {"value": round(V * 192 * 8 / dt / 1e9, 3), "unit": "GB/s", "cores": oracle.num_threads(),
           "kind": "oracle",
           "sample": f"FP64 oracle Wilson-clover operator on a 16^3x32 lattice (eps=0.5, csw=1), median of {n} "
                     f"applications; algorithmic 192 reals/site as on the GPU",
           "ms_per_apply": round(dt * 1e3, 3),
           "gflops_operator": round(1848.0 * V / dt / 1e9, 2),
           "sap_cycle_16x16x16x32_ms": round(sap_s * 1e3, 1),
           "sap_cycle_gflops": round(10584.0 * V / sap_s / 1e9, 2),
           "solve_8x8x8x8": {"time_s": round(c1_s, 3), "iterations": info1["iterations"],
                             "rel_residual": info1["rel_residual"],
                             "params": "FGMRES(20), SAP ncy=12 nmr=4, m0=-0.2, eps=0.3, tol 1e-10"}}
    if full and workload is not None:
        wd = workload["dims"]
        log(f"cpu baseline: the oracle on the workload lattice {wd}")
        Vw = synth.volume(wd)
        Uw = synth.random_su3_links(wd, workload["eps"], seed=0)
        Cw = oracle.clover_field(wd, Uw, workload["csw"])
        pw = synth.gaussian_spinor(wd, seed=1)
        t1 = time.perf_counter()
        oracle.apply_D(wd, Uw, Cw, workload["m0"], pw)
        dw = time.perf_counter() - t1
        t1 = time.perf_counter()
        oracle.sap(wd, (4, 4, 4, 4), Uw, Cw, workload["m0"], pw, 1, 4)
        sw = time.perf_counter() - t1
        out["workload_lattice"] = {"lattice": "x".join(map(str, wd)), "apply_ms": round(dw * 1e3, 1),
                                   "apply_gbs": round(Vw * 192 * 8 / dw / 1e9, 3),
                                   "sap_cycle_ms": round(sw * 1e3, 1)}
        del Uw, Cw, pw
        log(f"cpu baseline: workload lattice apply {dw * 1e3:.0f} ms, one SAP cycle {sw:.1f} s; "
            "now the full 32^3x64 oracle solve")
        d2 = (32, 32, 32, 64)
        U2 = synth.random_su3_links(d2, 0.5, seed=0)
        C2 = oracle.clover_field(d2, U2, 1.0)
        b2 = synth.gaussian_spinor(d2, seed=0)
        t1 = time.perf_counter()
        _, info2 = oracle.fgmres(d2, (4, 4, 4, 4), U2, C2, -0.35, b2, m=20, tol=1e-10, ncy=12, nmr=4)
        out["solve_32x32x32x64"] = {"time_s": round(time.perf_counter() - t1, 2), "iterations": info2["iterations"],
                                    "rel_residual": info2["rel_residual"],
                                    "params": "FGMRES(20), SAP ncy=12 nmr=4, m0=-0.35, eps=0.5, tol 1e-10"}
    return out


def make_rhs(w, V, dims):
    from paper_1710_07041_amd import synth
    if w["source"] == "point":
        return synth.point_sources(dims)
    b = synth.gaussian_spinor(dims, seed=0)
    return b[None] if w["nrhs"] == 1 else np.stack([synth.gaussian_spinor(dims, seed=k) for k in range(w["nrhs"])])


def roofline_entry(name, st, peak_gbs=HBM_PEAK_GBS):
    avg_ms = st["total_ms"] / st["launches"]
    bytes_per = st["bytes"] / st["launches"]
    flops_per = st["flops"] / st["launches"]
    gbs = bytes_per / (avg_ms * 1e-3) / 1e9
    tfl = flops_per / (avg_ms * 1e-3) / 1e12
    return {"kernel": name, "avg_ms": round(avg_ms, 4), "launches": st["launches"], "bytes_per_launch": bytes_per,
            "flops_per_launch": flops_per, "gbs": round(gbs, 1), "tflops": round(tfl, 2),
            "frac_hbm": round(gbs / peak_gbs, 4)}


def dslash_standalone(ctx, dims, reps=20, copy_gbs=None, cases=None):
    """The operator alone in every precision, for one and (up to 32^3x64) for
    12 fused right-hand sides (or the given (precision, nrhs) cases), timed
    with HIP events on the context stream: GB/s vs the roofline (and vs the
    measured copy bandwidth)."""
    import torch
    from paper_1710_07041_amd import synth
    res = {}
    V = synth.volume(dims)
    if cases is None:
        cases = [("f64", 1), ("f32", 1), ("f16", 1)]
        if V <= 32 ** 3 * 64:
            cases += [("f64", 12), ("f32", 12), ("f16", 12)]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(3)
    for prec, n in cases:
        x = torch.randn((n, V, 4, 3), dtype=torch.complex128, device="cuda", generator=gen)
        xb, yb = ctx.empty_blocked(prec, n), ctx.empty_blocked(prec, n)
        ctx.pack(x, xb, prec, n)
        del x
        m0 = np.full(n, -0.35)
        ctx.apply_D(m0, xb, yb, prec, n)
        ctx.profile_enable(True)
        for _ in range(reps):
            ctx.apply_D(m0, xb, yb, prec, n)
        st = ctx.profile_read()
        ctx.profile_enable(False)
        (name, v), = st.items()
        e = roofline_entry(name, v)
        res[f"{prec}_x{n}"] = {"gbs": e["gbs"], "frac": e["frac_hbm"], "avg_ms": e["avg_ms"],
                               "gflops": round(e["tflops"] * 1e3, 1),
                               **({"frac_of_copy": round(e["gbs"] / copy_gbs, 4)} if copy_gbs else {})}
        del xb, yb
        torch.cuda.empty_cache()
    return res


SERVE_FIELDS = [((16, 16, 16, 16), 0.5, 1), ((24, 24, 24, 48), 0.5, 2), ((32, 32, 32, 64), 0.5, 3)]


def serve_main(args):
    """Serving workload: three resident fields (16^4, 24^3x48, 32^3x64), requests on a uniformly chosen
    field with m0 ~ U[-0.38,-0.2] per right-hand side and 1..12 Gaussian right-hand sides, solved to 1e-10.
    First a closed loop that keeps the server saturated (at most --serve-inflight requests outstanding)
    gives the saturation throughput; then Poisson arrivals at 0.5x and 0.9x that request rate give
    p50/p99 latency (overall and per lattice); the plain FP64 GPU path (FP64 smoother) serves a shorter
    saturated run for comparison.  Right-hand sides are generated on the device when a request is
    submitted and freed when it is delivered, so device memory stays bounded."""
    import torch
    from paper_1710_07041_amd import ddsap, synth
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    fields = [(dims, synth.random_su3_links(dims, eps, seed=seed)) for dims, eps, seed in SERVE_FIELDS]
    vols = [synth.volume(dims) for dims, _ in fields]
    names = ["x".join(map(str, dims)) for dims, _ in fields]
    log(f"serving fields generated in {time.perf_counter() - t0:.1f} s")
    gen = torch.Generator(device="cuda")

    def make_server(prec):
        srv = ddsap.Server(hbm_budget_bytes=args.serve_budget_gb * 10 ** 9, max_width=12, use_graphs=1,
                           sap_prec=prec, sap_half_fields=1 if args.sap_half_fields and prec == "f32" else 0)
        fids = [srv.add_field(dims, U, 1.0) for dims, U in fields]
        return srv, fids, [srv.field_info(f)[0] for f in fids]

    def plan(seed, n):
        rng = np.random.default_rng(seed)
        reqs = []
        for k in range(n):
            fi = int(rng.integers(0, len(fields)))
            nrhs = int(rng.integers(1, 13))
            reqs.append((fi, rng.uniform(-0.38, -0.2, size=nrhs), 1000 * seed + k))
        return reqs

    def run(srv, fids, reqs, arrivals=None, inflight=None):
        """Submit reqs at their arrival times (seconds from the start) or, without arrivals, whenever
        fewer than `inflight` are outstanding; deliver completed ones as they finish."""
        out = {}  # rid -> (fi, nrhs, b, x)
        lat, lat_f, res = [], [[] for _ in fields], 0.0
        nrhs_tot = 0

        def deliver(block):
            nonlocal res
            for rid in list(out):
                fi, n, b, x = out[rid]
                if block:
                    st, info, l = srv.wait(rid)
                    done = True
                else:
                    done, st, info, l = srv.poll(rid)
                if not done:
                    continue
                if st != ddsap.DD_OK:
                    raise RuntimeError(f"served solve failed: {ddsap.STATUS_NAMES[st]}")
                lat.append(l)
                lat_f[fi].append(l)
                res = max(res, max(i["rel_residual"] for i in info))
                del out[rid]
                if block:
                    return

        held = lambda: sum(2 * o[1] * vols[o[0]] * 192 for o in out.values())  # bytes of b and x
        capped = 0
        t_start = time.perf_counter()
        for k, (fi, m0, seed) in enumerate(reqs):
            if arrivals is not None:
                while True:
                    deliver(False)
                    dt = t_start + arrivals[k] - time.perf_counter()
                    if dt <= 0:
                        break
                    time.sleep(min(dt, 0.002))
            else:
                deliver(False)
                while len(out) >= inflight:
                    deliver(True)
            if out and held() > args.serve_hold_gb * 10 ** 9:
                capped += 1  # device memory for requests in flight: wait for one to finish
                while out and held() > args.serve_hold_gb * 10 ** 9:
                    deliver(True)
            gen.manual_seed(seed)
            n = len(m0)
            b = torch.randn((n, vols[fi], 4, 3), dtype=torch.complex128, device="cuda", generator=gen)
            x = torch.zeros_like(b)
            out[srv.submit(fids[fi], m0, b, x)] = (fi, n, b, x)
            nrhs_tot += n
        while out:
            deliver(True)
        wall = time.perf_counter() - t_start
        pct = lambda v, q: round(float(np.percentile(v, q)), 2) if v else None
        return {"requests": len(reqs), "rhs": nrhs_tot, "wall_s": round(wall, 3),
                "requests_per_s": round(len(reqs) / wall, 3), "rhs_per_s": round(nrhs_tot / wall, 2),
                "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99), "mean_ms": round(float(np.mean(lat)), 2),
                "per_lattice": {names[f]: {"requests": len(lat_f[f]), "p50_ms": pct(lat_f[f], 50),
                                           "p99_ms": pct(lat_f[f], 99)} for f in range(len(fields))},
                "max_rel_residual": res, "submits_held_for_memory": capped}

    n = args.serve_requests
    srv, fids, widths = make_server(args.serve_prec)
    log(f"mixed server ({args.serve_prec} smoother): slots per field {widths}")
    sat = run(srv, fids, plan(7, n), inflight=args.serve_inflight)
    torch.cuda.empty_cache()
    log(f"saturation: {sat}")
    poisson = {}
    for k, load in enumerate((0.5, 0.9)):
        rate = load * sat["requests_per_s"]
        rng = np.random.default_rng(100 + k)
        arr = np.cumsum(rng.exponential(1.0 / rate, size=n))
        arr -= arr[0]
        poisson[f"{load}x"] = run(srv, fids, plan(8 + k, n), arrivals=list(arr))
        torch.cuda.empty_cache()
        log(f"poisson {load}x: {poisson[f'{load}x']}")
    st = srv.stats()
    srv.close()
    torch.cuda.empty_cache()
    # the plain FP64 GPU path on a shorter saturated run
    srv64, fids64, widths64 = make_server("f64")
    log(f"FP64 server: slots per field {widths64}")
    n64 = max(1, args.serve_fp64_requests)
    sat64 = run(srv64, fids64, plan(7, n64), inflight=args.serve_inflight)
    srv64.close()
    log(f"FP64 saturation: {sat64}")
    out = {
        "metric": "serving: RHS/s at saturation, p50/p99 latency under Poisson load (continuous batching)",
        "value": sat["rhs_per_s"], "unit": "RHS/s", "n_gpus": 1, "steps": n, "warmup": 0,
        "ms_per_step": round(1e3 * sat["wall_s"] / max(sat["requests"], 1), 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": "serving: resident 16^4, 24^3x48, 32^3x64 (eps=0.5, csw=1), m0~U[-0.38,-0.2], "
                               f"1-12 Gaussian RHS per request, SAP {args.serve_prec.upper()} + FGMRES(20) FP64 to 1e-10, "
                               f"{n} requests per phase, HBM budget {args.serve_budget_gb} GB",
                   "slots_per_field": widths, "saturation_inflight": args.serve_inflight,
                   **({"sap_half_fields": True} if args.sap_half_fields else {})},
        "serving": {"saturation": sat, "poisson": poisson, "server_stats": st,
                    "fp64_smoother": {"slots_per_field": widths64, "saturation": sat64,
                                      "mixed_over_fp64_rhs_per_s": round(sat["rhs_per_s"] / sat64["rhs_per_s"], 3)}},
    }
    print(json.dumps(out))


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the solver does not shard a lattice "
              "across GPUs (the domain decomposition over several GPUs is designed, not implemented)",
              file=sys.stderr)
        sys.exit(2)
    if args.serve:
        serve_main(args)
        return

    import torch
    from paper_1710_07041_amd import ddsap, synth

    w = WORKLOADS[args.workload]
    dims, nrhs = w["dims"], w["nrhs"]
    V = synth.volume(dims)
    torch.cuda.set_device(0)
    log(f"workload {args.workload}: {w['text']}")
    t0 = time.perf_counter()
    U = synth.random_su3_links(dims, w["eps"], seed=0)
    b = make_rhs(w, V, dims)
    log(f"fields generated in {time.perf_counter() - t0:.1f} s")
    ctx = ddsap.Context(dims, (1, 1, 1, -1))
    ctx.set_gauge(U, w["csw"])
    compressed = ctx.link_compression  # SU(3) links: two rows stored per link are read
    if args.sap_half_fields:
        ctx.set_sap_half_fields(True)
    del U
    bd = torch.from_numpy(np.ascontiguousarray(b)).to("cuda")
    xd = torch.zeros_like(bd)
    m0 = np.full(nrhs, w["m0"])

    def params(sap, eo=False, ncy=None, amg=False):
        p = ddsap.default_params()
        p.sap_prec = ddsap.PREC[sap]
        p.sap_eo = int(eo)
        p.amg = int(amg)
        # SAP cycles per preconditioner call: the count under test in a scan,
        # else the workload's own (picked by such a scan; library default 12)
        p.ncy = ncy if ncy is not None else w.get("ncy", p.ncy)
        return p

    def one_solve(sap, eo=False, ncy=None, amg=False):
        xd.zero_()
        st, info = ctx.solve(m0, bd, xd, nrhs, params(sap, eo, ncy, amg), raise_on_fail=False)
        if st != ddsap.DD_OK:
            raise RuntimeError(f"solve failed: {ddsap.STATUS_NAMES[st]} {info}")
        return info

    # a plain 1 GiB device copy (torch's): the reference a counter run scales
    # FETCH/WRITE by; and the achievable-bandwidth line, the library's own
    # streaming copy of 4 GiB (8 GiB moved per copy; median of 10)
    ca = torch.ones(256 << 20, dtype=torch.float32, device="cuda")
    cb = torch.empty_like(ca)
    cb.copy_(ca)
    del ca, cb
    sa = torch.ones(1 << 30, dtype=torch.float32, device="cuda")
    sb = torch.empty_like(sa)
    ddsap.stream_copy(sa, sb, sa.numel() * 4)
    torch.cuda.synchronize()
    ct = []
    for _ in range(10):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ddsap.stream_copy(sa, sb, sa.numel() * 4)
        e1.record()
        e1.synchronize()
        ct.append(e0.elapsed_time(e1) * 1e-3)
    copy_gbs = 2.0 * sa.numel() * 4 / float(np.median(ct)) / 1e9
    del sa, sb
    torch.cuda.empty_cache()
    log(f"streaming copy: {copy_gbs:.0f} GB/s")

    if args.standalone_only:
        cases = [(c.split("x")[0], int(c.split("x")[1])) for c in args.standalone_only.split(",")]
        res = dslash_standalone(ctx, dims, copy_gbs=copy_gbs, cases=cases)
        print(json.dumps({"workload": w["text"], "hbm_copy_gbs": round(copy_gbs, 1), "operator_alone": res}))
        return

    for i in range(args.warmup):
        info = one_solve(w["sap"])
        log(f"warmup {i}: {info[0]['iterations']} iterations, residual {info[0]['rel_residual']:.2e}")

    ctx.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos, tsteps = [], []
    for i in range(args.steps):
        t1 = time.perf_counter()
        infos.append(one_solve(w["sap"]))  # dd_solve synchronises
        tsteps.append(time.perf_counter() - t1)
        log(f"step {i}: {infos[-1][0]['iterations']} iterations, residual {infos[-1][0]['rel_residual']:.2e}")
    torch.cuda.synchronize()
    t_mixed = (time.perf_counter() - t0) / args.steps
    prof = ctx.profile_read()
    ctx.profile_enable(False)

    # FP64 GPU path (FP64 smoother), same algorithm, timed alongside
    t64 = None
    info64 = None
    t64s = []
    if args.fp64_steps > 0:
        one_solve("f64")
        torch.cuda.synchronize()
        for i in range(args.fp64_steps):
            t1 = time.perf_counter()
            info64 = one_solve("f64")
            t64s.append(time.perf_counter() - t1)
        t64 = float(np.median(t64s))
        log(f"fp64 path: {info64[0]['iterations']} iterations, median {t64 * 1e3:.1f} ms of {len(t64s)}")

    # the even-odd preconditioned smoother (a refinement beyond the paper's
    # plain block MR), mixed and FP64, timed alongside
    even_odd = None
    if args.eo_steps > 0:
        even_odd = {}
        for sap in (w["sap"], "f64"):
            one_solve(sap, eo=True)
            ctx.profile_enable(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(args.eo_steps):
                info_eo = one_solve(sap, eo=True)
            torch.cuda.synchronize()
            t_eo = (time.perf_counter() - t0) / args.eo_steps
            prof_eo = ctx.profile_read()
            ctx.profile_enable(False)
            cls = f"sap_sweep_eo_{sap}"
            sweep = prof_eo.get(cls)
            even_odd["mixed" if sap != "f64" else "fp64"] = {
                "time_s": round(t_eo, 4), "iterations": info_eo[0]["iterations"],
                "rel_residual": max(i["rel_residual"] for i in info_eo),
                "sweep_avg_ms": None if not sweep else round(sweep["total_ms"] / sweep["launches"], 4)}
            log(f"even-odd smoother {sap}: {info_eo[0]['iterations']} iterations, {t_eo * 1e3:.1f} ms")
        even_odd["mixed_speedup_over_plain"] = round(t_mixed / even_odd["mixed"]["time_s"], 3)

    # the two-level method: the coarse correction of DD-alpha-AMG over the
    # Schwarz smoother (FP32 post-smoothing for the FP32/FP16 workloads)
    two_level = None
    if args.amg_steps > 0:
        apar = ddsap.default_amg_params()
        gen = torch.Generator(device="cuda")
        gen.manual_seed(11)
        v0 = torch.randn((apar.nvec, V, 4, 3), dtype=torch.complex128, device="cuda", generator=gen)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.amg_setup(w["m0"], v0, apar)
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        del v0
        torch.cuda.empty_cache()
        sap_tl = "f64" if w["sap"] == "f64" else "f32"
        one_solve(sap_tl, amg=True)
        ctx.profile_enable(True)
        ttl = []
        for i in range(args.amg_steps):
            t1 = time.perf_counter()
            info_tl = one_solve(sap_tl, amg=True)
            ttl.append(time.perf_counter() - t1)
        prof_tl = ctx.profile_read()
        ctx.profile_enable(False)
        two_level = {
            "setup_s": round(t_setup, 3), "time_s": round(float(np.median(ttl)), 4), "time_min_s": round(min(ttl), 4),
            "repeats": len(ttl), "iterations": info_tl[0]["iterations"],
            "rel_residual": max(i["rel_residual"] for i in info_tl), "smoother": sap_tl,
            "speedup_over_sap_only": round(float(np.median(tsteps)) / float(np.median(ttl)), 3),
            "params": {f: getattr(apar, f) for f, _ in apar._fields_},
            "kernels_ms_per_solve": {k: round(v["total_ms"] / len(ttl), 3)
                                     for k, v in sorted(prof_tl.items(), key=lambda kv: -kv[1]["total_ms"])[:8]}}
        log(f"two-level: setup {t_setup:.2f} s, {info_tl[0]['iterations']} iterations, "
            f"{float(np.median(ttl)) * 1e3:.1f} ms")

    # sensitivity of the mixed solve to the SAP cycles per preconditioner call
    # (the paper leaves the count open; 12 is the default)
    ncy_scan = None
    if args.ncy_scan:
        ncy_scan = {}
        for k in [int(v) for v in args.ncy_scan.split(",") if v.strip()]:
            one_solve(w["sap"], ncy=k)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info_k = one_solve(w["sap"], ncy=k)
            torch.cuda.synchronize()
            t_k = time.perf_counter() - t0
            ncy_scan[str(k)] = {"time_s": round(t_k, 4), "iterations": info_k[0]["iterations"],
                                "rel_residual": max(i["rel_residual"] for i in info_k)}
            log(f"ncy={k}: {info_k[0]['iterations']} iterations, {t_k * 1e3:.1f} ms")

    # multi-RHS: the same right-hand sides solved one at a time, for the fusion gain
    sequential = None
    if nrhs > 1 and not args.no_sequential:
        bs = [bd[r:r + 1].clone() for r in range(nrhs)]
        xs = torch.zeros_like(bs[0])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for r in range(nrhs):
            xs.zero_()
            st, _ = ctx.solve(m0[r:r + 1], bs[r], xs, 1, params(w["sap"]), raise_on_fail=False)
        torch.cuda.synchronize()
        sequential = time.perf_counter() - t0
        del bs, xs
        log(f"{nrhs} right-hand sides one at a time: {sequential * 1e3:.1f} ms")

    standalone = None if args.no_standalone else dslash_standalone(ctx, dims, copy_gbs=copy_gbs)
    log(f"operator alone: {standalone}")

    # operator launches inside the timed solves
    dsl = {k: v for k, v in prof.items() if k in ("dslash_f64", "dslash_f32in_f64")}
    d_bytes = sum(v["bytes"] for v in dsl.values())
    d_ms = sum(v["total_ms"] for v in dsl.values())
    d_launch = sum(v["launches"] for v in dsl.values())
    dslash_gbs = d_bytes / (d_ms * 1e-3) / 1e9
    main_cls = max(dsl, key=lambda k: dsl[k]["total_ms"])
    rd = roofline_entry(main_cls, dsl[main_cls])

    total_ms = sum(v["total_ms"] for v in prof.values())
    dom = max(prof, key=lambda k: prof[k]["total_ms"])
    rdom = roofline_entry(dom, prof[dom])
    if dom.startswith("sap"):
        # smoother: arithmetic intensity above the FP32 ridge -> priced against
        # the vector ALU peak.  Algorithmic work per launch: the method's
        # count, 10,584 flops per site and SAP cycle (four MR steps of 2,184
        # and the block residual of 1,848), times the V/2 sites x nrhs one
        # colour sweep covers; the kernel's own count (the carried residual
        # needs no residual application) beside it.
        nmr = ddsap.default_params().nmr
        alg_flops = V / 2 * nrhs * (nmr * 2184.0 + 1848.0)
        alg_tf = alg_flops / (rdom["avg_ms"] * 1e-3) / 1e12
        peak = FP32_VEC_TFLOPS if not dom.endswith("f64") else FP64_VEC_TFLOPS
        roof = {"bound": "alu", "kernel": dom, "achieved": round(alg_tf, 2), "peak": round(peak, 1),
                "unit": "TFLOP/s", "frac": round(alg_tf / peak, 4), "traffic": None,
                "flops_per_launch": alg_flops, "flop_count": "10584 per site and SAP cycle (nmr=4)",
                "achieved_kernel_count": rdom["tflops"], "frac_kernel_count": round(rdom["tflops"] / peak, 4),
                "kernel_flops_per_launch": rdom["flops_per_launch"],
                "hbm_gbs": rdom["gbs"], "hbm_frac": rdom["frac_hbm"], "avg_ms": rdom["avg_ms"],
                "launches": rdom["launches"]}
        # a visit's memory phase (fields, psi, residual and faces in and out)
        # and its MR steps follow each other in a workgroup and, measured, do
        # not overlap across the workgroups of a CU: the sum of the HBM time
        # of the algorithmic bytes and the ALU time of the algorithmic flops
        # is the floor of this structure
        add_ms = (prof[dom]["bytes"] / prof[dom]["launches"] / (HBM_PEAK_GBS * 1e9)
                  + alg_flops / (peak * 1e12)) * 1e3
        roof["additive_bound_ms"] = round(add_ms, 4)
        roof["frac_additive"] = round(add_ms / rdom["avg_ms"], 4)
    else:
        roof = {"bound": "hbm", "kernel": dom, "achieved": rdom["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": rdom["frac_hbm"], "traffic": None, "avg_ms": rdom["avg_ms"]}

    # measured HBM traffic per launch (rocprofv3 FETCH_SIZE / WRITE_SIZE runs of
    # this workload, copy-calibrated), valid only for the kernel sources it was taken on
    traffic = {}
    try:
        from paper_1710_07041_amd import traffic as tmod
        rec = json.load(open(os.path.join(ROOT, "profiles", f"traffic_{args.workload}.json")))
        if rec.get("source_digest") == tmod.source_digest():
            traffic = {k: v["traffic_bytes"] for k, v in rec["kernels"].items()}
    except (OSError, ValueError, KeyError):
        traffic = {}
    roof["traffic"] = traffic.get(roof["kernel"])
    if roof["traffic"]:
        roof["traffic_over_algorithmic"] = round(roof["traffic"] / prof[dom]["bytes"] * prof[dom]["launches"], 3)

    breakdown = {k: {"launches": v["launches"], "ms_per_step": round(v["total_ms"] / args.steps, 3),
                     "share": round(v["total_ms"] / total_ms, 4),
                     "gbs": round(v["bytes"] / (v["total_ms"] * 1e-3) / 1e9, 1) if v["total_ms"] > 0 else None}
                 for k, v in sorted(prof.items(), key=lambda kv: -kv[1]["total_ms"])}

    cpu = None if args.no_cpu_baseline else cpu_baseline(args.cpu_seconds, w, args.cpu_full)

    out = {
        "metric": "Dslash GB/s & % HBM roofline; time-to-1e-10 SAP-FGMRES solve (mixed vs FP64)",
        "value": round(dslash_gbs, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_mixed * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic (seeded random SU(3) links, Gaussian right-hand sides)",
        "config": {"workload": w["text"] + ("; the FP64 GPU path (FP64 smoother, same parameters) timed alongside"
                                            if args.fp64_steps > 0 else ""),
                   "sap_cycles": params(w["sap"]).ncy,
                   "lattice": "x".join(map(str, dims)), "nrhs": nrhs,
                   "smoother": w["sap"], "parallelism": "single GPU", "link_compression": compressed,
                   **({"sap_half_fields": True} if args.sap_half_fields else {})},
        "hbm_copy_gbs": round(copy_gbs, 1),
        "roofline": roof,
        "roofline_dslash": {"bound": "hbm", "kernel": main_cls, "achieved": rd["gbs"], "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": rd["frac_hbm"], "frac_of_copy": round(rd["gbs"] / copy_gbs, 4),
                            "traffic": traffic.get(main_cls),
                            "avg_ms": rd["avg_ms"], "bytes_per_launch": rd["bytes_per_launch"],
                            # with gauge compression the kernel reads 48 of the 72 link reals per site
                            # that the algorithmic figure counts
                            "format_bytes_per_launch": rd["bytes_per_launch"] - (24 * 8 * V if compressed else 0)},
        "dslash_frac_hbm": round(dslash_gbs / HBM_PEAK_GBS, 4),
        "dslash_standalone": standalone,
        "time_to_solution_s": {"mixed": round(float(np.median(tsteps)), 4), "mixed_min": round(min(tsteps), 4),
                               "mixed_repeats": len(tsteps),
                               "fp64": None if t64 is None else round(t64, 4),
                               "fp64_min": None if t64 is None else round(min(t64s), 4),
                               "fp64_repeats": len(t64s),
                               "fp64_over_mixed": None if t64 is None else round(t64 / float(np.median(tsteps)), 3)},
        "multi_rhs": None if sequential is None else {
            "nrhs": nrhs, "fused_s": round(t_mixed, 4), "one_at_a_time_s": round(sequential, 4),
            "speedup": round(sequential / t_mixed, 3)},
        "iterations": {"mixed": infos[-1][0]["iterations"],
                       "fp64": None if info64 is None else info64[0]["iterations"]},
        "even_odd": even_odd,
        "two_level": two_level,
        **({"ncy_sensitivity": ncy_scan} if ncy_scan else {}),
        "final_rel_residual": max(i["rel_residual"] for i in infos[-1]),
        "kernels": breakdown,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
