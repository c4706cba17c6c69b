"""CPU test of the serving scheduler's bookkeeping (the FIFO of requests, the
admission of right-hand sides into the free slots of their field's executor,
completion accounting and latency statistics) with the oracle's FGMRES as a
fake executor in place of the GPU slot engines.  The same header drives the
server; this test needs no GPU.

The executor holds each slot for as many scheduler steps as the oracle's solve
took Arnoldi steps, so right-hand sides of different masses finish out of
order and later ones take over the slots that free up.  Checked: every
right-hand side admitted exactly once, on its own field, never before its
request arrived, into a slot nobody holds; per field, admission in arrival
order (FIFO, no overtaking); no slot left idle while a right-hand side of its
field waits; every solution solves its own system (a mix-up of field, mass or
right-hand side fails the residual check); latencies and their quantiles; a
fatal error completing every outstanding request with the error code."""
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_1710_07041_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DIMS = (4, 4, 4, 8)
V = int(np.prod(DIMS))
WIDTH = 3
DD_HIP_ERROR = 3  # dd_status value of a failed HIP call (ddsap.h)
FIELDS = [(0.4, 21, 1.0), (0.3, 22, 1.2)]  # (gauge disorder, seed, c_sw)
# (field, right-hand sides, arrival step): more right-hand sides per field
# than slots, arrivals while earlier requests run
REQUESTS = [(0, 2, 0), (1, 1, 0), (0, 3, 0), (0, 1, 0), (1, 4, 1), (0, 2, 4), (1, 1, 6), (1, 2, 6), (0, 1, 9)]


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    lib = oracle.build()
    out = tmp_path_factory.mktemp("serve_core") / "serve_core_test"
    subprocess.run(["g++", "-O2", "-std=c++17", "-Wall", "-Werror", "-pthread",
                    os.path.join(ROOT, "tests", "serve_core_test.cpp"), "-o", str(out),
                    "-L", str(lib.parent), "-loracle", "-Wl,-rpath," + str(lib.parent)], check=True)
    return out


@pytest.fixture(scope="module")
def world():
    Us, Cs = [], []
    for eps, seed, csw in FIELDS:
        U = synth.random_su3_links(DIMS, eps, seed=seed)
        Us.append(U)
        Cs.append(oracle.clover_field(DIMS, U, csw))
    rng = np.random.default_rng(5)
    bs, m0s = [], []
    for k, (_, n, _) in enumerate(REQUESTS):
        bs.append(synth.gaussian_spinor(DIMS, nrhs=n, seed=300 + k).reshape(n, V, 4, 3))
        m0s.append(rng.uniform(-0.3, 0.3, size=n))
    return Us, Cs, bs, m0s


def run(exe, world, tmp, mode, fail=(-1, -1)):
    Us, _, bs, m0s = world
    with open(tmp / "spec.txt", "w") as f:
        f.write("%d %d %d %d %d %d %d %d %d\n" % (*DIMS, len(FIELDS), WIDTH, len(REQUESTS), *fail))
        f.write(" ".join(str(c) for _, _, c in FIELDS) + "\n")
        for fi, n, st in REQUESTS:
            f.write("%d %d %d\n" % (fi, n, st))
    np.concatenate([np.ascontiguousarray(U, np.complex128).ravel() for U in Us]).tofile(tmp / "U.bin")
    np.concatenate([b.ravel() for b in bs]).astype(np.complex128).tofile(tmp / "b.bin")
    np.concatenate(m0s).astype(np.float64).tofile(tmp / "m0.bin")
    env = dict(os.environ, OMP_NUM_THREADS="1")
    p = subprocess.run([str(exe), str(tmp), mode], capture_output=True, text=True, env=env, timeout=300)
    assert p.returncode == 0, p.stderr
    ev = [ln.split() for ln in p.stdout.splitlines()]
    x = np.fromfile(tmp / "x.bin", np.complex128) if (tmp / "x.bin").exists() else None
    return ev, x


def check_slots(ev):
    """Replay admissions and completions per field: a slot is taken only when
    free and released by the right-hand side that holds it; every admission
    pass leaves no slot idle while a right-hand side of its field waits."""
    held = {}
    admitted = {}
    for e in ev:
        if e[0] == "admit":
            step, fi, slot, req, rhs = map(int, e[1:])
            assert (fi, slot) not in held, "slot taken twice"
            held[(fi, slot)] = (req, rhs)
            assert (req, rhs) not in admitted, "right-hand side admitted twice"
            admitted[(req, rhs)] = (step, fi)
        elif e[0] == "done":
            step, fi, slot, req, rhs, _ = map(int, e[1:])
            assert held.pop((fi, slot)) == (req, rhs)
        elif e[0] == "pass":
            _, _, nfree, waiting = map(int, e[1:])
            assert nfree == 0 or waiting == 0, "a slot idles while work waits"
    return admitted


def check_fifo(ev):
    per_field = {}
    for e in ev:
        if e[0] == "admit":
            fi, req, rhs = int(e[2]), int(e[4]), int(e[5])
            per_field.setdefault(fi, []).append((req, rhs))
    for fi, seq in per_field.items():
        assert seq == sorted(seq), "field %d admitted out of arrival order" % fi


def check_solutions(world, x, statuses):
    Us, Cs, bs, m0s = world
    x = x.reshape(-1, V, 4, 3)
    o = 0
    for k, (fi, n, _) in enumerate(REQUESTS):
        for j in range(n):
            if statuses[k] == 0:
                r = bs[k][j] - oracle.apply_D(DIMS, Us[fi], Cs[fi], m0s[k][j], x[o + j])
                assert np.linalg.norm(r) / np.linalg.norm(bs[k][j]) <= 1e-9, (k, j)
        o += n


def completes(ev):
    return {int(e[1]): (int(e[2]), float(e[3]), [int(v) for v in e[4:]]) for e in ev if e[0] == "complete"}


def test_steps_fifo_slots_results_latency(exe, world, tmp_path):
    ev, x = run(exe, world, tmp_path, "steps")
    admitted = check_slots(ev)
    check_fifo(ev)
    assert set(admitted) == {(k + 1, j) for k, (_, n, _) in enumerate(REQUESTS) for j in range(n)}
    for (req, rhs), (step, fi) in admitted.items():
        assert fi == REQUESTS[req - 1][0]
        assert step >= REQUESTS[req - 1][2], "admitted before it arrived"
    # a slot is held for exactly the solve's Arnoldi steps
    for e in ev:
        if e[0] == "done":
            step, req, rhs, iters = int(e[1]), int(e[4]), int(e[5]), int(e[6])
            assert step - admitted[(req, rhs)][0] == iters - 1
    # right-hand sides of one field finish out of admission order somewhere
    done_seq = [(int(e[4]), int(e[5])) for e in ev if e[0] == "done"]
    assert done_seq != sorted(done_seq)
    comp = completes(ev)
    assert sorted(comp) == list(range(1, len(REQUESTS) + 1))
    last_done = {}
    for e in ev:
        if e[0] == "done":
            last_done[int(e[4])] = int(e[1])
    lat = []
    for req, (st, ms, iters) in comp.items():
        assert st == 0
        assert len(iters) == REQUESTS[req - 1][1] and min(iters) > 0
        assert ms == pytest.approx(1e3 * (last_done[req] - REQUESTS[req - 1][2]))
        lat.append(ms)
    check_solutions(world, x, [0] * len(REQUESTS))
    stats = [e for e in ev if e[0] == "stats"][0]
    p50, p99, rhs_done, iters = float(stats[1]), float(stats[2]), int(stats[3]), int(stats[4])
    # completion order is the order the latencies were recorded in; the
    # quantiles do not depend on it
    assert p50 == pytest.approx(np.percentile(lat, 50), abs=1e-6)
    assert p99 == pytest.approx(np.percentile(lat, 99), abs=1e-6)
    assert rhs_done == sum(n for _, n, _ in REQUESTS)
    assert iters == sum(sum(v[2]) for v in comp.values())


def test_threads_results(exe, world, tmp_path):
    """One worker thread per field and a submitting thread, as in the server."""
    ev, x = run(exe, world, tmp_path, "threads")
    admitted = check_slots(ev)
    check_fifo(ev)
    assert len(admitted) == sum(n for _, n, _ in REQUESTS)
    for (req, _), (_, fi) in admitted.items():
        assert fi == REQUESTS[req - 1][0]
    comp = completes(ev)
    assert all(st == 0 for st, _, _ in comp.values())
    check_solutions(world, x, [0] * len(REQUESTS))


def test_fatal_error_completes_everything(exe, world, tmp_path):
    """Field 1's executor fails at step 40, after every arrival, with some
    requests of both fields finished and others running or queued: the
    finished ones keep their results, every other one completes with the
    error code."""
    ev, x = run(exe, world, tmp_path, "steps", fail=(1, 40))
    comp = completes(ev)
    assert sorted(comp) == list(range(1, len(REQUESTS) + 1))
    finished = {}
    for e in ev:
        if e[0] == "done":
            finished[int(e[4])] = finished.get(int(e[4]), 0) + 1
    statuses = []
    for req, (st, _, _) in sorted(comp.items()):
        whole = finished.get(req, 0) == REQUESTS[req - 1][1]
        assert st == (0 if whole else DD_HIP_ERROR)
        statuses.append(st)
    assert 0 in statuses and DD_HIP_ERROR in statuses
    check_solutions(world, x, statuses)
