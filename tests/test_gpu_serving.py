"""Serving loop on the GPU: results against the FP64 oracle, bitwise equality
alone vs in a mix, admission by HBM budget, cancellation, and an injected
launch fault that fails only the requests of the affected round."""
import os
import subprocess
import sys
import time

import numpy as np
import pytest

import oracle
import workloads as W
from tests.conftest import ROOT

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qs():
    import paper_2506_09198_amd as qs

    assert qs.qs_device_count() >= 1
    return qs


def _drain(qs, srv, ids, timeout=60.0, done=None):
    done = {} if done is None else done
    t_end = time.time() + timeout
    while len(done) < len(ids):
        for r in qs.qs_server_poll(srv):
            done[r["id"]] = r
        assert time.time() < t_end, f"serving did not finish: {len(done)}/{len(ids)}"
        time.sleep(0.0002)
    return done


def _mix(seed, ns=(4, 8, 11, 12, 13, 14, 16, 17, 18)):
    rng = np.random.default_rng(seed)
    out = []
    for n in ns:
        k = int(rng.integers(3))
        if k == 0:
            out.append(W.rqc_chain(n, int(rng.integers(2, 7)), int(rng.integers(100))))
        elif k == 1:
            out.append(W.qft(n, int(rng.integers(1 << n))))
        else:
            out.append(W.grover(n, int(rng.integers(1 << n))))
    return out


def _check(got, want, dt, what):
    got = got.astype(np.complex128)
    err = float(np.max(np.abs(got - want)))
    if dt == 2:
        assert err <= 1e-12, f"{what}: {err:.3e}"
    else:
        fid = abs(np.vdot(want, got)) ** 2
        assert fid >= 1 - 1e-6 and err <= 2e-5, f"{what}: fidelity {fid} err {err:.3e}"


@pytest.mark.parametrize("dt", [2, 1])
def test_server_results_match_oracle(qs, dt):
    srv = qs.qs_server_create(dtype=dt, hbm_budget=1 << 30)
    try:
        circs = _mix(1)
        ids = [qs.qs_server_submit(srv, c) for c in circs]
        done = _drain(qs, srv, ids)
        for rid, c in zip(ids, circs):
            assert done[rid]["status"] == 0
            assert done[rid]["t_submit_ms"] <= done[rid]["t_admit_ms"] <= done[rid]["t_done_ms"]
            _check(qs.qs_server_download(srv, rid, dt), oracle.run_circuit(c), dt, c.name)
            qs.qs_server_release(srv, rid)
        st = qs.qs_server_get_stats(srv)
        assert st["completed"] == len(circs) and st["used_bytes"] == 0 and st["rounds"] >= 1
    finally:
        qs.qs_server_destroy(srv)


@pytest.mark.parametrize("dt", [2, 1])
def test_server_alone_vs_mix_bitwise(qs, dt):
    probe = [W.rqc_chain(17, 5, 9), W.qft(12, 77), W.grover(15, 1234)]
    alone = []
    for c in probe:
        srv = qs.qs_server_create(dtype=dt, hbm_budget=1 << 28)
        try:
            rid = qs.qs_server_submit(srv, c)
            _drain(qs, srv, [rid])
            alone.append(qs.qs_server_download(srv, rid, dt))
        finally:
            qs.qs_server_destroy(srv)
    srv = qs.qs_server_create(dtype=dt, hbm_budget=1 << 30)
    try:
        ids, pids, early = [], [], {}
        others = _mix(5)
        for i, c in enumerate(others):
            ids.append(qs.qs_server_submit(srv, c))
            if i % 3 == 1:  # interleave the probes with the traffic, polling in between
                pids.append(qs.qs_server_submit(srv, probe[len(pids)]))
                for r in qs.qs_server_poll(srv):
                    early[r["id"]] = r
        done = _drain(qs, srv, ids + pids, done=early)
        for rid, ref, c in zip(pids, alone, probe):
            assert done[rid]["status"] == 0
            assert qs.qs_server_download(srv, rid, dt).tobytes() == ref.tobytes(), c.name
    finally:
        qs.qs_server_destroy(srv)


def test_server_admission_by_budget(qs):
    budget = 2 * (16 << 16) + 4096  # two 16-qubit complex128 states
    srv = qs.qs_server_create(dtype=2, hbm_budget=budget)
    try:
        circs = [W.rqc_chain(16, 3, s) for s in range(5)] + [W.qft(6, 3), W.grover(7, 9)]
        ids = [qs.qs_server_submit(srv, c) for c in circs]
        seen_queue = False
        done = {}
        t_end = time.time() + 60
        while len(done) < len(ids):
            for r in qs.qs_server_poll(srv):
                done[r["id"]] = r
                qs.qs_server_download(srv, r["id"], 2)
                qs.qs_server_release(srv, r["id"])  # frees room for the next request
            st = qs.qs_server_get_stats(srv)
            seen_queue |= st["queued"] > 0
            assert st["used_bytes"] <= st["budget_bytes"]
            assert time.time() < t_end
            time.sleep(0.0002)
        assert seen_queue and all(r["status"] == 0 for r in done.values())
        assert qs.qs_server_get_stats(srv)["peak_bytes"] <= budget
    finally:
        qs.qs_server_destroy(srv)


def test_server_rejects_oversize_and_cancels(qs):
    srv = qs.qs_server_create(dtype=2, hbm_budget=(16 << 12) + 256)
    try:
        with pytest.raises(qs.QSError) as e:
            qs.qs_server_submit(srv, W.qft(20, 1))
        assert e.value.status == qs.QS_ERR_OOM
        a = qs.qs_server_submit(srv, W.rqc_chain(12, 2, 1))  # takes the whole budget
        b = qs.qs_server_submit(srv, W.rqc_chain(12, 2, 2))  # must wait
        qs.qs_server_poll(srv)
        qs.qs_server_cancel(srv, b)
        done = _drain(qs, srv, [a, b])
        assert done[a]["status"] == 0 and done[b]["status"] == qs.QS_ERR_CANCELLED
        with pytest.raises(qs.QSError):
            qs.qs_server_cancel(srv, a)
    finally:
        qs.qs_server_destroy(srv)


def test_server_plan_larger_than_pool_fails(qs):
    """A request whose plan can never fit the plan pool finishes with
    QS_ERR_ARG instead of staying queued; a small one beside it is served."""
    srv = qs.qs_server_create(dtype=2, hbm_budget=1 << 28, plan_budget=256 << 10)
    try:
        big = W.rqc_chain(18, 200, 3)  # ~5400 gates: hundreds of KiB of plan
        small = W.qft(10, 77)
        a = qs.qs_server_submit(srv, big)
        b = qs.qs_server_submit(srv, small)
        done = _drain(qs, srv, [a, b])
        assert done[a]["status"] == qs.QS_ERR_ARG
        assert done[b]["status"] == 0
        _check(qs.qs_server_download(srv, b, 2), oracle.run_circuit(small), 2, "small beside the failed one")
    finally:
        qs.qs_server_destroy(srv)


FAULT_SCRIPT = r"""
import json, sys, time
sys.path.insert(0, sys.argv[1])
import paper_2506_09198_amd as qs
import workloads as W

srv = qs.qs_server_create(dtype=2, hbm_budget=1 << 28)
done = {}


def wait(ids):
    t_end = time.time() + 60
    while any(i not in done for i in ids) and time.time() < t_end:
        for r in qs.qs_server_poll(srv):
            done[r["id"]] = r["status"]
        time.sleep(0.0002)


first = qs.qs_server_submit(srv, W.qft(10, 3))          # launch 1: whole-circuit kernel
wait([first])
big = [qs.qs_server_submit(srv, W.rqc_chain(14, 2, s)) for s in range(3)]  # launches 2-4 init, 5 round
wait(big)
later = qs.qs_server_submit(srv, W.qft(10, 5))
wait([later])
print("STATUS " + json.dumps({"first": done.get(first), "big": [done.get(i) for i in big],
                              "later": done.get(later)}))
"""


def test_server_fault_fails_only_that_round():
    """The 5th launch reports an injected device error (no real GPU fault):
    the requests of that round fail, the one before and the one after succeed."""
    import json

    env = dict(os.environ, QS_FAULT_INJECT="launch:5")
    r = subprocess.run([sys.executable, "-c", FAULT_SCRIPT, ROOT], env=env, capture_output=True, text=True,
                       timeout=300)
    line = [l for l in r.stdout.splitlines() if l.startswith("STATUS ")]
    assert r.returncode == 0 and line, r.stdout + r.stderr
    st = json.loads(line[0][len("STATUS "):])
    assert st["first"] == 0
    assert st["big"] == [3, 3, 3]
    assert st["later"] == 0
