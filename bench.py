#!/usr/bin/env python3
"""Benchmark of the gate engine on one MI355X.

Workloads (``--workload``), each printing ONE JSON line:

- ``sweep`` (default): the per-target gate sweep on a 30-qubit complex128 state
  (16 GiB) -- one seeded U3 on every target 0..29, then seeded Haar-random 4x4
  unitaries on adjacent pairs (t, t+1) and far pairs (t, t+15), each once
  uncontrolled and once with one control: 118 gates, one launch each, state
  resident in HBM.  Value: amplitude-updates/s.  The same line carries, on
  the same state, the diagonal-gate sweep, the read-only passes (norm,
  marginals, expectation values, sampling) and the in-place ceiling probe,
  then compact batch (1024 circuits: fused complex64 vs per-gate complex128)
  and serving (p50/p99 latency, circuits/s) legs, and the oracle on the
  host's cores with one and with all threads.
- ``circuits``: 32-qubit random chain circuit (depth 20) and full QFT of a
  random basis state, complex64 in tile passes (register segments with fused
  register blocks), beside complex64 with 5-qubit fused blocks on matrix
  cores, complex128 tile passes and complex128 gate by gate.  Value:
  credited amplitude-updates/s of the complex64 tile passes.
- ``batch``: 4096 circuits (n log-uniform in [10, 22]; random chain / QFT /
  Grover) in one batch: fused complex64 against plain per-gate complex128 on
  8 streams and on 1 stream.  Value: circuits/s of the fused complex64 batch.
- ``serve``: Poisson stream of requests (n log-uniform in [8, 28]) admitted by
  HBM footprint, at 0.7x the saturated throughput, beside a 34-qubit complex64
  depth-24 chain circuit with fused blocks.  Value: served circuits/s, with
  p50/p99 latency.

Each line carries the roofline of the dominant kernel (HIP events recorded by
the library around its launches, or the batch's device time) and the FP64
oracle timed on host cores on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E, published
PEAK_FP64_TFLOPS = 78.6  # MI355X FP64 vector / matrix, published


def _args():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", choices=["sweep", "circuits", "batch", "serve"], default="sweep")
    p.add_argument("--n", type=int, default=0, help="qubits (0 = the workload's default: 30 / 32 / - / 34)")
    p.add_argument("--dtype", choices=["c128", "c64"], default="c128", help="sweep only")
    p.add_argument("--mode", choices=["pergate", "planned"], default="pergate", help="sweep only")
    p.add_argument("--count", type=int, default=0, help="circuits of the batch / requests of the stream")
    p.add_argument("--no-baselines", action="store_true",
                   help="circuits/batch: skip the per-gate complex128 comparison runs")
    p.add_argument("--no-tune", action="store_true", help="batch: skip the autotuner (library defaults)")
    p.add_argument("--only-head", action="store_true",
                   help="circuits / batch: run only the complex64 tile-pass variant / fused complex64 batch (no "
                        "comparisons, e.g. under a profiler)")
    p.add_argument("--qps-sweep", action="store_true", help="serve: also run 0.3x, 0.5x and 1.0x of saturation")
    p.add_argument("--big-blocks", type=int, default=256,
                   help="serve: workgroup cap of the large circuit's passes (0 = library default), which "
                        "leaves compute units to the request stream")
    p.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    p.add_argument("--tune-gates", action="store_true",
                   help="sweep: autotune the per-gate schedules on the state (qs_tune_gates) before the warm-up")
    p.add_argument("--no-side", action="store_true",
                   help="sweep: skip the compact batch and serving legs that follow the timed sweep")
    p.add_argument("--cpu-n", type=int, default=0, help="qubits of the oracle sample (0 = workload default)")
    p.add_argument("--oracle-n", type=int, default=30,
                   help="circuits: qubits of the chain circuit checked against the host oracle on every GPU path")
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run 3 torch copies of 4 GiB (reference for HBM byte counters) and exit")
    return p.parse_args()


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _updates(n, ops):
    """Amplitude-updates credited to a gate list: 2^(n - controls) per gate."""
    cm = np.ascontiguousarray(ops["cmask"], dtype=np.uint64)
    nc = np.unpackbits(cm.view(np.uint8)).reshape(-1, 64).sum(axis=1, dtype=np.int64)
    return int(np.sum(np.left_shift(np.int64(1), n - nc)))


def _header(a, metric, value, unit, ms_per_step, dtype, data, config, higher=True):
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
            "ms_per_step": ms_per_step, "higher_is_better": higher, "scaling": "weak", "vs_baseline": None,
            "dtype": dtype, "data": data, "config": config}


def _kinds(qs, recs):
    """Per kernel class totals from the library's launch trace."""
    kinds = {}
    for r in recs:
        k = qs.KIND_NAMES[int(r["kind"])]
        d = kinds.setdefault(k, {"launches": 0, "ms": 0.0, "bytes": 0})
        d["launches"] += 1
        d["ms"] += float(r["ms"])
        d["bytes"] += int(r["bytes"])
    for d in kinds.values():
        d["avg_ms"] = d["ms"] / d["launches"]
        d["avg_bytes"] = d["bytes"] / d["launches"]
        d["gbs"] = d["bytes"] / (d["ms"] * 1e-3) / 1e9
    return kinds


def _roofline(kinds, traffic=None):
    dom = max(kinds, key=lambda k: kinds[k]["ms"])
    D = kinds[dom]
    achieved = D["avg_bytes"] / (D["avg_ms"] * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
            "traffic_unit": "HBM bytes/launch (rocprofv3 FETCH_SIZE+WRITE_SIZE, copy-calibrated)",
            "algorithmic_bytes_per_launch": D["avg_bytes"]}


# ------------------------------------------------------------------ CPU legs

def host_cpu() -> dict:
    """Model, sockets and cores of the host (lscpu), and the CPUs this process may use."""
    import subprocess

    info = {}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
    except (OSError, subprocess.SubprocessError):
        txt = ""
    keys = {"Model name": "model", "Socket(s)": "sockets", "Core(s) per socket": "cores_per_socket",
            "Thread(s) per core": "threads_per_core", "CPU(s)": "cpus", "NUMA node(s)": "numa_nodes"}
    for line in txt.splitlines():
        k, _, v = line.partition(":")
        if k.strip() in keys and keys[k.strip()] not in info:
            info[keys[k.strip()]] = v.strip()
    try:
        info["physical_cores"] = int(info["sockets"]) * int(info["cores_per_socket"])
    except (KeyError, ValueError):
        pass
    info["usable_cpus"] = len(os.sched_getaffinity(0))
    return info


def cpu_baseline_gates(n_cpu: int = 30, reps_all: int = 5, reps_one: int = 3) -> dict:
    """The FP64 oracle on a bounded sample of the gate sweep at the GPU's size:
    six of its gates (U3 on t = 0, 15, 29; Haar 4x4 on (0,1), (14,15), (7,22))
    on a 2^30 complex128 state, timed per pass with all the threads the host
    gives this process and with one thread (U3 on t = 15 only); min and median
    of the repeated passes (the paper reports the minimum of 10)."""
    import oracle
    import workloads as W

    circ = W.gate_microbench(n_cpu)
    pick = [g for g in circ.gates if not g[2] and (g[0] in ((0,), (15,), (29,), (0, 1), (14, 15), (7, 22)))]
    psi = np.full(1 << n_cpu, 2.0 ** (-n_cpu / 2), dtype=np.complex128)  # timing does not depend on the values
    threads_all = oracle.num_threads()

    def passes(gates, reps):
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            for tg, u, cm, cv in gates:
                oracle.apply_op(n_cpu, psi, tg, u, cm, cv)
            ts.append(time.perf_counter() - t0)
        upd = len(gates) * float(1 << n_cpu)
        return {"threads": oracle.num_threads(), "reps": reps, "min_s": min(ts), "median_s": float(np.median(ts)),
                "amp_updates_per_s_best": upd / min(ts), "amp_updates_per_s_median": upd / float(np.median(ts))}

    try:
        allc = passes(pick, reps_all)
        oracle.set_threads(1)
        one = passes([g for g in pick if g[0] == (15,)], reps_one)
    finally:
        oracle.set_threads(threads_all)
    del psi
    return {"value": allc["amp_updates_per_s_best"], "unit": "amp-updates/s", "cores": allc["threads"],
            "kind": "oracle", "host": host_cpu(), "all_threads": allc, "one_thread": one,
            "sample": f"{len(pick)} gates of the sweep (U3 on t=0,15,29; Haar 4x4 on (0,1),(14,15),(7,22)) on the "
                      f"same n={n_cpu} complex128 size, {reps_all} passes with {allc['threads']} threads (value = "
                      f"best pass) and U3 on t=15 x{reps_one} with 1 thread"}


def cpu_baseline_sweep(n_cpu: int) -> dict:
    """The FP64 oracle on the same gate sweep at n_cpu qubits (bounded sample)."""
    import oracle
    import workloads as W

    c = W.gate_microbench(n_cpu)
    ops, mats = c.arrays()
    psi = np.ascontiguousarray(W.random_state(n_cpu, 2), dtype=np.complex128)
    passes, dt = 0, 0.0
    while passes < 4 and (passes == 0 or dt < 10.0):  # about 10-30 s of host work
        t0 = time.perf_counter()
        oracle.run_inplace(n_cpu, ops, mats, psi)
        dt += time.perf_counter() - t0
        passes += 1
    return {"value": passes * _updates(n_cpu, ops) / dt, "unit": "amp-updates/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"gate sweep at n={n_cpu} complex128 ({len(ops)} gates, {passes} passes, {dt:.1f} s)"}


def cpu_baseline_circuits(n_cpu: int) -> dict:
    """The oracle on the same two circuits at n_cpu qubits."""
    import oracle
    import workloads as W

    upd, dt = 0, 0.0
    for c in (W.rqc_chain(n_cpu, 20, 5), W.qft(n_cpu, 12345 % (1 << n_cpu))):
        ops, mats = c.arrays()
        t0 = time.perf_counter()
        oracle.run_circuit(c)
        dt += time.perf_counter() - t0
        upd += _updates(n_cpu, ops)
    return {"value": upd / dt, "unit": "amp-updates/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"depth-20 chain circuit + QFT at n={n_cpu} complex128 ({dt:.1f} s)"}


def cpu_baseline_mix(circs, budget_s: float = 15.0) -> dict:
    """The oracle on the circuits of the mix in order until budget_s is spent,
    skipping any whose estimated time exceeds what is left of the budget; its
    amplitude-update rate is scaled to circuits/s with the whole mix's mean
    amplitude-updates per circuit."""
    import oracle

    upd_all = [_updates(c.n, c.arrays()[0]) for c in circs]
    done, skipped, upd, dt, rate = 0, 0, 0, 0.0, 1e9
    for c, u in zip(circs, upd_all):
        if dt >= budget_s:
            break
        if u / rate > budget_s - dt:
            skipped += 1
            continue
        t0 = time.perf_counter()
        oracle.run_circuit(c)
        dt += time.perf_counter() - t0
        upd += u
        done += 1
        rate = upd / dt
    return {"value": rate / (sum(upd_all) / len(upd_all)), "unit": "circuits/s", "cores": oracle.num_threads(),
            "kind": "oracle", "amp_updates_per_s": rate,
            "sample": f"{done} circuits of the same mix in order ({skipped} skipped as too long for the "
                      f"{budget_s:.0f} s budget) in {dt:.1f} s, complex128; rate scaled by the mix's mean "
                      f"amplitude-updates per circuit"}


# ------------------------------------------------------------------ workloads

def _random_state_torch(torch, n, tdt, seed):
    """Seeded complex Gaussian state, normalised in FP64, generated on the device."""
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    psi = torch.empty(1 << n, dtype=tdt, device="cuda")
    chunk = 1 << 26
    nrm2 = 0.0
    for i in range(0, 1 << n, chunk):
        blk = torch.randn(min(chunk, (1 << n) - i), dtype=torch.complex128, device="cuda", generator=g)
        nrm2 += float((blk.real.square().sum() + blk.imag.square().sum()).item())
        psi[i:i + blk.numel()] = blk.to(tdt)
    psi /= math.sqrt(nrm2)
    return psi


def diag_sweep(qs, s, n, S, reps=3, seed=13):
    """CZ on (t, t+1) for t = 0..n-2 and CP(phi) with a seeded random control
    on every target, through the diagonal kernel; each changes 2^(n-2)
    amplitudes, so the algorithmic bytes are 2 S 2^(n-2) per gate."""
    rng = np.random.default_rng(seed)
    gates = [(t + 1, np.diag([1.0, -1.0]), 1 << t) for t in range(n - 1)]
    for t in range(n):
        c = int(rng.choice([q for q in range(n) if q != t]))
        gates.append((t, np.diag([1.0, np.exp(1j * rng.uniform(0, 2 * np.pi))]), 1 << c))
    qs.qs_trace_enable(s.h, True)
    for _ in range(reps):
        for t, u, cm in gates:
            qs.qs_apply_1q(s.h, t, u, cm, cm)
    recs = qs.qs_trace_read(s.h, 1 << 20)
    qs.qs_trace_enable(s.h, False)
    assert all(qs.KIND_NAMES[int(k)] == "diag" for k in recs["kind"])
    by, ms = float(recs["bytes"].sum()), float(recs["ms"].sum())
    return {"gates": len(gates), "reps": reps, "avg_ms": ms / len(recs),
            "gbs_algorithmic": by / ms / 1e6, "frac": by / ms / 1e6 / PEAK_HBM_GBS,
            "bytes_per_gate": 2 * S * (1 << (n - 2)),
            "traffic": measured_traffic("diag", f"diag_sweep_n{n}_c{8 * S}", DIAG_SRCS),
            "plain_path_bytes_per_gate": 2 * S * (1 << (n - 1)),
            "note": "CZ on neighbouring pairs and CP with random controls; pairs with a qubit below the "
                    "128-byte line (bit 3, complex128) read whole lines"}


# (slots per lane, log2 slot spread, workgroups per CU; 0 = no cap)
CEILING_SCHEDULES = ((1, 8, 0), (1, 8, 6), (2, 11, 0), (2, 11, 3), (2, 14, 3), (2, 14, 4), (4, 11, 2))


def ceiling_probe(qs, s, reps=3):
    """In-place read-modify-write ceiling on the same buffer: every 16-byte
    word read and written back once by the library's probe kernel, in the
    per-gate kernel's schedule family (slots per lane, slot spread,
    workgroups per CU); the best schedule's GB/s (2 x buffer bytes / launch
    time)."""
    recs = []
    for slots, sl, wg in CEILING_SCHEDULES:
        with qs.tunables(gate_wg_per_cu=wg):
            qs.qs_trace_enable(s.h, True)
            for _ in range(reps):
                qs.qs_probe_inplace(s.h, slots, sl)
            recs.append(qs.qs_trace_read(s.h, 64))
            qs.qs_trace_enable(s.h, False)
    gbs = np.array([[float(b) / float(m) / 1e6 for b, m in zip(r["bytes"], r["ms"])] for r in recs])
    best = gbs.max(axis=1)
    i = int(np.argmax(best))
    return {"gbs": float(best[i]), "schedule": dict(zip(("slots", "spread_log2", "wg_per_cu"), CEILING_SCHEDULES[i])),
            "per_schedule_gbs": {f"{a}x2^{b}/wg{c}": round(float(g)) for (a, b, c), g in zip(CEILING_SCHEDULES, best)},
            "bytes_per_launch": int(recs[0]["bytes"][0]),
            "note": "in-place read+write of every 16-byte word of the 16 GiB state (qs_probe_inplace), best of "
                    f"{reps} per schedule"}


def reductions(qs, s, n, S, reps=3, seed=17):
    """The read-only passes over the same state: squared norm, marginal
    probabilities over low / high / spread qubit sets, Pauli-string
    expectation values, and sampling (chunk sums, then one wave per shot).
    Kernel time from the library's HIP events; GB/s of the bytes each pass
    reads (S x 2^n per full pass, S x 4096 per shot)."""
    rng = np.random.default_rng(seed)
    cases = [("norm", lambda: qs.qs_norm(s.h)),
             ("probs_low_3", lambda: qs.qs_probabilities(s.h, [0, 1, 2])),
             ("probs_high_3", lambda: qs.qs_probabilities(s.h, [n - 3, n - 2, n - 1])),
             ("probs_spread_10", lambda: qs.qs_probabilities(s.h, list(range(0, n, 3))[:10])),
             ("probs_low_16", lambda: qs.qs_probabilities(s.h, list(range(16)))),
             ("expect_z_all", lambda: qs.qs_expect_pauli(s.h, 0, (1 << n) - 1)),
             ("expect_xz_mixed", lambda: qs.qs_expect_pauli(s.h, 0x2AAAAAAA & ((1 << n) - 1),
                                                           0x15555555 & ((1 << n) - 1))),
             ("sample_100k", lambda: qs.qs_sample(s.h, rng.random(100000)))]
    out = {}
    for name, fn in cases:
        fn()  # warm (scratch sized)
        qs.qs_trace_enable(s.h, True)
        for _ in range(reps):
            fn()
        recs = qs.qs_trace_read(s.h, 1 << 10)
        qs.qs_trace_enable(s.h, False)
        per = {}
        for r in recs:
            k = qs.KIND_NAMES[int(r["kind"])]
            d = per.setdefault(k, {"ms": [], "bytes": int(r["bytes"])})
            d["ms"].append(float(r["ms"]))
        out[name] = {k: {"ms": float(np.median(d["ms"])), "bytes": d["bytes"],
                         "gbs": d["bytes"] / float(np.median(d["ms"])) / 1e6} for k, d in per.items()}
    full = [v["reduce"]["gbs"] for v in out.values() if "reduce" in v]
    return {"cases": out, "min_gbs_full_pass": min(full), "frac_min": min(full) / PEAK_HBM_GBS,
            "note": f"n={n} complex128 state, median of {reps}; kind 'reduce' reads the whole state once, "
                    "'sample' reads 4096 amplitudes per shot"}


def _step_stats(recs, per_step, steps):
    """Device time of each timed step (sum of its launches' HIP-event times):
    min and median over the steps."""
    if len(recs) < per_step * steps or steps < 1:
        return None
    ms = np.array([float(r) for r in recs["ms"][:per_step * steps]]).reshape(steps, per_step).sum(axis=1)
    return {"min": float(ms.min()), "median": float(np.median(ms)), "steps": steps}


def per_target_table(gates, recs, steps):
    """GB/s per target index (median over the timed steps) for each gate of
    the sweep: 1q by target; 2q by first target, adjacent (t, t+1) and far
    (t, t+15), uncontrolled and with one control."""
    G = len(gates)
    if len(recs) < G * steps:
        return None
    ms = np.median(np.array([float(r) for r in recs["ms"][:G * steps]]).reshape(steps, G), axis=0)
    by = np.array([float(b) for b in recs["bytes"][:G]])
    gbs = by / ms / 1e6
    out = {"1q": [], "2q_adjacent": [], "2q_adjacent_ctrl": [], "2q_far": [], "2q_far_ctrl": []}
    for (tg, u, cm, cv), g in zip(gates, gbs):
        if len(tg) == 1:
            key = "1q"
        else:
            key = ("2q_adjacent" if tg[1] == tg[0] + 1 else "2q_far") + ("_ctrl" if cm else "")
        out[key].append(round(float(g)))
    out["note"] = "GB/s of algorithmic bytes per launch, index = first target"
    return out


def run_sweep(a, qs, torch, W):
    n = a.n or 30
    dt = qs.QS_C128 if a.dtype == "c128" else qs.QS_C64
    tdt = torch.complex128 if dt == qs.QS_C128 else torch.complex64
    S = 16 if dt == qs.QS_C128 else 8
    circ = W.gate_microbench(n)
    ops, mats = circ.arrays()
    gates = list(circ.gates)
    upd_step = _updates(n, ops)
    bytes_step = 2 * S * upd_step
    psi = _random_state_torch(torch, n, tdt, 2)
    torch.cuda.synchronize()
    s = qs.State.from_torch(psi)
    tuned = None
    if a.tune_gates and a.mode == "pergate":
        t0 = time.perf_counter()
        tuned = {"schedules": qs.qs_tune_gates(s.h), "seconds": time.perf_counter() - t0}
        _log(f"sweep: gate schedules tuned in {tuned['seconds']:.1f} s: {tuned['schedules']}")

    def step():
        if a.mode == "planned":
            s.run(ops, mats, mode=0)
        else:
            for tg, u, cm, cv in gates:
                if len(tg) == 1:
                    qs.qs_apply_1q(s.h, tg[0], u, cm, cv)
                else:
                    qs.qs_apply_2q(s.h, tg[0], tg[1], u, cm, cv)

    for _ in range(a.warmup):
        step()
    s.sync()
    torch.cuda.synchronize()
    qs.qs_trace_enable(s.h, True)
    t0 = time.perf_counter()
    for _ in range(a.steps):
        step()
    s.sync()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    recs = qs.qs_trace_read(s.h, 1 << 20)
    qs.qs_trace_enable(s.h, False)
    norm = s.norm()
    diag = diag_sweep(qs, s, n, S) if a.mode == "pergate" else None
    reds = reductions(qs, s, n, S) if a.mode == "pergate" else None
    ceiling = ceiling_probe(qs, s)
    s.close()
    kinds = _kinds(qs, recs)
    rl = _roofline(kinds)
    rl["ceiling_gbs"] = ceiling["gbs"]
    rl["frac_vs_ceiling"] = rl["achieved"] / ceiling["gbs"]
    per_target = per_target_table(gates, recs, a.steps) if a.mode == "pergate" else None
    if a.mode == "pergate":
        rl["traffic"] = measured_traffic(rl["kernel"], f"gate_sweep_n{n}_{a.dtype}")
    out = _header(a, "amplitude-updates/s", upd_step * a.steps / elapsed, "amp-updates/s",
                  elapsed * 1e3 / a.steps, "f64" if dt == qs.QS_C128 else "f32",
                  "synthetic (seeded complex Gaussian state, seeded U3 and Haar 4x4 gates)",
                  {"workload": f"gate sweep n={n} {a.dtype}: U3 on t=0..{n-1}, Haar 4x4 on (t,t+1) and "
                               f"(t,t+15), uncontrolled and 1-controlled; {len(gates)} gates/step",
                   "n": n, "state_bytes": (1 << n) * S, "gates_per_step": len(gates), "mode": a.mode})
    out.update({
        "hbm_gbs_algorithmic": bytes_step * a.steps / elapsed / 1e9,
        "hbm_frac_algorithmic": bytes_step * a.steps / elapsed / 1e9 / PEAK_HBM_GBS,
        "roofline": rl,
        "kernels": {k: {"launches": d["launches"], "avg_ms": round(d["avg_ms"], 4), "gbs": round(d["gbs"], 1)}
                    for k, d in kinds.items()},
        "event_coverage": sum(d["ms"] for d in kinds.values()) / (elapsed * 1e3),
        "step_device_ms": _step_stats(recs, len(gates), a.steps),
        "gate_schedules_tuned": tuned,
        "norm_minus_1": norm - 1.0,
        "per_target_gbs": per_target,
        "inplace_ceiling": ceiling,
        "diag_sweep": diag,
        "reductions": reds,
    })
    del psi
    torch.cuda.empty_cache()
    if a.mode == "pergate" and not a.no_side:
        out["batch"] = compact_batch(a, qs, W)
        out["serve"] = compact_serve(a, qs, W)
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline_gates(a.cpu_n or n)
    return out


def compact_batch(a, qs, W, count=1024, steps=3, warm=1):
    """Batched circuits (the 4096-circuit mix's recipe, first 1024 circuits of
    seed 7): the fused complex64 batch against the plain per-gate complex128
    path on 8 streams, both with the same warm-up and timed runs (medians),
    with a closed-form and oracle check of sampled results."""
    import oracle

    circs = W.circuit_mix(count, 7)
    arrs = [(c.n, *c.arrays(), c.init_basis) for c in circs]

    def leg(dt, mode, streams):
        for _ in range(warm):
            b = qs.qs_batch_submit(arrs, dtype=dt, mode=mode, streams=streams)
            qs.qs_batch_wait(b)
            qs.qs_batch_release(b)
        e2e, dev, keep = [], [], None
        for i in range(steps):
            t0 = time.perf_counter()
            b = qs.qs_batch_submit(arrs, dtype=dt, mode=mode, streams=streams)
            qs.qs_batch_wait(b)
            e2e.append(time.perf_counter() - t0)
            dev.append(qs.qs_batch_get_stats(b)["device_ms"])
            if i == steps - 1:
                keep = b
            else:
                qs.qs_batch_release(b)
        return {"circuits_per_s": count / float(np.median(e2e)), "end_to_end_ms": 1e3 * float(np.median(e2e)),
                "device_ms": float(np.median(dev)), "runs": steps, "warmup": warm}, keep

    fused, b64 = leg(qs.QS_C64, 0, 0)
    _log(f"batch (compact) c64 fused: {fused['circuits_per_s']:.0f} circuits/s")
    rng = np.random.default_rng(3)
    order = rng.permutation(count)
    closed = [i for i in order if circs[i].n <= 16 and _closed_form(circs[i]) is not None][:16]
    chains = [i for i in order if circs[i].n <= 14 and circs[i].name.startswith("rqc")][:4]
    fmin, emax = 1.0, 0.0
    for i in closed + chains:
        got = qs.qs_batch_download(b64, int(i), qs.QS_C64).astype(np.complex128)
        want = _closed_form(circs[i]) if i in closed else oracle.run_circuit(circs[i])
        fmin = min(fmin, abs(np.vdot(want, got)) ** 2)
        emax = max(emax, float(np.max(np.abs(got - want))))
    qs.qs_batch_release(b64)
    pergate, b = leg(qs.QS_C128, 1, 8)
    qs.qs_batch_release(b)
    _log(f"batch (compact) c128 per-gate 8 streams: {pergate['circuits_per_s']:.0f} circuits/s")
    return {"circuits": count, "c64_fused": fused, "c128_pergate_8streams": pergate,
            "ratio": fused["circuits_per_s"] / pergate["circuits_per_s"],
            "check": {"closed_form_circuits": len(closed), "oracle_circuits": len(chains),
                      "min_fidelity": fmin, "max_abs_err": emax},
            "note": "first 1024 circuits of the 4096-circuit mix (seed 7); --workload batch runs all 4096"}


def compact_serve(a, qs, W, count=120):
    """Serving: Poisson stream of requests (n log-uniform in [8, 28], seed 8),
    complex64, at 0.7x the saturated rate measured on the first 60 requests
    submitted at once; nothing else on the GPU (--workload serve adds the
    34-qubit circuit beside the stream)."""
    circs = W.circuit_mix(count, 8, n_lo=8, n_hi=28)
    dt = qs.QS_C64
    sat = _serve_stream(qs, circs[:60], np.zeros(60), dt)
    qps = 0.7 * sat["circuits_per_s"]
    main = _serve_stream(qs, circs, W.poisson_arrivals(count, qps, 8), dt)
    _log(f"serve (compact) at {qps:.1f} qps: p50 {main['p50_ms']:.1f} ms p99 {main['p99_ms']:.1f} ms")
    return {"requests": count, "qps": qps, "circuits_per_s": main["circuits_per_s"], "p50_ms": main["p50_ms"],
            "p99_ms": main["p99_ms"], "failed": main["failed"], "saturated_circuits_per_s": sat["circuits_per_s"],
            "note": "no large circuit beside the stream here; --workload serve runs it beside n=34"}


def _fidelity(torch, ref, x):
    """<ref|x> and ||x||^2 accumulated in FP64 over chunks; max |x - ref|."""
    acc, nx, err = 0j, 0.0, 0.0
    step = 1 << 26
    for i in range(0, ref.numel(), step):
        r = ref[i:i + step]
        b = x[i:i + step].to(torch.complex128)
        acc += complex(torch.vdot(r, b).item())
        nx += float((b.real.square().sum() + b.imag.square().sum()).item())
        err = max(err, float((b - r).abs().max().item()))
    return abs(acc) ** 2, nx - 1.0, err


def run_circuits(a, qs, torch, W):
    n = a.n or 32
    work = {"rqc_d20": W.rqc_chain(n, 20, 5),
            "qft": W.qft(n, int(np.random.default_rng(6).integers(1 << n)))}
    arrs = {k: c.arrays() for k, c in work.items()}
    upd = {k: _updates(n, arrs[k][0]) for k in work}
    head = "c64_tiles"
    variants = [(head, qs.QS_C64, 0, 0, a.steps, a.warmup)]
    if not a.only_head:
        variants += [("c64_mfma5", qs.QS_C64, 0, 5, 1, 1), ("c64_mfma5_fp32", qs.QS_C64, 0, 5, 1, 1),
                     ("c128_tiles", qs.QS_C128, 0, 0, 1, 1), ("c128_mfma5", qs.QS_C128, 0, 5, 1, 1)]
    if not a.no_baselines and not a.only_head:
        variants.append(("c128_pergate", qs.QS_C128, 1, 0, 1, 0))
    res, traces, states = {}, {}, {}
    for name, dt, mode, fk, steps, warm in variants:
        # FP32 matrix-core blocks (hi + bfloat16 lo) are a planner option
        os.environ["QS_FUSE_FP32"] = "1" if name.endswith("_fp32") else "0"
        tdt = torch.complex128 if dt == qs.QS_C128 else torch.complex64
        for k, c in work.items():
            ops, mats = arrs[k]
            psi = torch.empty(1 << n, dtype=tdt, device="cuda")
            s = qs.State.from_torch(psi)
            plan = qs.qs_plan_circuit(n, dt, ops, mats, mode=0, fuse_k=fk) if mode == 0 else None
            for _ in range(warm):
                s.init_basis(c.init_basis)
                s.run(ops, mats, mode=mode, fuse_k=fk)
            s.sync()
            if name == head:
                qs.qs_trace_enable(s.h, True)
            t0 = time.perf_counter()
            for _ in range(steps):
                s.init_basis(c.init_basis)
                s.run(ops, mats, mode=mode, fuse_k=fk)
            s.sync()
            el = (time.perf_counter() - t0) / steps
            if name == head:
                traces[k] = qs.qs_trace_read(s.h, 1 << 20)
                qs.qs_trace_enable(s.h, False)
            s.close()
            res.setdefault(name, {})[k] = {"ms": el * 1e3, "amp_updates_per_s": upd[k] / el,
                                           "gates": len(ops), "passes": None if plan is None else plan[0]}
            _log(f"circuits {name} {k}: {el * 1e3:.1f} ms")
            if name in (head, "c64_mfma5", "c128_tiles") and not a.only_head:
                states.setdefault(k, {})[name] = psi
            elif name == "c128_mfma5":  # both complex128 forms against each other
                ref = states[k].pop("c128_tiles")
                res[name][k]["max_abs_err_vs_c128_tiles"] = max(
                    float((psi[i:i + (1 << 26)] - ref[i:i + (1 << 26)]).abs().max().item())
                    for i in range(0, psi.numel(), 1 << 26))
                del ref, psi
                torch.cuda.empty_cache()
            else:
                del psi
        torch.cuda.synchronize()
        os.environ["QS_FUSE_FP32"] = "0"
        if name == "c128_tiles":  # both precisions of each circuit are resident: compare them
            for k in work:
                for v in (head, "c64_mfma5"):
                    f, dn, err = _fidelity(torch, states[k]["c128_tiles"], states[k][v])
                    res[v][k].update({"fidelity_vs_c128": f, "norm2_minus_1": dn, "max_abs_err_vs_c128": err})
                    del states[k][v]
            if work["qft"].name.startswith("qft"):  # c128 QFT against its closed form on samples
                x, N = work["qft"].init_basis, 1 << n
                y = np.random.default_rng(7).integers(0, N, size=1 << 16, dtype=np.int64)
                want = np.exp(2j * np.pi * ((x * y.astype(object)) % N).astype(np.float64) / N) / math.sqrt(N)
                got = states["qft"]["c128_tiles"][torch.from_numpy(y).cuda()].cpu().numpy()
                res["c128_tiles"]["qft"]["max_abs_err_closed_form_sampled"] = float(np.max(np.abs(got - want)))
            for k in work:  # the complex128 tile results stay for the matrix-core form
                states[k] = {"c128_tiles": states[k]["c128_tiles"]}
            torch.cuda.empty_cache()
    tot = sum(upd.values())
    ms64 = sum(r["ms"] for r in res[head].values())
    kinds = _kinds(qs, np.concatenate(list(traces.values())))
    out = _header(a, "amplitude-updates/s", tot / (ms64 * 1e-3), "amp-updates/s", ms64, "f64",
                  "synthetic (seeded chain circuit of sqrt(X)/sqrt(Y)/sqrt(W) + CZ layers; QFT of a seeded basis "
                  "state)",
                  {"workload": f"n={n}: depth-20 chain circuit ({len(arrs['rqc_d20'][0])} gates) + QFT "
                               f"({len(arrs['qft'][0])} gates); complex64 state in tile passes with fused register "
                               "blocks (FP64 arithmetic)",
                   "n": n, "state": "c64", "state_bytes_c64": 8 << n, "state_bytes_c128": 16 << n})
    for name in res:
        ms = sum(r["ms"] for r in res[name].values())
        res[name]["total_ms"] = ms
        res[name]["time_vs_head"] = ms / ms64
    rl = _roofline(kinds)
    fpa = tile_flops_per_amp()
    if fpa and rl["kernel"] == "tile":
        # the pass is bound by FP64 arithmetic issue: its executed FP64 flops per
        # amplitude (rocprofv3 counters of the same circuits) against 78.6 TF
        D = kinds["tile"]
        tf = fpa * (1 << n) / (D["avg_ms"] * 1e-3) / 1e12
        rl = {"bound": "alu", "kernel": "tile", "achieved": tf, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
              "frac": tf / PEAK_FP64_TFLOPS,
              "traffic": measured_traffic("tile", f"tile_circuits_n{n}_c64", TILE_SRCS),
              "traffic_unit": "HBM bytes per tile pass (rocprofv3 FETCH_SIZE+WRITE_SIZE, copy-calibrated)",
              "flops_per_amp_per_pass": fpa, "hbm_gbs_algorithmic": rl["achieved"],
              "hbm_frac": rl["achieved"] / PEAK_HBM_GBS,
              "note": "FP64 flops executed per amplitude per pass from profiles/tile_circuits_n30_c64_counters.txt "
                      "(2 x FP64 FMA + FP64 MUL, the same two circuits at n=30)"}
    out.update({"variants": res, "roofline": rl,
                "kernels": {k: {"launches": d["launches"], "avg_ms": round(d["avg_ms"], 4), "gbs": round(d["gbs"], 1)}
                            for k, d in kinds.items()}})
    if not a.only_head:
        out["oracle_check"] = circuits_vs_oracle(a, qs, W, min(n, a.oracle_n))
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline_circuits(a.cpu_n or 25)
    return out


def tile_flops_per_amp():
    """FP64 flops per amplitude per tile pass of the chain circuit + QFT, from
    the committed rocprofv3 counter summary (None when it is missing)."""
    path = os.path.join(ROOT, "profiles", "tile_circuits_n30_c64_counters.txt")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if "flop per pass" in line:
            return float(line.split()[0]) / float(1 << 30)
    return None


def circuits_vs_oracle(a, qs, W, n):
    """The depth-20 chain circuit at n qubits (30 by default: the host oracle
    takes about 100 s on 16 threads and the comparison needs about 60 GiB of
    host memory; 32 would take 7 minutes and over 200 GiB) on every GPU path,
    each against the FP64 oracle run on the host: max |psi - psi_oracle| and
    fidelity |<psi_oracle|psi>|^2 with psi as computed (not renormalised).
    The differences are taken in slices to bound the host memory."""
    import oracle

    c = W.rqc_chain(n, 20, 5)
    ops, mats = c.arrays()
    t0 = time.perf_counter()
    ref = oracle.run_circuit(c)
    t_or = time.perf_counter() - t0
    out = {"n": n, "gates": len(ops), "oracle_s": t_or, "oracle_threads": oracle.num_threads()}
    for name, dt, mode, fk in (("c64_tiles", qs.QS_C64, 0, 0), ("c64_mfma5", qs.QS_C64, 0, 5),
                               ("c64_mfma5_fp32", qs.QS_C64, 0, 5), ("c128_tiles", qs.QS_C128, 0, 0),
                               ("c128_mfma5", qs.QS_C128, 0, 5), ("c128_pergate", qs.QS_C128, 1, 0)):
        os.environ["QS_FUSE_FP32"] = "1" if name.endswith("_fp32") else "0"
        with qs.State.create(n, dt) as s:
            s.run(ops, mats, mode=mode, fuse_k=fk)
            got = s.download()
        os.environ["QS_FUSE_FP32"] = "0"
        ov, nrm, err = 0j, 0.0, 0.0
        for i in range(0, got.size, 1 << 24):
            g = got[i:i + (1 << 24)].astype(np.complex128)
            r = ref[i:i + (1 << 24)]
            ov += np.vdot(r, g)
            nrm += float(np.vdot(g, g).real)
            err = max(err, float(np.max(np.abs(g - r))))
        out[name] = {"fidelity": float(abs(ov) ** 2), "max_abs_err": err, "norm2_minus_1": nrm - 1.0}
        del got
    return out


def _closed_form(c):
    """QFT and Grover results in closed form (None for other circuits)."""
    n = c.n
    if c.name.startswith("qft"):
        x, N = c.init_basis, 1 << n
        yv = np.arange(N, dtype=np.int64)
        return np.exp(2j * np.pi * ((x * yv) % N) / N) / math.sqrt(N)
    if c.name.startswith("grover"):
        mark = int(c.name.split("_m")[1].split("_")[0])
        R = int(c.name.split("_r")[1])
        th = math.asin(2.0 ** (-n / 2))
        sg = (-1) ** R
        v = np.full(1 << n, sg * math.cos((2 * R + 1) * th) / math.sqrt((1 << n) - 1), dtype=complex)
        v[mark] = sg * math.sin((2 * R + 1) * th)
        return v
    return None


def run_batch(a, qs, torch, W):
    count = a.count or 4096
    t0 = time.perf_counter()
    circs = W.circuit_mix(count, 7)
    arrs = [(c.n, *c.arrays(), c.init_basis) for c in circs]
    _log(f"batch: generated {count} circuits in {time.perf_counter() - t0:.1f} s")
    upd_total = sum(_updates(c.n, x[1]) for c, x in zip(circs, arrs))

    tuned, tune_rows, tune_s = {}, None, None
    if not a.no_tune:
        rng = np.random.default_rng(11)
        sample = [arrs[i] for i in rng.permutation(count)[:min(256, count)]]
        t0 = time.perf_counter()
        tuned, tune_rows = qs.qs_batch_tune(sample, dtype=qs.QS_C64)
        tune_s = time.perf_counter() - t0
        _log(f"batch tuned on {len(sample)} circuits in {tune_s:.1f} s: {tuned}")

    def one(dt, mode, streams, steps, warm, **kw):
        for _ in range(warm):
            b = qs.qs_batch_submit(arrs, dtype=dt, mode=mode, streams=streams, **kw)
            qs.qs_batch_wait(b)
            qs.qs_batch_release(b)
        e2e, dev, keep = [], [], None
        for i in range(steps):
            t0 = time.perf_counter()
            b = qs.qs_batch_submit(arrs, dtype=dt, mode=mode, streams=streams, **kw)
            t1 = time.perf_counter()
            qs.qs_batch_wait(b)
            t2 = time.perf_counter()
            st = qs.qs_batch_get_stats(b)
            e2e.append(t2 - t0)
            dev.append(st["device_ms"])
            if i == steps - 1:
                keep = b
            else:
                qs.qs_batch_release(b)
        r = {"circuits_per_s": count / float(np.median(e2e)), "end_to_end_ms": 1e3 * float(np.median(e2e)),
             "device_ms": float(np.median(dev)), "submit_ms": 1e3 * (t1 - t0), "launches": st["launches"],
             "passes": st["passes"], "class_ms": st["class_ms"], "class_circuits": st["class_circuits"],
             "submit_phases_ms": st["submit_ms"], "amp_updates_per_s": upd_total / float(np.median(e2e))}
        return r, keep

    res = {}
    r, b64 = one(qs.QS_C64, 0, 0, a.steps, a.warmup, **tuned)
    r["options"] = dict(tuned) or "library defaults"
    res["c64_fused"] = r
    _log(f"batch c64 fused: {r['circuits_per_s']:.0f} circuits/s")
    # closed-form check of sampled QFT / Grover circuits of the fused complex64 batch
    rng = np.random.default_rng(3)
    pick = [i for i in rng.permutation(count) if circs[i].n <= 16 and _closed_form(circs[i]) is not None][:32]
    fmin, emax = 1.0, 0.0
    for i in pick:
        got = qs.qs_batch_download(b64, int(i), qs.QS_C64).astype(np.complex128)
        want = _closed_form(circs[i])
        fmin = min(fmin, abs(np.vdot(want, got)) ** 2)
        emax = max(emax, float(np.max(np.abs(got - want))))
    r["closed_form_check"] = {"circuits": len(pick), "min_fidelity": fmin, "max_abs_err": emax}
    qs.qs_batch_release(b64)
    if a.only_head:  # one fused complex64 batch only (e.g. under a profiler)
        return _header(a, "batched circuits/s", r["circuits_per_s"], "circuits/s", r["end_to_end_ms"], "f64",
                       "synthetic (seeded mix of chain circuits, QFTs and Grover searches)",
                       {"workload": f"{count} circuits, fused complex64 batch only", "circuits": count}) | {
                           "variants": res}
    # the same batch replayed from its HIP graph: device work only (planned and uploaded once)
    b = qs.qs_batch_submit(arrs, dtype=qs.QS_C64, mode=0, graph=1, **tuned)
    qs.qs_batch_wait(b)
    rt = []
    for _ in range(max(a.steps, 2)):
        t0 = time.perf_counter()
        qs.qs_batch_replay(b)
        qs.qs_batch_wait(b)
        rt.append(time.perf_counter() - t0)
    dev = qs.qs_batch_get_stats(b)["device_ms"]
    qs.qs_batch_release(b)
    res["c64_graph_replay"] = {"circuits_per_s": count / float(np.median(rt)), "wall_ms": 1e3 * float(np.median(rt)),
                               "device_ms": dev, "note": "same batch replayed from its captured HIP graph"}
    _log(f"batch c64 graph replay: {res['c64_graph_replay']['circuits_per_s']:.0f} circuits/s")
    r, b = one(qs.QS_C128, 0, 0, 1, 1)
    qs.qs_batch_release(b)
    res["c128_fused"] = r
    _log(f"batch c128 fused: {r['circuits_per_s']:.0f} circuits/s")
    if not a.no_baselines:
        for name, streams in (("c128_pergate_8streams", 8), ("c128_pergate_1stream", 1)):
            r, b = one(qs.QS_C128, 1, streams, 1, 0)
            qs.qs_batch_release(b)
            res[name] = r
            _log(f"batch {name}: {r['circuits_per_s']:.0f} circuits/s")
        res["c64_fused"]["ratio_vs_c128_pergate_8streams"] = (res["c64_fused"]["circuits_per_s"] /
                                                              res["c128_pergate_8streams"]["circuits_per_s"])
    v = res["c64_fused"]
    ns = np.array([c.n for c in circs])
    out = _header(a, "batched circuits/s", v["circuits_per_s"], "circuits/s", v["end_to_end_ms"], "f64",
                  "synthetic (seeded mix of chain circuits, QFTs and Grover searches)",
                  {"workload": f"{count} circuits, n log-uniform in [10,22] (mean {ns.mean():.1f}), one third each "
                               "chain circuit (depth 20-200), QFT, Grover (<=200 gates); complex64 states, FP64 "
                               "arithmetic, fused batch",
                   "circuits": count, "gates": int(sum(len(x[1]) for x in arrs))})
    # aggregate roofline: algorithmic bytes of every pass of every circuit over the batch's device time
    alg = 0
    for c, x in zip(circs, arrs):
        if c.n <= 13:  # whole circuit in LDS: one read of nothing, one write of the state
            alg += 8 << c.n
        else:
            alg += qs.qs_plan_circuit(c.n, qs.QS_C64, x[1], x[2], mode=0)[0] * (16 << c.n)
    ach = alg / (v["device_ms"] * 1e-3) / 1e9
    out.update({"tuning": {"sample": 256, "seconds": tune_s, "chosen": tuned, "candidates": tune_rows},
                "variants": res, "roofline": {
        "bound": "hbm", "kernel": "all batch launches (aggregate)", "achieved": ach, "peak": PEAK_HBM_GBS,
        "unit": "GB/s", "frac": ach / PEAK_HBM_GBS, "traffic": measured_traffic("batch", f"batch_{count}_c64", BATCH_SRCS),
        "traffic_unit": "HBM bytes per batch (rocprofv3 FETCH_SIZE+WRITE_SIZE over every batch kernel, copy-calibrated)",
        "algorithmic_bytes": alg,
        "note": "states of n<=22 (<=32 MiB) stay in L2/Infinity Cache, so HBM is a loose roof here"}})
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline_mix(circs)
    return out


def _serve_stream(qs, circs, arrivals, dt, budget=0, hook=None):
    """Submit each request at its arrival time; poll until every one is done
    (calling hook() between polls).  Returns latencies and the served rate."""
    srv = qs.qs_server_create(dtype=dt, hbm_budget=budget)
    done, ids = {}, []
    try:
        t0 = t_log = time.perf_counter()
        i = 0
        while len(done) < len(circs):
            now = time.perf_counter() - t0
            while i < len(circs) and arrivals[i] <= now:
                ids.append(qs.qs_server_submit(srv, circs[i]))
                i += 1
            for r in qs.qs_server_poll(srv):
                done[r["id"]] = r
                qs.qs_server_release(srv, r["id"])
            if hook is not None:
                hook()
            if i == len(circs) and time.perf_counter() - t0 > arrivals[-1] + 900:
                raise RuntimeError("serving did not drain")
            time.sleep(0.0001)
            if time.perf_counter() - t_log > 10:
                t_log = time.perf_counter()
                _log(f"serve: {len(done)}/{len(circs)} done, {i} submitted")
        st = qs.qs_server_get_stats(srv)
    finally:
        qs.qs_server_destroy(srv)
    lat = np.array([done[k]["t_done_ms"] - done[k]["t_submit_ms"] for k in ids])
    fails = sum(1 for k in ids if done[k]["status"] != 0)
    span = (max(done[k]["t_done_ms"] for k in ids) - min(done[k]["t_submit_ms"] for k in ids)) * 1e-3
    return {"requests": len(ids), "failed": fails, "circuits_per_s": len(ids) / span,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "rounds": st["rounds"], "launches": st["launches"],
            "peak_bytes": st["peak_bytes"], "budget_bytes": st["budget_bytes"]}


class _BigJob:
    """A large complex64 circuit kept running beside the request stream: it is
    run forward and then inverted (echo), and the cycle is enqueued again
    whenever the previous one has finished, until stop()."""

    def __init__(self, qs, torch, W, n, fuse_k=0, max_blocks=0):
        self.qs, self.torch, self.n, self.fuse_k, self.max_blocks = qs, torch, n, fuse_k, max_blocks
        c = W.rqc_chain(n, 24, 9)
        self.ops, self.mats = c.arrays()
        self.iops, self.imats = c.inverse().arrays()
        self.side = torch.cuda.Stream()
        self.psi = torch.zeros(1 << n, dtype=torch.complex64, device="cuda")
        self.psi[0] = 1
        torch.cuda.synchronize()
        self.s = qs.State.from_torch(self.psi, stream=self.side.cuda_stream)
        self.cycles = []  # (ev_start, ev_forward_done, ev_echo_done)
        self.enqueue()

    def enqueue(self):
        ev = [self.torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record(self.side)
        self.s.run(self.ops, self.mats, mode=0, fuse_k=self.fuse_k, max_blocks=self.max_blocks)
        ev[1].record(self.side)
        self.s.run(self.iops, self.imats, mode=0, fuse_k=self.fuse_k, max_blocks=self.max_blocks)
        ev[2].record(self.side)
        self.cycles.append(ev)

    def hook(self):
        if self.cycles[-1][2].query():
            self.enqueue()

    def stop(self):
        self.side.synchronize()
        qs = self.qs
        a0 = complex(self.psi[0].item())
        fw = [c[0].elapsed_time(c[1]) for c in self.cycles]
        ec = [c[1].elapsed_time(c[2]) for c in self.cycles]
        out = {"n": self.n, "dtype": "c64", "gates": len(self.ops), "cycles": len(self.cycles),
               "forward_ms": fw, "echo_ms": ec, "echo_prob_0": abs(a0) ** 2, "norm2_minus_1": self.s.norm() - 1.0,
               "fuse_k": self.fuse_k, "max_blocks": self.max_blocks,
               "passes": qs.qs_plan_circuit(self.n, qs.QS_C64, self.ops, self.mats, mode=0, fuse_k=self.fuse_k)[0]}
        out["pass_gbs_algorithmic"] = out["passes"] * (16 << self.n) / (float(np.median(fw)) * 1e-3) / 1e9
        self.s.close()
        del self.psi
        self.torch.cuda.empty_cache()
        return out


def run_serve(a, qs, torch, W):
    nb = 34 if a.n == 0 else a.n
    count = a.count or 120
    circs = W.circuit_mix(count, 8, n_lo=8, n_hi=28)
    _log(f"serve: {count} requests, {sum(len(c) for c in circs)} gates")
    dt = qs.QS_C64
    sat_n = min(count, 60)
    # saturated throughput with nothing alongside: the first requests all at once
    alone = _serve_stream(qs, circs[:sat_n], np.zeros(sat_n), dt)
    _log(f"serve saturated, alone: {alone['circuits_per_s']:.1f} circuits/s")
    # the same requests as one fused batch: what the device does without the loop
    t0 = time.perf_counter()
    bb = qs.qs_batch_submit(circs[:sat_n], dtype=dt, mode=0)
    qs.qs_batch_wait(bb)
    t_b = time.perf_counter() - t0
    as_batch = {"circuits_per_s": sat_n / t_b, "end_to_end_ms": 1e3 * t_b,
                "device_ms": qs.qs_batch_get_stats(bb)["device_ms"]}
    qs.qs_batch_release(bb)
    _log(f"serve: the same {sat_n} requests as one batch: {as_batch['circuits_per_s']:.1f} circuits/s")
    big, hook, sat = None, None, alone
    if nb > 0:
        big = _BigJob(qs, torch, W, nb, max_blocks=a.big_blocks)
        hook = big.hook
        sat = _serve_stream(qs, circs[:sat_n], np.zeros(sat_n), dt, hook=hook)
        _log(f"serve saturated, beside n={nb}: {sat['circuits_per_s']:.1f} circuits/s")
    qps = 0.7 * sat["circuits_per_s"]
    main = _serve_stream(qs, circs, W.poisson_arrivals(count, qps, 8), dt, hook=hook)
    main["qps"] = qps
    _log(f"serve at {qps:.1f} qps: p50 {main['p50_ms']:.1f} ms p99 {main['p99_ms']:.1f} ms")
    sweep = {}
    if a.qps_sweep:
        for f in (0.3, 0.5, 1.0):
            r = _serve_stream(qs, circs, W.poisson_arrivals(count, f * sat["circuits_per_s"], 8), dt, hook=hook)
            sweep[str(f)] = {k: r[k] for k in ("circuits_per_s", "p50_ms", "p99_ms", "failed")}
    if big is not None:
        big = big.stop()
    ns = np.array([c.n for c in circs])
    out = _header(a, "served circuits/s", main["circuits_per_s"], "circuits/s", None, "f64",
                  "synthetic (seeded Poisson arrivals; seeded mix of chain circuits, QFTs and Grover searches)",
                  {"workload": f"{count} requests, n log-uniform in [8,28] (mean {ns.mean():.1f}), complex64, "
                               f"Poisson at 0.7x the saturated rate" +
                               (f", beside an n={nb} complex64 depth-24 chain circuit in tile passes with fused "
                                "register blocks, run forward and back for the whole stream" if nb else ""),
                   "requests": count, "qps": qps})
    out.update({"latency_ms": {"p50": main["p50_ms"], "p99": main["p99_ms"]}, "stream": main,
                "saturated": sat, "saturated_alone": alone, "same_requests_as_batch": as_batch,
                "big_circuit": big, "qps_sweep": sweep or None})
    if big:
        ach = big["pass_gbs_algorithmic"]
        out["roofline"] = {"bound": "hbm", "kernel": f"tile passes of the n={nb} circuit (beside the stream)",
                           "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": ach / PEAK_HBM_GBS,
                           "traffic": None}
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline_mix(circs)
    return out


GATE_SRCS = ("paper_2506_09198_amd/csrc/gates.hip", "paper_2506_09198_amd/csrc/device_common.h")
DIAG_SRCS = ("paper_2506_09198_amd/csrc/diag.hip", "paper_2506_09198_amd/csrc/device_common.h")
TILE_SRCS = ("paper_2506_09198_amd/csrc/tile.hip", "paper_2506_09198_amd/csrc/tile_device.h",
             "paper_2506_09198_amd/csrc/planner.cpp")
BATCH_SRCS = ("paper_2506_09198_amd/csrc/tile_batch.hip", "paper_2506_09198_amd/csrc/tile_device.h",
              "paper_2506_09198_amd/csrc/planner.cpp", "paper_2506_09198_amd/csrc/batch.cpp")


def measured_traffic(kernel_class: str, tag: str, srcs=GATE_SRCS):
    """HBM bytes per launch of a kernel class from the committed rocprofv3
    counter summary, or None when the summary is missing or the kernel source
    (the files srcs) has changed since the counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"{tag}_hbm_bytes.txt")
    if not os.path.exists(path):
        return None
    rec = None
    for line in open(path):
        if line.startswith("TRAFFIC_JSON "):
            rec = json.loads(line[len("TRAFFIC_JSON "):])
    if rec is None:
        return None
    sha = hashlib.sha256(b"".join(open(os.path.join(ROOT, f), "rb").read() for f in srcs)).hexdigest()[:16]
    if sha != rec.get("src_sha"):
        return None
    c = rec["classes"].get(kernel_class)
    return None if c is None else c["traffic_bytes_per_launch"]


def main():
    a = _args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {a.gpus} is not supported "
              "(the library runs on one GPU; sharding across GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)
    import torch

    if a.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.complex128, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_per_copy": src.numel() * 16, "copies": 3}))
        return

    import paper_2506_09198_amd as qs
    import workloads as W

    fn = {"sweep": run_sweep, "circuits": run_circuits, "batch": run_batch, "serve": run_serve}[a.workload]
    out = fn(a, qs, torch, W)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
