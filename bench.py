#!/usr/bin/env python3
"""Benchmark of the gate engine on one MI355X.

Default workload (one "step"): the per-target gate sweep on a 30-qubit
complex128 state (16 GiB) -- one seeded U3 on every target 0..29, then seeded
Haar-random 4x4 unitaries on adjacent pairs (t, t+1) and far pairs (t, t+15),
each once uncontrolled and once with one control: 118 gates, each one launch
of the per-gate kernels, state resident in HBM.

Prints ONE JSON line: amplitude-updates/s (value), algorithmic HBM GB/s, the
roofline of the dominant kernel measured with HIP events recorded by the
library around every launch in the timed region, and the FP64 oracle timed on
host cores on a bounded sample of the same workload.
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


def _args():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--n", type=int, default=30)
    p.add_argument("--dtype", choices=["c128", "c64"], default="c128")
    p.add_argument("--mode", choices=["pergate", "planned"], default="pergate")
    p.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    p.add_argument("--cpu-n", type=int, default=26, help="qubits of the oracle sample")
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run 3 torch copies of 4 GiB (reference for HBM byte counters) and exit")
    return p.parse_args()


def cpu_baseline(n_cpu: int) -> dict:
    """The FP64 oracle on the same gate sweep at n_cpu qubits (bounded sample)."""
    import oracle
    import workloads as W

    c = W.gate_microbench(n_cpu)
    ops, mats = c.arrays()
    psi = W.random_state(n_cpu, 2)
    t0 = time.perf_counter()
    oracle.run(n_cpu, ops, mats, psi)
    dt = time.perf_counter() - t0
    updates = sum(1 << (n_cpu - bin(int(o["cmask"])).count("1")) for o in ops)
    return {"value": updates / dt, "unit": "amp-updates/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"gate sweep at n={n_cpu} complex128 ({len(ops)} gates, one pass, {dt:.1f} s)"}


def measured_traffic(kernel_class: str, tag: str):
    """HBM bytes per launch of a kernel class from the committed rocprofv3
    counter summary, or None when the summary is missing or the kernel source
    has changed since the counters were taken."""
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
    srcs = ["paper_2506_09198_amd/csrc/gates.hip", "paper_2506_09198_amd/csrc/device_common.h"]
    sha = hashlib.sha256(b"".join(open(os.path.join(ROOT, f), "rb").read() for f in srcs)).hexdigest()[:16]
    if sha != rec.get("src_sha"):
        return None
    c = rec["classes"].get(kernel_class)
    return None if c is None else c["traffic_bytes_per_launch"]


def main():
    a = _args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {a.gpus} is not supported "
              "(multi-GPU sharding is a design note, not part of this build)", file=sys.stderr)
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

    n = a.n
    dt = qs.QS_C128 if a.dtype == "c128" else qs.QS_C64
    tdt = torch.complex128 if dt == qs.QS_C128 else torch.complex64
    S = 16 if dt == qs.QS_C128 else 8
    circ = W.gate_microbench(n)
    ops, mats = circ.arrays()
    gates = [(tg, u, cm, cv) for (tg, u, cm, cv) in circ.gates]
    upd_step = sum(1 << (n - bin(cm).count("1")) for (_, _, cm, _) in gates)
    bytes_step = 2 * S * upd_step

    # seeded synthetic input, resident in HBM: complex Gaussian normalised in FP64
    g = torch.Generator(device="cuda")
    g.manual_seed(2)
    psi = torch.empty(1 << n, dtype=tdt, device="cuda")
    chunk = 1 << 26
    nrm2 = 0.0
    for i in range(0, 1 << n, chunk):
        blk = torch.randn(min(chunk, (1 << n) - i), dtype=torch.complex128, device="cuda", generator=g)
        nrm2 += float((blk.real.square().sum() + blk.imag.square().sum()).item())
        psi[i:i + blk.numel()] = blk.to(tdt)
    psi /= math.sqrt(nrm2)
    torch.cuda.synchronize()
    s = qs.State.from_torch(psi)

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
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        step()
    s.sync()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    recs = qs.qs_trace_read(s.h, 1 << 20)
    qs.qs_trace_enable(s.h, False)
    norm = s.norm()

    value = upd_step * a.steps / elapsed
    # per kernel class, from the HIP events around each launch
    kinds = {}
    for r in recs:
        k = qs.KIND_NAMES[int(r["kind"])]
        d = kinds.setdefault(k, {"launches": 0, "ms": 0.0, "bytes": 0})
        d["launches"] += 1
        d["ms"] += float(r["ms"])
        d["bytes"] += int(r["bytes"])
    for k, d in kinds.items():
        d["avg_ms"] = d["ms"] / d["launches"]
        d["avg_bytes"] = d["bytes"] / d["launches"]
        d["gbs"] = d["bytes"] / (d["ms"] * 1e-3) / 1e9
    dom = max(kinds, key=lambda k: kinds[k]["ms"])
    D = kinds[dom]
    achieved = D["avg_bytes"] / (D["avg_ms"] * 1e-3) / 1e9
    kern_ms = sum(d["ms"] for d in kinds.values())
    out = {
        "metric": "amplitude-updates/s",
        "value": value,
        "unit": "amp-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": elapsed * 1e3 / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if dt == qs.QS_C128 else "f32",
        "data": "synthetic (seeded complex Gaussian state, seeded U3 and Haar 4x4 gates)",
        "config": {"workload": f"gate sweep n={n} {a.dtype}: U3 on t=0..{n-1}, Haar 4x4 on (t,t+1) and "
                               f"(t,t+15), uncontrolled and 1-controlled; {len(gates)} gates/step",
                   "n": n, "state_bytes": (1 << n) * S, "gates_per_step": len(gates), "mode": a.mode},
        "hbm_gbs_algorithmic": bytes_step * a.steps / elapsed / 1e9,
        "hbm_frac_algorithmic": bytes_step * a.steps / elapsed / 1e9 / PEAK_HBM_GBS,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS,
                     "traffic": (measured_traffic(dom, f"gate_sweep_n{n}_{a.dtype}") if a.mode == "pergate" else None),
                     "traffic_unit": "HBM bytes/launch (rocprofv3 FETCH_SIZE+WRITE_SIZE, copy-calibrated)",
                     "algorithmic_bytes_per_launch": D["avg_bytes"]},
        "kernels": {k: {"launches": d["launches"], "avg_ms": round(d["avg_ms"], 4), "gbs": round(d["gbs"], 1)}
                    for k, d in kinds.items()},
        "event_coverage": kern_ms / (elapsed * 1e3),
        "norm_minus_1": norm - 1.0,
    }
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(a.cpu_n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
