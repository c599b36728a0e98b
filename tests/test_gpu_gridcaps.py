"""Block-loop paths against the oracle, and grid-size independence.

Every looping kernel (per-gate and diagonal gates, tile passes, batch and
serving rounds, the restore pass, grid-stride helpers) is driven with its
workgroup cap forced down to a few blocks, so that each workgroup walks many
chunks, tiles or entries.  Each run is compared element by element with the
FP64 oracle, and runs under different caps must agree bit for bit: every
amplitude is produced by exactly one lane from the same inputs in the same
order whatever the grid, so the grid can change nothing (the race guard of
the batch and serving rounds)."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TOL128 = 1e-12
CAPS = [1, 3, 5, None]  # None = library default


@pytest.fixture(scope="module")
def qs():
    import paper_2506_09198_amd as qs

    assert qs.qs_device_count() >= 1, "no HIP device visible"
    return qs


def _check(got, want, dt, what):
    got = got.astype(np.complex128)
    err = float(np.max(np.abs(got - want)))
    if dt == 2:
        assert err <= TOL128, f"{what}: max abs err {err:.3e}"
    else:
        fid = abs(np.vdot(want, got)) ** 2
        assert fid >= 1 - 1e-6 and err <= 2e-5, f"{what}: fidelity {fid!r} err {err:.3e}"


def _knobs(cap):
    if cap is None:
        return {}
    return {"gate_grid_cap": cap, "tile_grid_cap": cap, "round_grid_cap": cap, "aux_grid_cap": cap}


CIRCS = {
    "rqc16": lambda: W.rqc_chain(16, 8, 21),
    "qft17": lambda: W.qft(17, 70001),
    "grover14": lambda: W.grover(14, 9999),
    "bench16": lambda: W.gate_microbench(16, far=7),
    "u3cnot15": lambda: W.random_u3_cnot(15, 120, seed=4),
}


@pytest.mark.parametrize("dt", [2, 1])
@pytest.mark.parametrize("name", list(CIRCS))
@pytest.mark.parametrize("mode,tq", [(1, 0), (0, 0), (0, 9)])
def test_circuit_block_loops(qs, dt, name, mode, tq):
    c = CIRCS[name]()
    n = c.n
    ops, mats = c.arrays()
    psi0 = W.random_state(n, 31) if name in ("rqc16", "bench16") else None
    want = oracle.run(n, ops, mats, psi0, c.init_basis)
    outs = []
    for cap in CAPS:
        with qs.tunables(**_knobs(cap)):
            with qs.State.create(n, dt) as s:
                if psi0 is not None:
                    s.upload(psi0)
                else:
                    s.init_basis(c.init_basis)
                s.run(ops, mats, mode=mode, tile_qubits=tq)
                got = s.download()
        _check(got, want, dt, f"{name} mode={mode} tq={tq} cap={cap}")
        outs.append(got)
    for cap, o in zip(CAPS[1:], outs[1:]):
        assert o.tobytes() == outs[0].tobytes(), f"{name}: cap {cap} differs bitwise from cap {CAPS[0]}"


@pytest.mark.parametrize("dt", [2, 1])
def test_restore_pass_block_loop(qs, dt):
    """The QFT with SWAP relabeling forced ends with restore passes; with a
    grid of 1-5 workgroups they loop over every tile pair."""
    n = 16
    c = W.qft(n, 4242)
    ops, mats = c.arrays()
    assert len(qs.qs_plan_restore(n, dt, ops, mats)) >= 1
    want = oracle.run_circuit(c)
    outs = []
    for cap in CAPS:
        with qs.tunables(**_knobs(cap)):
            with qs.State.create(n, dt) as s:
                s.init_basis(c.init_basis)
                s.run(ops, mats, mode=0)
                got = s.download()
        _check(got, want, dt, f"qft16 remap cap={cap}")
        outs.append(got)
    assert all(o.tobytes() == outs[0].tobytes() for o in outs[1:])


def _mix():
    # n 17/18 are pass-major (one block per tile per round); smaller ones take
    # the whole-in-LDS and persistent classes
    return [W.rqc_chain(18, 6, 5), W.qft(17, 12345), W.grover(17, 777), W.rqc_chain(17, 9, 8),
            W.qft(11, 99), W.rqc_chain(14, 5, 3), W.grover(12, 1000)]


@pytest.mark.parametrize("dt", [2, 1])
def test_batch_round_block_loop(qs, dt):
    circs = _mix()
    wants = [oracle.run_circuit(c) for c in circs]
    outs = []
    for cap in CAPS:
        with qs.tunables(**_knobs(cap)):
            b = qs.qs_batch_submit(circs, dtype=dt, mode=0)
            try:
                qs.qs_batch_wait(b)
                got = [qs.qs_batch_download(b, i, dt) for i in range(len(circs))]
            finally:
                qs.qs_batch_release(b)
        for c, g, w in zip(circs, got, wants):
            _check(g, w, dt, f"batch {c.name} cap={cap}")
        outs.append(got)
    for got in outs[1:]:
        for c, a, b in zip(circs, got, outs[0]):
            assert a.tobytes() == b.tobytes(), c.name


@pytest.mark.parametrize("dt", [2, 1])
def test_serving_round_block_loop(qs, dt):
    import time

    circs = _mix()
    wants = [oracle.run_circuit(c) for c in circs]
    outs = []
    for cap in CAPS:
        with qs.tunables(**_knobs(cap)):
            srv = qs.qs_server_create(dtype=dt, hbm_budget=1 << 30)
            try:
                ids = [qs.qs_server_submit(srv, c) for c in circs]
                done = {}
                t_end = time.time() + 60
                while len(done) < len(ids):
                    for r in qs.qs_server_poll(srv):
                        done[r["id"]] = r
                    assert time.time() < t_end, "serving loop did not finish"
                    time.sleep(0.0005)
                assert all(done[i]["status"] == 0 for i in ids)
                got = [qs.qs_server_download(srv, i, dt) for i in ids]
            finally:
                qs.qs_server_destroy(srv)
        for c, g, w in zip(circs, got, wants):
            _check(g, w, dt, f"serve {c.name} cap={cap}")
        outs.append(got)
    for got in outs[1:]:
        for c, a, b in zip(circs, got, outs[0]):
            assert a.tobytes() == b.tobytes(), c.name


SCHEDULES = [
    {},
    {"gate_low_in_regs": 0},
    {"gate_low_in_regs": 2},
    {"gate_xcd_swizzle": 1},
    {"gate_xcd_swizzle": 2},
    {"gate_wg_per_cu": 1},
    {"gate_wg_per_cu": 8},
    {"slots_no_high": 1, "slots_one_high": 2, "slots_two_high": 4},
    {"slots_no_high": 2, "slots_one_high": 4, "slots_two_high": 2},
    {"gate_grid_cap": 3, "gate_xcd_swizzle": 2, "gate_low_in_regs": 2},
]


def _pergate_list(n, rng):
    """Every 1q target with and without controls (including controls inside a
    128-byte line), and 2q pairs: both inside a line, one inside, adjacent,
    far, with controls."""
    gates = []
    for t in range(n):
        gates.append(((t,), W.haar_unitary(2, rng), 0, 0))
        for cm_bits in ((0,), (1,), (2, 5), (n - 1,)):
            cs = [c for c in cm_bits if c != t and c < n]
            if cs:
                cm = sum(1 << c for c in cs)
                gates.append(((t,), W.haar_unitary(2, rng), cm, cm & ~(1 << cs[0]) if len(cs) > 1 else cm))
    for t0, t1 in ((0, 1), (1, 0), (0, 2), (2, 4), (3, 4), (5, 6), (0, n - 1), (n - 1, 4), (6, 7), (n - 2, n - 1)):
        gates.append(((t0, t1), W.haar_unitary(4, rng), 0, 0))
        others = [q for q in (0, 1, 3, 9) if q not in (t0, t1)]
        cm = (1 << others[0]) | (1 << others[1])
        gates.append(((t0, t1), W.haar_unitary(4, rng), cm, 1 << others[0]))
    return gates


@pytest.mark.parametrize("dt", [2, 1])
@pytest.mark.parametrize("n", [10, 16])
def test_pergate_schedules(qs, dt, n):
    """The per-gate kernel under every schedule knob (registers vs shuffles
    for low targets, chunk order by XCD, workgroups per CU, slots per lane,
    a looping grid) against the oracle, and bitwise the same across them."""
    rng = np.random.default_rng(600 + n)
    gates = _pergate_list(n, rng)
    psi0 = W.random_state(n, 61)
    want = psi0.copy()
    for tg, u, cm, cv in gates:
        oracle.apply_op(n, want, tg, u, cm, cv)
    outs = []
    for knobs in SCHEDULES:
        with qs.tunables(**knobs):
            with qs.State.create(n, dt) as s:
                s.upload(psi0 if dt == 2 else psi0.astype(np.complex64))
                for tg, u, cm, cv in gates:
                    if len(tg) == 1:
                        qs.qs_apply_1q(s.h, tg[0], u, cm, cv)
                    else:
                        qs.qs_apply_2q(s.h, tg[0], tg[1], u, cm, cv)
                got = s.download()
        _check(got, want, dt, f"n={n} {knobs}")
        outs.append(got)
    for knobs, o in zip(SCHEDULES[1:], outs[1:]):
        assert o.tobytes() == outs[0].tobytes(), f"{knobs} differs bitwise from the default schedule"


@pytest.mark.parametrize("dt", [2, 1])
@pytest.mark.parametrize("name", ["rqc16", "qft17", "u3cnot15"])
def test_tile_waves4_bitwise(qs, dt, name):
    """Tile passes of 2^11 amplitudes with the kernel held to 4 waves per SIMD
    and with the compiler-sized kernel: both against the oracle and bitwise
    the same (the register limit changes where values live, not the
    arithmetic)."""
    c = CIRCS[name]()
    ops, mats = c.arrays()
    psi0 = W.random_state(c.n, 32) if name == "rqc16" else None
    want = oracle.run(c.n, ops, mats, psi0, c.init_basis)
    outs = []
    for w4 in (0, 1):
        with qs.tunables(tile_waves4=w4):
            with qs.State.create(c.n, dt) as s:
                if psi0 is not None:
                    s.upload(psi0 if dt == 2 else psi0.astype(np.complex64))
                else:
                    s.init_basis(c.init_basis)
                s.run(ops, mats, mode=0, tile_qubits=11)
                got = s.download()
        _check(got, want, dt, f"{name} tile_waves4={w4}")
        outs.append(got)
    assert outs[0].tobytes() == outs[1].tobytes()


@pytest.mark.parametrize("dt", [2, 1])
def test_reduction_block_order_bitwise(qs, dt):
    """The reductions with their chunks in workgroup order and in XCD-
    contiguous order: the same partial sums in the same places, so bitwise
    the same marginals, norm and Pauli expectations, and both within the FP64
    bar of the oracle."""
    n = 17
    psi0 = W.random_state(n, 71)
    sets = [[], [0, 1, 2], [n - 3, n - 2, n - 1], [0, 5, 9, 14], list(range(8))]
    paulis = [(0, (1 << n) - 1), (0x5555 & ((1 << n) - 1), 0x2AAA & ((1 << n) - 1))]
    outs = []
    for order in (1, 2):
        with qs.tunables(reduce_xcd_order=order):
            with qs.State.create(n, dt) as s:
                s.upload(psi0 if dt == 2 else psi0.astype(np.complex64))
                host = s.download().astype(np.complex128)
                res = [s.probabilities(q) for q in sets if q] + [np.array([s.norm()])]
                res += [np.array([qs.qs_expect_pauli(s.h, x, z)]) for x, z in paulis]
        for q, r in zip([q for q in sets if q], res):
            want = oracle.probabilities(n, host, q)
            assert float(np.max(np.abs(r - want))) <= 1e-13, (order, q)
        outs.append(res)
    for a, b in zip(outs[0], outs[1]):
        assert a.tobytes() == b.tobytes()


@pytest.mark.parametrize("dt", [2, 1])
def test_gate_schedule_tuner_and_cache(qs, dt, tmp_path):
    """qs_tune_gates times every schedule candidate per gate class on the
    caller's state and leaves the state bitwise as it was; the chosen
    schedules are installed (gates still match the oracle and equal the
    built-in schedule's results bit for bit), written to the cache file and
    read back from it by the next call without timing."""
    import json

    n = 16
    cache = str(tmp_path / "gate_sched.jsonl")
    psi0 = W.random_state(n, 81)
    base = psi0 if dt == 2 else psi0.astype(np.complex64)
    rng = np.random.default_rng(82)
    gates = _pergate_list(n, rng)
    want = psi0.copy() if dt == 2 else psi0.astype(np.complex64).astype(np.complex128)
    for tg, u, cm, cv in gates:
        oracle.apply_op(n, want, tg, u, cm, cv)

    def run_gates(s):
        for tg, u, cm, cv in gates:
            if len(tg) == 1:
                qs.qs_apply_1q(s.h, tg[0], u, cm, cv)
            else:
                qs.qs_apply_2q(s.h, tg[0], tg[1], u, cm, cv)
        return s.download()

    qs.qs_tune_gates_reset()
    try:
        with qs.State.create(n, dt) as s:
            s.upload(base)
            ref = run_gates(s)  # built-in schedules
        with qs.State.create(n, dt) as s:
            s.upload(base)
            rows = qs.qs_tune_gates(s.h, cache)
            assert s.download().tobytes() == base.tobytes()  # tuning left the state as it was
            assert [r["cls"] for r in rows] == [0, 1, 2, 3]
            assert all(r["slots"] in (1, 2, 4, 8) and r["gbs"] > 0 and not r["from_cache"] for r in rows)
            assert all(r["slots"] != 8 for r in rows[1:])
            got = run_gates(s)
        _check(got, want, dt, "tuned schedules")
        assert got.tobytes() == ref.tobytes()
        lines = [json.loads(l) for l in open(cache)]
        assert len(lines) == 4 and len({l["key"] for l in lines}) == 1 and f"n{n}" in lines[0]["key"]
        qs.qs_tune_gates_reset()
        with qs.State.create(n, dt) as s:
            again = qs.qs_tune_gates(s.h, cache)
        assert all(r["from_cache"] for r in again)
        assert [(r["slots"], r["wg_per_cu"], r["xcd"]) for r in again] == \
            [(r["slots"], r["wg_per_cu"], r["xcd"]) for r in rows]
        with pytest.raises(qs.QSError):
            with qs.State.create(8, dt) as s:
                qs.qs_tune_gates(s.h, None)
    finally:
        qs.qs_tune_gates_reset()


@pytest.mark.parametrize("dt", [2, 1])
def test_restore_pass_run_lengths(qs, dt):
    """The qubit-order restore pass with runs of 2^4, 2^5 and (complex64)
    2^6 amplitudes: each against the oracle and bitwise the same (a pure
    permutation moves every amplitude unchanged)."""
    n = 17
    c = W.qft(n, 31337)
    ops, mats = c.arrays()
    assert len(qs.qs_plan_restore(n, dt, ops, mats)) >= 1
    want = oracle.run_circuit(c)
    outs = []
    for run in ((4, 5) if dt == 2 else (4, 5, 6)):
        with qs.tunables(perm_run_log2=run):
            with qs.State.create(n, dt) as s:
                s.init_basis(c.init_basis)
                s.run(ops, mats, mode=0)
                got = s.download()
        _check(got, want, dt, f"qft17 restore runs 2^{run}")
        outs.append(got)
    assert all(o.tobytes() == outs[0].tobytes() for o in outs[1:])
