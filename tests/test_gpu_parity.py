"""GPU parity: every kernel path against the FP64 oracle on the same seeded
inputs, through the C ABI.

Bars: complex128 max |psi - psi_oracle| <= 1e-12; complex64 fidelity
|<psi_oracle|psi>|^2 >= 1 - 1e-6 (and max abs error <= 2e-5); integer-like
results (basis states, permutations, untouched amplitudes) bit-exact.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TOL128 = 1e-12


@pytest.fixture(scope="module")
def qs():
    import paper_2506_09198_amd as qs

    assert qs.qs_device_count() >= 1, "no HIP device visible"
    return qs


def _state(qs, n, dt, psi0=None, basis=0):
    s = qs.State.create(n, dt)
    if psi0 is not None:
        s.upload(psi0)
    elif basis:
        s.init_basis(basis)
    return s


def _check(got, want, dt, what=""):
    got = got.astype(np.complex128)
    err = float(np.max(np.abs(got - want))) if got.size else 0.0
    if dt == 2:
        assert err <= TOL128, f"{what}: max abs err {err:.3e}"
    else:
        fid = abs(np.vdot(want, got)) ** 2 / max(abs(np.vdot(want, want)) ** 2, 1e-300)
        assert fid >= 1 - 1e-6 and err <= 2e-5, f"{what}: fidelity {fid!r} err {err:.3e}"
    return err


def _rand(n, seed):
    return W.random_state(n, seed)


DTS = [2, 1]  # QS_C128, QS_C64


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("n", [1, 2, 3, 5, 7, 8, 9, 12, 15])
def test_1q_every_target(qs, dt, n):
    rng = np.random.default_rng(100 + n)
    psi0 = _rand(n, n)
    s = _state(qs, n, dt, psi0)
    want = psi0.copy()
    for t in range(n):
        u = W.haar_unitary(2, rng)
        s.apply_1q(t, u)
        oracle.apply_op(n, want, [t], u)
    _check(s.download(), want, dt, f"n={n}")


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("n", [4, 9, 14])
def test_1q_controls(qs, dt, n):
    rng = np.random.default_rng(7 * n)
    psi0 = _rand(n, 3 * n)
    s = _state(qs, n, dt, psi0)
    want = psi0.copy()
    for t in range(n):
        others = [q for q in range(n) if q != t]
        for nc in (1, 2, 3):
            ctrl = list(rng.choice(others, size=min(nc, len(others)), replace=False))
            cm = sum(1 << int(c) for c in ctrl)
            cv = cm if nc != 2 else (1 << int(ctrl[0]))
            u = W.haar_unitary(2, rng)
            s.apply_1q(t, u, cm, cv)
            oracle.apply_op(n, want, [t], u, cm, cv)
    _check(s.download(), want, dt, f"n={n}")


@pytest.mark.parametrize("dt", DTS)
def test_2q_all_pairs(qs, dt):
    n = 6
    rng = np.random.default_rng(5)
    psi0 = _rand(n, 77)
    s = _state(qs, n, dt, psi0)
    want = psi0.copy()
    for t0, t1 in itertools.permutations(range(n), 2):
        u = W.haar_unitary(4, rng)
        s.apply_2q(t0, t1, u)
        oracle.apply_op(n, want, [t0, t1], u)
        others = [q for q in range(n) if q not in (t0, t1)]
        c = int(rng.choice(others))
        s.apply_2q(t0, t1, u, 1 << c)
        oracle.apply_op(n, want, [t0, t1], u, 1 << c, 1 << c)
    _check(s.download(), want, dt)


@pytest.mark.parametrize("dt", DTS)
def test_2q_large(qs, dt):
    n = 16
    rng = np.random.default_rng(9)
    psi0 = _rand(n, 78)
    s = _state(qs, n, dt, psi0)
    want = psi0.copy()
    pairs = [(0, 1), (1, 0), (0, 15), (15, 3), (7, 8), (14, 15), (2, 9)]
    for t0, t1 in pairs:
        u = W.haar_unitary(4, rng)
        others = [q for q in range(n) if q not in (t0, t1)]
        cm = (1 << int(others[3])) | (1 << int(others[-1]))
        s.apply_2q(t0, t1, u)
        oracle.apply_op(n, want, [t0, t1], u)
        s.apply_2q(t0, t1, u, cm, 1 << int(others[3]))
        oracle.apply_op(n, want, [t0, t1], u, cm, 1 << int(others[3]))
    _check(s.download(), want, dt)


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_fused_k(qs, dt, k):
    n = 11
    rng = np.random.default_rng(k)
    psi0 = _rand(n, k)
    s = _state(qs, n, dt, psi0)
    want = psi0.copy()
    for trial in range(3):
        tg = [int(x) for x in rng.permutation(n)[:k]]
        u = W.haar_unitary(1 << k, rng)
        others = [q for q in range(n) if q not in tg]
        cm = (1 << others[0]) if trial == 1 else 0
        s.apply_fused(tg, u, cm)
        oracle.apply_op(n, want, tg, u, cm, cm)
    _check(s.download(), want, dt, f"k={k}")


def test_fused_equals_kron_of_1q(qs):
    n = 10
    rng = np.random.default_rng(1)
    a, b = W.haar_unitary(2, rng), W.haar_unitary(2, rng)
    psi0 = _rand(n, 5)
    s1 = _state(qs, n, 2, psi0)
    s1.apply_fused([3, 8], np.kron(b, a))  # targets[0] = 3 is the low bit
    s2 = _state(qs, n, 2, psi0)
    s2.apply_1q(3, a)
    s2.apply_1q(8, b)
    assert np.max(np.abs(s1.download() - s2.download())) < 1e-14


CIRCS = {
    "u3cnot12": lambda: W.random_u3_cnot(12, 200, seed=1),
    "qft13": lambda: W.qft(13, 4321),
    "rqc14": lambda: W.rqc_chain(14, 12, 3),
    "grover12": lambda: W.grover(12, 2047),
    "bench16": lambda: W.gate_microbench(16, far=7),
}


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("name", list(CIRCS))
@pytest.mark.parametrize("mode,tq", [(1, 0), (0, 0), (0, 6), (0, 9), (0, 12), (0, 13)])
def test_circuits(qs, dt, name, mode, tq):
    c = CIRCS[name]()
    n = c.n
    ops, mats = c.arrays()
    psi0 = _rand(n, 11) if name in ("rqc14", "bench16") else None
    want = oracle.run(n, ops, mats, psi0, c.init_basis)
    s = _state(qs, n, dt, psi0, c.init_basis)
    s.run(ops, mats, mode=mode, tile_qubits=tq)
    _check(s.download(), want, dt, f"{name} mode={mode} tq={tq}")


def _phase_circuit(n, count, seed):
    """Random controlled phases, CZ and one-qubit diagonals (some with a
    further control): every form a diagonal factor group can take."""
    rng = np.random.default_rng(seed)
    c = W.Circuit(n, f"phases{n}")
    for q in range(n):
        c.g1(q, W.H)
    for _ in range(count):
        a, b, e = (int(x) for x in rng.choice(n, 3, replace=False))
        kind = int(rng.integers(4))
        if kind == 0:
            c.g1(a, W.phase(float(rng.uniform(0, 2 * np.pi))), controls=(b,))
        elif kind == 1:
            c.g1(a, W.Z, controls=(b,))
        elif kind == 2:
            c.g1(a, np.diag(np.exp(1j * rng.uniform(0, 2 * np.pi, 2))))
        else:
            c.g1(a, W.phase(float(rng.uniform(0, 2 * np.pi))), controls=(b, e))
    return c


def _groups(qs, c, dt, tq):
    """(thread positions, register bits kept) of every diagonal factor group
    in the plan."""
    from tests.tile_model import SO_DGROUP

    ops, mats = c.arrays()
    tops = qs.qs_plan_export(c.n, dt, ops, mats, tile_qubits=tq)[1]
    return [(int(t["dj"]) & 255, bin((int(t["dj"]) >> 16) & 15).count("1")) for t in tops
            if (int(t["rsv"]) >> 16) == SO_DGROUP]


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("tq", [10, 11, 12])
def test_diag_groups_against_oracle(qs, dt, tq):
    """Diagonal factor groups gathered per thread, with factors that skip
    register bits, against the oracle (random phases, CZ and controlled
    phases on 17 qubits)."""
    c = _phase_circuit(17, 400, 7)
    g = _groups(qs, c, dt, tq)
    assert any(k > 0 for k, _ in g) and any(d < min(4, tq - 8) for _, d in g), g
    ops, mats = c.arrays()
    psi0 = _rand(c.n, 21)
    want = oracle.run(c.n, ops, mats, psi0)
    s = _state(qs, c.n, dt, psi0)
    s.run(ops, mats, mode=0, tile_qubits=tq)
    _check(s.download(), want, dt, f"phases tq={tq}")


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("tq", [10, 11, 12])
def test_diag_groups_uniform_qft25(qs, dt, tq):
    """At 25 qubits the QFT's plan has groups with no thread position (read
    with uniform loads) beside per-thread ones: closed form."""
    n, x = 25, 9876543
    c = W.qft(n, x)
    g = _groups(qs, c, dt, tq)
    assert any(k == 0 for k, _ in g) and any(k > 0 for k, _ in g), g
    ops, mats = c.arrays()
    s = _state(qs, n, dt, basis=x)
    s.run(ops, mats, mode=0, tile_qubits=tq)
    N = 1 << n
    y = np.arange(N, dtype=np.int64)
    want = np.exp(2j * np.pi * ((x * y) % N) / N) / math.sqrt(N)
    _check(s.download(), want, dt, f"qft25 tq={tq}")


def test_config1_parity_and_determinism(qs):
    c = W.random_u3_cnot(12, 200, seed=1)
    ops, mats = c.arrays()
    want = oracle.run(12, ops, mats)
    outs = []
    for mode in (1, 0, 0):
        s = _state(qs, 12, 2)
        s.run(ops, mats, mode=mode)
        outs.append(s.download())
        assert np.max(np.abs(outs[-1] - want)) <= TOL128
    assert outs[1].tobytes() == outs[2].tobytes()


@pytest.mark.parametrize("dt", DTS)
def test_qft_closed_form_n20(qs, dt):
    n, x = 20, 777777
    c = W.qft(n, x)
    s = _state(qs, n, dt, basis=x)
    s.run_circuit(c)
    N = 1 << n
    y = np.arange(N, dtype=np.int64)
    want = np.exp(2j * np.pi * ((x * y) % N) / N) / math.sqrt(N)
    _check(s.download(), want, dt, "qft20")


def test_permutations_bit_exact(qs):
    n = 13
    rng = np.random.default_rng(3)
    s = _state(qs, n, 2)
    for _ in range(20):
        x = int(rng.integers(1 << n))
        a, b = (int(v) for v in rng.choice(n, 2, replace=False))
        s.init_basis(x)
        s.apply_1q(b, W.X, 1 << a)
        s.apply_2q(a, b, W.SWAP)
        y = x ^ (1 << b) if (x >> a) & 1 else x
        ba, bb = (y >> a) & 1, (y >> b) & 1
        y = (y & ~((1 << a) | (1 << b))) | (bb << a) | (ba << b)
        got = s.download()
        assert np.array_equal(got, oracle.basis(n, y))


def test_controls_leave_other_amplitudes_bitwise(qs):
    n = 12
    psi0 = _rand(n, 4)
    s = _state(qs, n, 2, psi0)
    s.apply_1q(2, W.haar_unitary(2, np.random.default_rng(0)), 1 << 9)
    got = s.download()
    keep = ((np.arange(1 << n) >> 9) & 1) == 0
    assert np.array_equal(got[keep], psi0[keep])


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("ctl", [(0,), (1,), (2,), (3,), (1, 2), (2, 3), (0, 11)])
def test_inline_controls_bitwise(qs, dt, ctl):
    """Controls on bits inside a 128-byte line (tested per lane; the lanes
    that fail write their amplitudes back or skip the store, by run size):
    amplitudes whose controls fail stay bitwise equal, the others match the
    oracle, for 1q and 2q gates with high and low targets."""
    n = 14
    rng = np.random.default_rng(90 + sum(ctl))
    psi0 = _rand(n, 5)
    start = psi0 if dt == 2 else psi0.astype(np.complex64).astype(np.complex128)
    cm = sum(1 << c for c in ctl)
    cv = cm & ~(1 << ctl[0]) if len(ctl) > 1 else cm  # first control on |0>, the rest on |1>
    free = [q for q in range(n) if q not in ctl]
    for tg in ([free[0]], [free[-1]], [free[0], free[1]], [free[1], free[-1]], [free[-2], free[-1]]):
        u = W.haar_unitary(1 << len(tg), rng)
        s = _state(qs, n, dt, psi0)
        if len(tg) == 1:
            qs.qs_apply_1q(s.h, tg[0], u, cm, cv)
        else:
            qs.qs_apply_2q(s.h, tg[0], tg[1], u, cm, cv)
        got = s.download()
        s.close()
        want = start.copy()
        oracle.apply_op(n, want, tuple(tg), u, cm, cv)
        keep = (np.arange(1 << n) & cm) != cv
        base = psi0 if dt == 2 else psi0.astype(np.complex64)
        assert np.array_equal(got[keep], base[keep]), (tg, ctl)
        _check(got, want, dt, f"targets {tg} controls {ctl}")


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("n", [1, 5, 13, 18])
def test_probabilities(qs, dt, n):
    psi0 = _rand(n, 21)
    s = _state(qs, n, dt, psi0)
    ref_in = psi0 if dt == 2 else psi0.astype(np.complex64).astype(np.complex128)
    rng = np.random.default_rng(n)
    sets = [[], [0], [n - 1], list(rng.permutation(n)[: min(3, n)]), list(range(min(n, 10)))]
    for qb in sets:
        qb = [int(q) for q in qb]
        got = s.probabilities(qb)
        want = oracle.probabilities(n, ref_in, qb)
        assert np.max(np.abs(got - want)) <= 1e-13, qb
        again = s.probabilities(qb)
        assert got.tobytes() == again.tobytes()
    assert abs(s.norm() - oracle.norm2(n, ref_in)) <= 1e-13


def test_torch_external_state(qs):
    import torch

    n = 10
    t = torch.zeros(1 << n, dtype=torch.complex128, device="cuda")
    t[0] = 1
    s = qs.State.from_torch(t)
    for q in range(n):
        s.apply_1q(q, W.H)
    s.sync()
    assert torch.allclose(t, torch.full_like(t, 2 ** (-n / 2)), atol=1e-15)
    s.close()


def test_trace_records(qs):
    n = 14
    s = _state(qs, n, 2)
    qs.qs_trace_enable(s.h, True)
    s.apply_1q(0, W.H)
    s.apply_1q(13, W.H)
    s.apply_2q(3, 9, W.SWAP)
    recs = qs.qs_trace_read(s.h)
    assert [qs.KIND_NAMES[k] for k in recs["kind"]] == ["1q_lo", "1q_hi", "2q"]
    assert (recs["bytes"] == 2 * 16 * (1 << n)).all() and (recs["ms"] > 0).all()


def test_error_leaves_state_untouched(qs):
    n = 8
    psi0 = _rand(n, 9)
    s = _state(qs, n, 2, psi0)
    with pytest.raises(qs.QSError):
        s.apply_1q(8, W.H)
    with pytest.raises(qs.QSError):
        s.apply_2q(1, 1, np.eye(4))
    with pytest.raises(qs.QSError):
        s.apply_1q(1, W.H, 1 << 1)
    assert np.array_equal(s.download(), psi0)


@pytest.mark.parametrize("dt,fp32", [(1, 0), (2, 0), (1, 1)])
@pytest.mark.parametrize("name", list(CIRCS))
@pytest.mark.parametrize("fk,tq,fmin", [(4, 0, 1), (5, 0, 1), (5, 9, 1), (4, 8, 2), (5, 13, 3)])
def test_fused_mfma_blocks(qs, dt, fp32, name, fk, tq, fmin, monkeypatch):
    """Fused dense blocks on FP64 matrix cores, both amplitude types, and
    (complex64) on FP32 matrix cores with the hi + bfloat16 lo split, against
    the oracle (complex128 to the FP64 bar)."""
    monkeypatch.setenv("QS_FUSE_MIN", str(fmin))
    monkeypatch.setenv("QS_FUSE_FP32", str(fp32))
    c = CIRCS[name]()
    n = c.n
    ops, mats = c.arrays()
    npass, nops = qs.qs_plan_circuit(n, dt, ops, mats, fuse_k=fk, tile_qubits=tq)
    psi0 = _rand(n, 11) if name in ("rqc14", "bench16") else None
    want = oracle.run(n, ops, mats, psi0, c.init_basis)
    s = _state(qs, n, dt, psi0, c.init_basis)
    s.run(ops, mats, mode=0, fuse_k=fk, tile_qubits=tq)
    _check(s.download(), want, dt, f"{name} fuse_k={fk} tq={tq} ({nops} ops in {npass} passes)")


def _batch_mix(seed):
    rng = np.random.default_rng(seed)
    circs = []
    for n in (3, 7, 10, 12, 13, 14, 15, 16, 17, 18):
        kind = int(rng.integers(3))
        if kind == 0:
            c = W.rqc_chain(n, int(rng.integers(3, 9)), int(rng.integers(1000)))
        elif kind == 1:
            c = W.qft(n, int(rng.integers(1 << n)))
        else:
            c = W.grover(n, int(rng.integers(1 << n)))
        circs.append(c)
    circs.append(W.random_u3_cnot(11, 150, seed=5))
    return circs


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("mode", [0, 1])
def test_batch_matches_oracle(qs, dt, mode):
    circs = _batch_mix(3)
    b = qs.qs_batch_submit(circs, dtype=dt, mode=mode, streams=4)
    try:
        qs.qs_batch_wait(b)
        st = qs.qs_batch_get_stats(b)
        assert st["launches"] >= 1 and st["device_ms"] > 0
        for i, c in enumerate(circs):
            want = oracle.run_circuit(c)
            got = qs.qs_batch_download(b, i, dt)
            _check(got, want, dt, f"batch mode={mode} circuit {i} {c.name}")
    finally:
        qs.qs_batch_release(b)


@pytest.mark.parametrize("dt", DTS)
def test_batch_result_independent_of_co_residents(qs, dt):
    circs = _batch_mix(4)
    b = qs.qs_batch_submit(circs, dtype=dt, mode=0)
    try:
        qs.qs_batch_wait(b)
        together = [qs.qs_batch_download(b, i, dt) for i in range(len(circs))]
    finally:
        qs.qs_batch_release(b)
    for i in (0, 3, 5, 8):
        b1 = qs.qs_batch_submit([circs[i]], dtype=dt, mode=0)
        try:
            alone = qs.qs_batch_download(b1, 0, dt)
        finally:
            qs.qs_batch_release(b1)
        assert alone.tobytes() == together[i].tobytes(), circs[i].name


def test_batch_rejects_invalid_circuit_before_any_work(qs):
    good = W.qft(6, 1)
    bad = W.Circuit(4).g1(5, W.H)
    with pytest.raises(qs.QSError) as e:
        qs.qs_batch_submit([good, bad])
    assert e.value.status == qs.QS_ERR_ARG and "circuit 1" in str(e.value)


@pytest.mark.parametrize("dt", [1, 2])
@pytest.mark.parametrize("graph", [0, 1])
def test_batch_replay_bitwise(qs, dt, graph):
    """A fused batch replayed (from its HIP graph or by re-enqueueing) gives
    bitwise the first run's states, every time, with eager device work and
    synchronisations between the replays; the first run matches the oracle."""
    import torch

    circs = [W.qft(n, 5 * n + 1) for n in (9, 12, 14, 17)] + [W.rqc_chain(n, 6, n) for n in (10, 13, 15, 16, 18)] + \
            [W.grover(n, 3 * n) for n in (11, 15)]
    b = qs.qs_batch_submit(circs, dtype=dt, mode=0, graph=graph)
    try:
        qs.qs_batch_wait(b)
        first = [qs.qs_batch_download(b, i, dt) for i in range(len(circs))]
        for i, c in enumerate(circs):
            want = oracle.run_circuit(c)
            got = first[i].astype(np.complex128)
            if dt == 2:
                assert float(np.max(np.abs(got - want))) <= 1e-12, c.name
            else:
                assert abs(np.vdot(want, got)) ** 2 >= 1 - 1e-6, c.name
        x = torch.randn(1 << 20, device="cuda")
        for rep in range(3):
            y = (x * (rep + 1)).sum()  # the program's own eager work between replays
            torch.cuda.synchronize()
            qs.qs_batch_replay(b)
            qs.qs_batch_wait(b)
            for i in range(len(circs)):
                assert qs.qs_batch_download(b, i, dt).tobytes() == first[i].tobytes(), (rep, circs[i].name)
            assert float(y.item()) == float(y.item())
        st = qs.qs_batch_get_stats(b)
        assert st["device_ms"] > 0
    finally:
        qs.qs_batch_release(b)


def test_batch_replay_rejects_per_gate(qs):
    b = qs.qs_batch_submit([W.qft(8, 3)], dtype=2, mode=1)
    try:
        qs.qs_batch_wait(b)
        with pytest.raises(qs.QSError) as e:
            qs.qs_batch_replay(b)
        assert e.value.status == qs.QS_ERR_UNSUPPORTED
    finally:
        qs.qs_batch_release(b)


@pytest.mark.parametrize("dt", [1, 2])
def test_batch_tune(qs, dt):
    """The autotuner times every candidate on a sample and returns one of them;
    a batch with the tuned options matches the oracle."""
    sample = [W.rqc_chain(n, 8, 100 + n) for n in (14, 15, 16, 17, 18)] + [W.qft(n, n) for n in (15, 17)]
    best, rows = qs.qs_batch_tune(sample, dtype=dt)
    expect = 9 + 5  # tile x fusion, then five workgroup-class variants
    assert len(rows) == expect and all(r["device_ms"] > 0 for r in rows)
    keys = ("tile_qubits", "fuse_k", "whole_max", "persist_max")
    fastest = min(rows, key=lambda r: r["device_ms"])
    assert tuple(best[k] for k in keys) == tuple(fastest[k] for k in keys)
    stage1 = min(rows[:expect - 5], key=lambda r: r["device_ms"])
    assert all((r["tile_qubits"], r["fuse_k"]) == (stage1["tile_qubits"], stage1["fuse_k"]) for r in rows[expect - 5:])
    b = qs.qs_batch_submit(sample, dtype=dt, mode=0, **best)
    try:
        qs.qs_batch_wait(b)
        for i, c in enumerate(sample):
            got = qs.qs_batch_download(b, i, dt).astype(np.complex128)
            want = oracle.run_circuit(c)
            if dt == 2:
                assert float(np.max(np.abs(got - want))) <= 1e-12, c.name
            else:
                assert abs(np.vdot(want, got)) ** 2 >= 1 - 1e-6, c.name
    finally:
        qs.qs_batch_release(b)


@pytest.mark.parametrize("dt", DTS)
def test_batch_probabilities_and_norm(qs, dt):
    """Per-circuit marginals and norms of a fused batch, computed on the
    device, against the oracle's reductions of the downloaded final states."""
    circs = _batch_mix(21)
    arrs = [(c.n, *c.arrays(), c.init_basis) for c in circs]
    b = qs.qs_batch_submit(arrs, dtype=dt, mode=0)
    qs.qs_batch_wait(b)
    rng = np.random.default_rng(4)
    for i, c in enumerate(circs):
        got_state = qs.qs_batch_download(b, i, dt).astype(np.complex128)
        for qb in ([], [0], list(rng.permutation(c.n)[: min(3, c.n)]), list(range(c.n))):
            qb = [int(q) for q in qb]
            got = qs.qs_batch_probabilities(b, i, qb)
            want = oracle.probabilities(c.n, got_state, qb)
            assert np.max(np.abs(got - want)) <= 1e-13, (c.name, qb)
        assert abs(qs.qs_batch_norm(b, i) - oracle.norm2(c.n, got_state)) <= 1e-13
    with pytest.raises(qs.QSError):
        qs.qs_batch_probabilities(b, len(circs), [0])
    with pytest.raises(qs.QSError):
        qs.qs_batch_probabilities(b, 0, [0, 0])
    with pytest.raises(qs.QSError):
        qs.qs_batch_probabilities(b, 0, list(range(circs[0].n + 1)))
    qs.qs_batch_release(b)


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("whole,persist", [(8, 12), (3, 9), (11, 18)])
def test_batch_workgroup_classes(qs, dt, whole, persist):
    """Non-default class boundaries (whole-in-LDS / persistent / pass-major),
    including a whole-circuit limit below the tile size, match the oracle."""
    circs = _batch_mix(6)
    b = qs.qs_batch_submit(circs, dtype=dt, mode=0, whole_max=whole, persist_max=persist)
    try:
        qs.qs_batch_wait(b)
        for i, c in enumerate(circs):
            _check(qs.qs_batch_download(b, i, dt), oracle.run_circuit(c), dt, f"classes {whole}/{persist} {c.name}")
    finally:
        qs.qs_batch_release(b)
    with pytest.raises(qs.QSError):
        qs.qs_batch_submit(circs, dtype=dt, mode=0, whole_max=14)
    with pytest.raises(qs.QSError):
        qs.qs_batch_submit(circs, dtype=dt, mode=0, whole_max=10, persist_max=9)
