"""The pass planner's gate order, checked on the CPU (no GPU needed).

The planner may reorder gates that commute, so that one tile pass absorbs
more of them.  Here the planned order is checked to be a permutation that
keeps every pass's dense targets inside its tile, and the FP64 oracle applied
in the planned order must give the state of the circuit order (gates that do
not commute keep their order, so the two agree to rounding).  A swap of two
gates that do not commute is shown to change the result, so the comparison
can fail."""
import numpy as np
import pytest

import oracle
import workloads as W


@pytest.fixture(scope="module")
def qs():
    import paper_2506_09198_amd as qs

    return qs


def _random_mixed(n, count, seed):
    """Dense and diagonal gates with and without controls (control values 0 or 1)."""
    rng = np.random.default_rng(seed)
    c = W.Circuit(n, f"mixed_n{n}_s{seed}")
    for _ in range(count):
        kind = int(rng.integers(6))
        k = {0: 1, 1: 2, 2: 1, 3: 2, 4: 3, 5: 1}[kind]
        qs_ = [int(x) for x in rng.permutation(n)[: k + int(rng.integers(0, 3))]]
        tg, ctl = qs_[:k], qs_[k:]
        cv = sum(int(b) << q for b, q in zip(rng.integers(0, 2, size=len(ctl)), ctl))
        if kind in (0, 5):
            u = W.u3(*rng.uniform(0, 2 * np.pi, 3))
        elif kind in (1, 4):
            u = W.haar_unitary(1 << k, rng)
        else:
            u = np.diag(np.exp(1j * rng.uniform(0, 2 * np.pi, 1 << k)))
        c.add(tg, u, ctl, cv)
    return c


def _circuits():
    return [W.random_u3_cnot(9, 150, seed=3), W.rqc_chain(10, 8, 4), W.qft(9, 300), W.grover(8, 77),
            _random_mixed(9, 160, 5), _random_mixed(10, 200, 6), _random_mixed(12, 250, 7), W.rqc_chain(12, 10, 8),
            W.rqc_chain(13, 2, 632), W.rqc_chain(12, 3, 2), W.swap_network(11, 120, 9)]


@pytest.mark.parametrize("tq,low", [(4, 2), (5, 3), (6, 0), (10, 3), (11, 5)])
@pytest.mark.parametrize("ci", range(11))
def test_planned_order_matches_oracle(qs, monkeypatch, ci, tq, low):
    monkeypatch.setenv("QS_TILE_LOW", str(low))
    c = _circuits()[ci]
    ops, mats = c.arrays()
    order, pass_of, masks = qs.qs_plan_order(c.n, qs.QS_C128, ops, mats, tile_qubits=tq)
    assert sorted(order.tolist()) == list(range(len(ops)))
    assert np.all(np.diff(pass_of) >= 0)
    assert len(masks) == qs.qs_plan_circuit(c.n, qs.QS_C128, ops, mats, tile_qubits=tq, remap=1)[0]
    for g, p in zip(order, pass_of):
        o = ops[g]
        dense = not np.allclose(np.diag(np.diag(c.gates[g][1])), c.gates[g][1], atol=0, rtol=0)
        if dense:
            tm = sum(1 << int(t) for t in o["t"][: o["nt"]])
            assert tm & ~int(masks[p]) == 0, (g, p)
        assert bin(int(masks[p])).count("1") <= max(tq, int(o["nt"]))
    ref = oracle.run_circuit(c)
    got = oracle.run(c.n, ops[order], mats, oracle.basis(c.n, c.init_basis))
    assert float(np.max(np.abs(got - ref))) <= 1e-12


def test_reordering_pays_for_chain_circuits(qs):
    r = W.rqc_chain(32, 20, 5)
    ops, mats = r.arrays()
    order, pass_of, _ = qs.qs_plan_order(32, qs.QS_C128, ops, mats, tile_qubits=11)
    assert pass_of[-1] + 1 <= 45  # in circuit order it takes 90
    assert not np.array_equal(order, np.arange(len(ops)))


def test_single_tile_keeps_circuit_order(qs):
    c = _random_mixed(8, 120, 9)
    ops, mats = c.arrays()
    order, pass_of, _ = qs.qs_plan_order(8, qs.QS_C128, ops, mats, tile_qubits=8)
    assert np.array_equal(order, np.arange(len(ops))) and pass_of.max() == 0


def test_noncommuting_swap_is_detected():
    """The oracle comparison above is sharp: exchanging two adjacent
    uncontrolled dense gates that share a target changes the state far beyond
    rounding.  (Controlled gates can commute by their control values alone.)"""
    c = _random_mixed(6, 40, 11)
    ops, mats = c.arrays()
    ref = oracle.run_circuit(c)
    for i in range(len(ops) - 1):
        a = set(ops[i]["t"][: ops[i]["nt"]].tolist())
        b = set(ops[i + 1]["t"][: ops[i + 1]["nt"]].tolist())
        da = np.allclose(np.diag(np.diag(c.gates[i][1])), c.gates[i][1], atol=0, rtol=0)
        db = np.allclose(np.diag(np.diag(c.gates[i + 1][1])), c.gates[i + 1][1], atol=0, rtol=0)
        if a & b and not da and not db and ops[i]["cmask"] == 0 and ops[i + 1]["cmask"] == 0:
            perm = np.arange(len(ops))
            perm[i], perm[i + 1] = i + 1, i
            got = oracle.run(c.n, ops[perm], mats, oracle.basis(c.n, c.init_basis))
            assert float(np.max(np.abs(got - ref))) > 1e-6
            return
    pytest.fail("no adjacent non-commuting pair in the sample circuit")


@pytest.mark.parametrize("dt", [1, 2])
@pytest.mark.parametrize("tq,low", [(10, 5), (11, 6), (12, 5), (13, 6), (0, 5)])
@pytest.mark.parametrize("ci", range(11))
def test_encoded_plan_matches_oracle(qs, monkeypatch, ci, tq, low, dt):
    """The planner's encoded passes (segments, fused register blocks, the
    diagonal forms) and restoring passes, executed by a host model of the
    kernels, give the oracle's state; tile sizes up to the whole state (tq =
    0: tile = n)."""
    from tests.tile_model import run_plan

    monkeypatch.setenv("QS_TILE_LOW", str(low))
    c = _circuits()[ci]
    t = c.n if tq == 0 else tq
    ops, mats = c.arrays()
    passes, tops, pool = qs.qs_plan_export(c.n, dt, ops, mats, tile_qubits=t)
    restore = qs.qs_plan_restore(c.n, dt, ops, mats, tile_qubits=t)
    got = run_plan(c.n, passes, tops, pool, oracle.basis(c.n, c.init_basis), restore)
    ref = oracle.run_circuit(c)
    assert float(np.max(np.abs(got - ref))) <= 1e-12


def _swap_circuits():
    return [W.qft(9, 300), W.qft(12, 1234), W.swap_network(11, 120, 9), W.swap_network(12, 200, 10),
            W.swap_network(7, 60, 11)]


@pytest.mark.parametrize("dt", [1, 2])
@pytest.mark.parametrize("tq,low", [(4, 2), (6, 3), (10, 5), (11, 6)])
@pytest.mark.parametrize("ci", range(5))
def test_relabeled_plan_matches_oracle(qs, monkeypatch, ci, tq, low, dt):
    """With every uncontrolled SWAP turned into a relabeling (forced), the
    passes on physical positions followed by the restoring involutions give
    the oracle's state, and the plan has no SWAP left in it."""
    from tests.tile_model import run_plan

    monkeypatch.setenv("QS_TILE_LOW", str(low))
    monkeypatch.setenv("QS_REMAP_ALWAYS", "1")
    c = _swap_circuits()[ci]
    ops, mats = c.arrays()
    passes, tops, pool = qs.qs_plan_export(c.n, dt, ops, mats, tile_qubits=tq)
    restore = qs.qs_plan_restore(c.n, dt, ops, mats, tile_qubits=tq)
    assert 1 <= len(restore) <= 2
    for tau in restore:  # involutions of bit positions
        assert sorted(tau.tolist()) == list(range(c.n)) and all(tau[tau[p]] == p for p in range(c.n))
    got = run_plan(c.n, passes, tops, pool, oracle.basis(c.n, c.init_basis), restore)
    ref = oracle.run_circuit(c)
    assert float(np.max(np.abs(got - ref))) <= 1e-12
    # dropping the restore passes must break the comparison (the qubits are permuted)
    bad = run_plan(c.n, passes, tops, pool, oracle.basis(c.n, c.init_basis))
    assert float(np.max(np.abs(bad - ref))) > 1e-6


def test_long_swap_cycle_needs_two_involutions(qs, monkeypatch):
    """A 5-cycle of qubits (four SWAPs) is not an involution: two restoring
    passes; QFT's swaps pair disjoint qubits: one."""
    monkeypatch.setenv("QS_REMAP_ALWAYS", "1")
    c = W.Circuit(8, "cycle5")
    for q in range(8):
        c.g1(q, W.H)
    for a in range(4):
        c.g2(a, a + 1, W.SWAP)
    c.g1(0, W.X)
    ops, mats = c.arrays()
    assert len(qs.qs_plan_restore(8, 2, ops, mats, tile_qubits=4)) == 2
    q = W.qft(10, 3)
    ops, mats = q.arrays()
    assert len(qs.qs_plan_restore(10, 2, ops, mats, tile_qubits=4)) == 1


def test_swap_relabeling_pays_for_qft(qs):
    """32-qubit QFT: relabeling its 16 SWAPs saves tile passes, at the cost of
    one restoring pass; remap = 1 keeps the SWAPs as gates."""
    c = W.qft(32, 5)
    ops, mats = c.arrays()
    for dt in (1, 2):
        auto = qs.qs_plan_circuit(32, dt, ops, mats)[0]
        plain = qs.qs_plan_circuit(32, dt, ops, mats, remap=1)[0]
        assert auto + 2 <= plain, (dt, auto, plain)
        assert len(qs.qs_plan_restore(32, dt, ops, mats)) == 1
        assert qs.qs_plan_restore(32, dt, ops, mats, remap=1) == []
    with pytest.raises(qs.QSError):
        qs.qs_plan_circuit(32, 1, ops, mats, remap=2)


@pytest.mark.parametrize("tq", [10, 11, 12])
def test_diag_groups_drop_unused_register_bits(qs, tq):
    """A diagonal group's factor table leaves out the register bits its
    product does not depend on (the QFT's phase groups mostly touch one or
    two of them), and some groups use no thread position at all; the
    compacted plans still give the oracle's state (host model)."""
    from tests.tile_model import SO_DGROUP, run_plan

    r = min(4, tq - 8)
    big = W.qft(25, 4321)
    ops, mats = big.arrays()
    tops = qs.qs_plan_export(big.n, 2, ops, mats, tile_qubits=tq)[1]
    groups = [t for t in tops if (int(t["rsv"]) >> 16) == SO_DGROUP]
    assert groups
    dep = [(int(t["dj"]) >> 16) & 15 for t in groups]
    kt = [int(t["dj"]) & 255 for t in groups]
    kg = [(int(t["dj"]) >> 8) & 255 for t in groups]
    assert all(d < (1 << r) for d in dep)
    assert any(bin(d).count("1") < r for d in dep), dep
    assert any(k == 0 for k in kt), kt
    for t, d, a, b in zip(groups, dep, kt, kg):
        assert int(t["k"]) == bin(d).count("1") + a + b
    c = W.qft(14, 4321)
    ops, mats = c.arrays()
    passes, tops, pool = qs.qs_plan_export(c.n, 2, ops, mats, tile_qubits=tq)
    got = run_plan(c.n, passes, tops, pool, oracle.basis(c.n, c.init_basis),
                   qs.qs_plan_restore(c.n, 2, ops, mats, tile_qubits=tq))
    assert float(np.max(np.abs(got - oracle.run_circuit(c)))) <= 1e-12


@pytest.mark.parametrize("fp32", [0, 1])
@pytest.mark.parametrize("dt", [1, 2])
@pytest.mark.parametrize("fk,tq", [(4, 10), (5, 11), (5, 12)])
def test_fused_blocks_encoded_match_oracle(qs, monkeypatch, fk, tq, dt, fp32):
    """Passes with fused matrix-core blocks, their fragments decoded back into
    matrices by the host model: the oracle's state, to FP64 rounding for the
    FP64 fragments and to the bfloat16 remainder (about 2^-33 of each entry)
    for the FP32 hi + lo fragments (complex64 only; complex128 keeps FP64)."""
    from tests.tile_model import run_plan

    monkeypatch.setenv("QS_FUSE_MIN", "1")
    monkeypatch.setenv("QS_FUSE_FP32", str(fp32))
    for c in (W.rqc_chain(14, 8, 41), W.qft(13, 77), W.grover(12, 123)):
        ops, mats = c.arrays()
        passes, tops, pool = qs.qs_plan_export(c.n, dt, ops, mats, tile_qubits=tq, fuse_k=fk)
        assert any(int(t["kind"]) == 4 for t in tops), c.name
        assert all(int(t["dclass"]) == (fp32 if dt == 1 else 0) for t in tops if int(t["kind"]) == 4)
        restore = qs.qs_plan_restore(c.n, dt, ops, mats, tile_qubits=tq, fuse_k=fk)
        got = run_plan(c.n, passes, tops, pool, oracle.basis(c.n, c.init_basis), restore)
        err = float(np.max(np.abs(got - oracle.run_circuit(c))))
        assert err <= (1e-8 if (fp32 and dt == 1) else 1e-12), (c.name, err)


def test_fp32_fragments_split_the_fp64_matrix(qs, monkeypatch):
    """The FP32 form's hi + lo parts reproduce the FP64 form's matrix to the
    bfloat16 remainder, and hi alone is each entry rounded to FP32."""
    from tests.tile_model import mfma_matrix

    monkeypatch.setenv("QS_FUSE_MIN", "1")
    c = W.rqc_chain(14, 6, 5)
    ops, mats = c.arrays()
    monkeypatch.setenv("QS_FUSE_FP32", "0")
    _, t64, p64 = qs.qs_plan_export(c.n, 1, ops, mats, tile_qubits=11, fuse_k=5)
    monkeypatch.setenv("QS_FUSE_FP32", "1")
    _, t32, p32 = qs.qs_plan_export(c.n, 1, ops, mats, tile_qubits=11, fuse_k=5)
    m64 = [mfma_matrix(t, p64) for t in t64 if int(t["kind"]) == 4]
    m32 = [mfma_matrix(t, p32) for t in t32 if int(t["kind"]) == 4]
    assert len(m64) == len(m32) > 0
    diffs = []
    for a, b in zip(m64, m32):
        d = float(np.max(np.abs(a - b)))
        assert d <= 2.0 ** -32 * float(np.max(np.abs(a))), d
        assert np.allclose(a @ a.conj().T, np.eye(a.shape[0]), atol=1e-12)
        diffs.append(d)
    # blocks of sqrt(X)/sqrt(Y) gates only are exact in FP32; those with
    # sqrt(W) (entries with 1/sqrt(2)) need the lo part
    assert max(diffs) > 0.0
