"""Pins for the FP64 oracle against facts that do not come from the oracle itself:
hand-worked examples of the paper's update formulas, dense Kronecker-product
operators, closed forms (H^n, GHZ, QFT of a basis state, Grover), exact
permutations, invariants, and brute force on tiny inputs."""
import itertools
import math

import numpy as np
import pytest

import workloads as W
import oracle
from oracle import dense
from tests.conftest import golden

TOL = 1e-13


def _rand_state(n, seed):
    g = np.random.default_rng(seed)
    v = g.standard_normal(1 << n) + 1j * g.standard_normal(1 << n)
    return v / np.linalg.norm(v)


def _parse_pairs(vals):
    v = [float(x) for x in vals]
    return np.array(v[0::2]) + 1j * np.array(v[1::2])


def _read_fixture(name):
    rows = []
    with open(golden(name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


# ---------------------------------------------------------------- golden

def test_golden_hadamard_alg1(orc):
    rows = _read_fixture("hadamard_alg1_n2.txt")
    n = int(rows[0][1])
    psi_in = _parse_pairs(rows[1][1:])
    i = 2
    checked = 0
    while i < len(rows):
        t = int(rows[i][1])
        want = _parse_pairs(rows[i + 1][1:])
        got = orc.apply_op(n, psi_in.copy(), [t], W.H)
        assert np.max(np.abs(got - want)) < 1e-15
        checked += 1
        i += 2
    assert checked == 2


def test_golden_controlled_skip(orc):
    rows = _read_fixture("controlled_x_n3.txt")
    n, c, t = int(rows[0][1]), int(rows[1][1]), int(rows[2][1])
    psi = _parse_pairs(rows[3][1:])
    want = _parse_pairs(rows[4][1:])
    got = orc.apply_op(n, psi.copy(), [t], W.X, cmask=1 << c)
    assert np.array_equal(got, want)


def test_golden_cnot_truth_table(orc):
    rows = _read_fixture("cnot_truth_n2.txt")
    for a, b in rows:
        psi = orc.basis(2, int(a))
        orc.apply_op(2, psi, [0], W.X, cmask=1 << 1)
        assert np.array_equal(psi, orc.basis(2, int(b)))


# ---------------------------------------------------------------- gate data

def test_gate_definitions():
    for p, s in ((W.X, W.SQRT_X), (W.Y, W.SQRT_Y), (W.W, W.SQRT_W)):
        assert np.allclose(s @ s, p, atol=1e-15)
        assert np.allclose(s.conj().T @ s, np.eye(2), atol=1e-15)
    # U3 reduces to textbook gates
    assert np.allclose(W.u3(math.pi, 0, math.pi), W.X, atol=1e-15)
    assert np.allclose(W.u3(math.pi / 2, 0, math.pi), W.H, atol=1e-15)
    assert np.allclose(W.u3(math.pi, math.pi / 2, math.pi / 2), W.Y, atol=1e-15)
    rng = np.random.default_rng(0)
    for d in (2, 4, 8):
        u = W.haar_unitary(d, rng)
        assert np.allclose(u.conj().T @ u, np.eye(d), atol=1e-13)
    assert np.array_equal(W.SWAP @ W.SWAP, np.eye(4))


# ---------------------------------------------------------------- dense pins

@pytest.mark.parametrize("n", [1, 3, 5])
def test_1q_every_target_vs_dense(orc, n):
    rng = np.random.default_rng(10 + n)
    for t in range(n):
        u = W.haar_unitary(2, rng)
        psi = _rand_state(n, 100 * n + t)
        want = dense.embed(n, [t], u) @ psi
        got = orc.apply_op(n, psi.copy(), [t], u)
        assert np.max(np.abs(got - want)) < TOL, t


def test_1q_controls_and_values_vs_dense(orc):
    n = 5
    rng = np.random.default_rng(7)
    for t in range(n):
        others = [q for q in range(n) if q != t]
        for nc in (1, 2, 4):
            for ctrl in itertools.islice(itertools.combinations(others, nc), 3):
                cm = sum(1 << c for c in ctrl)
                for cv in (cm, 0, cm & (0b10101)):
                    u = W.haar_unitary(2, rng)
                    psi = _rand_state(n, t * 31 + nc * 7 + cv)
                    want = dense.embed(n, [t], u, cm, cv) @ psi
                    got = orc.apply_op(n, psi.copy(), [t], u, cm, cv)
                    assert np.max(np.abs(got - want)) < TOL


def test_2q_every_ordered_pair_vs_dense(orc):
    n = 4
    rng = np.random.default_rng(3)
    for t0, t1 in itertools.permutations(range(n), 2):
        u = W.haar_unitary(4, rng)
        psi = _rand_state(n, t0 * 5 + t1)
        want = dense.embed(n, [t0, t1], u) @ psi
        got = orc.apply_op(n, psi.copy(), [t0, t1], u)
        assert np.max(np.abs(got - want)) < TOL, (t0, t1)
        others = [q for q in range(n) if q not in (t0, t1)]
        cm = 1 << others[0]
        want = dense.embed(n, [t0, t1], u, cm, cm) @ psi
        got = orc.apply_op(n, psi.copy(), [t0, t1], u, cm, cm)
        assert np.max(np.abs(got - want)) < TOL


@pytest.mark.parametrize("k", [3, 4, 5, 6])
def test_kq_vs_dense(orc, k):
    n = 7
    rng = np.random.default_rng(k)
    for trial in range(3):
        targets = list(rng.permutation(n)[:k])
        u = W.haar_unitary(1 << k, rng)
        psi = _rand_state(n, 50 + trial)
        others = [q for q in range(n) if q not in targets]
        cm = (1 << others[0]) if trial == 2 else 0
        want = dense.embed(n, targets, u, cm, cm) @ psi
        got = orc.apply_op(n, psi.copy(), targets, u, cm, cm)
        assert np.max(np.abs(got - want)) < TOL


def test_circuits_vs_dense(orc):
    n = 6
    circs = [W.random_u3_cnot(n, 60, seed=11), W.rqc_chain(n, 6, 5), W.qft(n, 13),
             W.grover(n, 42)]
    g = W.gate_microbench(n=6, far=3)
    circs.append(g)
    for c in circs:
        psi0 = _rand_state(n, 9)
        want = dense.run(c, psi0)
        got = orc.run_circuit(c, psi0)
        assert np.max(np.abs(got - want)) < 1e-12, c.name


def test_pins_detect_planted_mistakes(orc):
    """Each plausible slip (transposed matrix, conjugated entries, swapped target
    order, a control dropped, a target off by one) changes the result far beyond
    the pin tolerance, so the dense pin cannot pass a wrong oracle."""
    n = 4
    rng = np.random.default_rng(77)
    u2 = W.haar_unitary(2, rng)
    u4 = W.haar_unitary(4, rng)
    psi = _rand_state(n, 1)
    ref1 = dense.embed(n, [2], u2) @ psi
    ref2 = dense.embed(n, [1, 3], u4) @ psi
    ref2c = dense.embed(n, [1, 3], u4, 1, 1) @ psi
    mutants = [
        (orc.apply_op(n, psi.copy(), [2], u2.T), ref1),
        (orc.apply_op(n, psi.copy(), [2], u2.conj()), ref1),
        (orc.apply_op(n, psi.copy(), [1], u2), ref1),
        (orc.apply_op(n, psi.copy(), [3, 1], u4), ref2),
        (orc.apply_op(n, psi.copy(), [1, 3], u4.T), ref2),
        (orc.apply_op(n, psi.copy(), [1, 3], u4), ref2c),
    ]
    for got, ref in mutants:
        assert np.max(np.abs(got - ref)) > 1e-3


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("n", [1, 4, 12, 16])
def test_hadamard_all_uniform(orc, n):
    c = W.Circuit(n)
    for q in range(n):
        c.g1(q, W.H)
    psi = orc.run_circuit(c)
    assert np.max(np.abs(psi - 2.0 ** (-n / 2))) < 1e-15 * n


@pytest.mark.parametrize("n", [2, 10, 20])
def test_ghz(orc, n):
    c = W.Circuit(n).g1(0, W.H)
    for q in range(n - 1):
        c.g1(q + 1, W.X, controls=(q,))
    psi = orc.run_circuit(c)
    want = np.zeros(1 << n, dtype=complex)
    want[0] = want[-1] = W.SQ2
    assert np.max(np.abs(psi - want)) < 1e-15


@pytest.mark.parametrize("n,x", [(3, 5), (8, 77), (12, 2345), (16, 40000)])
def test_qft_basis_closed_form(orc, n, x):
    c = W.qft(n, x)
    assert len(c) == n + n * (n - 1) // 2 + n // 2
    psi = orc.run_circuit(c)
    N = 1 << n
    y = np.arange(N, dtype=np.int64)
    want = np.exp(2j * np.pi * ((x * y) % N) / N) / math.sqrt(N)
    assert np.max(np.abs(psi - want)) < 1e-12


def test_qft_gate_count_at_32():
    c = W.qft(32)
    assert len(c) == 544


@pytest.mark.parametrize("n,mark", [(6, 37), (10, 1000), (14, 123)])
def test_grover_closed_form(orc, n, mark):
    R = W.grover_rounds(n)
    c = W.grover(n, mark)
    assert len(c) == n + R * (2 * n + 2) and len(c) <= 200
    psi = orc.run_circuit(c)
    th = math.asin(2.0 ** (-n / 2))
    s = (-1) ** R
    want = np.full(1 << n, s * math.cos((2 * R + 1) * th) / math.sqrt((1 << n) - 1), dtype=complex)
    want[mark] = s * math.sin((2 * R + 1) * th)
    assert np.max(np.abs(psi - want)) < 1e-12


def test_grover_round_counts():
    assert [W.grover_rounds(n) for n in (10, 14, 18, 22)] == [8, 6, 4, 3]


# ---------------------------------------------------------------- invariants

def test_permutations_exact(orc):
    n = 10
    rng = np.random.default_rng(5)
    for _ in range(50):
        x = int(rng.integers(1 << n))
        a, b = (int(v) for v in rng.choice(n, 2, replace=False))
        psi = orc.basis(n, x)
        orc.apply_op(n, psi, [b], W.X, cmask=1 << a)
        y = x ^ (1 << b) if (x >> a) & 1 else x
        assert np.array_equal(psi, orc.basis(n, y))
        psi = orc.basis(n, x)
        orc.apply_op(n, psi, [a, b], W.SWAP)
        ba, bb = (x >> a) & 1, (x >> b) & 1
        y = (x & ~((1 << a) | (1 << b))) | (bb << a) | (ba << b)
        assert np.array_equal(psi, orc.basis(n, y))


def test_control_zero_amplitudes_untouched(orc):
    n = 8
    psi = _rand_state(n, 3)
    out = orc.apply_op(n, psi.copy(), [1], W.haar_unitary(2, np.random.default_rng(1)), cmask=1 << 6)
    idx = np.arange(1 << n)
    keep = ((idx >> 6) & 1) == 0
    assert np.array_equal(out[keep], psi[keep])


def test_echo_and_norm(orc):
    n = 14
    c = W.random_u3_cnot(n, 300, seed=3)
    psi0 = _rand_state(n, 4)
    psi = orc.run_circuit(c, psi0)
    assert abs(orc.norm2(n, psi) - 1.0) < 1e-13
    back = orc.run_circuit(c.inverse(), psi)
    assert np.max(np.abs(back - psi0)) < 1e-13


# ---------------------------------------------------------------- reductions

def test_probabilities_brute_force(orc):
    n = 7
    psi = _rand_state(n, 8)
    p = np.abs(psi) ** 2
    for qubits in ([], [0], [6], [3, 1], [0, 2, 4, 6], list(range(n)), [5, 0, 3]):
        got = orc.probabilities(n, psi, qubits)
        want = np.zeros(1 << len(qubits))
        for i in range(1 << n):
            o = 0
            for j, q in enumerate(qubits):
                o |= ((i >> q) & 1) << j
            want[o] += p[i]
        assert np.max(np.abs(got - want)) < 1e-15
    assert np.array_equal(orc.probabilities(n, psi, list(range(n))),
                          psi.real ** 2 + psi.imag ** 2)
    assert abs(orc.norm2(n, psi) - 1.0) < 1e-15


def test_outputs_at_matches_full_run(orc):
    n = 9
    rng = np.random.default_rng(21)
    psi = _rand_state(n, 2)
    cases = [([4], W.haar_unitary(2, rng), 0, 0), ([2, 7], W.haar_unitary(4, rng), 1 << 5, 1 << 5),
             ([8], W.haar_unitary(2, rng), 0b11, 0b01), ([0, 1, 3], W.haar_unitary(8, rng), 0, 0)]
    for tg, u, cm, cv in cases:
        full = orc.apply_op(n, psi.copy(), tg, u, cm, cv)
        idx = rng.integers(0, 1 << n, size=64).astype(np.uint64)
        got = orc.outputs_at(idx, tg, u, cm, cv, lambda j: psi[j.astype(np.int64)])
        assert np.max(np.abs(got - full[idx.astype(np.int64)])) < 1e-15


# ---------------------------------------------------------------- generators

def test_generators_deterministic():
    a = W.random_u3_cnot(12, 200, seed=1).arrays()
    b = W.random_u3_cnot(12, 200, seed=1).arrays()
    assert a[0].tobytes() == b[0].tobytes() and a[1].tobytes() == b[1].tobytes()
    c = W.gate_microbench(30)
    assert len(c) == 30 + 2 * (29 + 15)
    r = W.rqc_chain(32, 20, 5)
    assert len(r) == 640 + 310
    s1 = W.random_state(12, 7)
    s2 = W.random_state(12, 7)
    assert np.array_equal(s1, s2) and abs(np.vdot(s1, s1).real - 1) < 1e-14
    m1 = W.circuit_mix(16, 7)
    m2 = W.circuit_mix(16, 7)
    assert [x.name for x in m1] == [x.name for x in m2]


# ---------------------------------------------------------------- Pauli expectations and sampling

_PAULI = {"I": np.eye(2), "X": np.array([[0, 1], [1, 0]], complex), "Y": np.array([[0, -1j], [1j, 0]]),
          "Z": np.diag([1.0, -1.0]).astype(complex)}


def _pauli_dense(n, x, z):
    """Kronecker product of single-qubit Paulis, qubit 0 the rightmost factor."""
    M = np.eye(1, dtype=complex)
    for q in reversed(range(n)):
        xb, zb = (x >> q) & 1, (z >> q) & 1
        M = np.kron(M, _PAULI["Y" if xb and zb else ("X" if xb else ("Z" if zb else "I"))])
    return M


def test_expect_pauli_matches_dense_operator():
    rng = np.random.default_rng(21)
    for n in (1, 2, 4, 6):
        psi = W.random_state(n, 30 + n)
        for _ in range(12):
            x, z = int(rng.integers(1 << n)), int(rng.integers(1 << n))
            want = np.vdot(psi, _pauli_dense(n, x, z) @ psi)
            got = oracle.expect_pauli(n, psi, x, z)
            assert abs(got - want) <= 1e-13, (n, x, z)
            assert abs(got.imag) <= 1e-13  # Hermitian


def test_expect_pauli_closed_forms():
    n = 5
    for xb in (0, 7, 19, 31):  # basis states: <Z^z> = (-1)^|x & z|, <X on any bit> = 0
        psi = oracle.basis(n, xb)
        for z in (1, 6, 31):
            assert oracle.expect_pauli(n, psi, 0, z) == (-1) ** bin(xb & z).count("1")
        assert oracle.expect_pauli(n, psi, 4, 0) == 0
    ghz = np.zeros(1 << n, complex)
    ghz[0] = ghz[-1] = 2 ** -0.5
    assert abs(oracle.expect_pauli(n, ghz, (1 << n) - 1, 0) - 1) < 1e-15   # <X...X> = 1
    assert abs(oracle.expect_pauli(n, ghz, 0, 3) - 1) < 1e-15              # <Z0 Z1> = 1
    assert abs(oracle.expect_pauli(n, ghz, 0, 1)) < 1e-15                  # <Z0> = 0
    plus_i = np.array([1, 1j]) / 2 ** 0.5                                   # Y eigenstate
    assert abs(oracle.expect_pauli(1, plus_i, 1, 1) - 1) < 1e-15


def test_sample_closed_forms_and_brute_force():
    n = 6
    u = np.random.default_rng(5).random(400)
    assert np.all(oracle.sample(n, oracle.basis(n, 37), u) == 37)
    uni = np.full(1 << n, 2 ** (-n / 2), complex)                           # H^n|0>: index = floor(u 2^n)
    away = np.abs(u * (1 << n) - np.round(u * (1 << n))) > 1e-9
    assert np.array_equal(oracle.sample(n, uni, u)[away], np.floor(u * (1 << n))[away].astype(np.uint64))
    ghz = np.zeros(1 << n, complex)
    ghz[0] = ghz[-1] = 2 ** -0.5
    assert np.array_equal(oracle.sample(n, ghz, u), np.where(u < 0.5, 0, (1 << n) - 1).astype(np.uint64))
    for seed in range(5):                                                   # plain numpy inversion
        psi = W.random_state(n, 40 + seed)
        C = np.cumsum(np.abs(psi) ** 2)
        want = np.searchsorted(C, u * C[-1], side="right")
        assert np.array_equal(oracle.sample(n, psi, u), want.astype(np.uint64))


def test_sample_and_expectation_detect_slips():
    """A conjugation slip or a dropped sign breaks the dense comparison; a
    cumulative distribution taken in reverse order breaks the inversion."""
    n = 3
    psi = W.random_state(n, 77)
    want = np.vdot(psi, _pauli_dense(n, 5, 3) @ psi)
    assert abs(np.vdot(psi.conj(), _pauli_dense(n, 5, 3) @ psi.conj()) - want) > 1e-3
    assert abs(oracle.expect_pauli(n, psi, 5, 3) + want) > 1e-3
    u = np.random.default_rng(1).random(200)
    rev = (1 << n) - 1 - oracle.sample(n, psi[::-1].copy(), u).astype(np.int64)
    assert not np.array_equal(rev, oracle.sample(n, psi, u).astype(np.int64))
