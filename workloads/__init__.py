"""Seeded synthetic inputs shared by the GPU path, the oracle, the tests and the bench.

This module only *describes* work: gate matrices (as data), circuits as a flat
list of operations, random initial states and request streams.  It performs no
state-vector arithmetic; applying gates, fusing them and reducing states belong
to the simulator (and, separately, to the oracle).

Circuit IR
----------
A circuit is ``(n, ops, mats)``:

* ``ops`` is a numpy structured array of ``OP_DTYPE`` records (64 bytes each):
  ``nt`` target count (1..6), ``t[6]`` target qubits (``t[0]`` is the least
  significant bit of the matrix index, the same little-endian convention as the
  state index), ``flags`` (0), ``cmask`` control bitmask, ``cvals`` required
  values of the control bits (a subset of ``cmask``), ``moff`` offset in doubles
  of the op's matrix inside ``mats``.
* ``mats`` is one float64 array; each op's matrix is ``2^nt x 2^nt`` complex,
  row-major, interleaved ``(re, im)``.

Qubit ``q`` is bit ``q`` of the amplitude index (the paper's Alg. 1 pairs index
``i`` with ``i + 2^q`` for target ``q``, Section II-C).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

OP_DTYPE = np.dtype(
    [
        ("nt", "<i4"),
        ("t", "<i4", (6,)),
        ("flags", "<u4"),
        ("cmask", "<u8"),
        ("cvals", "<u8"),
        ("moff", "<u8"),
        ("rsv", "<u8"),
    ],
    align=False,
)
assert OP_DTYPE.itemsize == 64

# ---------------------------------------------------------------------------
# Gate matrices (data).  Definitions follow the standard conventions; the paper
# writes out only the Hadamard update (Alg. 1, Alg. 8) and names Pauli-Y and
# CNOT (Fig. ben3).
# ---------------------------------------------------------------------------

SQ2 = 1.0 / math.sqrt(2.0)
I2 = np.eye(2, dtype=np.complex128)
H = np.array([[SQ2, SQ2], [SQ2, -SQ2]], dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
W = (X + Y) * SQ2
SWAP = np.array(
    [[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], dtype=np.complex128
)


def u3(theta: float, phi: float, lam: float) -> np.ndarray:
    """OpenQASM 2 U3(theta, phi, lambda)."""
    c, s = math.cos(theta / 2.0), math.sin(theta / 2.0)
    return np.array(
        [
            [c, -np.exp(1j * lam) * s],
            [np.exp(1j * phi) * s, np.exp(1j * (phi + lam)) * c],
        ],
        dtype=np.complex128,
    )


def sqrt_pauli(p: np.ndarray) -> np.ndarray:
    """Principal square root of an involutory Pauli-like P: (1+i)/2 I + (1-i)/2 P."""
    return 0.5 * (1 + 1j) * I2 + 0.5 * (1 - 1j) * p


SQRT_X = sqrt_pauli(X)
SQRT_Y = sqrt_pauli(Y)
SQRT_W = sqrt_pauli(W)


def phase(phi: float) -> np.ndarray:
    """diag(1, e^{i phi}); as a controlled 1q gate it is CP(phi)."""
    return np.array([[1, 0], [0, np.exp(1j * phi)]], dtype=np.complex128)


def haar_unitary(d: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-random d x d unitary: QR of a complex Gaussian with the phases of R's
    diagonal moved into Q (Mezzadri's correction)."""
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) * SQ2
    q, r = np.linalg.qr(z)
    dg = np.diagonal(r)
    return q * (dg / np.abs(dg))[np.newaxis, :]


# ---------------------------------------------------------------------------
# Circuits
# ---------------------------------------------------------------------------


@dataclass
class Circuit:
    n: int
    name: str = "circuit"
    init_basis: int = 0
    gates: list = field(default_factory=list)  # (targets, matrix, cmask, cvals)

    def add(self, targets, u, controls=(), cvals=None):
        targets = tuple(int(t) for t in targets)
        u = np.asarray(u, dtype=np.complex128)
        d = 1 << len(targets)
        assert u.shape == (d, d), (u.shape, targets)
        cmask = 0
        for c in controls:
            cmask |= 1 << int(c)
        if cvals is None:
            cv = cmask
        else:  # cvals given as a bitmask over the same positions
            cv = int(cvals) & cmask
        self.gates.append((targets, u, cmask, cv))
        return self

    # convenience builders
    def g1(self, t, u, controls=(), cvals=None):
        return self.add((t,), u, controls, cvals)

    def g2(self, t0, t1, u, controls=(), cvals=None):
        return self.add((t0, t1), u, controls, cvals)

    def __len__(self):
        return len(self.gates)

    def arrays(self):
        """Pack into (ops, mats) in the IR described in the module docstring."""
        G = len(self.gates)
        ops = np.zeros(G, dtype=OP_DTYPE)
        if G == 0:
            return ops, np.zeros(0, dtype=np.float64)
        nt = np.fromiter((len(g[0]) for g in self.gates), dtype=np.int32, count=G)
        t = np.full((G, 6), -1, dtype=np.int32)
        for k in range(1, 7):
            sel = np.nonzero(nt == k)[0]
            if sel.size:
                t[sel, :k] = np.array([self.gates[i][0] for i in sel], dtype=np.int32)
        sizes = 2 * (1 << (2 * nt.astype(np.int64)))
        moff = np.zeros(G, dtype=np.uint64)
        moff[1:] = np.cumsum(sizes[:-1]).astype(np.uint64)
        ops["nt"] = nt
        ops["t"] = t
        ops["cmask"] = np.fromiter((g[2] for g in self.gates), dtype=np.uint64, count=G)
        ops["cvals"] = np.fromiter((g[3] for g in self.gates), dtype=np.uint64, count=G)
        ops["moff"] = moff
        mats = np.concatenate([np.ascontiguousarray(g[1], dtype=np.complex128).ravel().view(np.float64)
                               for g in self.gates])
        return ops, mats

    def inverse(self) -> "Circuit":
        """The adjoint circuit: reversed order, each matrix conjugate-transposed."""
        c = Circuit(self.n, self.name + "_inv", self.init_basis)
        for tg, u, cm, cv in reversed(self.gates):
            c.gates.append((tg, u.conj().T.copy(), cm, cv))
        return c


def _rng(seed, stream):
    return np.random.default_rng([int(seed), int(stream)])


def random_u3_cnot(n=12, depth=200, seed=1, leading_h=True) -> Circuit:
    """H on every qubit, then `depth` gates: with probability 1/2 a U3 with angles
    uniform in [0, 2pi) on a uniform target, else a CNOT on a uniform ordered pair
    of distinct qubits (control, target)."""
    rng = _rng(seed, 0)
    c = Circuit(n, f"u3cnot_n{n}_s{seed}")
    if leading_h:
        for q in range(n):
            c.g1(q, H)
    for _ in range(depth):
        if rng.random() < 0.5:
            t = int(rng.integers(n))
            th, ph, la = rng.uniform(0.0, 2.0 * math.pi, 3)
            c.g1(t, u3(th, ph, la))
        else:
            ct, tg = rng.choice(n, 2, replace=False)
            c.g1(int(tg), X, controls=(int(ct),))
    return c


def gate_microbench(n=30, seed_u3=2, seed_haar=3, seed_ctrl=4, far=15) -> Circuit:
    """The per-target gate sweep: one U3 per target, then Haar 4x4 unitaries on
    adjacent pairs (t, t+1) and far pairs (t, t+far), each once uncontrolled and
    once with one control drawn uniformly from the remaining qubits."""
    c = Circuit(n, f"gatebench_n{n}")
    r1 = _rng(seed_u3, 1)
    for t in range(n):
        th, ph, la = r1.uniform(0.0, 2.0 * math.pi, 3)
        c.g1(t, u3(th, ph, la))
    rh, rc = _rng(seed_haar, 1), _rng(seed_ctrl, 1)
    pairs = [(t, t + 1) for t in range(n - 1)] + [(t, t + far) for t in range(max(0, n - far))]
    for t0, t1 in pairs:
        u = haar_unitary(4, rh)
        c.g2(t0, t1, u)
        others = [q for q in range(n) if q not in (t0, t1)]
        if others:
            ctl = int(others[int(rc.integers(len(others)))])
            c.g2(t0, t1, u, controls=(ctl,))
    return c


def rqc_chain(n: int, depth: int, seed: int) -> Circuit:
    """Random circuit on a 1D chain: each layer applies an i.i.d. uniform choice of
    sqrt(X)/sqrt(Y)/sqrt(W) to every qubit, then CZ on (2j, 2j+1) in even layers
    and on (2j+1, 2j+2) in odd layers (open chain).  The choices of all layers
    are drawn at once, layer-major, from Generator([seed, 2])."""
    rng = _rng(seed, 2)
    pick = rng.integers(3, size=(depth, n))
    c = Circuit(n, f"rqc_n{n}_d{depth}_s{seed}")
    choices = (SQRT_X, SQRT_Y, SQRT_W)
    gates = c.gates
    for layer in range(depth):
        row = pick[layer]
        for q in range(n):
            gates.append(((q,), choices[row[q]], 0, 0))
        for a in range(layer % 2, n - 1, 2):
            m = 1 << a
            gates.append(((a + 1,), Z, m, m))
    return c


def qft(n: int, basis: int = 0) -> Circuit:
    """Iterative QFT, little-endian: for j = n-1 .. 0: H(j) then CP(pi / 2^(j-k))
    controlled by k on target j for k = j-1 .. 0; then SWAP(q, n-1-q)."""
    c = Circuit(n, f"qft_n{n}", init_basis=int(basis))
    for j in range(n - 1, -1, -1):
        c.g1(j, H)
        for k in range(j - 1, -1, -1):
            c.g1(j, phase(math.pi / (1 << (j - k))), controls=(k,))
    for q in range(n // 2):
        c.g2(q, n - 1 - q, SWAP)
    return c


def grover_rounds(n: int, gate_cap: int = 200) -> int:
    full = int(math.floor(math.pi / 4.0 * math.sqrt(2.0 ** n)))
    capped = (gate_cap - n) // (2 * n + 2)
    return max(0, min(full, capped))


def grover(n: int, mark: int, rounds: int | None = None, gate_cap: int = 200) -> Circuit:
    """H on every qubit, then R rounds of [phase -1 on |mark>; H^n; phase -1 on
    |0..0>; H^n].  Each phase flip is one multi-controlled 1q gate on qubit n-1
    whose controls are the other qubits with the required control values."""
    if rounds is None:
        rounds = grover_rounds(n, gate_cap)
    c = Circuit(n, f"grover_n{n}_m{mark}_r{rounds}")
    full = (1 << n) - 1
    top = n - 1
    others = [q for q in range(n) if q != top]
    flip_if_one = np.array([[1, 0], [0, -1]], dtype=np.complex128)
    flip_if_zero = np.array([[-1, 0], [0, 1]], dtype=np.complex128)
    for q in range(n):
        c.g1(q, H)
    for _ in range(rounds):
        u = flip_if_one if (mark >> top) & 1 else flip_if_zero
        c.g1(top, u, controls=others, cvals=mark & (full >> 1))
        for q in range(n):
            c.g1(q, H)
        c.g1(top, flip_if_zero, controls=others, cvals=0)
        for q in range(n):
            c.g1(q, H)
    return c


def swap_network(n: int, count: int, seed: int) -> Circuit:
    """A U3 on every qubit, then `count` gates drawn from Generator([seed, 4]):
    uncontrolled SWAPs that walk a random cycle of the qubits (so their
    product is a long permutation) or join a random pair, controlled SWAPs,
    Haar 4x4 gates and controlled phases."""
    rng = _rng(seed, 4)
    c = Circuit(n, f"swapnet_n{n}_c{count}_s{seed}")
    for q in range(n):
        c.g1(q, u3(*rng.uniform(0, 2 * np.pi, 3)))
    cyc = [int(q) for q in rng.permutation(n)]
    for i in range(count):
        r = int(rng.integers(6))
        if r < 2:
            c.g2(cyc[i % n], cyc[(i + 1) % n], SWAP)
        elif r == 2:
            a, b = (int(x) for x in rng.choice(n, 2, replace=False))
            c.g2(a, b, SWAP)
        elif r == 3:
            a, b, k = (int(x) for x in rng.choice(n, 3, replace=False))
            c.add([a, b], SWAP, [k], 0 if rng.random() < 0.5 else 1 << k)
        elif r == 4:
            a, b = (int(x) for x in rng.choice(n, 2, replace=False))
            c.g2(a, b, haar_unitary(4, rng))
        else:
            t, k = (int(x) for x in rng.choice(n, 2, replace=False))
            c.add([t], phase(rng.uniform(0, 2 * np.pi)), [k], 1 << k)
    return c


# ---------------------------------------------------------------------------
# States and mixes
# ---------------------------------------------------------------------------


def random_state(n: int, seed: int, dtype=np.complex128, block_log2: int = 22) -> np.ndarray:
    """Complex Gaussian amplitudes normalised in float64.  Generated in blocks of
    2^block_log2 amplitudes, block b from Generator(PCG64([seed, 3, b])), so the
    result does not depend on how many blocks are drawn at once."""
    N = 1 << n
    out = np.empty(N, dtype=np.complex128)
    bs = min(N, 1 << block_log2)
    for b in range(N // bs):
        g = np.random.default_rng([int(seed), 3, b])
        v = g.standard_normal(2 * bs)
        out[b * bs:(b + 1) * bs] = v[0::2] + 1j * v[1::2]
    nrm = math.sqrt(float(np.sum(out.real ** 2) + np.sum(out.imag ** 2)))
    out /= nrm
    return out.astype(dtype, copy=False)


def log_uniform_n(rng: np.random.Generator, lo: int, hi: int) -> int:
    """n = floor(exp(U(ln lo, ln(hi+1)))), so P(n) is proportional to ln((n+1)/n)."""
    v = int(math.floor(math.exp(rng.uniform(math.log(lo), math.log(hi + 1)))))
    return min(max(v, lo), hi)


def circuit_mix(count: int, seed: int, n_lo: int = 10, n_hi: int = 22,
                d_lo: int = 20, d_hi: int = 200) -> list:
    """A batch of circuits: n log-uniform in [n_lo, n_hi]; type uniform over
    {random chain circuit with depth ~ U{d_lo..d_hi} layers, full QFT on a random
    basis state, Grover capped at 200 gates with a random marked state}."""
    rng = _rng(seed, 4)
    out = []
    for i in range(count):
        n = log_uniform_n(rng, n_lo, n_hi)
        kind = int(rng.integers(3))
        if kind == 0:
            d = int(rng.integers(d_lo, d_hi + 1))
            c = rqc_chain(n, d, seed * 1000003 + i)
        elif kind == 1:
            c = qft(n, int(rng.integers(1 << n)))
        else:
            c = grover(n, int(rng.integers(1 << n)))
        out.append(c)
    return out


def poisson_arrivals(count: int, qps: float, seed: int) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson stream at rate qps."""
    rng = _rng(seed, 5)
    return np.cumsum(rng.exponential(1.0 / qps, size=count))
