"""Dense operator checks (n <= 8): the independent pin for the oracle.

TEST INFRASTRUCTURE ONLY.  Each gate is built as a full 2^n x 2^n matrix from
Kronecker products, with qubit 0 as the rightmost factor (qubit q is bit q of
the amplitude index), and the circuit operator is the ordered matrix product.
Nothing here shares code with ``qs_oracle.c``: it reaches the same definition by
a different route (linear algebra on the full operator instead of index walks).
"""
from __future__ import annotations

import numpy as np

P0 = np.array([[1, 0], [0, 0]], dtype=np.complex128)
P1 = np.array([[0, 0], [0, 1]], dtype=np.complex128)
I2 = np.eye(2, dtype=np.complex128)


def _kron_list(factors_msb_first):
    out = np.ones((1, 1), dtype=np.complex128)
    for f in factors_msb_first:
        out = np.kron(out, f)
    return out


def embed(n: int, targets, U: np.ndarray, cmask: int = 0, cvals: int | None = None) -> np.ndarray:
    """Full operator of a (controlled) gate.

    Uncontrolled: U acts on the targets' subspace with targets[j] as bit j of
    U's row/column index.  Built as a sum over the 2^k x 2^k matrix units:
    sum_{r,m} U[r,m] * (x)_q F_q with F_{targets[j]} = |r_j><m_j| and F_q = I
    elsewhere.  Controls: with projector Pc onto the control condition,
    G = Pc (x) (that operator) + (1 - Pc) (x) I, which as operators on the full
    space reads G = Pc * A + (I - Pc) for the Pc diagonal.
    """
    if cvals is None:
        cvals = cmask
    targets = list(targets)
    k = len(targets)
    d = 1 << k
    A = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    for r in range(d):
        for m in range(d):
            if U[r, m] == 0:
                continue
            fac = [I2] * n
            for j, t in enumerate(targets):
                e = np.zeros((2, 2), dtype=np.complex128)
                e[(r >> j) & 1, (m >> j) & 1] = 1.0
                fac[t] = e
            A += U[r, m] * _kron_list(fac[::-1])
    if cmask == 0:
        return A
    diag = np.array([1.0 if (i & cmask) == cvals else 0.0 for i in range(1 << n)])
    Pc = np.diag(diag).astype(np.complex128)
    return Pc @ A + (np.eye(1 << n) - Pc)


def circuit_operator(circ) -> np.ndarray:
    n = circ.n
    G = np.eye(1 << n, dtype=np.complex128)
    for tg, u, cm, cv in circ.gates:
        G = embed(n, tg, u, cm, cv) @ G
    return G


def run(circ, psi0: np.ndarray) -> np.ndarray:
    return circuit_operator(circ) @ psi0
