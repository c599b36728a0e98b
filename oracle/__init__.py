"""Correctness oracle for the GPU gate engine.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
bench's ``cpu_baseline`` leg, never by the product package.  It shares no code
with the GPU path; both sides read the same circuit IR (``workloads``).

* ``expect_pauli`` and ``sample`` (Pauli-string expectation values; sampling
  by inverting the cumulative distribution at caller-given uniforms).
* ``run``/``apply_op``/``probabilities``/``norm2`` call ``qs_oracle.c``: plain
  FP64 loops that apply each gate operator in order (the pair update of Alg. 1
  generalised to any 2x2 / 2^k x 2^k matrix, controls as in Fig. control6q2).
* ``outputs_at`` computes single output amplitudes of one gate from the input
  amplitudes it depends on, so results at sizes too large for a full host state
  can be checked on samples.
* ``dense`` holds the independent pin: full 2^n x 2^n operators from Kronecker
  products (n <= 8).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-std=c99"]


def build(force: bool = True) -> str:
    """Compile qs_oracle.c with gcc (a plain host build; no GPU code)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build(force=False)
            L = ctypes.CDLL(_LIB)
            dp = ctypes.POINTER(ctypes.c_double)
            L.orc_init_basis.argtypes = [ctypes.c_int, dp, ctypes.c_uint64]
            L.orc_apply_1q.argtypes = [ctypes.c_int, dp, ctypes.c_int, dp, ctypes.c_uint64, ctypes.c_uint64]
            L.orc_apply_kq.argtypes = [ctypes.c_int, dp, ctypes.c_int, ctypes.c_void_p, dp,
                                       ctypes.c_uint64, ctypes.c_uint64]
            L.orc_run.argtypes = [ctypes.c_int, dp, ctypes.c_void_p, ctypes.c_int64, dp]
            L.orc_probabilities.argtypes = [ctypes.c_int, dp, ctypes.c_void_p, ctypes.c_int, dp]
            L.orc_norm2.argtypes = [ctypes.c_int, dp]
            L.orc_norm2.restype = ctypes.c_double
            L.orc_num_threads.restype = ctypes.c_int
            L.orc_set_threads.argtypes = [ctypes.c_int]
            L.orc_expect_pauli.argtypes = [ctypes.c_int, dp, ctypes.c_uint64, ctypes.c_uint64, dp]
            L.orc_sample.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int64, ctypes.c_void_p]
            assert L.orc_op_size() == 64
            _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype in (np.float64, np.complex128) and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_threads(t: int) -> None:
    """Threads of the OpenMP loops from now on (the results do not depend on it)."""
    lib().orc_set_threads(int(t))


def basis(n: int, x: int = 0) -> np.ndarray:
    psi = np.empty(1 << n, dtype=np.complex128)
    lib().orc_init_basis(n, _dp(psi), int(x))
    return psi


def run(n: int, ops: np.ndarray, mats: np.ndarray, psi: np.ndarray | None = None,
        init_basis: int = 0) -> np.ndarray:
    """Apply every op of the IR in order; returns the final state (complex128)."""
    if psi is None:
        psi = basis(n, init_basis)
    else:
        psi = np.ascontiguousarray(psi, dtype=np.complex128).copy()
    assert psi.size == 1 << n
    mats = np.ascontiguousarray(mats, dtype=np.float64)
    if len(ops):
        ops = np.ascontiguousarray(ops)
        assert ops.dtype.itemsize == 64
        lib().orc_run(n, _dp(psi), ops.ctypes.data, len(ops), _dp(mats) if mats.size else None)
    return psi


def run_inplace(n: int, ops: np.ndarray, mats: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """As run(), but applies the ops to psi itself (C-contiguous complex128,
    2^n amplitudes) without copying it first."""
    assert psi.dtype == np.complex128 and psi.flags.c_contiguous and psi.size == 1 << n
    mats = np.ascontiguousarray(mats, dtype=np.float64)
    if len(ops):
        ops = np.ascontiguousarray(ops)
        assert ops.dtype.itemsize == 64
        lib().orc_run(n, _dp(psi), ops.ctypes.data, len(ops), _dp(mats) if mats.size else None)
    return psi


def run_circuit(circ, psi: np.ndarray | None = None) -> np.ndarray:
    ops, mats = circ.arrays()
    return run(circ.n, ops, mats, psi, circ.init_basis)


def apply_op(n: int, psi: np.ndarray, targets, U: np.ndarray, cmask: int = 0, cvals: int | None = None):
    """Apply one gate in place (psi complex128, U complex 2^k x 2^k)."""
    if cvals is None:
        cvals = cmask
    U = np.ascontiguousarray(U, dtype=np.complex128)
    t = np.asarray(list(targets), dtype=np.int32)
    if len(t) == 1:
        lib().orc_apply_1q(n, _dp(psi), int(t[0]), _dp(U), int(cmask), int(cvals))
    else:
        lib().orc_apply_kq(n, _dp(psi), len(t), t.ctypes.data, _dp(U), int(cmask), int(cvals))
    return psi


def probabilities(n: int, psi: np.ndarray, qubits) -> np.ndarray:
    q = np.asarray(list(qubits), dtype=np.int32)
    out = np.empty(1 << len(q), dtype=np.float64)
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    lib().orc_probabilities(n, _dp(psi), q.ctypes.data if len(q) else None, len(q), _dp(out))
    return out


def norm2(n: int, psi: np.ndarray) -> float:
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    return float(lib().orc_norm2(n, _dp(psi)))


def expect_pauli(n: int, psi: np.ndarray, x: int, z: int) -> complex:
    """<psi|P|psi> for P = i^|x&z| X^x Z^z (Y where a bit is in both masks)."""
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    out = np.zeros(2, dtype=np.float64)
    lib().orc_expect_pauli(n, _dp(psi), int(x), int(z), _dp(out))
    return complex(out[0], out[1])


def sample(n: int, psi: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Indices drawn by inverting the cumulative |psi|^2 at the given uniforms."""
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(u.size, dtype=np.uint64)
    lib().orc_sample(n, _dp(psi), _dp(u), u.size, out.ctypes.data)
    return out


def outputs_at(idx: np.ndarray, targets, U: np.ndarray, cmask: int, cvals: int, fetch):
    """Output amplitudes at indices ``idx`` of one gate, from its inputs.

    ``fetch(j)`` returns input amplitudes (complex128) at an integer array of
    indices.  Output i equals input i when the control test fails; otherwise
    with r = the target bits of i and b = i with those bits cleared,
    out_i = sum_m U[r, m] * in[b | bits(m)]  (the definition the C loops apply).
    """
    idx = np.asarray(idx, dtype=np.uint64)
    targets = [int(t) for t in targets]
    k = len(targets)
    U = np.asarray(U, dtype=np.complex128)
    r = np.zeros(idx.shape, dtype=np.int64)
    base = idx.copy()
    for j, t in enumerate(targets):
        bit = (idx >> np.uint64(t)) & np.uint64(1)
        r |= bit.astype(np.int64) << j
        base &= ~np.uint64(1 << t)
    out = np.zeros(idx.shape, dtype=np.complex128)
    for m in range(1 << k):
        a = base.copy()
        for j, t in enumerate(targets):
            if (m >> j) & 1:
                a |= np.uint64(1 << t)
        out += U[r, m] * fetch(a)
    active = (idx & np.uint64(cmask)) == np.uint64(cvals)
    same = fetch(idx)
    return np.where(active, out, same)
