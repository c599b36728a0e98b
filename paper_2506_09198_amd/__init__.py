"""Python binding of libqs.so, the gfx950 state-vector gate engine.

Argument marshalling only: every step runs in the library's HIP kernels.  The
functions carry the C ABI's names (``include/qs.h``) and raise ``QSError`` on
any status other than QS_OK.  Importing this package fails loudly if
``libqs.so`` has not been built (``python -m paper_2506_09198_amd._build``).

PyTorch is optional plumbing: ``State.from_torch`` wraps a torch complex tensor's
device memory and current stream so kernels run on torch's stream.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# QS_LIB selects another build of the same library (e.g. the host-AddressSanitizer
# build, libqs_asan.so); there is no fallback when it is missing.
LIB_PATH = os.environ.get("QS_LIB") or os.path.join(_HERE, "libqs.so")

QS_OK, QS_ERR_ARG, QS_ERR_OOM, QS_ERR_DEVICE, QS_ERR_BUSY, QS_ERR_UNSUPPORTED, QS_ERR_CANCELLED, \
    QS_ERR_TIMEOUT = range(8)
QS_C64, QS_C128 = 1, 2
QS_MAX_QUBITS = 34
QS_MAX_FUSED = 6
KIND_NAMES = {0: "init", 1: "1q_hi", 2: "1q_lo", 3: "2q", 4: "kq", 5: "tile", 6: "mfma", 7: "reduce", 8: "diag", 9: "perm",
              10: "probe", 11: "sample"}

TRACE_DTYPE = np.dtype([("kind", "<i4"), ("n", "<i4"), ("t0", "<i4"), ("t1", "<i4"), ("nctrl", "<i4"),
                        ("dtype", "<i4"), ("bytes", "<u8"), ("updates", "<u8"), ("ms", "<f4"),
                        ("rsv", "<i4")])
assert TRACE_DTYPE.itemsize == 48


class QSError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"qs status {status}: {msg}")
        self.status = status


class _Circuit(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("want", ctypes.c_int32), ("init_basis", ctypes.c_uint64),
                ("ops", ctypes.c_void_p), ("n_ops", ctypes.c_int64), ("mats", ctypes.c_void_p),
                ("n_mats", ctypes.c_int64), ("init_state", ctypes.c_void_p), ("out", ctypes.c_void_p)]


QS_WANT_NONE, QS_WANT_STATE, QS_WANT_PROBS, QS_WANT_NORM = 0, 1, 2, 3


class _BatchOpts(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("mode", ctypes.c_int32), ("streams", ctypes.c_int32),
                ("fuse_k", ctypes.c_int32), ("tile_qubits", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("whole_max", ctypes.c_int32), ("persist_max", ctypes.c_int32)]


class _TuneEntry(ctypes.Structure):
    _fields_ = [("tile_qubits", ctypes.c_int32), ("fuse_k", ctypes.c_int32), ("whole_max", ctypes.c_int32),
                ("persist_max", ctypes.c_int32), ("device_ms", ctypes.c_double)]


class _GateSched(ctypes.Structure):
    _fields_ = [("cls", ctypes.c_int32), ("slots", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32),
                ("xcd", ctypes.c_int32), ("gbs", ctypes.c_double), ("from_cache", ctypes.c_int32)]


QS_GATE_CLASSES = 4


class _BatchStats(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_uint64), ("passes", ctypes.c_uint64), ("device_ms", ctypes.c_double),
                ("class_ms", ctypes.c_double * 3), ("class_circuits", ctypes.c_uint32 * 3), ("rsv", ctypes.c_uint32),
                ("submit_ms", ctypes.c_double * 4)]


class _ServerOpts(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("rounds_ahead", ctypes.c_int32), ("hbm_budget", ctypes.c_uint64),
                ("plan_budget", ctypes.c_uint64), ("tile_qubits", ctypes.c_int32), ("fuse_k", ctypes.c_int32),
                ("rsv", ctypes.c_int32 * 4)]


class _Result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("status", ctypes.c_int32), ("n", ctypes.c_int32),
                ("t_submit_ms", ctypes.c_double), ("t_admit_ms", ctypes.c_double), ("t_done_ms", ctypes.c_double)]


class _ServerStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in ("submitted", "admitted", "completed", "failed", "cancelled",
                                               "rounds", "launches", "budget_bytes", "used_bytes", "peak_bytes")] + \
               [("queued", ctypes.c_uint32), ("active", ctypes.c_uint32)]


class _RunOpts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("fuse_k", ctypes.c_int32), ("tile_qubits", ctypes.c_int32),
                ("max_blocks", ctypes.c_int32), ("remap", ctypes.c_int32), ("rsv", ctypes.c_int32 * 3)]


def _load():
    # PyTorch-ROCm ships its own HIP runtime under the same soname
    # (libamdhip64.so.7).  The first one loaded serves the whole process, so
    # when torch is installed it is imported first: libqs then binds to the
    # runtime torch uses and both share one device context.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2506_09198_amd._build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, u64, i32, dp = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(ctypes.c_double)
    sig = {
        "qs_version": ([], ctypes.c_int),
        "qs_last_error": ([], ctypes.c_char_p),
        "qs_device_count": ([], ctypes.c_int),
        "qs_create": ([i32, i32, ctypes.POINTER(vp)], i32),
        "qs_create_external": ([i32, i32, vp, u64, vp, ctypes.POINTER(vp)], i32),
        "qs_destroy": ([vp], i32),
        "qs_set_stream": ([vp, vp], i32),
        "qs_get_info": ([vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(vp)], i32),
        "qs_init_basis": ([vp, u64], i32),
        "qs_upload": ([vp, vp, u64, u64], i32),
        "qs_download": ([vp, vp, u64, u64], i32),
        "qs_apply_1q": ([vp, i32, dp, u64, u64], i32),
        "qs_apply_2q": ([vp, i32, i32, dp, u64, u64], i32),
        "qs_apply_fused": ([vp, ctypes.POINTER(i32), i32, dp, u64, u64], i32),
        "qs_apply_diag": ([vp, ctypes.POINTER(i32), i32, dp, u64, u64], i32),
        "qs_run_circuit": ([vp, vp, ctypes.c_int64, dp, ctypes.c_int64, ctypes.POINTER(_RunOpts)], i32),
        "qs_plan_circuit": ([i32, i32, vp, ctypes.c_int64, dp, ctypes.c_int64, ctypes.POINTER(_RunOpts),
                             ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)], i32),
        "qs_plan_order": ([i32, i32, vp, ctypes.c_int64, dp, ctypes.c_int64, ctypes.POINTER(_RunOpts),
                           ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(i32), ctypes.POINTER(u64)], i32),
        "qs_plan_restore": ([i32, i32, vp, ctypes.c_int64, dp, ctypes.c_int64, ctypes.POINTER(_RunOpts),
                             ctypes.POINTER(i32), ctypes.POINTER(i32)], i32),
        "qs_plan_export": ([i32, i32, vp, ctypes.c_int64, dp, ctypes.c_int64, ctypes.POINTER(_RunOpts),
                            ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_int64), vp, ctypes.POINTER(ctypes.c_int64),
                            dp, ctypes.POINTER(ctypes.c_int64)], i32),
        "qs_batch_replay": ([vp], i32),
        "qs_batch_tune": ([ctypes.POINTER(_Circuit), i32, ctypes.POINTER(_BatchOpts), ctypes.POINTER(_TuneEntry), i32,
                           ctypes.POINTER(i32)], i32),
        "qs_expect_pauli": ([vp, u64, u64, dp], i32),
        "qs_sample": ([vp, dp, ctypes.c_int64, ctypes.c_void_p], i32),
        "qs_probabilities": ([vp, ctypes.POINTER(i32), i32, dp], i32),
        "qs_norm": ([vp, dp], i32),
        "qs_probabilities_noalloc": ([vp, ctypes.POINTER(i32), i32, vp], i32),
        "qs_sync": ([vp], i32),
        "qs_batch_submit": ([ctypes.POINTER(_Circuit), i32, ctypes.POINTER(_BatchOpts), ctypes.POINTER(vp)], i32),
        "qs_batch_wait": ([vp, i32], i32),
        "qs_batch_state": ([vp, i32, ctypes.POINTER(vp), ctypes.POINTER(i32)], i32),
        "qs_batch_download": ([vp, i32, vp], i32),
        "qs_batch_get_stats": ([vp, ctypes.POINTER(_BatchStats)], i32),
        "qs_batch_probabilities": ([vp, i32, ctypes.POINTER(i32), i32, dp], i32),
        "qs_batch_norm": ([vp, i32, dp], i32),
        "qs_batch_release": ([vp], i32),
        "qs_server_create": ([ctypes.POINTER(_ServerOpts), ctypes.POINTER(vp)], i32),
        "qs_server_submit": ([vp, ctypes.POINTER(_Circuit), ctypes.POINTER(ctypes.c_uint64)], i32),
        "qs_server_poll": ([vp, ctypes.POINTER(_Result), i32, ctypes.POINTER(i32)], i32),
        "qs_server_state": ([vp, ctypes.c_uint64, ctypes.POINTER(vp), ctypes.POINTER(i32)], i32),
        "qs_server_download": ([vp, ctypes.c_uint64, vp], i32),
        "qs_server_release": ([vp, ctypes.c_uint64], i32),
        "qs_server_cancel": ([vp, ctypes.c_uint64], i32),
        "qs_server_get_stats": ([vp, ctypes.POINTER(_ServerStats)], i32),
        "qs_server_destroy": ([vp], i32),
        "qs_trace_enable": ([vp, i32], i32),
        "qs_trace_read": ([vp, vp, i32, ctypes.POINTER(i32)], i32),
        "qs_probe_inplace": ([vp, i32, i32], i32),
        "qs_tune_gates": ([vp, ctypes.c_char_p, ctypes.POINTER(_GateSched), i32, ctypes.POINTER(i32)], i32),
        "qs_tune_gates_reset": ([], i32),
        "qs_tunable_set": ([ctypes.c_char_p, ctypes.c_int64], i32),
        "qs_tunable_get": ([ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64)], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    return L


lib = _load()


def _check(st: int):
    if st != QS_OK:
        raise QSError(st, lib.qs_last_error().decode(errors="replace"))


def _mask(c) -> int:
    if c is None:
        return 0
    if isinstance(c, (int, np.integer)):
        return int(c)
    m = 0
    for q in c:
        m |= 1 << int(q)
    return m


def _mat(U, k: int):
    a = np.ascontiguousarray(U, dtype=np.complex128)
    if a.shape != (1 << k, 1 << k):
        raise ValueError(f"matrix shape {a.shape} != {(1 << k, 1 << k)}")
    f = a.view(np.float64).ravel()
    return f, f.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _np_dtype(dt: int):
    return np.complex128 if dt == QS_C128 else np.complex64


# ------------------------------------------------------------------ ABI calls

def qs_version() -> int:
    return lib.qs_version()


def qs_last_error() -> str:
    return lib.qs_last_error().decode(errors="replace")


def qs_device_count() -> int:
    return lib.qs_device_count()


def qs_create(n: int, dtype: int = QS_C128) -> int:
    h = ctypes.c_void_p()
    _check(lib.qs_create(n, dtype, ctypes.byref(h)))
    return h.value


def qs_create_external(n: int, dtype: int, dev_ptr: int, nbytes: int, stream: int | None = None) -> int:
    h = ctypes.c_void_p()
    _check(lib.qs_create_external(n, dtype, ctypes.c_void_p(dev_ptr), nbytes, ctypes.c_void_p(stream or 0),
                                  ctypes.byref(h)))
    return h.value


def qs_destroy(s: int):
    _check(lib.qs_destroy(ctypes.c_void_p(s)))


def qs_set_stream(s: int, stream: int | None):
    _check(lib.qs_set_stream(ctypes.c_void_p(s), ctypes.c_void_p(stream or 0)))


def qs_get_info(s: int):
    n, dt, p = ctypes.c_int(), ctypes.c_int(), ctypes.c_void_p()
    _check(lib.qs_get_info(ctypes.c_void_p(s), ctypes.byref(n), ctypes.byref(dt), ctypes.byref(p)))
    return n.value, dt.value, p.value


def qs_tunable_set(name: str, value: int):
    """Set a launch knob (value < 0 restores its default / environment value)."""
    _check(lib.qs_tunable_set(name.encode(), int(value)))


def qs_tunable_get(name: str) -> int:
    v = ctypes.c_int64()
    _check(lib.qs_tunable_get(name.encode(), ctypes.byref(v)))
    return v.value


class tunables:
    """Context manager that sets launch knobs and restores them on exit:
    ``with tunables(gate_grid_cap=3, tile_grid_cap=2): ...``."""

    def __init__(self, **knobs):
        self.knobs = knobs
        self.saved = {}

    def __enter__(self):
        for k, v in self.knobs.items():
            self.saved[k] = qs_tunable_get(k)
            qs_tunable_set(k, v)
        return self

    def __exit__(self, *exc):
        for k, v in self.saved.items():
            qs_tunable_set(k, v)
        return False


def qs_init_basis(s: int, x: int):
    _check(lib.qs_init_basis(ctypes.c_void_p(s), int(x)))


def qs_upload(s: int, host: np.ndarray, first: int = 0):
    n, dt, _ = qs_get_info(s)
    a = np.ascontiguousarray(host, dtype=_np_dtype(dt))
    _check(lib.qs_upload(ctypes.c_void_p(s), ctypes.c_void_p(a.ctypes.data), first, a.size))


def qs_download(s: int, first: int = 0, count: int | None = None) -> np.ndarray:
    n, dt, _ = qs_get_info(s)
    if count is None:
        count = (1 << n) - first
    out = np.empty(count, dtype=_np_dtype(dt))
    _check(lib.qs_download(ctypes.c_void_p(s), ctypes.c_void_p(out.ctypes.data), first, count))
    return out


def qs_apply_1q(s: int, target: int, U, ctrl_mask=0, ctrl_vals=None):
    cm = _mask(ctrl_mask)
    cv = cm if ctrl_vals is None else _mask(ctrl_vals)
    f, p = _mat(U, 1)
    _check(lib.qs_apply_1q(ctypes.c_void_p(s), int(target), p, cm, cv))


def qs_apply_2q(s: int, t0: int, t1: int, U, ctrl_mask=0, ctrl_vals=None):
    cm = _mask(ctrl_mask)
    cv = cm if ctrl_vals is None else _mask(ctrl_vals)
    f, p = _mat(U, 2)
    _check(lib.qs_apply_2q(ctypes.c_void_p(s), int(t0), int(t1), p, cm, cv))


def qs_apply_fused(s: int, targets, U, ctrl_mask=0, ctrl_vals=None):
    t = np.ascontiguousarray(list(targets), dtype=np.int32)
    cm = _mask(ctrl_mask)
    cv = cm if ctrl_vals is None else _mask(ctrl_vals)
    f, p = _mat(U, len(t))
    _check(lib.qs_apply_fused(ctypes.c_void_p(s), t.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), len(t), p,
                              cm, cv))


def qs_apply_diag(s: int, targets, diag, ctrl_mask=0, ctrl_vals=None):
    """psi[i] *= diag[j] (bit b of j = bit targets[b] of i) where the controls match."""
    t = np.ascontiguousarray(list(targets), dtype=np.int32)
    d = np.ascontiguousarray(diag, dtype=np.complex128)
    if d.shape != (1 << len(t),):
        raise ValueError(f"diagonal shape {d.shape} != {(1 << len(t),)}")
    cm = _mask(ctrl_mask)
    cv = cm if ctrl_vals is None else _mask(ctrl_vals)
    f = d.view(np.float64)
    _check(lib.qs_apply_diag(ctypes.c_void_p(s), t.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), len(t),
                             f.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), cm, cv))


def qs_run_circuit(s: int, ops: np.ndarray, mats: np.ndarray, mode: int = 0, fuse_k: int = 0,
                   tile_qubits: int = 0, max_blocks: int = 0, remap: int = 0):
    ops = np.ascontiguousarray(ops)
    if ops.dtype.itemsize != 64:
        raise ValueError("ops must be 64-byte records (workloads.OP_DTYPE)")
    mats = np.ascontiguousarray(mats, dtype=np.float64)
    o = _RunOpts(mode, fuse_k, tile_qubits, max_blocks, remap)
    _check(lib.qs_run_circuit(ctypes.c_void_p(s), ctypes.c_void_p(ops.ctypes.data if len(ops) else 0), len(ops),
                              mats.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), mats.size, ctypes.byref(o)))


def qs_plan_circuit(n: int, dtype: int, ops: np.ndarray, mats: np.ndarray, mode: int = 0, fuse_k: int = 0,
                    tile_qubits: int = 0, remap: int = 0):
    """Host-only planning: returns (state passes incl. restoring ones, ops inside tile passes)."""
    ops = np.ascontiguousarray(ops)
    mats = np.ascontiguousarray(mats, dtype=np.float64)
    o = _RunOpts(mode, fuse_k, tile_qubits, 0, remap)
    npass, nops = ctypes.c_int64(), ctypes.c_int64()
    _check(lib.qs_plan_circuit(n, dtype, ctypes.c_void_p(ops.ctypes.data if len(ops) else 0), len(ops),
                               mats.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), mats.size, ctypes.byref(o),
                               ctypes.byref(npass), ctypes.byref(nops)))
    return npass.value, nops.value


def qs_plan_order(n: int, dtype: int, ops: np.ndarray, mats: np.ndarray, tile_qubits: int = 0):
    """Host-only: (order, pass_of, tile_masks) of the planned execution."""
    ops = np.ascontiguousarray(ops)
    mats = np.ascontiguousarray(mats, dtype=np.float64)
    k = len(ops)
    order = np.zeros(max(k, 1), dtype=np.int64)
    pass_of = np.zeros(max(k, 1), dtype=np.int32)
    masks = np.zeros(max(k, 1), dtype=np.uint64)
    o = _RunOpts(0, 0, tile_qubits)
    _check(lib.qs_plan_order(n, dtype, ctypes.c_void_p(ops.ctypes.data if k else 0), k,
                             mats.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), mats.size, ctypes.byref(o),
                             order.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                             pass_of.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                             masks.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))))
    npass = int(pass_of[:k].max()) + 1 if k else 0
    return order[:k], pass_of[:k], masks[:npass]


TILE_OP_DTYPE = np.dtype([("kind", "<i4"), ("k", "<i4"), ("p", "<i4", (6,)), ("lcm", "<u8"), ("lcv", "<u8"),
                          ("gcm", "<u8"), ("gcv", "<u8"), ("moff", "<u8"), ("lp", "i1", (6,)), ("dclass", "i1"),
                          ("dbit", "i1"), ("dj", "<i4"), ("rsv", "<i4")])
assert TILE_OP_DTYPE.itemsize == 88


def qs_plan_restore(n: int, dtype: int, ops: np.ndarray, mats: np.ndarray, tile_qubits: int = 0, fuse_k: int = 0,
                    remap: int = 0):
    """Host-only: the qubit-order restoring involutions run after the tile
    passes (a list of 0-2 arrays tau, tau[p] = the position p exchanges with)."""
    ops = np.ascontiguousarray(ops)
    mats = np.ascontiguousarray(mats, dtype=np.float64)
    o = _RunOpts(0, fuse_k, tile_qubits, 0, remap)
    tau = np.zeros(128, dtype=np.int32)
    nr = ctypes.c_int32(0)
    _check(lib.qs_plan_restore(n, dtype, ctypes.c_void_p(ops.ctypes.data if len(ops) else 0), len(ops),
                               mats.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), mats.size, ctypes.byref(o),
                               tau.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(nr)))
    return [tau[64 * i:64 * i + n].copy() for i in range(nr.value)]


def qs_plan_export(n: int, dtype: int, ops: np.ndarray, mats: np.ndarray, tile_qubits: int = 0, fuse_k: int = 0,
                   remap: int = 0):
    """Host-only: (passes, tile_ops, pool) as planned for mode 0.  passes is a
    list of dicts {m, L, op0, nops, Q}; qubit positions are physical (see
    qs_plan_restore)."""
    ops = np.ascontiguousarray(ops)
    mats = np.ascontiguousarray(mats, dtype=np.float64)
    o = _RunOpts(0, fuse_k, tile_qubits, 0, remap)
    np_, nt, npool = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
    args = (n, dtype, ctypes.c_void_p(ops.ctypes.data if len(ops) else 0), len(ops),
            mats.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), mats.size, ctypes.byref(o))
    _check(lib.qs_plan_export(*args, None, ctypes.byref(np_), None, ctypes.byref(nt), None, ctypes.byref(npool)))
    desc = np.zeros((max(np_.value, 1), 36), dtype=np.int32)
    tops = np.zeros(max(nt.value, 1), dtype=TILE_OP_DTYPE)
    pool = np.zeros(max(npool.value, 1), dtype=np.float64)
    _check(lib.qs_plan_export(*args, desc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(np_),
                              ctypes.c_void_p(tops.ctypes.data), ctypes.byref(nt),
                              pool.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(npool)))
    passes = [{"m": int(d[0]), "L": int(d[1]), "op0": int(d[2]), "nops": int(d[3]),
               "Q": [int(q) for q in d[4:4 + d[0]]]} for d in desc[:np_.value]]
    return passes, tops[:nt.value], pool[:npool.value]


def qs_expect_pauli(s: int, x_mask: int, z_mask: int) -> complex:
    out = np.zeros(2, dtype=np.float64)
    _check(lib.qs_expect_pauli(ctypes.c_void_p(s), int(x_mask), int(z_mask),
                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return complex(out[0], out[1])


def qs_sample(s: int, u: np.ndarray) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(u.size, dtype=np.uint64)
    _check(lib.qs_sample(ctypes.c_void_p(s), u.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), u.size,
                         ctypes.c_void_p(out.ctypes.data)))
    return out


def qs_probabilities(s: int, qubits) -> np.ndarray:
    q = np.ascontiguousarray(list(qubits), dtype=np.int32)
    out = np.empty(1 << len(q), dtype=np.float64)
    _check(lib.qs_probabilities(ctypes.c_void_p(s), q.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), len(q),
                                out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out


def qs_norm(s: int) -> float:
    v = ctypes.c_double()
    _check(lib.qs_norm(ctypes.c_void_p(s), ctypes.byref(v)))
    return v.value


def qs_probabilities_noalloc(s: int, qubits, dev_out: int):
    """Enqueue the marginal probabilities into device memory at address
    ``dev_out`` (2^m doubles) without any allocation; returns at once."""
    q = np.ascontiguousarray(list(qubits), dtype=np.int32)
    _check(lib.qs_probabilities_noalloc(ctypes.c_void_p(s), q.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), len(q),
                                        ctypes.c_void_p(int(dev_out))))


def qs_sync(s: int):
    _check(lib.qs_sync(ctypes.c_void_p(s)))


def _circuit_array(circuits):
    """Circuits as qs_circuit records.  Each item is a workloads.Circuit, a
    tuple (n, ops, mats, basis), or (n, ops, mats, basis, init_state, want,
    out): init_state a device address (int; 0 = start from |basis>), want a
    QS_WANT_* value and out a C-contiguous numpy array that receives it (the
    caller keeps it alive until the result is written)."""
    keep, arr = [], (_Circuit * max(1, len(circuits)))()
    for i, c in enumerate(circuits):
        init, want, out = 0, QS_WANT_NONE, None
        if hasattr(c, "arrays"):
            n, (ops, mats), basis = c.n, c.arrays(), c.init_basis
        elif len(c) == 7:
            n, ops, mats, basis, init, want, out = c
        else:
            n, ops, mats, basis = c
        ops = np.ascontiguousarray(ops)
        mats = np.ascontiguousarray(mats, dtype=np.float64)
        keep.append((ops, mats))
        if out is not None and not out.flags.c_contiguous:
            raise ValueError("result buffer must be C-contiguous")
        arr[i] = _Circuit(n, int(want), int(basis), ops.ctypes.data if len(ops) else 0, len(ops),
                          mats.ctypes.data if mats.size else 0, mats.size, int(init or 0),
                          out.ctypes.data if out is not None else 0)
    return keep, arr


def qs_batch_submit(circuits, dtype: int = QS_C128, mode: int = 0, streams: int = 0, fuse_k: int = 0,
                    tile_qubits: int = 0, graph: int = 0, whole_max: int = 0, persist_max: int = 0) -> int:
    """circuits: iterable of (n, ops, mats, init_basis) or objects with .n/.arrays()/.init_basis."""
    keep, arr = _circuit_array(circuits)
    o = _BatchOpts(dtype, mode, streams, fuse_k, tile_qubits, graph, whole_max, persist_max)
    h = ctypes.c_void_p()
    _check(lib.qs_batch_submit(arr, len(circuits), ctypes.byref(o), ctypes.byref(h)))
    return h.value


def qs_batch_replay(b: int):
    _check(lib.qs_batch_replay(ctypes.c_void_p(b)))


def qs_batch_tune(sample, dtype: int = QS_C128, streams: int = 0):
    """Time candidate (tile_qubits, fuse_k, whole_max, persist_max) on a sample;
    returns (best dict, all timings)."""
    keep, arr = _circuit_array(sample)
    o = _BatchOpts(dtype, 0, streams, 0, 0, 0)
    out = (_TuneEntry * 32)()
    k = ctypes.c_int()
    _check(lib.qs_batch_tune(arr, len(sample), ctypes.byref(o), out, 32, ctypes.byref(k)))
    keys = ("tile_qubits", "fuse_k", "whole_max", "persist_max")
    rows = [{**{x: getattr(e, x) for x in keys}, "device_ms": e.device_ms} for e in out[:k.value]]
    return {x: getattr(o, x) for x in keys}, rows


def qs_batch_wait(b: int, timeout_ms: int = -1):
    _check(lib.qs_batch_wait(ctypes.c_void_p(b), timeout_ms))


def qs_batch_state(b: int, i: int):
    p, n = ctypes.c_void_p(), ctypes.c_int()
    _check(lib.qs_batch_state(ctypes.c_void_p(b), i, ctypes.byref(p), ctypes.byref(n)))
    return p.value, n.value


def qs_batch_download(b: int, i: int, dtype: int = QS_C128) -> np.ndarray:
    _, n = qs_batch_state(b, i)
    out = np.empty(1 << n, dtype=_np_dtype(dtype))
    _check(lib.qs_batch_download(ctypes.c_void_p(b), i, ctypes.c_void_p(out.ctypes.data)))
    return out


def qs_batch_get_stats(b: int) -> dict:
    st = _BatchStats()
    _check(lib.qs_batch_get_stats(ctypes.c_void_p(b), ctypes.byref(st)))
    return {"launches": st.launches, "passes": st.passes, "device_ms": st.device_ms,
            "class_ms": list(st.class_ms), "class_circuits": list(st.class_circuits),
            "submit_ms": dict(zip(("alloc", "plan", "pack", "enqueue"), st.submit_ms))}


def qs_batch_probabilities(b: int, i: int, qubits) -> np.ndarray:
    q = np.ascontiguousarray(list(qubits), dtype=np.int32)
    out = np.empty(1 << len(q), dtype=np.float64)
    _check(lib.qs_batch_probabilities(ctypes.c_void_p(b), int(i), q.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                      len(q), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out


def qs_batch_norm(b: int, i: int) -> float:
    out = np.zeros(1, dtype=np.float64)
    _check(lib.qs_batch_norm(ctypes.c_void_p(b), int(i), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return float(out[0])


def qs_batch_release(b: int):
    _check(lib.qs_batch_release(ctypes.c_void_p(b)))


def qs_server_create(dtype: int = QS_C128, hbm_budget: int = 0, rounds_ahead: int = 0, tile_qubits: int = 0,
                     fuse_k: int = 0, plan_budget: int = 0) -> int:
    o = _ServerOpts(dtype, rounds_ahead, hbm_budget, plan_budget, tile_qubits, fuse_k)
    h = ctypes.c_void_p()
    _check(lib.qs_server_create(ctypes.byref(o), ctypes.byref(h)))
    return h.value


def qs_server_submit(srv: int, circ) -> int:
    """Queue one request (a circuit in any form _circuit_array takes)."""
    keep, arr = _circuit_array([circ])
    rid = ctypes.c_uint64()
    _check(lib.qs_server_submit(ctypes.c_void_p(srv), ctypes.byref(arr[0]), ctypes.byref(rid)))
    return rid.value


def qs_server_poll(srv: int, max_results: int = 256) -> list:
    out = (_Result * max_results)()
    c = ctypes.c_int()
    _check(lib.qs_server_poll(ctypes.c_void_p(srv), out, max_results, ctypes.byref(c)))
    return [{"id": r.id, "status": r.status, "n": r.n, "t_submit_ms": r.t_submit_ms, "t_admit_ms": r.t_admit_ms,
             "t_done_ms": r.t_done_ms} for r in out[: c.value]]


def qs_server_state(srv: int, rid: int):
    p, n = ctypes.c_void_p(), ctypes.c_int()
    _check(lib.qs_server_state(ctypes.c_void_p(srv), rid, ctypes.byref(p), ctypes.byref(n)))
    return p.value, n.value


def qs_server_download(srv: int, rid: int, dtype: int = QS_C128) -> np.ndarray:
    _, n = qs_server_state(srv, rid)
    out = np.empty(1 << n, dtype=_np_dtype(dtype))
    _check(lib.qs_server_download(ctypes.c_void_p(srv), rid, ctypes.c_void_p(out.ctypes.data)))
    return out


def qs_server_release(srv: int, rid: int):
    _check(lib.qs_server_release(ctypes.c_void_p(srv), rid))


def qs_server_cancel(srv: int, rid: int):
    _check(lib.qs_server_cancel(ctypes.c_void_p(srv), rid))


def qs_server_get_stats(srv: int) -> dict:
    st = _ServerStats()
    _check(lib.qs_server_get_stats(ctypes.c_void_p(srv), ctypes.byref(st)))
    return {k: getattr(st, k) for k, _ in _ServerStats._fields_}


def qs_server_destroy(srv: int):
    _check(lib.qs_server_destroy(ctypes.c_void_p(srv)))


def qs_trace_enable(s: int, on: bool = True):
    _check(lib.qs_trace_enable(ctypes.c_void_p(s), 1 if on else 0))


def qs_trace_read(s: int, max_records: int = 1 << 16) -> np.ndarray:
    out = np.zeros(max_records, dtype=TRACE_DTYPE)
    c = ctypes.c_int()
    _check(lib.qs_trace_read(ctypes.c_void_p(s), ctypes.c_void_p(out.ctypes.data), max_records, ctypes.byref(c)))
    return out[: c.value]


def qs_probe_inplace(s: int, slots: int = 4, spread_log2: int = 11):
    """Enqueue the in-place read-modify-write ceiling probe over the state's
    buffer (leaves it unchanged; timed through the trace as kind "probe")."""
    _check(lib.qs_probe_inplace(ctypes.c_void_p(s), int(slots), int(spread_log2)))


def qs_tune_gates(s: int, cache_path: str | None = None) -> list:
    """Autotune the per-gate kernel's schedule for this state's type and size
    (see include/qs.h); returns one dict per gate class."""
    out = (_GateSched * QS_GATE_CLASSES)()
    n = ctypes.c_int(0)
    path = cache_path.encode() if cache_path else None
    _check(lib.qs_tune_gates(ctypes.c_void_p(s), path, out, QS_GATE_CLASSES, ctypes.byref(n)))
    return [{"cls": int(r.cls), "slots": int(r.slots), "wg_per_cu": int(r.wg_per_cu), "xcd": int(r.xcd),
             "gbs": float(r.gbs), "from_cache": bool(r.from_cache)} for r in out[:n.value]]


def qs_tune_gates_reset() -> None:
    _check(lib.qs_tune_gates_reset())


# ------------------------------------------------------------------ convenience

class State:
    """Owning wrapper around a qs_state handle."""

    def __init__(self, handle: int, tensor=None):
        self.h = handle
        self.tensor = tensor  # keeps torch-owned memory alive
        self.n, self.dtype, self.ptr = qs_get_info(handle)

    @classmethod
    def create(cls, n: int, dtype: int = QS_C128) -> "State":
        return cls(qs_create(n, dtype))

    @classmethod
    def from_torch(cls, tensor, stream=None) -> "State":
        import torch

        if tensor.dtype == torch.complex128:
            dt = QS_C128
        elif tensor.dtype == torch.complex64:
            dt = QS_C64
        else:
            raise TypeError("state tensor must be complex64 or complex128")
        n = int(tensor.numel()).bit_length() - 1
        if tensor.numel() != 1 << n or not tensor.is_contiguous() or not tensor.is_cuda:
            raise ValueError("need a contiguous CUDA tensor with 2^n elements")
        if stream is None:
            stream = torch.cuda.current_stream(tensor.device).cuda_stream
        nbytes = tensor.numel() * tensor.element_size()
        return cls(qs_create_external(n, dt, tensor.data_ptr(), nbytes, stream), tensor)

    def close(self):
        if self.h:
            qs_destroy(self.h)
            self.h = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def apply_1q(self, t, U, controls=0, cvals=None):
        qs_apply_1q(self.h, t, U, controls, cvals)

    def apply_2q(self, t0, t1, U, controls=0, cvals=None):
        qs_apply_2q(self.h, t0, t1, U, controls, cvals)

    def apply_fused(self, targets, U, controls=0, cvals=None):
        qs_apply_fused(self.h, targets, U, controls, cvals)

    def apply_diag(self, targets, diag, controls=0, cvals=None):
        qs_apply_diag(self.h, targets, diag, controls, cvals)

    def run(self, ops, mats, **kw):
        qs_run_circuit(self.h, ops, mats, **kw)

    def run_circuit(self, circ, **kw):
        ops, mats = circ.arrays()
        qs_run_circuit(self.h, ops, mats, **kw)

    def init_basis(self, x=0):
        qs_init_basis(self.h, x)

    def upload(self, host, first=0):
        qs_upload(self.h, host, first)

    def download(self, first=0, count=None):
        return qs_download(self.h, first, count)

    def probabilities(self, qubits):
        return qs_probabilities(self.h, qubits)

    def norm(self):
        return qs_norm(self.h)

    def sync(self):
        qs_sync(self.h)
