"""C-ABI checks that need no GPU: the library loads, exports every entry point
the header declares, rejects bad arguments before touching the device, and the
host-side planner groups gates as designed."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import workloads as W
from tests.conftest import ROOT


@pytest.fixture(scope="module")
def qs():
    lib = os.path.join(ROOT, "paper_2506_09198_amd", "libqs.so")
    if not os.path.exists(lib):
        from paper_2506_09198_amd import _build

        _build.build()
    import paper_2506_09198_amd as qs

    return qs


def _declared_functions():
    hdr = open(os.path.join(ROOT, "include", "qs.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    return sorted(set(re.findall(r"\b(qs_[a-z0-9_]+)\s*\(", hdr)))


def test_exports_every_declared_symbol(qs):
    names = _declared_functions()
    assert len(names) >= 20
    out = subprocess.run(["nm", "-D", "--defined-only", qs.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (qs_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert hasattr(qs, n), n  # the binding carries the same names


def test_version_and_errors(qs):
    assert qs.qs_version() >= 1
    with pytest.raises(qs.QSError) as e:
        qs.qs_create(0, qs.QS_C128)
    assert e.value.status == qs.QS_ERR_ARG and "outside" in qs.qs_last_error()
    for bad in (-1, 35, 64):
        with pytest.raises(qs.QSError) as e:
            qs.qs_create(bad, qs.QS_C64)
        assert e.value.status == qs.QS_ERR_ARG
    with pytest.raises(qs.QSError) as e:
        qs.qs_create(4, 7)
    assert e.value.status == qs.QS_ERR_ARG


def test_null_handle_rejected(qs):
    for call in (lambda: qs.qs_apply_1q(0, 0, np.eye(2)), lambda: qs.qs_norm(0), lambda: qs.qs_sync(0),
                 lambda: qs.qs_init_basis(0, 0)):
        with pytest.raises(qs.QSError) as e:
            call()
        assert e.value.status == qs.QS_ERR_ARG
    qs.qs_destroy(0)  # NULL is accepted


def test_create_without_device_reports_device_error(qs):
    if qs.qs_device_count() > 0:
        pytest.skip("a GPU is visible")
    with pytest.raises(qs.QSError) as e:
        qs.qs_create(4, qs.QS_C128)
    assert e.value.status == qs.QS_ERR_DEVICE


def test_plan_validation(qs):
    c = W.Circuit(4).g1(0, W.H).g2(1, 2, W.SWAP)
    ops, mats = c.arrays()
    bad = ops.copy()
    bad[0]["t"][0] = 4
    with pytest.raises(qs.QSError):
        qs.qs_plan_circuit(4, qs.QS_C128, bad, mats)
    bad = ops.copy()
    bad[1]["t"][1] = 1  # duplicate target
    with pytest.raises(qs.QSError):
        qs.qs_plan_circuit(4, qs.QS_C128, bad, mats)
    bad = ops.copy()
    bad[0]["cmask"] = 1  # control equals target
    with pytest.raises(qs.QSError):
        qs.qs_plan_circuit(4, qs.QS_C128, bad, mats)
    bad = ops.copy()
    bad[0]["cmask"] = 2
    bad[0]["cvals"] = 4  # value outside mask
    with pytest.raises(qs.QSError):
        qs.qs_plan_circuit(4, qs.QS_C128, bad, mats)
    bad = ops.copy()
    bad[1]["moff"] = mats.size  # matrix out of the pool
    with pytest.raises(qs.QSError):
        qs.qs_plan_circuit(4, qs.QS_C128, bad, mats)


def test_planner_groups_gates(qs):
    # every gate inside the tile: one pass
    c = W.random_u3_cnot(10, 200, seed=2)
    ops, mats = c.arrays()
    npass, nops = qs.qs_plan_circuit(10, qs.QS_C128, ops, mats, tile_qubits=10)
    assert npass == 1 and nops <= len(ops)  # register blocks absorb runs of gates
    # diagonal gates never force a new pass
    q = W.qft(24)
    ops, mats = q.arrays()
    npass, nops = qs.qs_plan_circuit(24, qs.QS_C128, ops, mats, tile_qubits=11)
    assert nops <= len(ops)
    n_dense = 24 + 12  # Hadamards and swaps
    assert npass < n_dense // 2
    # per-gate mode is not planned into tiles but validates the same way
    r = W.rqc_chain(32, 20, 5)
    ops, mats = r.arrays()
    npass, nops = qs.qs_plan_circuit(32, qs.QS_C64, ops, mats, tile_qubits=12)
    assert nops <= len(ops) and npass <= 20 * 6


@pytest.mark.parametrize("dt", [1, 2])
def test_planner_fuses_blocks(qs, dt, monkeypatch):
    monkeypatch.setenv("QS_FUSE_MIN", "2")
    monkeypatch.setenv("QS_REG_SEGMENTS", "0")  # compare matrix-core blocks with ops one by one
    r = W.rqc_chain(20, 10, 1)
    ops, mats = r.arrays()
    plain = qs.qs_plan_circuit(20, dt, ops, mats, tile_qubits=12)
    fused = qs.qs_plan_circuit(20, dt, ops, mats, tile_qubits=12, fuse_k=5)
    assert fused[0] == plain[0] and fused[1] < 0.6 * plain[1]
    # blocks need tiles of at least fuse_k + 4 qubits
    assert qs.qs_plan_circuit(20, dt, ops, mats, tile_qubits=8, fuse_k=5) == \
        qs.qs_plan_circuit(20, dt, ops, mats, tile_qubits=8)
    with pytest.raises(qs.QSError):
        qs.qs_plan_circuit(20, dt, ops, mats, fuse_k=3)


def test_new_entry_points_reject_null_handles(qs):
    for call in (lambda: qs.qs_apply_diag(0, [0], np.array([1, -1])),
                 lambda: qs.qs_expect_pauli(0, 1, 0),
                 lambda: qs.qs_sample(0, np.array([0.5]))):
        with pytest.raises(qs.QSError) as e:
            call()
        assert e.value.status == qs.QS_ERR_ARG


def test_plan_restore_validation_and_shape(qs):
    c = W.qft(12, 7)
    ops, mats = c.arrays()
    with pytest.raises(qs.QSError):
        qs.qs_plan_restore(12, qs.QS_C64, ops, mats, remap=3)
    bad = ops.copy()
    bad[0]["t"][0] = 12
    with pytest.raises(qs.QSError):
        qs.qs_plan_restore(12, qs.QS_C64, bad, mats)
    taus = qs.qs_plan_restore(12, qs.QS_C64, ops, mats, tile_qubits=6)
    assert len(taus) <= 2
    for tau in taus:
        assert tau.shape == (12,) and all(tau[tau[p]] == p for p in range(12))
    # no SWAP gate: nothing to restore, with or without relabeling
    r = W.rqc_chain(14, 6, 3)
    ops, mats = r.arrays()
    assert qs.qs_plan_restore(14, qs.QS_C64, ops, mats) == []


def test_batch_stats_layout(qs):
    import ctypes

    # launches, passes, device_ms, class_ms[3], class_circuits[3], rsv, submit_ms[4]
    assert ctypes.sizeof(qs._BatchStats) == 8 * 3 + 8 * 3 + 4 * 3 + 4 + 8 * 4
    assert ctypes.sizeof(qs._RunOpts) == 4 * 8


def test_unitarity_check_is_opt_in(qs, monkeypatch):
    c = W.Circuit(3).g1(0, W.H).g2(1, 2, W.SWAP)
    ops, mats = c.arrays()
    bad = mats.copy()
    bad[:8] = [1, 0, 1, 0, 1, 0, -1, 0]  # H without its 1/sqrt(2)
    qs.qs_plan_circuit(3, qs.QS_C128, ops, bad)  # not checked by default
    monkeypatch.setenv("QS_CHECK_UNITARY", "1")
    with pytest.raises(qs.QSError) as e:
        qs.qs_plan_circuit(3, qs.QS_C128, ops, bad)
    assert e.value.status == qs.QS_ERR_ARG and "unitary" in qs.qs_last_error()
    qs.qs_plan_circuit(3, qs.QS_C128, ops, mats)  # the real gates pass


def test_tunables_roundtrip_and_validation():
    import paper_2506_09198_amd as qs

    d = qs.qs_tunable_get("gate_grid_cap")
    qs.qs_tunable_set("gate_grid_cap", 7)
    assert qs.qs_tunable_get("gate_grid_cap") == 7
    with qs.tunables(gate_grid_cap=3, tile_grid_cap=2):
        assert qs.qs_tunable_get("gate_grid_cap") == 3 and qs.qs_tunable_get("tile_grid_cap") == 2
    assert qs.qs_tunable_get("gate_grid_cap") == 7
    qs.qs_tunable_set("gate_grid_cap", -1)
    assert qs.qs_tunable_get("gate_grid_cap") == d
    with pytest.raises(qs.QSError):
        qs.qs_tunable_set("gate_grid_cap", 0)
    with pytest.raises(qs.QSError):
        qs.qs_tunable_set("slots_one_high", 9)
    with pytest.raises(qs.QSError):
        qs.qs_tunable_set("no_such_knob", 1)


def test_circuit_record_and_want_validation(qs):
    """qs_circuit is 64 bytes (want, init_state and out after the original
    fields); a wanted result needs a host buffer and a known kind; the
    checks run before any device work."""
    import workloads as W

    assert ctypes.sizeof(qs._Circuit) == 64
    c = W.qft(8, 1)
    with pytest.raises(qs.QSError) as e:
        qs.qs_batch_submit([(c.n, *c.arrays(), 0, 0, qs.QS_WANT_STATE, None)])
    assert e.value.status == qs.QS_ERR_ARG
    with pytest.raises(qs.QSError) as e:
        qs.qs_batch_submit([(c.n, *c.arrays(), 0, 0, 7, np.zeros(1))])
    assert e.value.status == qs.QS_ERR_ARG
    big = W.qft(25, 0)
    with pytest.raises(qs.QSError) as e:
        qs.qs_batch_submit([(big.n, *big.arrays(), 0, 0, qs.QS_WANT_PROBS, np.zeros(1))])
    assert e.value.status == qs.QS_ERR_ARG
