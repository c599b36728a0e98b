"""GPU parity of SWAP relabeling: tile passes on physical qubit positions
followed by the in-place restoring passes, against the FP64 oracle.

Forced relabeling (QS_REMAP_ALWAYS=1) exercises one and two restoring
passes on circuits whose SWAPs form long cycles; remap = 1 keeps SWAPs as
gates; the default decides by pass count.  The same bars as every circuit:
complex128 max abs error <= 1e-12, complex64 fidelity >= 1 - 1e-6.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qs():
    import paper_2506_09198_amd as qs

    assert qs.qs_device_count() >= 1, "no HIP device visible"
    return qs


def _check(got, want, dt, what=""):
    got = got.astype(np.complex128)
    err = float(np.max(np.abs(got - want)))
    if dt == 2:
        assert err <= 1e-12, f"{what}: max abs err {err:.3e}"
    else:
        fid = abs(np.vdot(want, got)) ** 2
        assert fid >= 1 - 1e-6 and err <= 2e-5, f"{what}: fidelity {fid!r} err {err:.3e}"


CIRCS = {
    "qft14": lambda: W.qft(14, 9876),
    "qft17": lambda: W.qft(17, 4321),
    "swapnet12": lambda: W.swap_network(12, 200, 10),
    "swapnet16": lambda: W.swap_network(16, 300, 12),
    "swapnet19": lambda: W.swap_network(19, 240, 13),
    "swapnet7": lambda: W.swap_network(7, 60, 11),
}


@pytest.mark.parametrize("dt", [2, 1])
@pytest.mark.parametrize("name", list(CIRCS))
@pytest.mark.parametrize("how", ["forced", "auto", "off"])
def test_relabeled_circuits_match_oracle(qs, monkeypatch, dt, name, how):
    c = CIRCS[name]()
    ops, mats = c.arrays()
    remap = 1 if how == "off" else 0
    if how == "forced":
        monkeypatch.setenv("QS_REMAP_ALWAYS", "1")
    tq = 6 if c.n <= 12 else 0
    restore = qs.qs_plan_restore(c.n, dt, ops, mats, tile_qubits=tq, remap=remap)
    if how == "forced":
        assert 1 <= len(restore) <= 2
    if how == "off":
        assert restore == []
    s = qs.State.create(c.n, dt)
    s.init_basis(c.init_basis)
    qs.qs_trace_enable(s.h, True)
    s.run_circuit(c, tile_qubits=tq, remap=remap)
    kinds = [qs.KIND_NAMES[k] for k in qs.qs_trace_read(s.h)["kind"]]
    assert kinds.count("perm") == len(restore)
    assert kinds.count("tile") + len(restore) == qs.qs_plan_circuit(c.n, dt, ops, mats, tile_qubits=tq,
                                                                    remap=remap)[0]
    _check(s.download(), oracle.run_circuit(c), dt, f"{name} {how}")
    s.close()


@pytest.mark.parametrize("dt", [2, 1])
def test_qft_n24_relabeled_closed_form(qs, dt):
    """24-qubit QFT of a basis state (default planning relabels its SWAPs):
    every amplitude against the closed form, and the restoring pass moved
    the qubits back (without it the amplitudes would be bit-reversed)."""
    n, x = 24, 0xA5C3E1
    c = W.qft(n, x)
    ops, mats = c.arrays()
    assert len(qs.qs_plan_restore(n, dt, ops, mats)) == 1
    s = qs.State.create(n, dt)
    s.init_basis(x)
    s.run_circuit(c)
    got = s.download().astype(np.complex128)
    y = np.arange(1 << n, dtype=np.int64)
    want = np.exp(2j * np.pi * ((x * y) % (1 << n)) / (1 << n)) / math.sqrt(1 << n)
    err = float(np.max(np.abs(got - want)))
    assert err <= (1e-12 if dt == 2 else 2e-6), err
    s.close()
