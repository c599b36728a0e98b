"""Degenerate and boundary inputs on the GPU, each against the oracle:
one- and two-qubit states, circuits without gates, circuits of diagonal gates
only, batches and serving requests of those, and reductions over every qubit
of a small state."""
import time

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

DTS = [2, 1]


@pytest.fixture(scope="module")
def qs():
    import paper_2506_09198_amd as qs

    assert qs.qs_device_count() >= 1, "no HIP device visible"
    return qs


def _check(got, want, dt):
    got = got.astype(np.complex128)
    err = float(np.max(np.abs(got - want))) if got.size else 0.0
    assert err <= (1e-12 if dt == 2 else 2e-6), err


@pytest.mark.parametrize("dt", DTS)
def test_one_and_two_qubit_states(qs, dt):
    rng = np.random.default_rng(3)
    for n in (1, 2):
        psi0 = W.random_state(n, 10 + n)
        start = psi0 if dt == 2 else psi0.astype(np.complex64).astype(np.complex128)
        with qs.State.create(n, dt) as s:
            s.upload(psi0)
            want = start.copy()
            for t in range(n):
                u = W.haar_unitary(2, rng)
                qs.qs_apply_1q(s.h, t, u, 0, 0)
                oracle.apply_op(n, want, (t,), u)
            if n == 2:
                u = W.haar_unitary(4, rng)
                qs.qs_apply_2q(s.h, 1, 0, u, 0, 0)
                oracle.apply_op(n, want, (1, 0), u)
                u = W.haar_unitary(2, rng)
                qs.qs_apply_1q(s.h, 0, u, 1 << 1, 0)  # control on |0>
                oracle.apply_op(n, want, (0,), u, 1 << 1, 0)
            _check(s.download(), want, dt)
            host = s.download().astype(np.complex128)
            for qb in ([0], list(range(n)), list(range(n))[::-1]):
                got = s.probabilities(qb)
                assert float(np.max(np.abs(got - oracle.probabilities(n, host, qb)))) <= 1e-13
            assert abs(s.norm() - oracle.norm2(n, host)) <= 1e-13
            shots = qs.qs_sample(s.h, np.array([0.0, 0.25, 0.5, 0.999999]))
            assert np.array_equal(shots, oracle.sample(n, host, np.array([0.0, 0.25, 0.5, 0.999999])))


@pytest.mark.parametrize("dt", DTS)
def test_circuit_without_gates_leaves_state(qs, dt):
    n = 13
    psi0 = W.random_state(n, 4)
    c = W.Circuit(n, "empty")
    ops, mats = c.arrays()
    for mode in (0, 1):
        with qs.State.create(n, dt) as s:
            s.upload(psi0)
            before = s.download()
            s.run(ops, mats, mode=mode)
            assert s.download().tobytes() == before.tobytes()


@pytest.mark.parametrize("dt", DTS)
def test_diagonal_only_circuit(qs, dt):
    """CZ / CP / Z / RZ-type gates only: tile passes of diagonal groups and the
    per-gate diagonal kernel against the oracle."""
    n = 15
    rng = np.random.default_rng(6)
    c = W.Circuit(n, "diag")
    for _ in range(60):
        a, b = (int(x) for x in rng.choice(n, 2, replace=False))
        kind = int(rng.integers(3))
        if kind == 0:
            c.g1(a, W.Z, controls=(b,))
        elif kind == 1:
            c.g1(a, W.phase(float(rng.uniform(0, 2 * np.pi))), controls=(b,))
        else:
            c.g1(a, np.diag(np.exp(1j * rng.uniform(0, 2 * np.pi, 2))))
    ops, mats = c.arrays()
    psi0 = W.random_state(n, 7)
    want = oracle.run(n, ops, mats, psi0)
    for mode in (0, 1):
        with qs.State.create(n, dt) as s:
            s.upload(psi0)
            s.run(ops, mats, mode=mode)
            _check(s.download(), want, dt)


@pytest.mark.parametrize("dt", DTS)
def test_batch_and_server_degenerate_circuits(qs, dt):
    """A batch and a server holding a gate-free circuit, a one-qubit circuit
    and an ordinary one: every result against the oracle."""
    rng = np.random.default_rng(8)
    c0 = W.Circuit(5, "nogates", init_basis=19)
    c1 = W.Circuit(1, "oneq", init_basis=1).g1(0, W.haar_unitary(2, rng))
    c2 = W.rqc_chain(12, 4, 3)
    circs = [c0, c1, c2]
    wants = [oracle.run_circuit(c) for c in circs]
    b = qs.qs_batch_submit(circs, dtype=dt, mode=0)
    try:
        qs.qs_batch_wait(b)
        for i, w in enumerate(wants):
            _check(qs.qs_batch_download(b, i, dt), w, dt)
    finally:
        qs.qs_batch_release(b)
    srv = qs.qs_server_create(dtype=dt, hbm_budget=1 << 28)
    try:
        ids = [qs.qs_server_submit(srv, c) for c in circs]
        done, t_end = {}, time.time() + 60
        while len(done) < len(ids):
            for r in qs.qs_server_poll(srv):
                done[r["id"]] = r
            assert time.time() < t_end, "serving loop did not finish"
            time.sleep(0.0005)
        assert all(done[i]["status"] == 0 for i in ids)
        for i, w in zip(ids, wants):
            _check(qs.qs_server_download(srv, i, dt), w, dt)
    finally:
        qs.qs_server_destroy(srv)
