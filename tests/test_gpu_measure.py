"""Pauli expectation values and sampling on the GPU against the FP64 oracle
(small and ragged sizes, many chunks) and against closed forms at 28 qubits."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qs():
    import paper_2506_09198_amd as qs

    assert qs.qs_device_count() >= 1
    return qs


def _state(qs, n, dt, seed):
    psi = W.random_state(n, seed)
    s = qs.State.create(n, dt)
    s.upload(psi.astype(np.complex64 if dt == 1 else np.complex128))
    host = s.download(0, 1 << n).astype(np.complex128)  # what the device holds (complex64 rounded)
    return s, host


@pytest.mark.parametrize("dt", [2, 1])
@pytest.mark.parametrize("n", [1, 5, 12, 13, 17])
def test_expect_pauli_matches_oracle(qs, n, dt):
    rng = np.random.default_rng(n)
    s, host = _state(qs, n, dt, 50 + n)
    try:
        masks = [(0, 0), (0, (1 << n) - 1), ((1 << n) - 1, 0), ((1 << n) - 1, (1 << n) - 1)]
        masks += [(int(rng.integers(1 << n)), int(rng.integers(1 << n))) for _ in range(8)]
        for x, z in masks:
            got = qs.qs_expect_pauli(s.h, x, z)
            want = oracle.expect_pauli(n, host, x, z)
            assert abs(got - want) <= 1e-12, (x, z, got, want)
    finally:
        s.close()


@pytest.mark.parametrize("dt", [2, 1])
@pytest.mark.parametrize("n", [1, 3, 11, 12, 13, 17])
def test_sample_matches_oracle(qs, n, dt):
    s, host = _state(qs, n, dt, 60 + n)
    try:
        u = np.random.default_rng(n + 100 * dt).random(20000)
        got = qs.qs_sample(s.h, u)
        want = oracle.sample(n, host, u)
        assert np.array_equal(got, want)
    finally:
        s.close()


def test_sample_edges_and_errors(qs):
    with qs.State.create(8, 2) as s:
        s.init_basis(77)
        assert np.all(qs.qs_sample(s.h, np.array([0.0, 0.5, 0.999999999])) == 77)
        assert qs.qs_sample(s.h, np.zeros(0)).size == 0
        for bad in (np.array([1.0]), np.array([-0.1]), np.array([np.nan])):
            with pytest.raises(qs.QSError):
                qs.qs_sample(s.h, bad)
        with pytest.raises(qs.QSError):
            qs.qs_expect_pauli(s.h, 1 << 8, 0)
        assert qs.qs_expect_pauli(s.h, 0, 0b1001101) == (-1) ** bin(77 & 0b1001101).count("1")


def test_closed_forms_at_28_qubits(qs):
    """Uniform superposition: every sample is floor(u 2^n) (complex128; the
    amplitudes are 2^-14 up to ~1e-15 relative, so only u within 1e-4 of a bin
    edge may land one bin off); GHZ: <X..X> = <Z0 Z27> = 1, <Z0> = 0, samples
    0 or 2^n - 1."""
    n = 28
    with qs.State.create(n, 2) as s:
        c = W.Circuit(n, "h_all")
        for q in range(n):
            c.g1(q, W.u3(np.pi / 2, 0, np.pi))  # Hadamard
        s.run_circuit(c)
        u = np.random.default_rng(9).random(100000)
        got = qs.qs_sample(s.h, u).astype(np.int64)
        want = np.floor(u * (1 << n)).astype(np.int64)
        frac = u * (1 << n) - want
        inner = (frac > 1e-4) & (frac < 1 - 1e-4)
        assert np.array_equal(got[inner], want[inner]) and np.all(np.abs(got - want) <= 1)
        assert abs(qs.qs_expect_pauli(s.h, (1 << n) - 1, 0) - 1) < 1e-12  # <X..X> = 1 on |+>^n
        s.init_basis(0)
        g = W.Circuit(n, "ghz")
        g.g1(0, W.u3(np.pi / 2, 0, np.pi))
        for q in range(n - 1):
            g.g1(q + 1, np.array([[0, 1], [1, 0]], complex), controls=(q,))
        s.run_circuit(g)
        assert abs(qs.qs_expect_pauli(s.h, (1 << n) - 1, 0) - 1) < 1e-12
        assert abs(qs.qs_expect_pauli(s.h, 0, 1 | (1 << 27)) - 1) < 1e-12
        assert abs(qs.qs_expect_pauli(s.h, 0, 1)) < 1e-12
        smp = qs.qs_sample(s.h, u[:1000])
        assert np.array_equal(smp, np.where(u[:1000] < 0.5, 0, (1 << n) - 1).astype(np.uint64))
