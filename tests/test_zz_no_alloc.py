"""The no-allocation marginal-probability entry point against the allocating
one (bitwise: same kernels, same order) and against the FP64 oracle, on two
calls in a row, the second with a smaller state; plus its argument checks."""
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


def _noalloc(qs, torch, s, qubits):
    out = torch.full((1 << len(qubits),), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    qs.qs_probabilities_noalloc(s.h, qubits, out.data_ptr())
    s.sync()
    return out.cpu().numpy()


@pytest.mark.parametrize("first,second", [((20, 2, [3, 17, 0]), (13, 1, [])),
                                          ((16, 1, list(range(16))), (12, 2, [11, 4]))])
def test_noalloc_matches_probabilities(qs, first, second):
    import torch

    for n, dt, qubits in (first, second):  # the second call takes a smaller input
        psi = W.random_state(n, 40 + n)
        host = psi if dt == 2 else psi.astype(np.complex64)
        with qs.State.create(n, dt) as s:
            s.upload(host)
            got = _noalloc(qs, torch, s, qubits)
            ref = s.probabilities(qubits)
        assert got.tobytes() == ref.tobytes(), (n, dt, qubits)
        want = oracle.probabilities(n, host.astype(np.complex128), qubits)
        assert float(np.max(np.abs(got - want))) <= 1e-13, (n, dt, qubits)


def test_noalloc_rejects(qs):
    import torch

    with qs.State.create(24, 1) as s:
        out = torch.empty(1 << 23, dtype=torch.float64, device="cuda")
        with pytest.raises(qs.QSError):
            qs.qs_probabilities_noalloc(s.h, list(range(23)), out.data_ptr())  # 2^23 > 2^22 doubles
        with pytest.raises(qs.QSError):
            qs.qs_probabilities_noalloc(s.h, [1], 0)  # null device output
        with pytest.raises(qs.QSError):
            qs.qs_probabilities_noalloc(s.h, [1, 1], out.data_ptr())  # duplicate qubit
        # the state is still usable after the rejected calls
        got = _noalloc(qs, torch, s, [0])
        assert abs(float(got.sum()) - 1.0) < 1e-12
