"""GPU parity of the diagonal (phase-only) kernel against the FP64 oracle.

Diagonal gates reach the kernel from qs_apply_diag and from qs_apply_1q /
qs_apply_2q / qs_apply_fused whenever the matrix has no nonzero off-diagonal
entry.  Only amplitudes whose factor differs from 1 are read; the rest must
stay bitwise unchanged.  Bars as for every gate: complex128 max abs error
<= 1e-12, complex64 fidelity >= 1 - 1e-6; untouched amplitudes bit-exact.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TOL128 = 1e-12
DTS = [2, 1]  # QS_C128, QS_C64


@pytest.fixture(scope="module")
def qs():
    import paper_2506_09198_amd as qs

    assert qs.qs_device_count() >= 1, "no HIP device visible"
    return qs


def _check(got, want, dt, what=""):
    got = got.astype(np.complex128)
    err = float(np.max(np.abs(got - want)))
    if dt == 2:
        assert err <= TOL128, f"{what}: max abs err {err:.3e}"
    else:
        fid = abs(np.vdot(want, got)) ** 2 / abs(np.vdot(want, want)) ** 2
        assert fid >= 1 - 1e-6 and err <= 2e-5, f"{what}: fidelity {fid!r} err {err:.3e}"


def _phase_diag(rng, k, unit_frac):
    """2^k unit-modulus entries; about unit_frac of them exactly 1."""
    d = np.exp(1j * rng.uniform(0, 2 * np.pi, 1 << k))
    d[rng.random(1 << k) < unit_frac] = 1.0
    return d


def _gates(n, rng):
    """A mixed list of diagonal gates (targets, diagonal, cmask, cvals, route)."""
    out = []
    for t in range(n):
        out.append(([t], np.array([1, -1]), 0, 0, "1q"))                                 # Z
        th = rng.uniform(0, 2 * np.pi)
        out.append(([t], np.exp(1j * np.array([-th / 2, th / 2])), 0, 0, "1q"))           # RZ
    pairs = [(a, b) for a in range(n) for b in range(n) if a != b]
    if len(pairs) > 40:
        pairs = [pairs[i] for i in rng.choice(len(pairs), 40, replace=False)]
    for c, t in pairs:
        phi = rng.uniform(0, 2 * np.pi)
        out.append(([t], np.array([1, np.exp(1j * phi)]), 1 << c, 1 << c, "1q"))          # CP as controlled phase
        out.append(([t], np.array([1, -1]), 1 << c, 0, "1q"))                             # CZ on control value 0
        out.append(([c, t], np.array([1, 1, 1, np.exp(1j * phi)]), 0, 0, "2q"))           # CP as 4x4 diagonal
        out.append(([c, t], _phase_diag(rng, 2, 0.3), 0, 0, "2q"))
    if n >= 2:
        for _ in range(4):                                                                # multi-controlled Z
            t = int(rng.integers(n))
            others = [q for q in range(n) if q != t]
            cm = sum(1 << q for q in others)
            cv = int(rng.integers(0, 1 << n)) & cm
            out.append(([t], np.array([1, -1]), cm, cv, "1q"))
    for k in range(1, min(n, 6) + 1):
        for route in ("fused", "diag"):
            perm = [int(q) for q in rng.permutation(n)]
            tg, rest = perm[:k], perm[k:]
            nc = min(len(rest), int(rng.integers(0, 3)))
            cm = sum(1 << q for q in rest[:nc])
            cv = int(rng.integers(0, 1 << n)) & cm
            out.append((tg, _phase_diag(rng, k, 0.5), cm, cv, route))
    return out


def _apply(qs, s, tg, d, cm, cv, route):
    if route == "1q":
        s.apply_1q(tg[0], np.diag(d), cm, cv)
    elif route == "2q":
        s.apply_2q(tg[0], tg[1], np.diag(d), cm, cv)
    elif route == "fused":
        s.apply_fused(tg, np.diag(d), cm, cv)
    else:
        s.apply_diag(tg, d, cm, cv)


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 9, 13, 17])
def test_diagonal_gates_match_oracle(qs, dt, n):
    rng = np.random.default_rng(500 + n)
    psi0 = W.random_state(n, 40 + n)
    want = psi0.copy()
    s = qs.State.create(n, dt)
    s.upload(psi0.astype(np.complex128 if dt == 2 else np.complex64))
    for i, (tg, d, cm, cv, route) in enumerate(_gates(n, rng)):
        _apply(qs, s, tg, d, cm, cv, route)
        oracle.apply_op(n, want, tg, np.diag(d), cm, cv)
        if i % 16 == 0:
            _check(s.download(), want, dt, f"n={n} gate {i} {route} targets {tg}")
    _check(s.download(), want, dt, f"n={n} end")
    s.close()


def _factor_is_one(n, tg, d, cm, cv):
    i = np.arange(1 << n, dtype=np.int64)
    j = np.zeros_like(i)
    for b, q in enumerate(tg):
        j |= ((i >> q) & 1) << b
    ctl = (i & cm) == cv
    return ~ctl | (d[j] == 1)


@pytest.mark.parametrize("dt", DTS)
def test_untouched_amplitudes_stay_bitwise(qs, dt):
    """Amplitudes whose factor is 1 keep their bits, also those that share a
    128-byte line with changed ones (low fixed bits are written back)."""
    n = 12
    ct = np.complex128 if dt == 2 else np.complex64
    psi0 = W.random_state(n, 77).astype(ct)
    cases = [([5], np.array([1, -1]), 1 << 0, 1 << 0), ([0], np.array([1, 1j]), 1 << 1, 1 << 1),
             ([2], np.array([1, -1]), 1 << 9, 0), ([11], np.array([1, -1]), ((1 << 11) - 1), 0b10110011001),
             ([1, 7], np.array([1, 1, np.exp(0.3j), 1]), 0, 0)]
    for tg, d, cm, cv in cases:
        s = qs.State.create(n, dt)
        s.upload(psi0)
        s.apply_diag(tg, d, cm, cv)
        got = s.download()
        keep = _factor_is_one(n, tg, d, cm, cv)
        assert np.array_equal(got[keep].view(np.uint8), psi0[keep].view(np.uint8)), (tg, cm, cv)
        want = psi0.astype(np.complex128)
        oracle.apply_op(n, want, tg, np.diag(d), cm, cv)
        _check(got, want, dt, f"{tg}")
        s.close()


def test_identity_diagonal_launches_nothing(qs):
    n = 10
    psi0 = W.random_state(n, 5)
    s = qs.State.create(n, 2)
    s.upload(psi0)
    qs.qs_trace_enable(s.h, True)
    s.apply_1q(3, np.eye(2))
    s.apply_diag([1, 4], np.ones(4), 1 << 7, 0)
    s.apply_fused([0, 2, 5], np.eye(8))
    assert len(qs.qs_trace_read(s.h)) == 0
    assert np.array_equal(s.download(), psi0)
    s.close()


def test_trace_kind_and_algorithmic_bytes(qs):
    n = 14
    s = qs.State.create(n, 2)
    qs.qs_trace_enable(s.h, True)
    s.apply_1q(9, W.phase(0.7), 1 << 3)                     # CP: a quarter of the state
    s.apply_2q(3, 9, np.diag([1, 1, 1, -1]))                # CZ as a 4x4 diagonal
    s.apply_1q(5, np.diag(np.exp([-0.2j, 0.2j])))           # RZ: every amplitude
    s.apply_1q(13, np.diag([1, -1]), (1 << 13) - 1, 0)      # multi-controlled Z: one amplitude
    s.apply_diag([0, 6, 12], np.array([1, 1, 1, 1, 1, 1, 1j, -1j]))  # two entries of eight
    recs = qs.qs_trace_read(s.h)
    assert [qs.KIND_NAMES[k] for k in recs["kind"]] == ["diag"] * 5
    S = 16
    assert recs["bytes"].tolist() == [2 * S * (1 << (n - 2))] * 2 + [2 * S * (1 << n), 2 * S, 2 * S * (1 << (n - 2))]
    assert (recs["ms"] > 0).all()
    s.close()


def test_apply_diag_rejects_bad_arguments(qs):
    n = 6
    psi0 = W.random_state(n, 8)
    s = qs.State.create(n, 2)
    s.upload(psi0)
    bad = [([], np.ones(1)), ([0, 1, 2, 3, 4, 5, 6][:7], np.ones(128)), ([1, 1], np.ones(4)), ([6], np.ones(2)),
           ([2], np.array([1, np.nan])), ([2], np.array([np.inf, 1]))]
    for tg, d in bad:
        with pytest.raises((qs.QSError, ValueError)):
            s.apply_diag(tg, d)
    with pytest.raises(qs.QSError):
        s.apply_diag([2], np.array([1, -1]), 1 << 2, 1 << 2)    # control equals target
    with pytest.raises(qs.QSError):
        s.apply_diag([2], np.array([1, -1]), 1 << 3, 1 << 4)    # value outside the mask
    with pytest.raises(ValueError):
        s.apply_diag([2, 3], np.ones(2))                        # shape does not match k
    assert np.array_equal(s.download(), psi0)
    s.close()


@pytest.mark.parametrize("dt", DTS)
def test_per_gate_circuits_take_the_diagonal_kernel(qs, dt):
    """QFT and Grover one launch per gate: every controlled phase and phase
    flip runs as a diagonal launch, and the result matches the oracle."""
    for c in (W.qft(11, 1234), W.grover(9, 300)):
        s = qs.State.create(c.n, dt)
        s.init_basis(c.init_basis)
        qs.qs_trace_enable(s.h, True)
        s.run_circuit(c, mode=1)
        kinds = [qs.KIND_NAMES[k] for k in qs.qs_trace_read(s.h)["kind"]]
        ndiag = sum(1 for tg, u, cm, cv in c.gates if np.count_nonzero(u - np.diag(np.diag(u))) == 0
                    and not np.array_equal(np.diag(u), np.ones(u.shape[0])))
        assert kinds.count("diag") == ndiag > 0
        _check(s.download(), oracle.run_circuit(c), dt, c.name)
        s.close()


def _torch_state(n, seed):
    import torch

    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    psi = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
    chunk = 1 << 26
    nrm2 = 0.0
    for i in range(0, 1 << n, chunk):
        blk = torch.randn(min(chunk, (1 << n) - i), dtype=torch.complex128, device="cuda", generator=g)
        nrm2 += float((blk.real.square().sum() + blk.imag.square().sum()).item())
        psi[i:i + blk.numel()] = blk
    psi /= math.sqrt(nrm2)
    return psi


def test_diagonal_sweep_n30_c128_sampled(qs):
    """30 qubits complex128 in the launch configuration the bench times: CZ
    on neighbouring and distant pairs (control below and above a sector),
    CP, RZ, a multi-controlled Z, 2- and 3-qubit diagonals, each checked on
    4096 sampled outputs (half of them drawn among the changed amplitudes)
    against the oracle's per-amplitude definition."""
    import torch

    n = 30
    psi = _torch_state(n, 31)
    prev = torch.empty_like(psi)
    s = qs.State.from_torch(psi)
    rng = np.random.default_rng(32)
    gates = [([t + 1], np.array([1, -1]), 1 << t, 1 << t) for t in (0, 1, 2, 3, 14, 28)]
    gates += [([t], np.array([1, np.exp(0.37j)]), 1 << c, 1 << c) for c, t in ((29, 0), (2, 20), (7, 3))]
    gates += [([t], np.exp(1j * np.array([-0.4, 0.4])), 0, 0) for t in (0, 17)]
    gates += [([29], np.array([1, -1]), (1 << 29) - 1, 0x2A5A5A5A & ((1 << 29) - 1))]
    gates += [([1, 25], _phase_diag(rng, 2, 0.3), 0, 0), ([0, 12, 27], _phase_diag(rng, 3, 0.5), 1 << 5, 0)]
    for g, (tg, d, cm, cv) in enumerate(gates):
        prev.copy_(psi)
        qs.qs_apply_diag(s.h, tg, d, cm, cv)
        s.sync()
        idx = rng.integers(0, 1 << n, size=4096, dtype=np.uint64)
        # force half of the samples onto amplitudes the gate changes
        fixed = cm
        val = cv
        j = rng.integers(0, 1 << len(tg), size=2048)
        j = np.array([x for x in j if d[x] != 1] or [int(np.argmax(d != 1))], dtype=np.int64)
        h = idx[:j.size] & ~np.uint64(fixed)
        h |= np.uint64(val)
        for b, q in enumerate(tg):
            h &= ~np.uint64(1 << q)
            h |= ((j >> b) & 1).astype(np.uint64) << np.uint64(q)
        idx[:j.size] = h

        def fetch(x):
            t = torch.from_numpy(x.astype(np.int64)).to("cuda")
            return prev[t].cpu().numpy()

        want = oracle.outputs_at(idx, tg, np.diag(d), cm, cv, fetch)
        got = psi[torch.from_numpy(idx.astype(np.int64)).to("cuda")].cpu().numpy()
        err = float(np.max(np.abs(got - want)))
        assert err <= TOL128, f"gate {g} targets {tg} ctrl {cm:#x}: {err:.3e}"
    s.close()
    assert abs(float((psi.abs() ** 2).sum().item()) - 1.0) < 1e-10
