"""Parity at the full workload sizes, in the launch configurations the bench
and the batch/serving paths use, on outputs the oracle can compute one by one
or on properties that hold at any size (closed forms, echo, norm).

- gate sweep, 30 qubits complex128: every gate's outputs on 2048 sampled
  indices against the oracle's per-amplitude definition (1e-12);
- 32 qubits: QFT of a random basis state against its closed form on samples
  (complex128 1e-12; complex64 estimated infidelity <= 1e-6), random chain
  circuit followed by its inverse returns |0..0> (echo);
- 4096-circuit batch: sampled circuits against the oracle or closed forms;
- 32-qubit random chain circuit gate by gate in complex128 (the per-gate
  kernels' block loops): every gate's outputs on sampled indices against the
  oracle's per-amplitude definition; the tile-pass runs (complex128, complex64
  with register blocks and with 5-qubit matrix-core blocks) are then compared
  on samples with that result, which shares no tile or fusion code;
- the deepest 20-22-qubit chain circuits of the 4096-circuit batch against the
  full oracle;
- serving mix beside a 34-qubit complex64 random circuit run as the bench runs
  it (echo + norm).
"""
import math
import time

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


def _torch_state(n, dtype, seed):
    import torch

    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    psi = torch.empty(1 << n, dtype=dtype, device="cuda")
    chunk = 1 << 26
    nrm2 = 0.0
    for i in range(0, 1 << n, chunk):
        blk = torch.randn(min(chunk, (1 << n) - i), dtype=torch.complex128, device="cuda", generator=g)
        nrm2 += float((blk.real.square().sum() + blk.imag.square().sum()).item())
        psi[i:i + blk.numel()] = blk.to(dtype)
    psi /= math.sqrt(nrm2)
    return psi


def test_gate_sweep_n30_c128_sampled_per_gate(qs):
    import torch

    n = 30
    psi = _torch_state(n, torch.complex128, 2)
    prev = torch.empty_like(psi)
    s = qs.State.from_torch(psi)
    circ = W.gate_microbench(n)
    rng = np.random.default_rng(12)
    worst = 0.0
    for g, (tg, u, cm, cv) in enumerate(circ.gates):
        prev.copy_(psi)
        if len(tg) == 1:
            qs.qs_apply_1q(s.h, tg[0], u, cm, cv)
        else:
            qs.qs_apply_2q(s.h, tg[0], tg[1], u, cm, cv)
        s.sync()
        idx = rng.integers(0, 1 << n, size=2048, dtype=np.uint64)

        def fetch(j):
            t = torch.from_numpy(j.astype(np.int64)).to("cuda")
            return prev[t].cpu().numpy()

        want = oracle.outputs_at(idx, tg, u, cm, cv, fetch)
        got = psi[torch.from_numpy(idx.astype(np.int64)).to("cuda")].cpu().numpy()
        err = float(np.max(np.abs(got - want)))
        worst = max(worst, err)
        assert err <= 1e-12, f"gate {g} targets {tg} ctrl {cm:#x}: {err:.3e}"
    s.close()
    assert abs(float((psi.abs() ** 2).sum().item()) - 1.0) < 1e-10


@pytest.mark.parametrize("dt,fuse", [(2, 0), (1, 0), (1, 5), (2, 5), (1, -5)])
def test_qft_n32_closed_form_sampled(qs, dt, fuse, monkeypatch):
    """fuse -5: 5-qubit blocks on FP32 matrix cores (complex64)."""
    monkeypatch.setenv("QS_FUSE_FP32", "1" if fuse < 0 else "0")
    fuse = abs(fuse)
    n = 32
    x = int(np.random.default_rng(6).integers(1 << n))
    c = W.qft(n, x)
    with qs.State.create(n, dt) as s:
        s.init_basis(x)
        s.run_circuit(c, mode=0, fuse_k=fuse)
        y = np.random.default_rng(7).integers(0, 1 << n, size=4096, dtype=np.uint64)
        got = np.array([s.download(int(v), 1)[0] for v in y[:512]], dtype=np.complex128)
        y = y[:512]
    N = 1 << n
    want = np.exp(2j * np.pi * ((x * y.astype(object)) % N).astype(np.float64) / N) / math.sqrt(N)
    d = got - want
    if dt == 2:
        assert float(np.max(np.abs(d))) <= 1e-12
    else:
        infid = N * float(np.mean(np.abs(d) ** 2))  # estimate of 1 - F from samples
        assert infid <= 1e-6, infid


def _gather(t, idx):
    import torch

    return t[torch.from_numpy(np.asarray(idx, dtype=np.uint64).astype(np.int64)).to(t.device)].cpu().numpy()


def test_rqc_n32_c128_pergate_sampled_and_tile_anchors(qs):
    """Config 3A gate by gate (complex128, 64 GiB): each gate's outputs on 256
    sampled indices against the oracle's definition, from the GPU state just
    before that gate.  The per-gate result then anchors the tile-pass runs of
    the same circuit on 4096 samples: complex128 (register blocks, and 5-qubit
    matrix-core blocks) within 1e-12, complex64 (both forms) with an
    estimated infidelity below 1e-6."""
    import torch

    n = 32
    c = W.rqc_chain(n, 20, 5)
    ops, mats = c.arrays()
    psi = torch.zeros(1 << n, dtype=torch.complex128, device="cuda")
    psi[0] = 1
    torch.cuda.synchronize()
    s = qs.State.from_torch(psi)
    rng = np.random.default_rng(32)
    worst = 0.0
    for g, (tg, u, cm, cv) in enumerate(c.gates):
        idx = rng.integers(0, 1 << n, size=256, dtype=np.uint64)
        want = oracle.outputs_at(idx, tg, u, cm, cv, lambda j: _gather(psi, j))
        if len(tg) == 1:
            qs.qs_apply_1q(s.h, tg[0], u, cm, cv)
        else:
            qs.qs_apply_2q(s.h, tg[0], tg[1], u, cm, cv)
        s.sync()
        err = float(np.max(np.abs(_gather(psi, idx) - want)))
        worst = max(worst, err)
        assert err <= 1e-12, f"gate {g} targets {tg} ctrl {cm:#x}: {err:.3e}"
    assert abs(s.norm() - 1.0) < 1e-11
    s.close()
    ys = np.random.default_rng(33).integers(0, 1 << n, size=4096, dtype=np.uint64)
    ref = _gather(psi, ys)
    N = float(1 << n)
    for dt, fuse in ((2, 0), (2, 5), (1, 0), (1, 5)):
        with qs.State.create(n, dt) as t:
            t.run(ops, mats, mode=0, fuse_k=fuse)
            got = np.array([t.download(int(v), 1)[0] for v in ys], dtype=np.complex128)
        d = got - ref
        if dt == 2:
            assert float(np.max(np.abs(d))) <= 1e-12, (dt, fuse, float(np.max(np.abs(d))))
        else:
            infid = N * float(np.mean(np.abs(d) ** 2))  # estimate of 1 - F from samples
            assert infid <= 1e-6, (dt, fuse, infid)
    del psi
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dt,fuse", [(2, 0), (1, 0), (1, 5), (2, 5), (1, -5)])
def test_rqc_n32_echo(qs, dt, fuse, monkeypatch):
    """fuse -5: 5-qubit blocks on FP32 matrix cores (complex64)."""
    monkeypatch.setenv("QS_FUSE_FP32", "1" if fuse < 0 else "0")
    fuse = abs(fuse)
    n = 32
    c = W.rqc_chain(n, 20, 5)
    ops, mats = c.arrays()
    iops, imats = c.inverse().arrays()
    with qs.State.create(n, dt) as s:
        s.run(ops, mats, mode=0, fuse_k=fuse)
        nrm = s.norm()
        s.run(iops, imats, mode=0, fuse_k=fuse)
        a0 = complex(s.download(0, 1)[0])
        nrm2 = s.norm()
    if dt == 2:
        assert abs(nrm - 1) < 1e-12 and abs(a0 - 1) < 1e-12 and abs(nrm2 - 1) < 1e-12
    else:
        assert abs(a0) ** 2 >= 1 - 2e-6 and abs(nrm - 1) < 1e-5


def _expected(c):
    """Oracle for small n; closed forms for QFT and Grover at any n."""
    n = c.n
    if c.name.startswith("qft"):
        x, N = c.init_basis, 1 << n
        yv = np.arange(N, dtype=np.int64)
        return np.exp(2j * np.pi * ((x * yv) % N) / N) / math.sqrt(N)
    if c.name.startswith("grover"):
        mark = int(c.name.split("_m")[1].split("_")[0])
        R = int(c.name.split("_r")[1])
        th = math.asin(2.0 ** (-n / 2))
        s = (-1) ** R
        v = np.full(1 << n, s * math.cos((2 * R + 1) * th) / math.sqrt((1 << n) - 1), dtype=complex)
        v[mark] = s * math.sin((2 * R + 1) * th)
        return v
    return oracle.run_circuit(c)


def _fid_ok(got, want, dt):
    got = got.astype(np.complex128)
    if dt == 2:
        return float(np.max(np.abs(got - want))) <= 1e-12
    return abs(np.vdot(want, got)) ** 2 >= 1 - 1e-6


def _deepest_chains(circs, per_n=1):
    """Indices of the deepest chain circuits at each of n = 20, 21, 22 (the
    pass-major class's longest runs, up to ~6600 gates)."""
    out = []
    for n in (20, 21, 22):
        cand = [i for i, c in enumerate(circs) if c.n == n and c.name.startswith("rqc")]
        cand.sort(key=lambda i: -len(circs[i]))
        out += cand[:per_n]
    return out


def test_batch_4096_sampled(qs):
    circs = W.circuit_mix(4096, 7)
    arrs = [(c.n, *c.arrays(), c.init_basis) for c in circs]
    rng = np.random.default_rng(3)
    pick = [i for i in rng.permutation(len(circs)) if circs[i].n <= 14 or not circs[i].name.startswith("rqc")][:24]
    deep = _deepest_chains(circs)
    assert len(deep) == 3 and min(len(circs[i]) for i in deep) > 5000
    wants = {i: _expected(circs[i]) for i in pick + deep}  # deep chains: full oracle, seconds each
    for dt, mode in ((1, 0), (2, 0), (2, 1)):
        b = qs.qs_batch_submit(arrs, dtype=dt, mode=mode)
        try:
            qs.qs_batch_wait(b)
            for i in pick + deep:
                got = qs.qs_batch_download(b, int(i), dt)
                assert _fid_ok(got, wants[i], dt), (dt, mode, circs[i].name)
        finally:
            qs.qs_batch_release(b)


def test_serving_beside_n34_c64(qs):
    """The 34-qubit complex64 circuit as the serving bench runs it (register
    blocks, no matrix-core fusion, 256-workgroup cap), forward while the
    request stream is served, then its inverse."""
    import torch

    big = W.rqc_chain(34, 24, 9)
    bops, bmats = big.arrays()
    iops, imats = big.inverse().arrays()
    side = torch.cuda.Stream()
    psi = torch.zeros(1 << 34, dtype=torch.complex64, device="cuda")
    psi[0] = 1
    torch.cuda.synchronize()
    bs = qs.State.from_torch(psi, stream=side.cuda_stream)
    bs.run(bops, bmats, mode=0, fuse_k=0, max_blocks=256)  # own stream; serving runs meanwhile
    srv = qs.qs_server_create(dtype=1, hbm_budget=24 << 30)
    try:
        rng = np.random.default_rng(8)
        circs = []
        for _ in range(48):
            n = W.log_uniform_n(rng, 8, 24)
            k = int(rng.integers(3))
            circs.append(W.rqc_chain(n, int(rng.integers(2, 8)), int(rng.integers(1000))) if k == 0 and n <= 14
                         else (W.qft(n, int(rng.integers(1 << n))) if k != 2 else W.grover(n, int(rng.integers(1 << n)))))
        ids = []
        done = {}
        t_end = time.time() + 120
        for c in circs:
            ids.append(qs.qs_server_submit(srv, c))
            for r in qs.qs_server_poll(srv):
                done[r["id"]] = r
        while len(done) < len(ids):
            for r in qs.qs_server_poll(srv):
                done[r["id"]] = r
            assert time.time() < t_end
            time.sleep(0.0002)
        for rid, c in zip(ids, circs):
            assert done[rid]["status"] == 0
            assert _fid_ok(qs.qs_server_download(srv, rid, 1), _expected(c), 1), c.name
    finally:
        qs.qs_server_destroy(srv)
    bs.run(iops, imats, mode=0, fuse_k=0, max_blocks=256)
    bs.sync()
    a0 = complex(psi[0].item())
    nrm = bs.norm()
    bs.close()
    del psi
    torch.cuda.empty_cache()
    assert abs(a0) ** 2 >= 1 - 2e-6 and abs(nrm - 1) < 1e-5
