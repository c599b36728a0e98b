"""A host model of what the tile kernels do with a planned pass (test
infrastructure).  It executes the planner's encoded operations -- tile
qubits, register segments, fused register blocks, diagonal forms -- on a
complex128 state with numpy, so a CPU test can compare the result with the
FP64 oracle and catch an encoding mistake without a GPU.  After SWAP
relabeling the passes act on physical qubit positions, and the restoring
involutions (one in-place exchange of bit pairs each) follow them.  It follows the
field meanings the kernels use; it does not model rounding or thread layout.
Fused matrix-core blocks are decoded from their fragment layouts (FP64
fragments, or FP32 hi + bfloat16 lo fragments) back into the dense matrix
they carry.
"""
import numpy as np

TK_DENSE1, TK_DENSE2, TK_DENSEK, TK_DIAG, TK_MFMA, TK_SEG = range(6)
SO_1Q, SO_2Q, SO_D0, SO_D1, SO_D2, SO_D1X, SO_D2X, SO_BLOCK, SO_DG, SO_DGROUP = 0, 8, 20, 21, 25, 31, 39, 63, 64, 65
SD_GATHER = 7


def _bit(x, pos):
    return (x >> pos) & 1


def _cmat(pool, moff, d):
    v = pool[moff:moff + 2 * d * d]
    return (v[0::2] + 1j * v[1::2]).reshape(d, d)


def _cvec(pool, moff, d):
    v = pool[moff:moff + 2 * d]
    return v[0::2] + 1j * v[1::2]


def _dense(T, tsel, esel, targets, U):
    """Apply U (index bit j = targets[j]) to the tile elements of the
    selected tiles whose group base passes esel (a mask over group bases)."""
    k = len(targets)
    E = T.shape[1]
    e = np.arange(E)
    tm = sum(1 << t for t in targets)
    g0 = e[(e & tm) == 0]
    g0 = g0[esel(g0)]
    if g0.size == 0 or not tsel.any():
        return
    offs = np.array([sum(_bit(mi, j) << targets[j] for j in range(k)) for mi in range(1 << k)])
    cols = g0[:, None] | offs[None, :]                 # (groups, D)
    V = T[np.ix_(tsel, cols.ravel())].reshape(int(tsel.sum()), g0.size, 1 << k)
    W = V @ U.T
    T[np.ix_(tsel, cols.ravel())] = W.reshape(int(tsel.sum()), -1)


def _diag(T, tsel, factor):
    """Multiply the selected tiles elementwise by factor (ntiles x E)."""
    T[tsel] *= factor[tsel]


def _member(T, base, R, op, pool):
    E = T.shape[1]
    e = np.arange(E)
    tsel = (base & int(op["gcm"])) == int(op["gcv"])
    opc = int(op["rsv"]) >> 16
    lcm, lcv = int(op["lcm"]), int(op["lcv"])
    ctl = lambda g: (g & lcm) == lcv
    if opc == SO_BLOCK:
        _dense(T, tsel, lambda g: np.ones(g.size, bool), list(R), _cmat(pool, int(op["moff"]), 1 << len(R)))
        return
    if opc < SO_D0:
        rb = int(op["rsv"]) & 0xFFFF
        if opc < SO_2Q:
            _dense(T, tsel, ctl, [R[rb & 255]], _cmat(pool, int(op["moff"]), 2))
        else:
            _dense(T, tsel, ctl, [R[rb & 255], R[(rb >> 8) & 255]], _cmat(pool, int(op["moff"]), 4))
        return
    k = int(op["k"])
    tab = _cvec(pool, int(op["moff"]), 1 << k)
    if opc == SO_DGROUP:
        tp = [q for q in range(32) if (int(op["lcm"]) >> q) & 1]
        gp = [q for q in range(64) if (int(op["lcv"]) >> q) & 1]
        rdep = (int(op["dj"]) >> 16) & 15  # register bits the factors depend on
        rq = [q for b, q in enumerate(R) if (rdep >> b) & 1]
        idx = np.zeros((T.shape[0], E), dtype=np.int64)
        for b, q in enumerate(rq):
            idx |= _bit(e, q)[None, :] << b
        for b, q in enumerate(tp):
            idx |= _bit(e, q)[None, :] << (len(rq) + b)
        for b, q in enumerate(gp):
            idx |= _bit(base, q)[:, None] << (len(rq) + len(tp) + b)
        _diag(T, tsel, tab[idx])
        return
    if opc == SO_DG:
        idx = np.zeros((T.shape[0], E), dtype=np.int64)
        for j in range(k):
            q = int(op["lp"][j])
            b = _bit(e, q)[None, :] if q >= 0 else _bit(base, int(op["p"][j]))[:, None]
            idx |= b << j
        f = np.where(((e & lcm) == lcv)[None, :], tab[idx], 1.0)
        _diag(T, tsel, f)
        return
    kr, kt = int(op["dj"]) & 15, (int(op["dj"]) >> 4) & 15
    ranks = [int(op["rsv"]) & 255, (int(op["rsv"]) >> 8) & 255]
    idx = np.zeros((T.shape[0], E), dtype=np.int64)
    for j in range(k):
        if j < kr:
            b = _bit(e, R[ranks[j]])[None, :]
        elif j < kr + kt:
            b = _bit(e, int(op["p"][j]))[None, :]
        else:
            b = _bit(base, int(op["p"][j]))[:, None]
        idx |= b << j
    f = tab[idx]
    if SO_D1X <= opc < SO_D2X:
        ri = (opc - SO_D1X) % 2
        keep = _bit(e, R[ranks[0]]) == ri
        f = np.where(keep[None, :], f, 1.0)
    elif SO_D2X <= opc < SO_D2X + 24:
        ri = (opc - SO_D2X) % 4
        keep = (_bit(e, R[ranks[0]]) | (_bit(e, R[ranks[1]]) << 1)) == ri
        f = np.where(keep[None, :], f, 1.0)
    _diag(T, tsel, f)


def mfma_matrix(op, pool):
    """The complex 2^k x 2^k matrix a fused matrix-core block carries, read
    back from its fragments: the real embedding A (rows and columns
    interleaved re/im) has A[2r][2c] = Re U[r][c] and A[2r+1][2c] = Im U[r][c].
    FP64 form: doubles [q][lane][2], fragment f = 2q + j = rb * KS + ks holds
    A[16rb + lane%16][4ks + lane/16].  FP32 form (dclass 1): FP32 hi
    fragments [f][lane], then bfloat16 lo fragments
    [rb * KB + kb][lane][4] holding A[16rb + lane%16][16kb + 4(lane/16) + j]."""
    k = int(op["k"])
    D = 1 << k
    DR, RB, KS = 2 * D, (2 * D) // 16, (2 * D) // 4
    KB, NF = KS // 4, RB * KS
    A = np.zeros((DR, DR))
    moff = int(op["moff"])
    lanes = np.arange(64)
    if int(op["dclass"]) == 0:
        fr = pool[moff:moff + NF * 64]
        for rb in range(RB):
            for ks in range(KS):
                f = rb * KS + ks
                A[16 * rb + lanes % 16, 4 * ks + lanes // 16] = fr[((f // 2) * 64 + lanes) * 2 + f % 2]
    else:
        raw = np.ascontiguousarray(pool[moff:]).view(np.uint8)
        hi = raw[:NF * 64 * 4].view(np.float32)
        lo16 = raw[NF * 64 * 4:NF * 64 * 4 + RB * KB * 64 * 8].view(np.uint16)
        lo = (lo16.astype(np.uint32) << 16).view(np.float32)
        for rb in range(RB):
            for ks in range(KS):
                f = rb * KS + ks
                A[16 * rb + lanes % 16, 4 * ks + lanes // 16] = hi[f * 64 + lanes]
            for kb in range(KB):
                for j in range(4):
                    A[16 * rb + lanes % 16, 16 * kb + 4 * (lanes // 16) + j] += \
                        lo[((rb * KB + kb) * 64 + lanes) * 4 + j].astype(np.float64)
    return A[0::2, 0::2] + 1j * A[1::2, 0::2]


def _top(T, base, op, pool):
    """An operation outside a segment, in the planner's original form."""
    E = T.shape[1]
    e = np.arange(E)
    kind, k = int(op["kind"]), int(op["k"])
    lcm, lcv = int(op["lcm"]), int(op["lcv"])
    if kind == TK_DIAG:
        tsel = (base & int(op["gcm"])) == int(op["gcv"])
        tab = _cvec(pool, int(op["moff"]), 1 << k)
        idx = np.zeros((T.shape[0], E), dtype=np.int64)
        for j in range(k):
            q = int(op["lp"][j])
            b = _bit(e, q)[None, :] if q >= 0 else _bit(base, int(op["p"][j]))[:, None]
            idx |= b << j
        _diag(T, tsel, np.where(((e & lcm) == lcv)[None, :], tab[idx], 1.0))
        return
    if kind == TK_MFMA:  # fused blocks carry no controls
        tsel = np.ones(T.shape[0], dtype=bool)
        _dense(T, tsel, lambda g: np.ones(g.shape, dtype=bool), [int(x) for x in op["p"][:k]],
               mfma_matrix(op, pool))
        return
    if kind in (TK_DENSE1, TK_DENSE2, TK_DENSEK):
        tsel = (base & int(op["gcm"])) == int(op["gcv"])
        _dense(T, tsel, lambda g: (g & lcm) == lcv, [int(x) for x in op["p"][:k]], _cmat(pool, int(op["moff"]), 1 << k))
        return
    raise NotImplementedError(f"op kind {kind} is not modelled")


def apply_involution(psi, n, tau):
    """The restoring pass: swap psi[y] with psi[y'] where y' is y with the bits
    at each exchanged pair of positions (p, tau[p]) swapped."""
    y = np.arange(1 << n, dtype=np.int64)
    z = y.copy()
    for p in range(n):
        q = int(tau[p])
        if q > p:
            diff = ((y >> p) ^ (y >> q)) & 1
            z ^= diff * ((1 << p) | (1 << q))
    return psi[z]


def run_plan(n, passes, tops, pool, psi, restore=()):
    """Apply the planned passes, then the restoring involutions, to psi
    (complex128, 2^n); returns the result."""
    psi = np.array(psi, dtype=np.complex128)
    for P in passes:
        m, Q = P["m"], P["Q"]
        others = [q for q in range(n) if q not in Q]
        e = np.arange(1 << m, dtype=np.int64)
        local = np.zeros(1 << m, dtype=np.int64)
        for j, q in enumerate(Q):
            local |= _bit(e, j) << q
        tau = np.arange(1 << (n - m), dtype=np.int64)
        base = np.zeros(tau.size, dtype=np.int64)
        for j, q in enumerate(others):
            base |= _bit(tau, j) << q
        idx = base[:, None] | local[None, :]
        T = psi[idx]
        ops = tops[P["op0"]:P["op0"] + P["nops"]]
        i = 0
        while i < len(ops):
            op = ops[i]
            if int(op["kind"]) == TK_SEG:
                R = [int(x) for x in op["p"][:int(op["k"])]]
                for mem in ops[i + 1:i + 1 + int(op["dj"])]:
                    _member(T, base, R, mem, pool)
                i += 1 + int(op["dj"])
                continue
            _top(T, base, op, pool)
            i += 1
        psi[idx] = T
    for tau in restore:
        psi = apply_involution(psi, n, tau)
    return psi
