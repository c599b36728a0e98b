// Circuit planner and tile-pass executor.
//
// A pass keeps a set Q of at most m tile qubits and takes every gate that is
// ready (all gates it does not commute with are done) and fits: a
// non-diagonal gate when its targets fit into Q (growing Q), a diagonal gate
// (CZ, controlled phases, phase flips) always, since it scales amplitudes
// elementwise and needs no tile qubits.  Gates that commute are reordered;
// gates that do not keep their circuit order.  A closed pass is padded with
// the lowest unused qubits so its tiles are built from the longest possible
// contiguous runs.  Each pass costs one read and one write of the state,
// against one per gate when gates are launched one by one.
#include "planner.h"

#include <algorithm>
#include <complex>
#include <cstring>
#include <set>

namespace qs {

using cd = std::complex<double>;

// ---------------------------------------------------------------- fusion
//
// Inside one pass, consecutive operations whose qubits (targets and local
// controls, all inside the tile, no per-tile controls) fit in K qubits are
// multiplied into one 2^K x 2^K matrix in FP64 and applied as a single dense
// block on matrix cores.  The product stays FP64 and is stored in the
// A-fragment order of v_mfma_f64_16x16x4f64 for the real embedding
// [[Ur, -Ui], [Ui, Ur]].

static bool op_local_bits(const TileOp& t, uint32_t* bits)
{
    if (t.gcm != 0) return false;
    uint32_t b = (uint32_t)t.lcm;
    if (t.kind == TK_DIAG) {
        for (int j = 0; j < t.k; ++j) {
            if (t.lp[j] < 0) return false;
            b |= 1u << t.lp[j];
        }
    } else if (t.kind == TK_DENSE1 || t.kind == TK_DENSE2 || t.kind == TK_DENSEK) {
        for (int j = 0; j < t.k; ++j) b |= 1u << t.p[j];
    } else {
        return false;
    }
    *bits = b;
    return true;
}

// G = op * G for a 2^K x 2^K matrix G (row-major) on the block whose qubits
// are the tile positions bq[0..K): the op's matrix acts on each column of G
// directly, so a k-qubit op costs 2^K * 2^K * 2^k multiply-adds.
static void embed_op(const TileOp& t, const std::vector<double>& pool, const int* bq, int K, std::vector<cd>& G)
{
    const int D = 1 << K;
    int bidx[32];
    for (int i = 0; i < 32; ++i) bidx[i] = -1;
    for (int j = 0; j < K; ++j) bidx[bq[j]] = j;
    uint32_t cbm = 0, cbv = 0;
    for (int q = 0; q < 32; ++q)
        if ((t.lcm >> q) & 1) {
            cbm |= 1u << bidx[q];
            if ((t.lcv >> q) & 1) cbv |= 1u << bidx[q];
        }
    const bool diag = t.kind == TK_DIAG;
    int tb[6];
    uint32_t tmask = 0;
    for (int j = 0; j < t.k; ++j) {
        tb[j] = bidx[diag ? t.lp[j] : t.p[j]];
        tmask |= 1u << tb[j];
    }
    const int dk = 1 << t.k;
    const double* U = pool.data() + t.moff;
    auto row_of = [&](uint32_t r0, int m) {
        uint32_t r = r0;
        for (int j = 0; j < t.k; ++j)
            if ((m >> j) & 1) r |= 1u << tb[j];
        return r;
    };
    if (diag) {
        for (int r = 0; r < D; ++r) {
            if (((uint32_t)r & cbm) != cbv) continue;
            int mi = 0;
            for (int j = 0; j < t.k; ++j) mi |= (int)((r >> tb[j]) & 1) << j;
            const cd f(U[2 * mi], U[2 * mi + 1]);
            cd* row = G.data() + (size_t)r * D;
            for (int c = 0; c < D; ++c) row[c] *= f;
        }
        return;
    }
    thread_local std::vector<cd> u;
    u.resize((size_t)dk * dk);
    for (int i = 0; i < dk * dk; ++i) u[i] = cd(U[2 * i], U[2 * i + 1]);
    cd v[64], w[64];
    for (uint32_t r0 = 0; r0 < (uint32_t)D; ++r0) {
        if ((r0 & tmask) != 0 || (r0 & cbm) != cbv) continue;
        uint32_t rows[64];
        for (int m = 0; m < dk; ++m) rows[m] = row_of(r0, m);
        for (int c = 0; c < D; ++c) {
            for (int m = 0; m < dk; ++m) v[m] = G[(size_t)rows[m] * D + c];
            for (int m = 0; m < dk; ++m) {
                cd acc = 0;
                for (int q = 0; q < dk; ++q) acc += u[m * dk + q] * v[q];
                w[m] = acc;
            }
            for (int m = 0; m < dk; ++m) G[(size_t)rows[m] * D + c] = w[m];
        }
    }
}

// Round to the nearest bfloat16 (ties to even): the upper half of the FP32
// bit pattern after rounding the lower half away.
static uint16_t bf16_rne(float x)
{
    uint32_t u;
    std::memcpy(&u, &x, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

static void fuse_pass(PlanPass& P, std::vector<double>& pool, int K, int min_dense, bool fp32)
{
    std::vector<TileOp> out;
    std::vector<int64_t> osrc;
    std::vector<size_t> blk;
    uint32_t bbits = 0;
    int bdense = 0;
    auto emit = [&]() {
        if (blk.empty()) return;
        if (bdense < min_dense) {
            for (size_t i : blk) {
                out.push_back(P.ops[i]);
                osrc.push_back(P.src[i]);
            }
        } else {
            uint32_t bits = bbits;
            for (int q = 0; __builtin_popcount(bits) < K && q < P.m; ++q) bits |= 1u << q;
            int bq[8], nb = 0;
            for (int q = 0; q < 32; ++q)
                if ((bits >> q) & 1) bq[nb++] = q;
            const int D = 1 << K;
            std::vector<cd> G((size_t)D * D, cd(0, 0));
            for (int i = 0; i < D; ++i) G[(size_t)i * D + i] = 1.0;
            for (size_t i : blk) embed_op(P.ops[i], pool, bq, K, G);
            const int DR = 2 * D, RB = DR / 16, KS = DR / 4, NF = RB * KS, KB = KS / 4;
            // the real embedding [[Ur, -Ui], [Ui, Ur]], interleaved rows and columns
            auto areal = [&](int row, int col) {
                const cd u = G[(size_t)(row / 2) * D + col / 2];
                if ((row & 1) == 0) return (col & 1) == 0 ? u.real() : -u.imag();
                return (col & 1) == 0 ? u.imag() : u.real();
            };
            std::vector<double> fr;
            if (!fp32) {
                fr.assign((size_t)NF * 64, 0.0); // [q][lane][2], fragment f = 2q + j
                for (int lane = 0; lane < 64; ++lane)
                    for (int rb = 0; rb < RB; ++rb)
                        for (int ks = 0; ks < KS; ++ks) {
                            const int f = rb * KS + ks;
                            fr[((size_t)(f / 2) * 64 + lane) * 2 + (f % 2)] =
                                areal(16 * rb + (lane % 16), 4 * ks + lane / 16);
                        }
            } else {
                // FP32 form: hi = the FP32 rounding of each entry, as
                // v_mfma_f32_16x16x4f32 A fragments ([f][lane] floats,
                // fragment f = rb * KS + ks, lane l: row 16rb + l%16, column
                // 4ks + l/16); lo = the remainder rounded to bfloat16,
                // as v_mfma_f32_16x16x16bf16 A fragments ([rb * KB + kb][lane]
                // x 4, lane l: row 16rb + l%16, columns 16kb + 4(l/16) + j).
                std::vector<float> hi((size_t)NF * 64);
                std::vector<uint16_t> lo((size_t)RB * KB * 64 * 4);
                for (int lane = 0; lane < 64; ++lane)
                    for (int rb = 0; rb < RB; ++rb) {
                        const int row = 16 * rb + (lane % 16);
                        for (int ks = 0; ks < KS; ++ks) {
                            const int f = rb * KS + ks;
                            hi[(size_t)f * 64 + lane] = (float)areal(row, 4 * ks + lane / 16);
                        }
                        for (int kb = 0; kb < KB; ++kb)
                            for (int j = 0; j < 4; ++j) {
                                const double a = areal(row, 16 * kb + 4 * (lane / 16) + j);
                                const float h = (float)a;
                                lo[(((size_t)(rb * KB + kb) * 64 + lane) * 4) + j] = bf16_rne((float)(a - (double)h));
                            }
                    }
                fr.assign((hi.size() * 4 + lo.size() * 2 + 7) / 8, 0.0);
                std::memcpy(fr.data(), hi.data(), hi.size() * 4);
                std::memcpy((char*)fr.data() + hi.size() * 4, lo.data(), lo.size() * 2);
            }
            TileOp t;
            std::memset(&t, 0, sizeof t);
            t.kind = TK_MFMA;
            t.k = K;
            t.dclass = fp32 ? 1 : 0; // 1: FP32 hi + bfloat16 lo fragments
            for (int j = 0; j < K; ++j) t.p[j] = bq[j];
            size_t off = pool.size();
            pool.resize(off + fr.size() + 2);
            // fragments start on a 16-byte boundary inside the pool
            if (off & 1) ++off;
            std::memcpy(pool.data() + off, fr.data(), fr.size() * sizeof(double));
            t.moff = off;
            out.push_back(t);
            osrc.push_back(-1);
        }
        blk.clear();
        bbits = 0;
        bdense = 0;
    };
    for (size_t i = 0; i < P.ops.size(); ++i) {
        uint32_t bits = 0;
        const bool ok = op_local_bits(P.ops[i], &bits);
        if (ok && __builtin_popcount(bbits | bits) <= K) {
            blk.push_back(i);
            bbits |= bits;
            bdense += P.ops[i].kind != TK_DIAG;
            continue;
        }
        emit();
        if (ok) {
            blk.push_back(i);
            bbits = bits;
            bdense = P.ops[i].kind != TK_DIAG;
        } else {
            out.push_back(P.ops[i]);
            osrc.push_back(P.src[i]);
        }
    }
    emit();
    P.ops.swap(out);
    P.src.swap(osrc);
}

// ------------------------------------------------------- register segments
//
// Inside a pass, ops are grouped into segments whose dense targets lie on at
// most r tile positions; the kernel then moves each thread's 2^r amplitudes
// between LDS and registers once per segment instead of once per op.  Ops
// are reordered within the pass by the commutation rule the pass scheduler
// uses (on tile-local positions); a diagonal op joins any segment.  k >= 3
// dense ops and fused blocks run on their own, in LDS.

// A diagonal op inside a segment is rewritten for the register kernel:
// local controls become extra targets (factor 1 where a control fails), and
// the targets are ordered register positions first (by register rank), then
// thread positions, then positions outside the tile.  dclass then holds the
// number of register targets kr (SD_GATHER when the fast form does not
// apply) and dbit the number of thread targets kt; the kernel reads the
// same from 32-bit fields: dj = kr | kt << 4 (SD_GATHER << 8 for the
// gather form), rsv = register ranks (target 0 | target 1 << 8), and p[j] =
// the tile position of a local target, the global position of one outside.

// Opcode of a segment member (rsv >> 16): one switch in the kernel picks the
// code with the member's register bits fixed at compile time.
static int seg_pair_index(int a, int b) // a < b < 4
{
    static const int idx[4][4] = {{-1, 0, 1, 3}, {-1, -1, 2, 4}, {-1, -1, -1, 5}, {-1, -1, -1, -1}};
    return idx[a][b];
}

// Diagonal member: SO_DG (gather), SO_D0 (no register target: one factor per
// thread), SO_D1 + rank, SO_D2 + pair (every register combination), or, when
// a single register combination ri has a factor other than 1 for every
// thread and outside bit, SO_D1X + 2 rank + ri / SO_D2X + 4 pair + ri (only
// those registers are multiplied).
static int seg_diag_opcode(const TileOp& t, const std::vector<double>& pool)
{
    if ((t.dj >> 8) == SD_GATHER) return SO_DG;
    const int kr = t.dj & 15;
    if (kr == 0) return SO_D0;
    const int nri = 1 << kr, D = 1 << t.k;
    const double* T = pool.data() + t.moff;
    uint32_t notone = 0;
    for (int i = 0; i < D; ++i)
        if (T[2 * i] != 1.0 || T[2 * i + 1] != 0.0) notone |= 1u << (i & (nri - 1));
    const int r0 = t.rsv & 255, r1 = (t.rsv >> 8) & 255;
    if (__builtin_popcount(notone) == 1) {
        const int ri = __builtin_ctz(notone);
        return kr == 1 ? SO_D1X + 2 * r0 + ri : SO_D2X + 4 * seg_pair_index(r0, r1) + ri;
    }
    return kr == 1 ? SO_D1 + r0 : SO_D2 + seg_pair_index(r0, r1);
}

static void seg_diag_form(TileOp& t, std::vector<double>& pool, uint32_t R, const int* rank)
{
    int reg[6], thr[6], glo[6], nr = 0, nt = 0, ng = 0;
    for (int j = 0; j < t.k; ++j) {
        const int q = t.lp[j];
        if (q < 0) glo[ng++] = j;
        else if ((R >> q) & 1) reg[nr++] = j;
        else thr[nt++] = j;
    }
    int creg[32], cthr[32], ncr = 0, nct = 0;
    for (uint32_t b = (uint32_t)t.lcm; b; b &= b - 1) {
        const int q = __builtin_ctz(b);
        if ((R >> q) & 1) creg[ncr++] = q;
        else cthr[nct++] = q;
    }
    const int kn = t.k + ncr + nct;
    if (kn > 6 || nr + ncr > 2 || nt + nct > 2) {
        t.dclass = SD_GATHER;
        t.dj = SD_GATHER << 8;
        return;
    }
    // new target list: (kind, old index or control position)
    struct Tg {
        int local; // tile position or -1
        int gpos;  // global position
        int oldj;  // index bit in the old table, or -1 for a control
        int cval;  // control value (controls only)
        int rk;    // register rank (register targets only)
    };
    Tg nl[6];
    int c = 0;
    auto add_reg_target = [&](int local, int gpos, int oldj, int cval) {
        nl[c++] = {local, gpos, oldj, cval, rank[local]};
    };
    for (int i = 0; i < nr; ++i) add_reg_target(t.lp[reg[i]], t.p[reg[i]], reg[i], 0);
    for (int i = 0; i < ncr; ++i) add_reg_target(creg[i], -1, -1, (int)((t.lcv >> creg[i]) & 1));
    if (c == 2 && nl[0].rk > nl[1].rk) std::swap(nl[0], nl[1]);
    for (int i = 0; i < nt; ++i) nl[c++] = {t.lp[thr[i]], t.p[thr[i]], thr[i], 0, -1};
    for (int i = 0; i < nct; ++i) nl[c++] = {cthr[i], -1, -1, (int)((t.lcv >> cthr[i]) & 1), -1};
    for (int i = 0; i < ng; ++i) nl[c++] = {-1, t.p[glo[i]], glo[i], 0, -1};
    const int D = 1 << kn;
    const size_t off = pool.size();
    pool.resize(off + 2 * (size_t)D);
    const double* U = pool.data() + t.moff;
    double* W = pool.data() + off;
    for (int ni = 0; ni < D; ++ni) {
        int oi = 0;
        bool on = true;
        for (int j = 0; j < kn; ++j) {
            const int b = (ni >> j) & 1;
            if (nl[j].oldj >= 0) oi |= b << nl[j].oldj;
            else if (b != nl[j].cval) on = false;
        }
        W[2 * ni] = on ? U[2 * oi] : 1.0;
        W[2 * ni + 1] = on ? U[2 * oi + 1] : 0.0;
    }
    t.moff = off;
    t.k = kn;
    for (int j = 0; j < kn; ++j) {
        t.lp[j] = (int8_t)nl[j].local;
        t.p[j] = nl[j].local >= 0 ? nl[j].local : nl[j].gpos; // tile position, or global outside the tile
    }
    t.lcm = t.lcv = 0;
    t.dclass = (int8_t)(nr + ncr);
    t.dbit = (int8_t)(nt + nct);
    t.dj = (nr + ncr) | ((nt + nct) << 4);
    t.rsv = (nr + ncr > 0 ? nl[0].rk : 0) | (nr + ncr > 1 ? nl[1].rk << 8 : 0);
}

static void segment_pass(PlanPass& P, std::vector<double>& pool, int r)
{
    const size_t N = P.ops.size();
    std::vector<uint32_t> nd(N), dq(N);
    std::vector<uint8_t> cap(N); // 0: dense in registers, 1: diagonal, 2: on its own
    for (size_t i = 0; i < N; ++i) {
        const TileOp& t = P.ops[i];
        uint32_t tm = 0;
        if (t.kind == TK_DIAG) {
            for (int j = 0; j < t.k; ++j)
                if (t.lp[j] >= 0) tm |= 1u << t.lp[j];
            nd[i] = 0;
            dq[i] = tm | (uint32_t)t.lcm;
            cap[i] = 1;
        } else {
            for (int j = 0; j < t.k; ++j) tm |= 1u << t.p[j];
            nd[i] = tm;
            dq[i] = (uint32_t)t.lcm;
            cap[i] = (t.kind == TK_DENSE1 || t.kind == TK_DENSE2) && t.k <= r ? 0 : 2;
        }
    }
    std::vector<std::pair<int, int>> edges;
    {
        int last_nd[32];
        std::vector<int> since[32];
        for (int q = 0; q < 32; ++q) last_nd[q] = -1;
        for (size_t g = 0; g < N; ++g) {
            for (uint32_t b = nd[g] | dq[g]; b; b &= b - 1) {
                const int q = __builtin_ctz(b);
                if (last_nd[q] >= 0) edges.push_back({last_nd[q], (int)g});
                if ((nd[g] >> q) & 1)
                    for (int h : since[q]) edges.push_back({h, (int)g});
            }
            for (uint32_t b = nd[g]; b; b &= b - 1) {
                const int q = __builtin_ctz(b);
                last_nd[q] = (int)g;
                since[q].clear();
            }
            for (uint32_t b = dq[g]; b; b &= b - 1) since[__builtin_ctz(b)].push_back((int)g);
        }
    }
    std::vector<int> eoff(N + 1, 0), esucc(edges.size()), indeg(N, 0);
    for (auto& e : edges) eoff[e.first + 1] += 1;
    for (size_t g = 0; g < N; ++g) eoff[g + 1] += eoff[g];
    {
        std::vector<int> fill(eoff.begin(), eoff.end() - 1);
        for (auto& e : edges) {
            esucc[fill[e.first]++] = e.second;
            indeg[e.second] += 1;
        }
    }
    std::set<int> ready;
    for (size_t g = 0; g < N; ++g)
        if (indeg[g] == 0) ready.insert((int)g);
    std::vector<TileOp> out;
    std::vector<int64_t> osrc, ord;
    auto unlock = [&](int g) {
        for (int e = eoff[g]; e < eoff[g + 1]; ++e)
            if (--indeg[esucc[e]] == 0) ready.insert(esucc[e]);
    };
    size_t done = 0;
    std::vector<int> mem;
    while (done < N) {
        uint32_t R = 0;
        mem.clear();
        for (auto it = ready.begin(); it != ready.end();) {
            const int g = *it;
            bool ok = cap[g] == 1;
            if (cap[g] == 0 && __builtin_popcount(R | nd[g]) <= r) {
                R |= nd[g];
                ok = true;
            }
            if (!ok) {
                ++it;
                continue;
            }
            mem.push_back(g);
            unlock(g);
            it = ready.erase(it);
            ++done;
        }
        if (mem.empty()) { // the first ready op runs on its own
            const int g = *ready.begin();
            ready.erase(ready.begin());
            unlock(g);
            ++done;
            out.push_back(P.ops[g]);
            osrc.push_back(P.src[g]);
            ord.push_back(P.src[g]);
            continue;
        }
        {
            // pad with the positions the segment's diagonal ops use most (a
            // diagonal op whose bits are register bits touches only the
            // registers it changes), then with high positions
            int freq[32] = {0};
            for (int g : mem)
                if (cap[g] == 1)
                    for (uint32_t b = dq[g]; b; b &= b - 1) freq[__builtin_ctz(b)] += 1;
            while (__builtin_popcount(R) < r) {
                int best = -1;
                for (int q = P.m - 1; q >= 0; --q)
                    if (!((R >> q) & 1) && (best < 0 || freq[q] > freq[best])) best = q;
                R |= 1u << best;
            }
        }
        TileOp h;
        std::memset(&h, 0, sizeof h);
        h.kind = TK_SEG;
        h.k = r;
        int rank[32], nr = 0;
        for (int q = 0; q < 32; ++q)
            if ((R >> q) & 1) {
                rank[q] = nr;
                h.p[nr++] = q;
            }
        const size_t hpos = out.size();
        out.push_back(h);
        osrc.push_back(-1);

        auto emit_member = [&](int g) {
            TileOp t = P.ops[g];
            ord.push_back(P.src[g]);
            if (t.kind == TK_DIAG) {
                seg_diag_form(t, pool, R, rank);
                t.rsv |= seg_diag_opcode(t, pool) << 16;
                out.push_back(t);
                osrc.push_back(P.src[g]);
                return;
            }
            const uint32_t lc = (uint32_t)t.lcm;
            t.dj = ((lc & R) ? 1 : 0) | ((lc & ~R) ? 2 : 0); // controls at register / thread positions
            if (t.kind == TK_DENSE1) {
                t.lp[0] = (int8_t)rank[t.p[0]];
                t.rsv = rank[t.p[0]];
            } else if (t.kind == TK_DENSE2) {
                int a = rank[t.p[0]], b = rank[t.p[1]];
                if (a > b) { // make target 0 the lower register bit: swap the matrix index bits
                    const size_t off = pool.size();
                    pool.resize(off + 32);
                    const double* U = pool.data() + t.moff;
                    double* W = pool.data() + off;
                    auto sw = [](int x) { return ((x & 1) << 1) | ((x >> 1) & 1); };
                    for (int rr = 0; rr < 4; ++rr)
                        for (int cc = 0; cc < 4; ++cc) {
                            W[2 * (rr * 4 + cc)] = U[2 * (sw(rr) * 4 + sw(cc))];
                            W[2 * (rr * 4 + cc) + 1] = U[2 * (sw(rr) * 4 + sw(cc)) + 1];
                        }
                    t.moff = off;
                    std::swap(t.p[0], t.p[1]);
                    std::swap(a, b);
                }
                t.lp[0] = (int8_t)a;
                t.lp[1] = (int8_t)b;
                t.rsv = a | (b << 8);
            }
            const bool ctl = t.dj != 0;
            int opc;
            if (t.kind == TK_DENSE1) opc = SO_1Q + (t.rsv & 255) + (ctl ? 4 : 0);
            else opc = SO_2Q + seg_pair_index(t.rsv & 255, (t.rsv >> 8) & 255) + (ctl ? 6 : 0);
            t.rsv |= opc << 16;
            out.push_back(t);
            osrc.push_back(P.src[g]);
        };

        // Runs of register-only ops (dense ops and diagonal ops whose qubits
        // and controls are all register positions, no outside control) are
        // multiplied into one 2^r x 2^r block when that is cheaper than the
        // ops one by one.  An op that cannot join moves after later run ops
        // it commutes with; otherwise it closes the run.
        auto absorbable = [&](int g) {
            const TileOp& t = P.ops[g];
            if (t.gcm != 0 || ((uint32_t)t.lcm & ~R) != 0) return false;
            if (t.kind == TK_DENSE1 || t.kind == TK_DENSE2) return true;
            if (t.kind != TK_DIAG) return false;
            for (int j = 0; j < t.k; ++j)
                if (t.lp[j] < 0 || !((R >> t.lp[j]) & 1)) return false;
            return true;
        };
        auto commute = [&](int x, int y) {
            return (nd[x] & (nd[y] | dq[y])) == 0 && (nd[y] & (nd[x] | dq[x])) == 0;
        };
        // Consecutive diagonal ops (they commute) as one factor table: index
        // bits = the register bits the product depends on (rank mask rdep,
        // ascending, compressed), then the thread positions they use, then
        // the positions outside the tile (targets or controls); at most
        // kGroupBits bits, counting the register ranks the ops touch.  Each
        // thread reads its 2^|rdep| factors as one contiguous slice (uniform
        // loads when no thread position is used); dj = kt | kg << 8 | rdep << 16.
        constexpr int kGroupBits = 12; // 64 KiB tables; a tile reads 2^(|rdep| + kt) entries
        auto diag_masks = [&](const int* gs, size_t cnt, uint32_t& rrm, uint32_t& tpm, uint64_t& gpm) {
            rrm = 0;
            tpm = 0;
            gpm = 0;
            for (size_t i = 0; i < cnt; ++i) {
                const TileOp& t = P.ops[gs[i]];
                for (int j = 0; j < t.k; ++j) {
                    if (t.lp[j] >= 0) {
                        if (!((R >> t.lp[j]) & 1)) tpm |= 1u << t.lp[j];
                        else rrm |= 1u << rank[t.lp[j]];
                    } else {
                        gpm |= 1ull << t.p[j];
                    }
                }
                for (uint32_t m = (uint32_t)t.lcm & R; m; m &= m - 1) rrm |= 1u << rank[__builtin_ctz(m)];
                tpm |= (uint32_t)t.lcm & ~R;
                gpm |= t.gcm;
            }
        };
        auto diag_group = [&](const int* gs, size_t cnt) -> bool {
            uint32_t rrm, tpm;
            uint64_t gpm;
            diag_masks(gs, cnt, rrm, tpm, gpm);
            const int kr0 = __builtin_popcount(rrm), kt = __builtin_popcount(tpm), kg = __builtin_popcountll(gpm);
            if (kr0 + kt + kg > kGroupBits) return false;
            int tpos[32], gpos[64];
            for (int i = 0, q = 0; q < 32; ++q)
                if ((tpm >> q) & 1) tpos[i++] = q;
            for (int i = 0, q = 0; q < 64; ++q)
                if ((gpm >> q) & 1) gpos[i++] = q;
            const int K = kr0 + kt + kg, D = 1 << K;
            size_t off = pool.size();
            if (off & 1) pool.push_back(0.0), ++off; // 16-byte aligned factors
            pool.resize(off + 2 * (size_t)D);
            // each op's targets and controls as bit positions of the index x
            struct Xop {
                int tb[6];
                int k;
                uint32_t cm, cv;
            };
            std::vector<Xop> xo(cnt);
            int xbit_local[32], xbit_glob[64];
            for (int q = 0; q < 32; ++q) xbit_local[q] = -1;
            for (int q = 0; q < 64; ++q) xbit_glob[q] = -1;
            for (int b = 0, i = 0; b < r; ++b)
                if ((rrm >> b) & 1) xbit_local[h.p[b]] = i++;
            for (int b = 0; b < kt; ++b) xbit_local[tpos[b]] = kr0 + b;
            for (int b = 0; b < kg; ++b) xbit_glob[gpos[b]] = kr0 + kt + b;
            for (size_t i = 0; i < cnt; ++i) {
                const TileOp& t = P.ops[gs[i]];
                Xop& x = xo[i];
                x.k = t.k;
                x.cm = x.cv = 0;
                for (int j = 0; j < t.k; ++j) x.tb[j] = t.lp[j] >= 0 ? xbit_local[t.lp[j]] : xbit_glob[t.p[j]];
                for (int q = 0; q < 32; ++q)
                    if (((uint32_t)t.lcm >> q) & 1) {
                        x.cm |= 1u << xbit_local[q];
                        if (((uint32_t)t.lcv >> q) & 1) x.cv |= 1u << xbit_local[q];
                    }
                for (int q = 0; q < 64; ++q)
                    if ((t.gcm >> q) & 1) {
                        x.cm |= 1u << xbit_glob[q];
                        if ((t.gcv >> q) & 1) x.cv |= 1u << xbit_glob[q];
                    }
            }
            // The product over the ops, in their order, entry by entry; an op
            // visits only the entries where its factor is not exactly 1 (its
            // controls pass and its targets spell a factor other than 1):
            // a controlled phase touches a quarter of the table.
            double* F = pool.data() + off;
            for (int x = 0; x < D; ++x) {
                F[2 * x] = 1.0;
                F[2 * x + 1] = 0.0;
            }
            for (size_t i = 0; i < cnt; ++i) {
                const Xop& o = xo[i];
                for (int v = 0; v < (1 << o.k); ++v) {
                    const double* T = pool.data() + P.ops[gs[i]].moff + 2 * v;
                    if (T[0] == 1.0 && T[1] == 0.0) continue;
                    uint32_t fix = o.cm, val = o.cv;
                    for (int j = 0; j < o.k; ++j) {
                        fix |= 1u << o.tb[j];
                        if ((v >> j) & 1) val |= 1u << o.tb[j];
                    }
                    const uint32_t fr_bits = (uint32_t)(D - 1) & ~fix; // free index bits
                    uint32_t y = 0;
                    do {
                        double* e = F + 2 * (size_t)(y | val);
                        const double nr = e[0] * T[0] - e[1] * T[1], ni = e[0] * T[1] + e[1] * T[0];
                        e[0] = nr;
                        e[1] = ni;
                        y = (y - fr_bits) & fr_bits;
                    } while (y != 0);
                }
            }
            // Register bits the factors do not depend on (bitwise equal
            // entries; a CZ pair can cancel) are dropped from the index as well.
            uint32_t dep = 0; // over the kr0 compressed register bits
            for (int b = 0; b < kr0; ++b)
                for (int x = 0; x < D; ++x)
                    if (!((x >> b) & 1) &&
                        (std::memcmp(&pool[off + 2 * (size_t)x], &pool[off + 2 * (size_t)(x | 1 << b)],
                                     2 * sizeof(double)) != 0)) {
                        dep |= 1u << b;
                        break;
                    }
            const int kr = __builtin_popcount(dep);
            if (kr < kr0) {
                const int Kc = kr + kt + kg;
                for (int y = 0; y < (1 << Kc); ++y) { // y <= x: compacting in place keeps unread entries
                    int x = (y >> kr) << kr0;
                    for (int b = 0, i = 0; b < kr0; ++b)
                        if ((dep >> b) & 1) x |= ((y >> i++) & 1) << b;
                    pool[off + 2 * (size_t)y] = pool[off + 2 * (size_t)x];
                    pool[off + 2 * (size_t)y + 1] = pool[off + 2 * (size_t)x + 1];
                }
                pool.resize(off + 2 * ((size_t)1 << Kc));
            }
            uint32_t rdep = 0; // rank mask
            for (int b = 0, i = 0; b < r; ++b)
                if ((rrm >> b) & 1)
                    if ((dep >> i++) & 1) rdep |= 1u << b;
            TileOp t;
            std::memset(&t, 0, sizeof t);
            t.kind = TK_DIAG;
            t.k = kr + kt + kg;
            t.lcm = tpm; // thread positions of the index
            t.lcv = gpm; // positions outside the tile
            t.moff = off;
            t.dj = kt | (kg << 8) | (int32_t)(rdep << 16);
            t.rsv = SO_DGROUP << 16;
            out.push_back(t);
            osrc.push_back(-1);
            for (size_t i = 0; i < cnt; ++i) ord.push_back(P.src[gs[i]]);
            return true;
        };
        auto op_cost = [&](int g) {
            const TileOp& t = P.ops[g];
            return t.kind == TK_DENSE1 ? 20.0 : (t.kind == TK_DENSE2 ? 40.0 : 8.0);
        };
        const double block_cost = 4.0 * (1 << r) + 10.0;
        std::vector<int> run, pend;
        auto flush = [&]() {
            double c = 0;
            for (int g : run) c += op_cost(g);
            if (run.size() >= 2 && c > block_cost) {
                const int D = 1 << r;
                std::vector<cd> G((size_t)D * D, cd(0, 0));
                for (int i = 0; i < D; ++i) G[(size_t)i * D + i] = 1.0;
                for (int g : run) {
                    embed_op(P.ops[g], pool, h.p, r, G);
                    ord.push_back(P.src[g]);
                }
                TileOp t;
                std::memset(&t, 0, sizeof t);
                t.kind = TK_DENSEK;
                t.k = r;
                for (int j = 0; j < r; ++j) t.p[j] = h.p[j];
                t.moff = pool.size();
                for (const cd& z : G) {
                    pool.push_back(z.real());
                    pool.push_back(z.imag());
                }
                t.rsv = SO_BLOCK << 16;
                out.push_back(t);
                osrc.push_back(-1);
            } else {
                for (int g : run) emit_member(g);
            }
            for (size_t i = 0; i < pend.size();) {
                // the longest run of diagonal ops from i whose factor table
                // fits (at most kGroupBits index bits)
                size_t j = i;
                uint32_t rrm = 0, tpm = 0;
                uint64_t gpm = 0;
                while (j < pend.size() && P.ops[pend[j]].kind == TK_DIAG) {
                    uint32_t r2, t2;
                    uint64_t g2;
                    diag_masks(pend.data() + j, 1, r2, t2, g2);
                    if (__builtin_popcount(rrm | r2) + __builtin_popcount(tpm | t2) + __builtin_popcountll(gpm | g2) >
                        kGroupBits)
                        break;
                    rrm |= r2;
                    tpm |= t2;
                    gpm |= g2;
                    ++j;
                }
                if (j - i >= 2) {
                    diag_group(pend.data() + i, j - i);
                    i = j;
                    continue;
                }
                emit_member(pend[i]);
                ++i;
            }
            run.clear();
            pend.clear();
        };
        for (int g : mem) {
            if (!absorbable(g)) {
                pend.push_back(g);
                continue;
            }
            bool ok = true;
            for (int q : pend) ok = ok && commute(q, g);
            if (!ok) flush();
            run.push_back(g);
        }
        flush();
        out[hpos].dj = (int32_t)(out.size() - hpos - 1);
    }
    P.ops.swap(out);
    P.src.swap(osrc);
    P.order.swap(ord);
}

static bool is_diagonal(const double* U, int nt)
{
    const int d = 1 << nt;
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c)
            if (r != c && (U[2 * (r * d + c)] != 0.0 || U[2 * (r * d + c) + 1] != 0.0)) return false;
    return true;
}

void plan_circuit(int n, const qs_op* ops, int64_t n_ops, const double* mats, const PlanOpts& po,
                  std::vector<PlanPass>& passes, std::vector<double>& pool, bool encode)
{
    const int m = std::min(std::max(po.m, 1), n);
    const int Lf = std::min(std::max(po.L, 0), m);
    const uint64_t lowQ = (Lf >= 64) ? ~0ull : ((1ull << Lf) - 1);
    passes.clear();
    pool.clear();

    struct Item {
        const qs_op* op;
        bool diag;
    };
    std::vector<Item> items;
    uint64_t qmask = 0;

    auto close = [&]() {
        if (items.empty()) return;
        for (int q = 0; __builtin_popcountll(qmask) < m && q < n; ++q) qmask |= 1ull << q;
        PlanPass P;
        P.m = m;
        int pos[64];
        for (int q = 0; q < n; ++q)
            if ((qmask >> q) & 1) {
                pos[q] = (int)P.Q.size();
                P.Q.push_back(q);
            }
        int L = 0;
        while (L < m && ((qmask >> L) & 1)) ++L;
        P.L = L;
        auto to_local = [&](uint64_t bits) {
            uint64_t r = 0;
            for (int q = 0; q < n; ++q)
                if ((bits >> q) & 1) r |= 1ull << pos[q];
            return r;
        };
        for (const Item& it : items) {
            const qs_op& o = *it.op;
            const double* U = mats + o.moff;
            const int d = 1 << o.nt;
            TileOp t;
            std::memset(&t, 0, sizeof t);
            t.k = o.nt;
            const uint64_t cin = o.cmask & qmask;
            t.lcm = to_local(cin);
            t.lcv = to_local(o.cvals & cin);
            t.gcm = o.cmask & ~qmask;
            t.gcv = o.cvals & ~qmask;
            t.moff = pool.size();
            if (it.diag) {
                t.kind = TK_DIAG;
                int nlt = 0;
                for (int j = 0; j < 6; ++j) t.lp[j] = -1;
                for (int j = 0; j < o.nt; ++j) {
                    t.p[j] = o.t[j];
                    if ((qmask >> o.t[j]) & 1) {
                        t.lp[j] = (int8_t)pos[o.t[j]];
                        ++nlt;
                        t.dj = j;
                        t.dbit = (int8_t)pos[o.t[j]];
                    }
                }
                const int nlc = __builtin_popcountll(t.lcm);
                if (nlt == 0 && nlc == 0) {
                    t.dclass = DG_UNIFORM;
                } else if (nlt == 1 && nlc == 0) {
                    t.dclass = DG_LTARGET;
                } else if (nlt == 0 && nlc == 1) {
                    t.dclass = DG_LCONTROL;
                    t.dbit = (int8_t)__builtin_ctzll(t.lcm);
                } else if (nlt == 1 && nlc == 1) {
                    t.dclass = DG_CT;
                } else {
                    t.dclass = DG_GENERAL;
                }
                for (int r = 0; r < d; ++r) {
                    pool.push_back(U[2 * (r * d + r)]);
                    pool.push_back(U[2 * (r * d + r) + 1]);
                }
            } else {
                t.kind = o.nt == 1 ? TK_DENSE1 : (o.nt == 2 ? TK_DENSE2 : TK_DENSEK);
                for (int j = 0; j < o.nt; ++j) t.p[j] = pos[o.t[j]];
                pool.insert(pool.end(), U, U + 2 * d * d);
            }
            P.ops.push_back(t);
            P.src.push_back((int64_t)(it.op - ops));
            P.order.push_back((int64_t)(it.op - ops));
            P.gates += 1;
            P.updates += 1ull << (n - __builtin_popcountll(o.cmask));
        }
        if (encode && (po.fuse_k == 4 || po.fuse_k == 5) && m >= po.fuse_k + 4)
            fuse_pass(P, pool, po.fuse_k, po.fuse_min, po.fuse_fp32 && po.dt == QS_C64);
        const int r = po.segments ? seg_reg_qubits(po.dt, m) : 0;
        if (encode && r > 0) segment_pass(P, pool, r);
        passes.push_back(std::move(P));
        items.clear();
        qmask = 0;
    };

    // Dependencies.  A gate acts non-diagonally on its dense targets and
    // diagonally on its controls (and on a diagonal gate's targets); two
    // gates commute when neither acts non-diagonally on a qubit the other
    // touches.  Gate g waits for the last non-diagonal gate on each of its
    // qubits and, on its non-diagonal qubits, for the diagonal gates since.
    std::vector<uint8_t> isdiag((size_t)n_ops);
    std::vector<uint64_t> ndq((size_t)n_ops);
    std::vector<int> indeg((size_t)n_ops, 0);
    std::vector<std::pair<int, int>> edges;
    {
        int last_nd[64];
        std::vector<int> since[64];
        for (int q = 0; q < 64; ++q) last_nd[q] = -1;
        for (int64_t g = 0; g < n_ops; ++g) {
            const qs_op& o = ops[g];
            const bool diag = is_diagonal(mats + o.moff, o.nt);
            uint64_t tm = 0;
            for (int j = 0; j < o.nt; ++j) tm |= 1ull << o.t[j];
            const uint64_t nd = diag ? 0 : tm, dq = (diag ? tm : 0) | o.cmask;
            isdiag[g] = diag;
            ndq[g] = nd;
            for (uint64_t b = nd | dq; b; b &= b - 1) {
                const int q = __builtin_ctzll(b);
                if (last_nd[q] >= 0) edges.push_back({last_nd[q], (int)g});
                if ((nd >> q) & 1)
                    for (int h : since[q]) edges.push_back({h, (int)g});
            }
            for (uint64_t b = nd; b; b &= b - 1) {
                const int q = __builtin_ctzll(b);
                last_nd[q] = (int)g;
                since[q].clear();
            }
            for (uint64_t b = dq; b; b &= b - 1) since[__builtin_ctzll(b)].push_back((int)g);
        }
    }
    std::vector<int> eoff((size_t)n_ops + 1, 0), esucc(edges.size());
    for (auto& e : edges) eoff[e.first + 1] += 1;
    for (int64_t g = 0; g < n_ops; ++g) eoff[g + 1] += eoff[g];
    {
        std::vector<int> fill(eoff.begin(), eoff.end() - 1);
        for (auto& e : edges) {
            esucc[fill[e.first]++] = e.second;
            indeg[e.second] += 1;
        }
    }

    // Passes.  Each pass starts from the forced low qubits and takes the
    // ready gates in circuit order: a diagonal gate always (its qubits need
    // not be in the tile), a dense gate when its targets fit the tile, which
    // then grows by them.  Gates made ready inside the pass are considered in
    // the same sweep, so one pass runs as deep as its qubits allow (for a
    // nearest-neighbour chain, a staircase over several layers).  A circuit
    // that fits one tile keeps its original order.
    std::set<int> ready;
    for (int64_t g = 0; g < n_ops; ++g)
        if (indeg[g] == 0) ready.insert((int)g);
    const uint64_t nmask = n >= 64 ? ~0ull : ((1ull << n) - 1);
    int64_t done = 0;
    while (done < n_ops) {
        qmask = lowQ & nmask;
        bool dense_in = false;
        for (auto it = ready.begin(); it != ready.end();) {
            const int g = *it;
            bool ok = isdiag[g] != 0;
            if (!ok) {
                const uint64_t need = qmask | ndq[g];
                if (__builtin_popcountll(need) <= m) {
                    qmask = need;
                    ok = true;
                } else if (!dense_in) { // the gate alone: padding fills low qubits
                    qmask = ndq[g];
                    ok = true;
                }
                dense_in |= ok;
            }
            if (!ok) {
                ++it;
                continue;
            }
            items.push_back({&ops[g], isdiag[g] != 0});
            for (int e = eoff[g]; e < eoff[g + 1]; ++e)
                if (--indeg[esucc[e]] == 0) ready.insert(esucc[e]);
            it = ready.erase(it);
            ++done;
        }
        close();
    }
}

static bool is_swap(const qs_op& o, const double* U)
{
    if (o.nt != 2 || o.cmask != 0) return false;
    static const double S[32] = {1, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 0, 0, 0,
                                 0, 0, 1, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 0};
    for (int i = 0; i < 32; ++i)
        if (U[i] != S[i]) return false;
    return true;
}

bool remap_swaps(int n, const qs_op* ops, int64_t n_ops, const double* mats, Remap& r)
{
    bool any = false;
    for (int64_t g = 0; g < n_ops && !any; ++g) any = is_swap(ops[g], mats + ops[g].moff);
    if (!any) return false;
    int perm[64]; // logical qubit -> bit position holding it
    for (int q = 0; q < 64; ++q) perm[q] = q;
    auto map_bits = [&](uint64_t bits) {
        uint64_t out = 0;
        for (; bits; bits &= bits - 1) out |= 1ull << perm[__builtin_ctzll(bits)];
        return out;
    };
    r.ops.clear();
    r.src.clear();
    for (int64_t g = 0; g < n_ops; ++g) {
        const qs_op& o = ops[g];
        if (is_swap(o, mats + o.moff)) {
            std::swap(perm[o.t[0]], perm[o.t[1]]);
            continue;
        }
        qs_op m = o;
        for (int j = 0; j < o.nt; ++j) m.t[j] = perm[o.t[j]];
        m.cmask = map_bits(o.cmask);
        m.cvals = map_bits(o.cvals);
        r.ops.push_back(m);
        r.src.push_back(g);
    }
    // restoring permutation rho: position perm[q] -> q, as tau[1] o tau[0].
    // For a cycle c_0 -> c_1 -> ... -> c_{k-1} of rho, tau0(c_i) = c_{-i} and
    // tau1(c_i) = c_{1-i} (indices mod k) are involutions with
    // tau1(tau0(c_i)) = c_{i+1}.
    int rho[64], t0[64], t1[64];
    for (int q = 0; q < n; ++q) rho[perm[q]] = q;
    for (int p = 0; p < 64; ++p) t0[p] = t1[p] = p;
    bool seen[64] = {false};
    for (int p0 = 0; p0 < n; ++p0) {
        if (seen[p0]) continue;
        int c[64], k = 0;
        for (int p = p0; !seen[p]; p = rho[p]) {
            seen[p] = true;
            c[k++] = p;
        }
        for (int i = 0; i < k; ++i) {
            t0[c[i]] = c[(k - i) % k];
            t1[c[i]] = c[(k + 1 - i) % k];
        }
    }
    r.nrestore = 0;
    for (const int* t : {t0, t1}) {
        bool id = true;
        for (int p = 0; p < n; ++p) id &= t[p] == p;
        if (!id) std::memcpy(r.tau[r.nrestore++], t, sizeof t0);
    }
    return true;
}

void plan_circuit_remap(int n, const qs_op* ops, int64_t n_ops, const double* mats, const PlanOpts& po, int remap,
                        std::vector<PlanPass>& passes, std::vector<double>& pool, Remap& r)
{
    r.nrestore = 0;
    // QS_REMAP_ALWAYS=1 relabels whenever there is a SWAP gate (for tests)
    const bool always = env_int("QS_REMAP_ALWAYS", 0) != 0;
    Remap rr;
    if (remap != 0 || !remap_swaps(n, ops, n_ops, mats, rr)) {
        plan_circuit(n, ops, n_ops, mats, po, passes, pool);
        return;
    }
    // Compare the pass counts of both plans before encoding either: the
    // encoding (fused blocks, segments, diagonal factor tables) is most of
    // the planning time and only the chosen plan needs it.
    if (!always) {
        std::vector<PlanPass> p1, p2;
        std::vector<double> pool1, pool2;
        plan_circuit(n, ops, n_ops, mats, po, p1, pool1, false);
        if (!rr.ops.empty()) plan_circuit(n, rr.ops.data(), (int64_t)rr.ops.size(), mats, po, p2, pool2, false);
        if (p1.size() <= 1 || (double)p2.size() + 0.5 * rr.nrestore >= (double)p1.size()) {
            plan_circuit(n, ops, n_ops, mats, po, passes, pool);
            return;
        }
    }
    passes.clear();
    pool.clear();
    if (!rr.ops.empty()) plan_circuit(n, rr.ops.data(), (int64_t)rr.ops.size(), mats, po, passes, pool);
    for (PlanPass& P : passes) {
        for (int64_t& g : P.src)
            if (g >= 0) g = rr.src[(size_t)g];
        for (int64_t& g : P.order)
            if (g >= 0) g = rr.src[(size_t)g];
    }
    r = std::move(rr);
}

static int default_tile_qubits(int dt)
{
    const int e = env_int("QS_TILE_QUBITS", 0);
    if (e > 0) return e;
    return 11; // measured best for both types on the random chain and QFT circuits
}

// Qubits 0..L-1 are forced into every tile, so tiles load and store runs of
// 2^L amplitudes.  Measured on the 32-qubit chain circuit and QFT with
// 11-qubit tiles: L = 4 for complex128 (256-byte runs; 3 % faster than 5) and
// L = 5 for complex64 (256-byte runs; 8 % faster than 6) -- fewer forced
// qubits leave more room for gate qubits, so passes are fewer.
static int default_low_qubits(int dt)
{
    const int e = env_int("QS_TILE_LOW", -1);
    if (e >= 0) return e;
    return dt == QS_C128 ? 4 : 5;
}

static qs_status plan_opts(int dt, const qs_op* ops, int64_t n_ops, const qs_run_opts& o, PlanOpts& po)
{
    return plan_opts_for(dt, ops, n_ops, o.fuse_k, o.tile_qubits, po);
}

qs_status plan_opts_for(int dt, const qs_op* ops, int64_t n_ops, int fuse_k, int tile_qubits, PlanOpts& po)
{
    po.m = tile_qubits > 0 ? tile_qubits : default_tile_qubits(dt);
    if (po.m > 13) return set_err(QS_ERR_ARG, "tile_qubits=%d > 13", po.m);
    int maxk = 1;
    for (int64_t g = 0; g < n_ops; ++g) maxk = std::max(maxk, (int)ops[g].nt);
    po.m = std::max(po.m, maxk);
    po.L = default_low_qubits(dt);
    po.fuse_k = fuse_k > 0 ? fuse_k : env_int("QS_FUSE_K", 0);
    po.fuse_min = env_int("QS_FUSE_MIN", 3);
    po.dt = dt;
    po.segments = env_int("QS_REG_SEGMENTS", 1) != 0;
    po.fuse_fp32 = env_int("QS_FUSE_FP32", 0) != 0;
    if (po.fuse_k != 0 && po.fuse_k != 4 && po.fuse_k != 5)
        return set_err(QS_ERR_ARG, "fuse_k=%d: fused blocks have 4 or 5 qubits", po.fuse_k);
    return QS_OK;
}

qs_status run_planned(qs_state s, const qs_op* ops, int64_t n_ops, const double* mats, int64_t n_mats,
                      const qs_run_opts& o)
{
    (void)n_mats;
    if (n_ops == 0) return QS_OK;
    PlanOpts po;
    qs_status pst = plan_opts(s->dt, ops, n_ops, o, po);
    if (pst != QS_OK) return pst;
    if (o.remap != 0 && o.remap != 1) return set_err(QS_ERR_ARG, "remap=%d is not 0 or 1", o.remap);
    std::vector<PlanPass> passes;
    std::vector<double> pool;
    Remap rm;
    plan_circuit_remap(s->n, ops, n_ops, mats, po, o.remap, passes, pool, rm);

    // One staging copy: every pass's op table, then the FP64 matrix pool.
    size_t nops_total = 0;
    for (auto& p : passes) nops_total += p.ops.size();
    const size_t ops_bytes = ((nops_total * sizeof(TileOp)) + 255) & ~size_t(255);
    std::vector<char> host(ops_bytes + pool.size() * sizeof(double));
    size_t off = 0;
    for (auto& p : passes) {
        std::memcpy(host.data() + off, p.ops.data(), p.ops.size() * sizeof(TileOp));
        off += p.ops.size() * sizeof(TileOp);
    }
    std::memcpy(host.data() + ops_bytes, pool.data(), pool.size() * sizeof(double));
    const void* dev = nullptr;
    qs_status st = stage_bytes(s, host.data(), host.size(), &dev);
    if (st != QS_OK) return st;
    const TileOp* dops = (const TileOp*)dev;
    const void* dmats = (const char*)dev + ops_bytes;
    size_t op0 = 0;
    for (auto& p : passes) {
        qs_trace_rec rec;
        std::memset(&rec, 0, sizeof rec);
        rec.n = s->n;
        rec.t0 = p.m;
        rec.t1 = (int)p.ops.size();
        rec.dtype = s->dt;
        rec.bytes = 2ull * amp_bytes(s->dt) * (1ull << s->n);
        rec.updates = p.updates;
        const TileOp* pd = dops + op0;
        st = traced_launch(
            s, rec,
            [&](int* kind) {
                *kind = QS_K_TILE;
                return launch_tile_pass(s->d, s->dt, s->n, p, pd, dmats, o.max_blocks, s->st);
            },
            "tile pass launch");
        if (st != QS_OK) return st;
        op0 += p.ops.size();
    }
    for (int i = 0; i < rm.nrestore; ++i) {
        qs_trace_rec rec;
        std::memset(&rec, 0, sizeof rec);
        rec.n = s->n;
        rec.t0 = rec.t1 = -1;
        rec.dtype = s->dt;
        rec.bytes = 2ull * amp_bytes(s->dt) * involution_moved(s->n, rm.tau[i]);
        const int* tau = rm.tau[i];
        st = traced_launch(
            s, rec,
            [&](int* kind) {
                *kind = QS_K_PERM;
                return launch_bit_involution(s->d, s->dt, s->n, tau, s->st);
            },
            "qubit order restore launch");
        if (st != QS_OK) return st;
    }
    return QS_OK;
}

} // namespace qs

extern "C" qs_status qs_plan_circuit(int n, qs_dtype dt, const qs_op* ops, int64_t n_ops, const double* mats,
                                    int64_t n_mats, const qs_run_opts* opts, int64_t* n_passes,
                                    int64_t* n_ops_out)
{
    using namespace qs;
    if (!n_passes || !n_ops_out) return set_err(QS_ERR_ARG, "null output");
    if (n < 1 || n > QS_MAX_QUBITS) return set_err(QS_ERR_ARG, "n=%d outside [1, %d]", n, QS_MAX_QUBITS);
    if (dt != QS_C64 && dt != QS_C128) return set_err(QS_ERR_ARG, "unknown dtype %d", (int)dt);
    qs_status st = validate_circuit(n, ops, n_ops, mats, n_mats);
    if (st != QS_OK) return st;
    qs_run_opts o;
    std::memset(&o, 0, sizeof o);
    if (opts) o = *opts;
    PlanOpts po;
    if ((st = plan_opts(dt, ops, n_ops, o, po)) != QS_OK) return st;
    if (o.remap != 0 && o.remap != 1) return set_err(QS_ERR_ARG, "remap=%d is not 0 or 1", o.remap);
    std::vector<PlanPass> passes;
    std::vector<double> pool;
    Remap rm;
    if (n_ops > 0) plan_circuit_remap(n, ops, n_ops, mats, po, o.remap, passes, pool, rm);
    int64_t c = 0; // segment headers are bookkeeping, not operations
    for (auto& p : passes)
        for (auto& t : p.ops) c += t.kind != TK_SEG;
    *n_passes = (int64_t)passes.size() + rm.nrestore;
    *n_ops_out = c;
    return QS_OK;
}

extern "C" qs_status qs_plan_order(int n, qs_dtype dt, const qs_op* ops, int64_t n_ops, const double* mats,
                                  int64_t n_mats, const qs_run_opts* opts, int64_t* order, int32_t* pass_of,
                                  uint64_t* tile_mask)
{
    using namespace qs;
    if (n_ops > 0 && (!order || !pass_of)) return set_err(QS_ERR_ARG, "null output");
    if (n < 1 || n > QS_MAX_QUBITS) return set_err(QS_ERR_ARG, "n=%d outside [1, %d]", n, QS_MAX_QUBITS);
    if (dt != QS_C64 && dt != QS_C128) return set_err(QS_ERR_ARG, "unknown dtype %d", (int)dt);
    qs_status st = validate_circuit(n, ops, n_ops, mats, n_mats);
    if (st != QS_OK) return st;
    qs_run_opts o;
    std::memset(&o, 0, sizeof o);
    if (opts) o = *opts;
    PlanOpts po;
    if ((st = plan_opts(dt, ops, n_ops, o, po)) != QS_OK) return st;
    po.fuse_k = 0; // the order of the circuit's own gates
    std::vector<PlanPass> passes;
    std::vector<double> pool;
    if (n_ops > 0) plan_circuit(n, ops, n_ops, mats, po, passes, pool);
    int64_t c = 0;
    for (size_t p = 0; p < passes.size(); ++p) {
        uint64_t qm = 0;
        for (int q : passes[p].Q) qm |= 1ull << q;
        if (tile_mask) tile_mask[p] = qm;
        for (int64_t g : passes[p].order) {
            if (g < 0) continue;
            order[c] = g;
            pass_of[c] = (int32_t)p;
            ++c;
        }
    }
    return QS_OK;
}

extern "C" qs_status qs_plan_export(int n, qs_dtype dt, const qs_op* ops, int64_t n_ops, const double* mats,
                                   int64_t n_mats, const qs_run_opts* opts, int32_t* pass_desc,
                                   int64_t* n_passes, void* ops_out, int64_t* n_tile_ops, double* pool_out,
                                   int64_t* n_pool)
{
    using namespace qs;
    if (!n_passes || !n_tile_ops || !n_pool) return set_err(QS_ERR_ARG, "null size output");
    if (n < 1 || n > QS_MAX_QUBITS) return set_err(QS_ERR_ARG, "n=%d outside [1, %d]", n, QS_MAX_QUBITS);
    if (dt != QS_C64 && dt != QS_C128) return set_err(QS_ERR_ARG, "unknown dtype %d", (int)dt);
    qs_status st = validate_circuit(n, ops, n_ops, mats, n_mats);
    if (st != QS_OK) return st;
    qs_run_opts o;
    std::memset(&o, 0, sizeof o);
    if (opts) o = *opts;
    PlanOpts po;
    if ((st = plan_opts(dt, ops, n_ops, o, po)) != QS_OK) return st;
    if (o.remap != 0 && o.remap != 1) return set_err(QS_ERR_ARG, "remap=%d is not 0 or 1", o.remap);
    std::vector<PlanPass> passes;
    std::vector<double> pool;
    Remap rm;
    if (n_ops > 0) plan_circuit_remap(n, ops, n_ops, mats, po, o.remap, passes, pool, rm);
    int64_t total = 0;
    for (auto& p : passes) total += (int64_t)p.ops.size();
    const bool fill = pass_desc && ops_out && pool_out;
    if (fill && (*n_passes < (int64_t)passes.size() || *n_tile_ops < total || *n_pool < (int64_t)pool.size()))
        return set_err(QS_ERR_ARG, "export buffers too small");
    if (fill) {
        int64_t op0 = 0;
        for (size_t i = 0; i < passes.size(); ++i) {
            int32_t* d = pass_desc + 36 * i;
            const PlanPass& p = passes[i];
            d[0] = p.m;
            d[1] = p.L;
            d[2] = (int32_t)op0;
            d[3] = (int32_t)p.ops.size();
            for (int j = 0; j < 32; ++j) d[4 + j] = j < (int)p.Q.size() ? p.Q[j] : -1;
            std::memcpy((char*)ops_out + op0 * sizeof(TileOp), p.ops.data(), p.ops.size() * sizeof(TileOp));
            op0 += (int64_t)p.ops.size();
        }
        if (!pool.empty()) std::memcpy(pool_out, pool.data(), pool.size() * sizeof(double));
    }
    *n_passes = (int64_t)passes.size();
    *n_tile_ops = total;
    *n_pool = (int64_t)pool.size();
    return QS_OK;
}

extern "C" qs_status qs_plan_restore(int n, qs_dtype dt, const qs_op* ops, int64_t n_ops, const double* mats,
                                    int64_t n_mats, const qs_run_opts* opts, int32_t* tau, int32_t* n_restore)
{
    using namespace qs;
    if (!tau || !n_restore) return set_err(QS_ERR_ARG, "null output");
    if (n < 1 || n > QS_MAX_QUBITS) return set_err(QS_ERR_ARG, "n=%d outside [1, %d]", n, QS_MAX_QUBITS);
    if (dt != QS_C64 && dt != QS_C128) return set_err(QS_ERR_ARG, "unknown dtype %d", (int)dt);
    qs_status st = validate_circuit(n, ops, n_ops, mats, n_mats);
    if (st != QS_OK) return st;
    qs_run_opts o;
    std::memset(&o, 0, sizeof o);
    if (opts) o = *opts;
    PlanOpts po;
    if ((st = plan_opts(dt, ops, n_ops, o, po)) != QS_OK) return st;
    if (o.remap != 0 && o.remap != 1) return set_err(QS_ERR_ARG, "remap=%d is not 0 or 1", o.remap);
    std::vector<PlanPass> passes;
    std::vector<double> pool;
    Remap rm;
    if (n_ops > 0) plan_circuit_remap(n, ops, n_ops, mats, po, o.remap, passes, pool, rm);
    for (int i = 0; i < 2; ++i)
        for (int p = 0; p < 64; ++p) tau[64 * i + p] = (i < rm.nrestore && p < n) ? rm.tau[i][p] : p;
    *n_restore = rm.nrestore;
    return QS_OK;
}
