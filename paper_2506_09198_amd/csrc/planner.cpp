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

// Full 2^K x 2^K matrix (column-major product order: G = op * G) of one op in
// the block whose qubits are the local positions bq[0..K).
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
    int tb[6];
    const bool diag = t.kind == TK_DIAG;
    for (int j = 0; j < t.k; ++j) tb[j] = bidx[diag ? t.lp[j] : t.p[j]];
    const int dk = 1 << t.k;
    const double* U = pool.data() + t.moff;
    std::vector<cd> H((size_t)D * D, cd(0, 0));
    for (int c = 0; c < D; ++c) {
        if (((uint32_t)c & cbm) != cbv) {
            H[(size_t)c * D + c] = 1.0;
            continue;
        }
        int mi = 0, base = c;
        for (int j = 0; j < t.k; ++j) {
            mi |= ((c >> tb[j]) & 1) << j;
            base &= ~(1 << tb[j]);
        }
        if (diag) {
            H[(size_t)c * D + c] = cd(U[2 * mi], U[2 * mi + 1]);
            continue;
        }
        for (int r = 0; r < dk; ++r) {
            int row = base;
            for (int j = 0; j < t.k; ++j)
                if ((r >> j) & 1) row |= 1 << tb[j];
            H[(size_t)row * D + c] = cd(U[2 * (r * dk + mi)], U[2 * (r * dk + mi) + 1]);
        }
    }
    std::vector<cd> out((size_t)D * D, cd(0, 0));
    for (int r = 0; r < D; ++r)
        for (int k2 = 0; k2 < D; ++k2) {
            const cd h = H[(size_t)r * D + k2];
            if (h == cd(0, 0)) continue;
            for (int c = 0; c < D; ++c) out[(size_t)r * D + c] += h * G[(size_t)k2 * D + c];
        }
    G.swap(out);
}

static void fuse_pass(PlanPass& P, std::vector<double>& pool, int K, int min_dense)
{
    std::vector<TileOp> out;
    std::vector<size_t> blk;
    uint32_t bbits = 0;
    int bdense = 0;
    auto emit = [&]() {
        if (blk.empty()) return;
        if (bdense < min_dense) {
            for (size_t i : blk) out.push_back(P.ops[i]);
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
            const int DR = 2 * D, RB = DR / 16, KS = DR / 4, NF = RB * KS;
            std::vector<double> fr((size_t)NF * 64); // [q][lane][2], fragment f = 2q + j
            for (int lane = 0; lane < 64; ++lane)
                for (int rb = 0; rb < RB; ++rb)
                    for (int ks = 0; ks < KS; ++ks) {
                        const int row = 16 * rb + (lane % 16), col = 4 * ks + lane / 16;
                        const cd u = G[(size_t)(row / 2) * D + col / 2];
                        double v;
                        if ((row & 1) == 0)
                            v = (col & 1) == 0 ? u.real() : -u.imag();
                        else
                            v = (col & 1) == 0 ? u.imag() : u.real();
                        const int f = rb * KS + ks;
                        fr[((size_t)(f / 2) * 64 + lane) * 2 + (f % 2)] = v;
                    }
            TileOp t;
            std::memset(&t, 0, sizeof t);
            t.kind = TK_MFMA;
            t.k = K;
            for (int j = 0; j < K; ++j) t.p[j] = bq[j];
            size_t off = pool.size();
            pool.resize(off + fr.size() + 2);
            // fragments start on a 16-byte boundary inside the pool
            if (off & 1) ++off;
            std::memcpy(pool.data() + off, fr.data(), fr.size() * sizeof(double));
            t.moff = off;
            out.push_back(t);
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
        }
    }
    emit();
    P.ops.swap(out);
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
                  std::vector<PlanPass>& passes, std::vector<double>& pool)
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
            P.gates += 1;
            P.updates += 1ull << (n - __builtin_popcountll(o.cmask));
        }
        if ((po.fuse_k == 4 || po.fuse_k == 5) && po.dt == QS_C64 && m >= po.fuse_k + 4)
            fuse_pass(P, pool, po.fuse_k, po.fuse_min);
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

static int default_tile_qubits(int dt)
{
    const int e = env_int("QS_TILE_QUBITS", 0);
    if (e > 0) return e;
    return dt == QS_C128 ? 11 : 12;
}

static int default_low_qubits(int dt)
{
    const int e = env_int("QS_TILE_LOW", -1);
    if (e >= 0) return e;
    return dt == QS_C128 ? 5 : 6;
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
    std::vector<PlanPass> passes;
    std::vector<double> pool;
    plan_circuit(s->n, ops, n_ops, mats, po, passes, pool);

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
                return launch_tile_pass(s->d, s->dt, s->n, p, pd, dmats, s->st);
            },
            "tile pass launch");
        if (st != QS_OK) return st;
        op0 += p.ops.size();
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
    std::vector<PlanPass> passes;
    std::vector<double> pool;
    if (n_ops > 0) plan_circuit(n, ops, n_ops, mats, po, passes, pool);
    int64_t c = 0;
    for (auto& p : passes) c += (int64_t)p.ops.size();
    *n_passes = (int64_t)passes.size();
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
        for (int64_t g : passes[p].src) {
            order[c] = g;
            pass_of[c] = (int32_t)p;
            ++c;
        }
    }
    return QS_OK;
}
