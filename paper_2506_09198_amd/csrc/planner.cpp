// Circuit planner and tile-pass executor.
//
// Gates are taken strictly in circuit order.  A pass keeps a set Q of at most
// m tile qubits; a non-diagonal gate joins the current pass when its targets
// fit into Q (growing Q), otherwise the pass is closed and a new one starts.
// Diagonal gates (CZ, controlled phases, phase flips) join whatever pass is
// open: they scale amplitudes elementwise and need no tile qubits.  A closed
// pass is padded with the lowest unused qubits so its tiles are built from the
// longest possible contiguous runs.  Each pass costs one read and one write of
// the state, against one per gate when gates are launched one by one.
#include "planner.h"

#include <algorithm>
#include <cstring>

namespace qs {

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
                for (int j = 0; j < o.nt; ++j) t.p[j] = o.t[j];
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
            P.gates += 1;
            P.updates += 1ull << (n - __builtin_popcountll(o.cmask));
        }
        passes.push_back(std::move(P));
        items.clear();
        qmask = 0;
    };

    for (int64_t g = 0; g < n_ops; ++g) {
        const qs_op& o = ops[g];
        const bool diag = is_diagonal(mats + o.moff, o.nt);
        if (diag) {
            items.push_back({&o, true});
            continue;
        }
        uint64_t tm = 0;
        for (int j = 0; j < o.nt; ++j) tm |= 1ull << o.t[j];
        uint64_t need = qmask | tm | lowQ;
        if (__builtin_popcountll(need) > m) {
            close();
            need = tm | lowQ;
            if (__builtin_popcountll(need) > m) need = tm; // the gate alone: padding fills low qubits
        }
        qmask = need;
        items.push_back({&o, false});
    }
    if (qmask == 0 && !items.empty()) qmask = lowQ; // only diagonal gates
    close();
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
    po.m = o.tile_qubits > 0 ? o.tile_qubits : default_tile_qubits(dt);
    if (po.m > 13) return set_err(QS_ERR_ARG, "tile_qubits=%d > 13", po.m);
    int maxk = 1;
    for (int64_t g = 0; g < n_ops; ++g) maxk = std::max(maxk, (int)ops[g].nt);
    po.m = std::max(po.m, maxk);
    po.L = default_low_qubits(dt);
    po.fuse_k = o.fuse_k;
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

qs_status validate_circuit(int n, const qs_op* ops, int64_t n_ops, const double* mats, int64_t n_mats);

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
