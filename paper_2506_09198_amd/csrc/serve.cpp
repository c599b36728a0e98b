// Serving loop (qs_server_*): continuous batching of circuit requests.
//
// Requests wait in a FIFO until their state fits the HBM budget; admission
// allocates the state from the server's pool, plans the circuit and uploads
// the plan.  Work is enqueued in rounds on one stream: a round advances every
// active request by one tile pass (one launch for all of them) and runs newly
// admitted small requests (n <= the LDS tile) whole, one launch per n.  Up to
// `rounds_ahead` rounds are in flight; a request that arrives while others
// are on the GPU joins the next round built, and a finished request frees its
// place in later rounds at once (its state stays until qs_server_release).
// Each request's plan depends only on its own circuit and the server options,
// and every tile is computed the same way whoever shares the round, so a result
// is bitwise the same alone and in any mix.
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <unordered_map>
#include <vector>

#include "planner.h"
#include "runtime.h"

using namespace qs;

namespace {

// First-fit allocator over [0, size) with coalescing, 256-byte granularity.
struct Pool {
    std::map<uint64_t, uint64_t> free; // offset -> bytes
    uint64_t size = 0, used = 0, peak = 0;
    void init(uint64_t bytes)
    {
        size = bytes;
        free.clear();
        if (bytes) free[0] = bytes;
    }
    bool alloc(uint64_t bytes, uint64_t* off)
    {
        bytes = (bytes + 255) & ~255ull;
        for (auto it = free.begin(); it != free.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const uint64_t rest = it->second - bytes, o = it->first + bytes;
            free.erase(it);
            if (rest) free[o] = rest;
            used += bytes;
            if (used > peak) peak = used;
            return true;
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes)
    {
        bytes = (bytes + 255) & ~255ull;
        used -= bytes;
        auto it = free.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free.erase(nx);
        }
        if (it != free.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free.erase(it);
            }
        }
    }
};

enum { R_QUEUED = 0, R_ACTIVE = 1, R_DONE = 2, R_FAILED = 3, R_CANCELLED = 4 };

struct Req {
    uint64_t id = 0;
    int n = 0;
    uint64_t basis = 0;               // basis state, or kLoadInitial with init_state
    const void* init_state = nullptr; // caller's device copy of the initial state
    int want = QS_WANT_NONE;          // result written to `out` when the request is done
    void* out = nullptr;
    std::vector<qs_op> ops;
    std::vector<double> mats;
    int state = R_QUEUED;
    qs_status status = QS_OK;
    uint64_t s_off = 0, s_bytes = 0;
    uint64_t p_off = 0, p_bytes = 0;
    std::vector<char> plan_host; // kept until the request finishes (async upload source)
    int npass = 0, next_pass = 0;
    std::vector<uint8_t> pass_var; // tile-kernel variant of pass j (ops_variant)
    int max_var = 0;               // largest over the passes
    bool whole = false, whole_launched = false;
    int64_t last_round = -1;
    double t_submit = 0, t_admit = 0, t_done = 0;
    uint64_t passes_off = 0, ops_off = 0, mats_off = 0; // inside the plan region
};

struct Slot {
    ServeEntry* host = nullptr;
    ServeEntry* dev = nullptr;
    int cap = 0;
    hipEvent_t ev = nullptr;
    int64_t round = -1;
    bool busy = false;
    std::vector<uint64_t> ids;
};

} // namespace

struct qs_server_s {
    int dt = QS_C128;
    int m = 11, whole_max = 12, fuse_k = 0, tile_qubits = 0;
    int rounds_ahead = 3;
    char* pool = nullptr;
    char* plan = nullptr;
    Pool spool, ppool;
    hipStream_t st = nullptr;
    std::vector<Slot> slots;
    int64_t next_round = 0;
    uint64_t next_id = 1;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, Req> reqs;
    std::vector<uint64_t> active;
    std::deque<qs_result> completed;
    std::chrono::steady_clock::time_point t0;
    qs_server_stats stats;
    // delivery of wanted results: own stream (the rounds' stream may hold
    // rounds enqueued ahead) and reduction scratch
    hipStream_t rst = nullptr;
    double* red = nullptr;
    uint64_t red_cap = 0; // doubles
};

namespace {

double now_ms(qs_server s)
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - s->t0).count();
}

// Write a finished request's wanted result to its host buffer.  Its last
// round has completed (its event was seen), so the state in the pool is final.
qs_status deliver(qs_server s, const Req& r)
{
    hipError_t e = hipSuccess;
    if (!s->rst) {
        e = hipStreamCreateWithFlags(&s->rst, hipStreamNonBlocking);
        if (e != hipSuccess) {
            s->rst = nullptr;
            (void)hipGetLastError();
            return set_err(QS_ERR_DEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
        }
    }
    const char* psi = s->pool + r.s_off;
    if (r.want == QS_WANT_STATE) {
        e = hipMemcpyAsync(r.out, psi, amp_bytes(s->dt) << r.n, hipMemcpyDeviceToHost, s->rst);
    } else {
        const int m = r.want == QS_WANT_PROBS ? r.n : 0;
        std::vector<int> q((size_t)m);
        for (int j = 0; j < m; ++j) q[(size_t)j] = j;
        const uint64_t need = reduce_scratch_doubles(r.n, m) + (1ull << m);
        if (need > s->red_cap) {
            if (s->red) dev_free(s->red, s->red_cap * sizeof(double));
            s->red = nullptr;
            s->red_cap = 0;
            qs_status st = dev_alloc((void**)&s->red, need * sizeof(double), "serving reduction scratch");
            if (st != QS_OK) return st;
            s->red_cap = need;
        }
        double* dout = s->red + reduce_scratch_doubles(r.n, m);
        e = launch_probabilities(psi, s->dt, r.n, q.data(), m, s->red, dout, s->rst);
        if (e == hipSuccess) e = hipMemcpyAsync(r.out, dout, sizeof(double) << m, hipMemcpyDeviceToHost, s->rst);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s->rst);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_err(QS_ERR_DEVICE, "result delivery: %s", hipGetErrorString(e));
    }
    return QS_OK;
}

void finish(qs_server s, Req& r, qs_status st, int state)
{
    if (state == R_DONE && r.want != QS_WANT_NONE) {
        const qs_status d = deliver(s, r);
        if (d != QS_OK) {
            st = d;
            state = R_FAILED;
        }
    }
    r.state = state;
    r.status = st;
    r.t_done = now_ms(s);
    if (r.p_bytes) {
        s->ppool.release(r.p_off, r.p_bytes);
        r.p_bytes = 0;
    }
    r.plan_host.clear();
    r.plan_host.shrink_to_fit();
    r.ops.clear();
    r.mats.clear();
    qs_result res;
    std::memset(&res, 0, sizeof res);
    res.id = r.id;
    res.status = st;
    res.n = r.n;
    res.t_submit_ms = r.t_submit;
    res.t_admit_ms = r.t_admit;
    res.t_done_ms = r.t_done;
    s->completed.push_back(res);
    if (state == R_DONE)
        s->stats.completed += 1;
    else
        s->stats.failed += 1;
}

void drop_active(qs_server s, uint64_t id)
{
    for (size_t i = 0; i < s->active.size(); ++i)
        if (s->active[i] == id) {
            s->active.erase(s->active.begin() + i);
            return;
        }
}

// Fail every request with work in a round that could not be enqueued or ran
// into an error; free their states so the server keeps serving the others.
void fail_round(qs_server s, Slot& sl, qs_status st)
{
    for (uint64_t id : sl.ids) {
        auto it = s->reqs.find(id);
        if (it == s->reqs.end() || it->second.state != R_ACTIVE) continue;
        Req& r = it->second;
        drop_active(s, id);
        s->spool.release(r.s_off, r.s_bytes);
        r.s_bytes = 0;
        finish(s, r, st, R_FAILED);
    }
    sl.busy = false;
    sl.ids.clear();
}

void retire(qs_server s)
{
    for (;;) {
        // the oldest busy slot
        Slot* sl = nullptr;
        for (auto& x : s->slots)
            if (x.busy && (!sl || x.round < sl->round)) sl = &x;
        if (!sl) return;
        hipError_t e = hipEventQuery(sl->ev);
        if (e == hipErrorNotReady) {
            (void)hipGetLastError();
            return;
        }
        if (e != hipSuccess) {
            (void)hipGetLastError();
            fail_round(s, *sl, set_err(QS_ERR_DEVICE, "serving round failed: %s", hipGetErrorString(e)));
            continue;
        }
        for (uint64_t id : sl->ids) {
            auto it = s->reqs.find(id);
            if (it == s->reqs.end()) continue;
            Req& r = it->second;
            if (r.state == R_ACTIVE && r.last_round == sl->round) {
                drop_active(s, id);
                finish(s, r, QS_OK, R_DONE);
            }
        }
        sl->busy = false;
        sl->ids.clear();
    }
}

qs_status admit_one(qs_server s, Req& r)
{
    const uint64_t S = amp_bytes(s->dt);
    r.s_bytes = S << r.n;
    if (!s->spool.alloc(r.s_bytes, &r.s_off)) {
        r.s_bytes = 0;
        return QS_ERR_OOM;
    }
    PlanOpts po;
    qs_status st = plan_opts_for(s->dt, r.ops.data(), (int64_t)r.ops.size(), s->fuse_k, s->tile_qubits, po);
    if (st != QS_OK) return st;
    r.whole = r.n <= s->whole_max;
    po.m = r.whole ? r.n : s->m;
    std::vector<PlanPass> passes;
    std::vector<double> pool;
    if (!r.ops.empty()) plan_circuit(r.n, r.ops.data(), (int64_t)r.ops.size(), r.mats.data(), po, passes, pool);
    std::vector<BatchPass> bp;
    std::vector<TileOp> to;
    for (auto& p : passes) {
        BatchPass d;
        std::memset(&d, 0, sizeof d);
        d.m = p.m;
        d.L = p.L;
        uint64_t qm = 0;
        for (int j = 0; j < p.m; ++j) {
            d.q[j] = p.Q[j];
            qm |= 1ull << p.Q[j];
        }
        d.ip = make_insert_plan(qm);
        d.op0 = (int)to.size();
        d.nops = (int)p.ops.size();
        for (auto& t : p.ops) to.push_back(t);
        const int v = ops_variant(p.ops.data(), p.ops.size(), p.m);
        r.pass_var.push_back((uint8_t)v);
        r.max_var = std::max(r.max_var, v);
        bp.push_back(d);
    }
    auto al = [](uint64_t x) { return (x + 255) & ~255ull; };
    r.passes_off = 0;
    r.ops_off = al(bp.size() * sizeof(BatchPass));
    r.mats_off = al(r.ops_off + to.size() * sizeof(TileOp));
    r.p_bytes = al(r.mats_off + pool.size() * sizeof(double)) + 256;
    if (r.p_bytes > s->ppool.size) {
        // can never fit, however many requests finish: fail it, do not queue it forever
        s->spool.release(r.s_off, r.s_bytes);
        r.s_bytes = 0;
        const unsigned long long pb = r.p_bytes;
        r.p_bytes = 0;
        return set_err(QS_ERR_ARG, "plan of %llu bytes can never fit the serving plan pool of %llu bytes", pb,
                       (unsigned long long)s->ppool.size);
    }
    if (!s->ppool.alloc(r.p_bytes, &r.p_off)) {
        s->spool.release(r.s_off, r.s_bytes);
        r.s_bytes = 0;
        r.p_bytes = 0;
        return QS_ERR_OOM;
    }
    if (r.init_state) {
        // the caller's initial state into the pool, ahead of the request's rounds
        hipError_t e0 = hipMemcpyAsync(s->pool + r.s_off, r.init_state, amp_bytes(s->dt) << r.n,
                                       hipMemcpyDeviceToDevice, s->st);
        if (e0 != hipSuccess) return set_err(QS_ERR_DEVICE, "initial state copy: %s", hipGetErrorString(e0));
    }
    r.plan_host.assign(r.p_bytes, 0);
    std::memcpy(r.plan_host.data() + r.passes_off, bp.data(), bp.size() * sizeof(BatchPass));
    std::memcpy(r.plan_host.data() + r.ops_off, to.data(), to.size() * sizeof(TileOp));
    std::memcpy(r.plan_host.data() + r.mats_off, pool.data(), pool.size() * sizeof(double));
    hipError_t e = hipMemcpyAsync(s->plan + r.p_off, r.plan_host.data(), r.p_bytes, hipMemcpyHostToDevice, s->st);
    if (e != hipSuccess) return set_err(QS_ERR_DEVICE, "plan upload: %s", hipGetErrorString(e));
    r.npass = (int)passes.size();
    r.next_pass = 0;
    if (!r.whole && !r.init_state) {
        // tile passes read the state from HBM: start it as |basis>
        if (inject_fault_now()) return set_err(QS_ERR_DEVICE, "injected device fault (QS_FAULT_INJECT)");
        e = launch_init_basis(s->pool + r.s_off, s->dt, r.n, r.basis, s->st);
        s->stats.launches += 1;
        if (e != hipSuccess) return set_err(QS_ERR_DEVICE, "init launch: %s", hipGetErrorString(e));
    }
    r.state = R_ACTIVE;
    r.t_admit = now_ms(s);
    s->active.push_back(r.id);
    s->stats.admitted += 1;
    return QS_OK;
}

void admit(qs_server s)
{
    // FIFO; a request that does not fit yet is passed over by later ones at
    // most 64 times before admission stops behind it (no starvation of big ones)
    int bypassed = 0;
    for (auto it = s->queue.begin(); it != s->queue.end();) {
        Req& r = s->reqs[*it];
        qs_status st = admit_one(s, r);
        if (st == QS_OK) {
            it = s->queue.erase(it);
            continue;
        }
        if (st != QS_ERR_OOM) {
            const uint64_t id = *it;
            it = s->queue.erase(it);
            drop_active(s, id);
            if (r.s_bytes) s->spool.release(r.s_off, r.s_bytes);
            r.s_bytes = 0;
            finish(s, r, st, R_FAILED);
            continue;
        }
        if (++bypassed > 64) break;
        ++it;
    }
}

// Build and enqueue one round; false when there is nothing to do or no slot.
bool build_round(qs_server s)
{
    Slot* sl = nullptr;
    for (auto& x : s->slots)
        if (!x.busy) {
            sl = &x;
            break;
        }
    if (!sl) return false;
    std::vector<ServeEntry> whole_e, round_e;
    std::vector<int> whole_n;
    std::vector<uint8_t> whole_v; // per whole entry: tile-kernel variant
    int round_v = 0;
    std::vector<uint64_t> ids;
    uint32_t blocks = 0;
    for (uint64_t id : s->active) {
        Req& r = s->reqs[id];
        if (r.whole) {
            if (r.whole_launched) continue;
            ServeEntry en;
            std::memset(&en, 0, sizeof en);
            en.psi_off = r.s_off;
            en.pass_off = r.npass ? r.p_off + r.passes_off : ~0ull;
            en.ops_off = r.p_off + r.ops_off;
            en.mats_off = r.p_off + r.mats_off;
            en.basis = r.basis;
            en.n = r.n;
            whole_e.push_back(en);
            whole_n.push_back(r.n);
            whole_v.push_back((uint8_t)r.max_var);
            ids.push_back(id);
        } else if (r.next_pass < r.npass || (r.npass == 0 && r.last_round < 0)) {
            if (r.npass > 0) {
                ServeEntry en;
                std::memset(&en, 0, sizeof en);
                en.psi_off = r.s_off;
                en.pass_off = r.p_off + r.passes_off + (uint64_t)r.next_pass * sizeof(BatchPass);
                en.ops_off = r.p_off + r.ops_off;
                en.mats_off = r.p_off + r.mats_off;
                en.n = r.n;
                en.first_block = blocks;
                blocks += 1u << (r.n - s->m);
                round_e.push_back(en);
                round_v = std::max(round_v, (int)r.pass_var[(size_t)r.next_pass]);
            }
            ids.push_back(id);
        }
    }
    if (ids.empty()) return false;
    // whole entries grouped by n (each launch covers a contiguous run)
    std::vector<size_t> order(whole_e.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return whole_n[a] < whole_n[b]; });
    const size_t need = whole_e.size() + round_e.size();
    if ((int)need > sl->cap) {
        if (sl->host) (void)hipHostFree(sl->host);
        if (sl->dev) dev_free(sl->dev, (uint64_t)sl->cap * sizeof(ServeEntry));
        sl->host = nullptr;
        sl->dev = nullptr;
        int cap = 256;
        while ((size_t)cap < need) cap *= 2;
        if (hipHostMalloc((void**)&sl->host, cap * sizeof(ServeEntry), hipHostMallocDefault) != hipSuccess ||
            dev_alloc((void**)&sl->dev, cap * sizeof(ServeEntry), "serving round entries") != QS_OK) {
            (void)hipGetLastError();
            sl->cap = 0;
            return false;
        }
        sl->cap = cap;
    }
    for (size_t i = 0; i < order.size(); ++i) sl->host[i] = whole_e[order[i]];
    for (size_t i = 0; i < round_e.size(); ++i) sl->host[whole_e.size() + i] = round_e[i];
    sl->round = s->next_round++;
    sl->ids = ids;
    sl->busy = true;
    hipError_t e = hipMemcpyAsync(sl->dev, sl->host, need * sizeof(ServeEntry), hipMemcpyHostToDevice, s->st);
    qs_status st = QS_OK;
    if (e != hipSuccess) st = set_err(QS_ERR_DEVICE, "round upload: %s", hipGetErrorString(e));
    for (size_t i = 0; i < order.size() && st == QS_OK;) {
        size_t j = i;
        int var = 0;
        while (j < order.size() && whole_n[order[j]] == whole_n[order[i]]) var = std::max(var, (int)whole_v[order[j++]]);
        if (inject_fault_now()) {
            st = set_err(QS_ERR_DEVICE, "injected device fault (QS_FAULT_INJECT)");
            break;
        }
        e = launch_serve_whole(s->dt, whole_n[order[i]], s->pool, s->plan, sl->dev + i, (int)(j - i), var, s->st);
        s->stats.launches += 1;
        if (e != hipSuccess) st = set_err(QS_ERR_DEVICE, "whole launch: %s", hipGetErrorString(e));
        i = j;
    }
    if (st == QS_OK && !round_e.empty()) {
        if (inject_fault_now()) {
            st = set_err(QS_ERR_DEVICE, "injected device fault (QS_FAULT_INJECT)");
        } else {
            e = launch_serve_round(s->dt, s->m, s->pool, s->plan, sl->dev + whole_e.size(), (int)round_e.size(), blocks,
                                   round_v, s->st);
            s->stats.launches += 1;
            if (e != hipSuccess) st = set_err(QS_ERR_DEVICE, "round launch: %s", hipGetErrorString(e));
        }
    }
    if (st == QS_OK) {
        e = hipEventRecord(sl->ev, s->st);
        if (e != hipSuccess) st = set_err(QS_ERR_DEVICE, "hipEventRecord: %s", hipGetErrorString(e));
    }
    if (st != QS_OK) {
        (void)hipGetLastError();
        // the stream is still usable for injected faults; make sure nothing of
        // this round is waited on, and fail its requests
        (void)hipStreamSynchronize(s->st);
        fail_round(s, *sl, st);
        return true;
    }
    for (uint64_t id : ids) {
        Req& r = s->reqs[id];
        if (r.whole) {
            r.whole_launched = true;
            r.last_round = sl->round;
        } else {
            if (r.npass > 0) r.next_pass += 1;
            if (r.next_pass >= r.npass) r.last_round = sl->round;
        }
    }
    s->stats.rounds += 1;
    return true;
}

} // namespace

extern "C" {

qs_status qs_server_create(const qs_server_opts* opts, qs_server* out)
{
    if (!out) return set_err(QS_ERR_ARG, "null output pointer");
    *out = nullptr;
    qs_server_opts o;
    std::memset(&o, 0, sizeof o);
    if (opts) o = *opts;
    if (o.dtype == 0) o.dtype = QS_C128;
    if (o.dtype != QS_C64 && o.dtype != QS_C128) return set_err(QS_ERR_ARG, "unknown dtype %d", o.dtype);
    if (o.rounds_ahead <= 0) o.rounds_ahead = 3;
    if (o.rounds_ahead > 16) return set_err(QS_ERR_ARG, "rounds_ahead=%d > 16", o.rounds_ahead);
    if (o.tile_qubits != 0 && (o.tile_qubits < 9 || o.tile_qubits > 13))
        return set_err(QS_ERR_ARG, "tile_qubits=%d outside [9, 13]", o.tile_qubits);
    if (qs_device_count() < 1) return set_err(QS_ERR_DEVICE, "no HIP device available");
    uint64_t budget = o.hbm_budget;
    if (budget == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            (void)hipGetLastError();
            return set_err(QS_ERR_DEVICE, "hipMemGetInfo failed");
        }
        budget = fr / 2;
    }
    budget &= ~255ull;
    qs_server s = new qs_server_s();
    std::memset(&s->stats, 0, sizeof s->stats);
    s->dt = o.dtype;
    s->tile_qubits = o.tile_qubits;
    s->fuse_k = o.fuse_k;
    s->rounds_ahead = o.rounds_ahead;
    PlanOpts po;
    (void)plan_opts_for(s->dt, nullptr, 0, o.fuse_k, o.tile_qubits, po);
    s->m = std::min(std::max(po.m, 9), 13);
    s->whole_max = s->dt == QS_C128 ? 12 : 13;
    s->t0 = std::chrono::steady_clock::now();
    const uint64_t plan_bytes = o.plan_budget ? o.plan_budget : (256ull << 20);
    qs_status st = dev_alloc((void**)&s->pool, budget, "serving state pool");
    if (st == QS_OK) {
        s->spool.init(budget);
        st = dev_alloc((void**)&s->plan, plan_bytes, "serving plan pool");
        if (st == QS_OK) s->ppool.init(plan_bytes);
    }
    if (st != QS_OK) {
        qs_server_destroy(s);
        return st;
    }
    hipError_t e = hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking);
    if (e != hipSuccess) {
        qs_server_destroy(s);
        (void)hipGetLastError();
        return set_err(QS_ERR_DEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
    }
    s->slots.resize(s->rounds_ahead);
    for (auto& x : s->slots)
        if (hipEventCreate(&x.ev) != hipSuccess) {
            qs_server_destroy(s);
            (void)hipGetLastError();
            return set_err(QS_ERR_DEVICE, "hipEventCreate failed");
        }
    s->stats.budget_bytes = budget;
    *out = s;
    return QS_OK;
}

qs_status qs_server_submit(qs_server s, const qs_circuit* c, uint64_t* id)
{
    if (!s || !c || !id) return set_err(QS_ERR_ARG, "null argument");
    if (c->n < 1 || c->n > QS_MAX_QUBITS) return set_err(QS_ERR_ARG, "n=%d outside [1, %d]", c->n, QS_MAX_QUBITS);
    if (!c->init_state && c->init_basis >= (1ull << c->n)) return set_err(QS_ERR_ARG, "basis state out of range");
    if (c->want < QS_WANT_NONE || c->want > QS_WANT_NORM) return set_err(QS_ERR_ARG, "want=%d", c->want);
    if (c->want != QS_WANT_NONE && !c->out) return set_err(QS_ERR_ARG, "want without an output buffer");
    if (c->want == QS_WANT_PROBS && c->n > 24) return set_err(QS_ERR_ARG, "QS_WANT_PROBS needs n <= 24");
    qs_status st = validate_circuit(c->n, c->ops, c->n_ops, c->mats, c->n_mats);
    if (st != QS_OK) return st;
    const uint64_t need = ((amp_bytes(s->dt) << c->n) + 255) & ~255ull;
    if (need > s->spool.size)
        return set_err(QS_ERR_OOM, "state of %llu bytes can never fit the serving budget of %llu",
                       (unsigned long long)need, (unsigned long long)s->spool.size);
    Req r;
    r.id = s->next_id++;
    r.n = c->n;
    r.basis = c->init_state ? kLoadInitial : c->init_basis;
    r.init_state = c->init_state;
    r.want = c->want;
    r.out = c->out;
    r.ops.assign(c->ops, c->ops + c->n_ops);
    r.mats.assign(c->mats, c->mats + c->n_mats);
    r.t_submit = now_ms(s);
    s->reqs.emplace(r.id, std::move(r));
    s->queue.push_back(s->next_id - 1);
    s->stats.submitted += 1;
    *id = s->next_id - 1;
    return QS_OK;
}

qs_status qs_server_poll(qs_server s, qs_result* out, int max, int* count)
{
    if (!s || !count || (max > 0 && !out)) return set_err(QS_ERR_ARG, "null argument");
    retire(s);
    admit(s);
    int built = 0;
    while (built < s->rounds_ahead && build_round(s)) ++built;
    retire(s);
    int c = 0;
    while (c < max && !s->completed.empty()) {
        out[c++] = s->completed.front();
        s->completed.pop_front();
    }
    *count = c;
    s->stats.queued = (uint32_t)s->queue.size();
    s->stats.active = (uint32_t)s->active.size();
    s->stats.used_bytes = s->spool.used;
    s->stats.peak_bytes = s->spool.peak;
    return QS_OK;
}

static Req* find_done(qs_server s, uint64_t id)
{
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) {
        set_err(QS_ERR_ARG, "unknown request %llu", (unsigned long long)id);
        return nullptr;
    }
    if (it->second.state != R_DONE) {
        set_err(QS_ERR_BUSY, "request %llu is not finished", (unsigned long long)id);
        return nullptr;
    }
    return &it->second;
}

qs_status qs_server_state(qs_server s, uint64_t id, void** dev_ptr, int* n)
{
    if (!s) return set_err(QS_ERR_ARG, "null server");
    Req* r = find_done(s, id);
    if (!r) return s->reqs.count(id) ? QS_ERR_BUSY : QS_ERR_ARG;
    if (dev_ptr) *dev_ptr = s->pool + r->s_off;
    if (n) *n = r->n;
    return QS_OK;
}

qs_status qs_server_download(qs_server s, uint64_t id, void* host)
{
    if (!s || !host) return set_err(QS_ERR_ARG, "null argument");
    Req* r = find_done(s, id);
    if (!r) return s->reqs.count(id) ? QS_ERR_BUSY : QS_ERR_ARG;
    hipError_t e = hipMemcpyAsync(host, s->pool + r->s_off, amp_bytes(s->dt) << r->n, hipMemcpyDeviceToHost, s->st);
    if (e == hipSuccess) e = hipStreamSynchronize(s->st);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_err(QS_ERR_DEVICE, "download: %s", hipGetErrorString(e));
    }
    return QS_OK;
}

qs_status qs_server_release(qs_server s, uint64_t id)
{
    if (!s) return set_err(QS_ERR_ARG, "null server");
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return set_err(QS_ERR_ARG, "unknown request %llu", (unsigned long long)id);
    Req& r = it->second;
    if (r.state == R_QUEUED || r.state == R_ACTIVE)
        return set_err(QS_ERR_BUSY, "request %llu is still queued or running", (unsigned long long)id);
    if (r.s_bytes) s->spool.release(r.s_off, r.s_bytes);
    s->reqs.erase(it);
    return QS_OK;
}

qs_status qs_server_cancel(qs_server s, uint64_t id)
{
    if (!s) return set_err(QS_ERR_ARG, "null server");
    for (auto it = s->queue.begin(); it != s->queue.end(); ++it)
        if (*it == id) {
            s->queue.erase(it);
            Req& r = s->reqs[id];
            finish(s, r, QS_ERR_CANCELLED, R_CANCELLED);
            s->stats.failed -= 1;
            s->stats.cancelled += 1;
            return QS_OK;
        }
    return set_err(QS_ERR_BUSY, "request %llu is not queued (running, finished or unknown)", (unsigned long long)id);
}

qs_status qs_server_get_stats(qs_server s, qs_server_stats* out)
{
    if (!s || !out) return set_err(QS_ERR_ARG, "null argument");
    s->stats.queued = (uint32_t)s->queue.size();
    s->stats.active = (uint32_t)s->active.size();
    s->stats.used_bytes = s->spool.used;
    s->stats.peak_bytes = s->spool.peak;
    *out = s->stats;
    return QS_OK;
}

qs_status qs_server_destroy(qs_server s)
{
    if (!s) return QS_OK;
    if (s->st) (void)hipStreamSynchronize(s->st);
    for (auto& x : s->slots) {
        if (x.ev) (void)hipEventDestroy(x.ev);
        if (x.host) (void)hipHostFree(x.host);
        if (x.dev) dev_free(x.dev, (uint64_t)x.cap * sizeof(ServeEntry));
    }
    if (s->st) (void)hipStreamDestroy(s->st);
    if (s->rst) (void)hipStreamDestroy(s->rst);
    if (s->red) dev_free(s->red, s->red_cap * sizeof(double));
    if (s->pool) dev_free(s->pool, s->spool.size);
    if (s->plan) dev_free(s->plan, s->ppool.size);
    (void)hipGetLastError();
    delete s;
    return QS_OK;
}

} // extern "C"
