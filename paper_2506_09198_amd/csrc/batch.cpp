// Batched execution of many independent circuits (qs_batch_*).
//
// All final states live in one device arena.  Mode 0 (fused) sorts circuits by
// size:
//   - "whole": n at most the largest LDS tile -- each circuit runs entirely in
//     one workgroup's LDS; one launch per distinct n covers all of them, and
//     their states touch HBM once, when written;
//   - "persistent": medium n -- one workgroup per circuit walks the circuit's
//     tile passes over its state (block barriers only, no grid-wide sync);
//     one launch per tile size covers all of them;
//   - "streamed": large n -- pass-major rounds: launch r processes pass r of
//     every large circuit that has one (each block one tile), so the launch
//     count is the longest pass list, not the sum of all of them.
// Mode 1 launches every gate separately (the per-gate kernels), circuits spread
// over the streams: the unfused reference the fused mode is compared against.
#include <chrono>
#include <cstring>
#include <mutex>
#include <thread>
#include <utility>
#include <vector>

#include "planner.h"
#include "runtime.h"

using namespace qs;

struct qs_batch_s {
    int dt = QS_C128;
    int mode = 0;
    int count = 0;
    char* arena = nullptr;
    uint64_t arena_bytes = 0;
    char* dbuf = nullptr; // descriptors, passes, ops, matrices
    uint64_t dbuf_bytes = 0;
    char* hbuf = nullptr; // pinned staging for dbuf
    uint64_t hbuf_cap = 0;
    std::vector<uint64_t> off;
    std::vector<int> n;
    std::vector<hipStream_t> st;
    std::vector<hipEvent_t> done;
    hipEvent_t t0 = nullptr;
    hipEvent_t cls_done[3] = {nullptr, nullptr, nullptr};
    bool failed = false;
    qs_batch_stats stats;
    // the fused launch schedule, kept for qs_batch_replay (device data in dbuf)
    struct Sched {
        std::vector<std::pair<int, std::pair<size_t, int>>> whole_groups; // (n, (list offset, count))
        size_t persist_l0 = 0, stream_l0 = 0;
        int persist_count = 0, stream_count = 0, persist_m = 0, stream_m = 0;
        std::vector<std::pair<size_t, std::pair<int, uint32_t>>> rounds; // (entry offset, (count, blocks))
        // the tile-kernel variant each launch needs (ops_variant, largest over
        // the passes it covers): the lean kernel holds fewer registers
        std::vector<uint8_t> whole_var; // per whole group
        int persist_var = 0;
        std::vector<uint8_t> round_var; // per round
        const BatchCirc* dcirc = nullptr;
        const BatchPass* dpass = nullptr;
        const TileOp* dops = nullptr;
        const int32_t* dlist = nullptr;
        const RoundEntry* dents = nullptr;
        const double* dmats = nullptr;
    } sched;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    double* red = nullptr; // reduction scratch for qs_batch_probabilities
    uint64_t red_cap = 0;  // doubles
    // initial states given by the caller (circuit, device source), copied into
    // the arena before every run; results delivered to host buffers on
    // completion (circuit, want, out), once per run
    std::vector<std::pair<int, const void*>> init_src;
    std::vector<std::pair<int, std::pair<int, void*>>> wants;
    bool delivered = false;
};

namespace {

// One spare pinned staging buffer kept across batches: pinning a fresh
// gigabyte per submit costs far more than filling it.  A batch takes the spare
// when it is large enough (else allocates its own) and hands its buffer back
// on release; the larger of the two is kept.
std::mutex g_pin_mu;
char* g_pin = nullptr;
uint64_t g_pin_cap = 0;

qs_status pinned_acquire(uint64_t bytes, char** out, uint64_t* cap)
{
    {
        std::lock_guard<std::mutex> lk(g_pin_mu);
        if (g_pin && g_pin_cap >= bytes) {
            *out = g_pin;
            *cap = g_pin_cap;
            g_pin = nullptr;
            g_pin_cap = 0;
            return QS_OK;
        }
    }
    const uint64_t want = bytes + bytes / 4; // room for a slightly larger next batch
    if (hipHostMalloc((void**)out, want, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        *out = nullptr;
        return set_err(QS_ERR_OOM, "hipHostMalloc(%llu) failed", (unsigned long long)want);
    }
    *cap = want;
    return QS_OK;
}

void pinned_release(char* p, uint64_t cap)
{
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_pin_mu);
    if (!g_pin || cap > g_pin_cap) std::swap(g_pin, p), std::swap(g_pin_cap, cap);
    if (p) (void)hipHostFree(p);
}

qs_status bfail(qs_batch b, hipError_t e, const char* what)
{
    b->failed = true;
    (void)hipGetLastError();
    return set_err(QS_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

void release(qs_batch b)
{
    if (!b) return;
    for (hipStream_t s : b->st) (void)hipStreamSynchronize(s);
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (hipEvent_t e : b->done) (void)hipEventDestroy(e);
    if (b->t0) (void)hipEventDestroy(b->t0);
    for (hipEvent_t e : b->cls_done)
        if (e) (void)hipEventDestroy(e);
    for (hipStream_t s : b->st) (void)hipStreamDestroy(s);
    if (b->arena) dev_free(b->arena, b->arena_bytes);
    if (b->dbuf) dev_free(b->dbuf, b->dbuf_bytes);
    if (b->red) dev_free(b->red, b->red_cap * sizeof(double));
    pinned_release(b->hbuf, b->hbuf_cap); // the streams are idle: the upload is done
    (void)hipGetLastError();
    delete b;
}

// Enqueue the fused batch's device work from its kept schedule: arena
// init, whole circuits (stream 0), persistent circuits (stream 1), pass-major
// rounds (stream 2).  The streams must already be ordered after the upload.
// mark: record the per-class completion events (not inside a graph capture).
qs_status enqueue_fused(qs_batch b, bool mark)
{
    const qs_batch_s::Sched& S = b->sched;
    const int NS = (int)b->st.size();
    hipStream_t s0 = b->st[0], s1 = b->st[NS > 1 ? 1 : 0], sr = b->st[NS > 2 ? 2 : 0];
    auto launched = [&](hipError_t err, const char* what) -> qs_status {
        b->stats.launches += 1;
        if (err != hipSuccess) return bfail(b, err, what);
        return QS_OK;
    };
    auto mk = [&](int k, hipStream_t s) {
        if (!mark) return;
        if (!b->cls_done[k] && hipEventCreate(&b->cls_done[k]) != hipSuccess) return;
        (void)hipEventRecord(b->cls_done[k], s);
    };
    qs_status st = QS_OK;
    if (S.stream_count > 0 || !b->init_src.empty()) {
        // zero the arena and set the streamed circuits' basis amplitudes, then
        // copy the given initial states in, before any other stream reads or
        // writes a state there
        if (S.stream_count > 0) {
            hipError_t e = launch_batch_init(b->dt, b->arena, b->arena_bytes, S.dcirc, S.dlist + S.stream_l0,
                                             S.stream_count, s0);
            b->stats.launches += 2;
            if (e != hipSuccess) return bfail(b, e, "batch init launch");
        }
        for (const auto& is : b->init_src) {
            hipError_t e = hipMemcpyAsync(b->arena + b->off[is.first], is.second, amp_bytes(b->dt) << b->n[is.first],
                                          hipMemcpyDeviceToDevice, s0);
            if (e != hipSuccess) return bfail(b, e, "initial state copy");
        }
        hipEvent_t ev;
        if (hipEventCreate(&ev) == hipSuccess) {
            (void)hipEventRecord(ev, s0);
            (void)hipStreamWaitEvent(s1, ev, 0);
            (void)hipStreamWaitEvent(sr, ev, 0);
            (void)hipEventDestroy(ev);
        }
    }
    for (size_t gi = 0; gi < S.whole_groups.size(); ++gi) {
        const auto& g = S.whole_groups[gi];
        st = launched(launch_batch_whole(b->dt, g.first, b->arena, S.dcirc, S.dlist + g.second.first, g.second.second,
                                         S.dpass, S.dops, S.dmats, S.whole_var[gi], s0),
                      "batch whole launch");
        if (st != QS_OK) return st;
    }
    if (!S.whole_groups.empty()) mk(0, s0);
    if (S.persist_count > 0) {
        st = launched(launch_batch_persist(b->dt, S.persist_m, b->arena, S.dcirc, S.dlist + S.persist_l0,
                                           S.persist_count, S.dpass, S.dops, S.dmats, S.persist_var, s1),
                      "batch persistent launch");
        if (st != QS_OK) return st;
        mk(1, s1);
    }
    for (size_t r = 0; r < S.rounds.size(); ++r) {
        st = launched(launch_batch_round(b->dt, S.stream_m, b->arena, S.dcirc, S.dpass, S.dops, S.dmats,
                                         S.dents + S.rounds[r].first, S.rounds[r].second.first,
                                         S.rounds[r].second.second, S.round_var[r], sr),
                      "batch round launch");
        if (st != QS_OK) return st;
    }
    if (!S.rounds.empty()) mk(2, sr);
    return QS_OK;
}

// Capture enqueue_fused into a HIP graph (streams forked from and joined
// back to stream 0), keep it for replays, and launch it once.
qs_status capture_fused(qs_batch b)
{
    hipStream_t s0 = b->st[0];
    const int NS = (int)b->st.size();
    const int used = NS < 3 ? NS : 3;
    hipError_t e = hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return bfail(b, e, "hipStreamBeginCapture");
    std::vector<hipEvent_t> evs;
    auto ev = [&]() {
        hipEvent_t x = nullptr;
        if (hipEventCreateWithFlags(&x, hipEventDisableTiming) == hipSuccess) evs.push_back(x);
        return x;
    };
    hipEvent_t fork = ev();
    (void)hipEventRecord(fork, s0);
    for (int i = 1; i < used; ++i) (void)hipStreamWaitEvent(b->st[i], fork, 0);
    qs_status st = enqueue_fused(b, false);
    for (int i = 1; i < used; ++i) {
        hipEvent_t j = ev();
        (void)hipEventRecord(j, b->st[i]);
        (void)hipStreamWaitEvent(s0, j, 0);
    }
    e = hipStreamEndCapture(s0, &b->graph);
    for (hipEvent_t x : evs) (void)hipEventDestroy(x);
    if (st != QS_OK) return st;
    if (e != hipSuccess) return bfail(b, e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return bfail(b, e, "hipGraphInstantiate");
    e = hipGraphLaunch(b->gexec, s0);
    if (e != hipSuccess) return bfail(b, e, "hipGraphLaunch");
    return QS_OK;
}

int default_whole_max(int dt) { return dt == QS_C128 ? 12 : 13; } // 64 KiB of LDS
int default_persist_max(int dt) { return dt == QS_C128 ? 15 : 16; }

int whole_max(int dt, int opt)
{
    if (opt > 0) return opt;
    const int e = env_int("QS_BATCH_WHOLE_MAX", 0);
    return e > 0 ? e : default_whole_max(dt);
}

int persist_max(int dt, int opt)
{
    if (opt > 0) return opt;
    const int e = env_int("QS_BATCH_PERSIST_MAX", 0);
    return e > 0 ? e : default_persist_max(dt);
}

} // namespace

extern "C" {

qs_status qs_batch_submit(const qs_circuit* circuits, int count, const qs_batch_opts* opts, qs_batch* out)
{
    if (!out) return set_err(QS_ERR_ARG, "null output pointer");
    *out = nullptr;
    if (count < 0 || (count > 0 && !circuits)) return set_err(QS_ERR_ARG, "bad circuit list");
    qs_batch_opts o;
    std::memset(&o, 0, sizeof o);
    if (opts) o = *opts;
    if (o.dtype == 0) o.dtype = QS_C128;
    if (o.dtype != QS_C64 && o.dtype != QS_C128) return set_err(QS_ERR_ARG, "unknown dtype %d", o.dtype);
    if (o.mode != 0 && o.mode != 1) return set_err(QS_ERR_ARG, "unknown batch mode %d", o.mode);
    if (o.streams <= 0) o.streams = 8;
    if (o.streams > 64) return set_err(QS_ERR_ARG, "streams=%d > 64", o.streams);
    if (o.whole_max < 0 || o.whole_max > default_whole_max(o.dtype))
        return set_err(QS_ERR_ARG, "whole_max=%d outside [0, %d]", o.whole_max, default_whole_max(o.dtype));
    if (o.persist_max < 0 || o.persist_max > 20 || (o.persist_max > 0 && o.persist_max < o.whole_max))
        return set_err(QS_ERR_ARG, "persist_max=%d outside [whole_max, 20]", o.persist_max);
    for (int i = 0; i < count; ++i) {
        const qs_circuit& c = circuits[i];
        if (c.n < 1 || c.n > QS_MAX_QUBITS) return set_err(QS_ERR_ARG, "circuit %d: n=%d outside [1, %d]", i, c.n, QS_MAX_QUBITS);
        if (!c.init_state && c.init_basis >= (1ull << c.n))
            return set_err(QS_ERR_ARG, "circuit %d: basis state out of range", i);
        if (c.want < QS_WANT_NONE || c.want > QS_WANT_NORM) return set_err(QS_ERR_ARG, "circuit %d: want=%d", i, c.want);
        if (c.want != QS_WANT_NONE && !c.out) return set_err(QS_ERR_ARG, "circuit %d: want without an output", i);
        if (c.want == QS_WANT_PROBS && c.n > 24) return set_err(QS_ERR_ARG, "circuit %d: QS_WANT_PROBS needs n <= 24", i);
        qs_status st = validate_circuit(c.n, c.ops, c.n_ops, c.mats, c.n_mats);
        if (st != QS_OK) return set_err(st, "circuit %d: %s", i, qs_last_error());
    }
    if (qs_device_count() < 1) return set_err(QS_ERR_DEVICE, "no HIP device available");

    using clk = std::chrono::steady_clock;
    auto t_last = clk::now();
    auto phase = [&]() { // host milliseconds since the previous phase ended
        const auto t = clk::now();
        return std::chrono::duration<double, std::milli>(t - std::exchange(t_last, t)).count();
    };
    qs_batch b = new qs_batch_s();
    std::memset(&b->stats, 0, sizeof b->stats);
    b->dt = o.dtype;
    b->mode = o.mode;
    b->count = count;
    const uint64_t S = amp_bytes(b->dt);
    // arena layout
    uint64_t total = 0;
    for (int i = 0; i < count; ++i) {
        b->off.push_back(total);
        b->n.push_back(circuits[i].n);
        total += ((S << circuits[i].n) + 255) & ~255ull;
    }
    b->arena_bytes = total ? total : 256;
    qs_status st = dev_alloc((void**)&b->arena, b->arena_bytes, "batch arena");
    if (st != QS_OK) {
        release(b);
        return st;
    }
    for (int i = 0; i < o.streams; ++i) {
        hipStream_t s;
        hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e != hipSuccess) {
            qs_status r = bfail(b, e, "hipStreamCreate");
            release(b);
            return r;
        }
        b->st.push_back(s);
        hipEvent_t ev;
        e = hipEventCreate(&ev);
        if (e != hipSuccess) {
            qs_status r = bfail(b, e, "hipEventCreate");
            release(b);
            return r;
        }
        b->done.push_back(ev);
    }
    hipError_t e = hipEventCreate(&b->t0);
    if (e == hipSuccess) e = hipEventRecord(b->t0, b->st[0]);
    if (e != hipSuccess) {
        qs_status r = bfail(b, e, "hipEventRecord");
        release(b);
        return r;
    }
    for (size_t i = 1; i < b->st.size(); ++i) (void)hipStreamWaitEvent(b->st[i], b->t0, 0);

    b->stats.submit_ms[0] = phase();
    // ------------------------------------------------------------ plan
    enum { C_WHOLE = 0, C_PERSIST = 1, C_STREAM = 2 };
    std::vector<int> cls(count, C_STREAM);
    std::vector<BatchCirc> bc(count);
    int persist_m = 0, stream_m = 0;
    // classes and tile sizes first (the first circuit of a class fixes its
    // tile size), then the plans on host threads, then one concatenation
    std::vector<PlanOpts> popts(count);
    for (int i = 0; i < count; ++i) {
        const qs_circuit& c = circuits[i];
        std::memset(&bc[i], 0, sizeof(BatchCirc));
        bc[i].psi_off = b->off[i];
        bc[i].basis = c.init_state ? kLoadInitial : c.init_basis;
        bc[i].n = c.n;
        if (c.init_state) b->init_src.push_back({i, c.init_state});
        if (c.want != QS_WANT_NONE) b->wants.push_back({i, {c.want, c.out}});
        if (b->mode == 1) continue;
        PlanOpts& po = popts[i];
        st = plan_opts_for(b->dt, c.ops, c.n_ops, o.fuse_k, o.tile_qubits, po);
        if (st != QS_OK) {
            release(b);
            return st;
        }
        // a circuit smaller than its class's tile (possible when whole_max is
        // set below the tile size) runs whole in LDS: n < m <= 13 fits there
        const bool in_persist = c.n <= persist_max(b->dt, o.persist_max);
        const int class_m = in_persist ? (persist_m ? persist_m : std::min(po.m, 13))
                                       : (stream_m ? stream_m : std::min(po.m, 13));
        if (c.n <= whole_max(b->dt, o.whole_max) || c.n < class_m) {
            cls[i] = C_WHOLE;
            po.m = c.n;
        } else if (in_persist) {
            cls[i] = C_PERSIST;
            if (persist_m == 0) persist_m = std::min(po.m, 13);
            po.m = persist_m;
        } else {
            if (stream_m == 0) stream_m = std::min(po.m, 13);
            po.m = stream_m;
        }
    }
    std::vector<std::vector<PlanPass>> plans(b->mode == 0 ? count : 0);
    std::vector<std::vector<double>> pools(b->mode == 0 ? count : 0);
    if (b->mode == 0)
        parallel_for(count, [&](int i) {
            const qs_circuit& c = circuits[i];
            if (c.n_ops > 0) plan_circuit(c.n, c.ops, c.n_ops, c.mats, popts[i], plans[i], pools[i]);
        });
    b->stats.submit_ms[1] = phase();
    // Sizes first: each circuit's passes, ops and matrix pool get a fixed
    // place in the descriptor buffer, so host threads can fill it in parallel.
    std::vector<int64_t> pass0(count + 1, 0), opx0(count + 1, 0), mat0(count + 1, 0);
    for (int i = 0; i < count; ++i) {
        int64_t np = 0, no = 0, nm = 0;
        if (b->mode == 0) {
            np = (int64_t)plans[i].size();
            for (const PlanPass& p : plans[i]) no += (int64_t)p.ops.size();
            nm = (int64_t)pools[i].size();
        } else {
            nm = circuits[i].n_mats;
        }
        pass0[i + 1] = pass0[i] + np;
        opx0[i + 1] = opx0[i] + no;
        mat0[i + 1] = mat0[i] + ((nm + 1) & ~int64_t(1)); // keep 16-byte alignment
        bc[i].pass0 = (int)pass0[i];
        bc[i].npass = (int)np;
    }
    b->stats.passes = (uint64_t)pass0[count];
    // per-gate mode: dense k > 2 gates read their matrices from the pool
    std::vector<size_t> gate_pool_base(count, 0);
    if (b->mode == 1)
        for (int i = 0; i < count; ++i) gate_pool_base[i] = (size_t)mat0[i];
    // pass-major rounds over the streamed circuits: round r = pass r of each
    std::vector<RoundEntry> rents;
    std::vector<std::pair<size_t, std::pair<int, uint32_t>>> rounds; // (entry offset, (count, blocks))
    if (b->mode == 0) {
        int maxp = 0;
        for (int i = 0; i < count; ++i)
            if (cls[i] == C_STREAM) maxp = std::max(maxp, bc[i].npass);
        for (int r = 0; r < maxp; ++r) {
            const size_t e0 = rents.size();
            uint32_t blocks = 0;
            for (int i = 0; i < count; ++i) {
                if (cls[i] != C_STREAM || bc[i].npass <= r) continue;
                RoundEntry en;
                en.circ = i;
                en.pass = bc[i].pass0 + r;
                en.first_block = blocks;
                en.rsv = 0;
                rents.push_back(en);
                blocks += (uint32_t)(1u << (bc[i].n - stream_m));
            }
            rounds.push_back({e0, {(int)(rents.size() - e0), blocks}});
        }
    }
    std::vector<int32_t> lists;
    std::vector<std::pair<int, std::pair<size_t, int>>> whole_groups; // (n, (list offset, count))
    for (int nn = 1; nn <= 13; ++nn) {
        const size_t l0 = lists.size();
        for (int i = 0; i < count; ++i)
            if (cls[i] == C_WHOLE && bc[i].n == nn && b->mode == 0) lists.push_back(i);
        if (lists.size() > l0) whole_groups.push_back({nn, {l0, (int)(lists.size() - l0)}});
    }
    const size_t persist_l0 = lists.size();
    for (int i = 0; i < count; ++i)
        if (cls[i] == C_PERSIST && b->mode == 0) lists.push_back(i);
    const int persist_count = (int)(lists.size() - persist_l0);
    const size_t stream_l0 = lists.size();
    for (int i = 0; i < count; ++i)
        if (cls[i] == C_STREAM && b->mode == 0) lists.push_back(i);
    const int stream_count = (int)(lists.size() - stream_l0);

    // ------------------------------------------------------------ upload
    auto al = [](uint64_t x) { return (x + 255) & ~255ull; };
    const uint64_t o_circ = 0;
    const uint64_t o_pass = al(o_circ + bc.size() * sizeof(BatchCirc));
    const uint64_t o_ops = al(o_pass + (uint64_t)pass0[count] * sizeof(BatchPass));
    const uint64_t o_list = al(o_ops + (uint64_t)opx0[count] * sizeof(TileOp));
    const uint64_t o_ents = al(o_list + lists.size() * sizeof(int32_t));
    const uint64_t o_mats = al(o_ents + rents.size() * sizeof(RoundEntry));
    b->dbuf_bytes = al(o_mats + (uint64_t)mat0[count] * sizeof(double)) + 256;
    if ((st = dev_alloc((void**)&b->dbuf, b->dbuf_bytes, "batch descriptors")) != QS_OK) {
        release(b);
        return st;
    }
    if ((st = pinned_acquire(b->dbuf_bytes, &b->hbuf, &b->hbuf_cap)) != QS_OK) {
        release(b);
        return st;
    }
    std::vector<uint8_t> needs_var(count, 0);             // largest over the passes of circuit i
    std::vector<uint8_t> pass_var((size_t)pass0[count], 0); // per pass (global index)
    parallel_for(count, [&](int i) {
        double* M = (double*)(b->hbuf + o_mats) + mat0[i];
        if (b->mode == 1) {
            std::memcpy(M, circuits[i].mats, (size_t)circuits[i].n_mats * sizeof(double));
            return;
        }
        std::vector<PlanPass>& passes = plans[i];
        std::vector<double>& pool = pools[i];
        if (!pool.empty()) std::memcpy(M, pool.data(), pool.size() * sizeof(double));
        BatchPass* P = (BatchPass*)(b->hbuf + o_pass) + pass0[i];
        TileOp* T = (TileOp*)(b->hbuf + o_ops) + opx0[i];
        int64_t op = opx0[i];
        for (size_t j = 0; j < passes.size(); ++j) {
            const PlanPass& p = passes[j];
            BatchPass d;
            std::memset(&d, 0, sizeof d);
            d.m = p.m;
            d.L = p.L;
            uint64_t qm = 0;
            for (int k = 0; k < p.m; ++k) {
                d.q[k] = p.Q[k];
                qm |= 1ull << p.Q[k];
            }
            d.ip = make_insert_plan(qm);
            d.op0 = (int)op;
            d.nops = (int)p.ops.size();
            P[j] = d;
            for (TileOp t : p.ops) {
                t.moff += (uint64_t)mat0[i];
                *T++ = t;
            }
            const uint8_t v = (uint8_t)ops_variant(p.ops.data(), p.ops.size(), p.m);
            pass_var[(size_t)pass0[i] + j] = v;
            needs_var[i] = std::max(needs_var[i], v);
            op += (int64_t)p.ops.size();
        }
        std::vector<PlanPass>().swap(passes);
        std::vector<double>().swap(pool);
    });
    std::memcpy(b->hbuf + o_circ, bc.data(), bc.size() * sizeof(BatchCirc));
    std::memcpy(b->hbuf + o_list, lists.data(), lists.size() * sizeof(int32_t));
    std::memcpy(b->hbuf + o_ents, rents.data(), rents.size() * sizeof(RoundEntry));
    hipStream_t s0 = b->st[0];
    b->stats.submit_ms[2] = phase();
    e = hipMemcpyAsync(b->dbuf, b->hbuf, b->dbuf_bytes, hipMemcpyHostToDevice, s0);
    if (e != hipSuccess) {
        qs_status r = bfail(b, e, "batch upload");
        release(b);
        return r;
    }
    const BatchCirc* dcirc = (const BatchCirc*)(b->dbuf + o_circ);
    const BatchPass* dpass = (const BatchPass*)(b->dbuf + o_pass);
    const TileOp* dops = (const TileOp*)(b->dbuf + o_ops);
    const int32_t* dlist = (const int32_t*)(b->dbuf + o_list);
    const RoundEntry* dents = (const RoundEntry*)(b->dbuf + o_ents);
    const double* dmats = (const double*)(b->dbuf + o_mats);
    hipEvent_t up;
    (void)hipEventCreate(&up);
    (void)hipEventRecord(up, s0);
    for (size_t i = 1; i < b->st.size(); ++i) (void)hipStreamWaitEvent(b->st[i], up, 0);
    (void)hipEventDestroy(up);

    // ------------------------------------------------------------ launch
    auto launched = [&](hipError_t err, const char* what) -> qs_status {
        b->stats.launches += 1;
        if (err != hipSuccess) return bfail(b, err, what);
        return QS_OK;
    };
    const int NS = (int)b->st.size();
    if (b->mode == 0) {
        qs_batch_s::Sched& S = b->sched;
        S.whole_groups = whole_groups;
        S.persist_l0 = persist_l0;
        S.persist_count = persist_count;
        S.persist_m = persist_m;
        S.stream_l0 = stream_l0;
        S.stream_count = stream_count;
        S.stream_m = stream_m;
        S.rounds = rounds;
        S.whole_var.assign(whole_groups.size(), 0);
        for (size_t gi = 0; gi < whole_groups.size(); ++gi)
            for (int k = 0; k < whole_groups[gi].second.second; ++k)
                S.whole_var[gi] = std::max(S.whole_var[gi], needs_var[lists[whole_groups[gi].second.first + k]]);
        S.persist_var = 0;
        for (int k = 0; k < persist_count; ++k) S.persist_var = std::max(S.persist_var, (int)needs_var[lists[persist_l0 + k]]);
        S.round_var.assign(rounds.size(), 0);
        for (size_t r = 0; r < rounds.size(); ++r)
            for (int k = 0; k < rounds[r].second.first; ++k)
                S.round_var[r] = std::max(S.round_var[r], pass_var[(size_t)rents[rounds[r].first + k].pass]);
        S.dcirc = dcirc;
        S.dpass = dpass;
        S.dops = dops;
        S.dlist = dlist;
        S.dents = dents;
        S.dmats = dmats;
        for (int i = 0; i < count; ++i) b->stats.class_circuits[cls[i]] += 1;
        st = o.graph ? capture_fused(b) : enqueue_fused(b, true);
    } else {
        for (int i = 0; i < count && st == QS_OK; ++i) {
            const qs_circuit& c = circuits[i];
            hipStream_t s = b->st[i % NS];
            void* psi = b->arena + b->off[i];
            if (c.init_state)
                st = launched(hipMemcpyAsync(psi, c.init_state, amp_bytes(b->dt) << c.n, hipMemcpyDeviceToDevice, s),
                              "initial state copy");
            else
                st = launched(launch_init_basis(psi, b->dt, c.n, c.init_basis, s), "batch init launch");
            for (int64_t g = 0; g < c.n_ops && st == QS_OK; ++g) {
                const qs_op& op = c.ops[g];
                const double* U = c.mats + op.moff;
                int kind;
                hipError_t err;
                DiagPlan dp;
                if (diag_plan_matrix(c.n, op.t, op.nt, U, op.cmask, op.cvals, &dp)) {
                    if (dp.identity) continue;
                    err = launch_diag(psi, b->dt, dp, s);
                } else if (op.nt == 1)
                    err = launch_apply_1q(psi, b->dt, c.n, op.t[0], U, op.cmask, op.cvals, s, &kind);
                else if (op.nt == 2)
                    err = launch_apply_2q(psi, b->dt, c.n, op.t[0], op.t[1], U, op.cmask, op.cvals, s, &kind);
                else
                    err = launch_apply_kq_dev(psi, b->dt, c.n, op.t, op.nt, dmats + gate_pool_base[i] + op.moff,
                                              op.cmask, op.cvals, s, &kind);
                st = launched(err, "batch gate launch");
            }
        }
    }
    for (int i = 0; i < NS; ++i) {
        e = hipEventRecord(b->done[i], b->st[i]);
        if (e != hipSuccess && st == QS_OK) st = bfail(b, e, "hipEventRecord");
    }
    b->stats.submit_ms[3] = phase();
    if (st != QS_OK) {
        release(b);
        return st;
    }
    *out = b;
    return QS_OK;
}

} // extern "C"

namespace {

qs_status wait_done(qs_batch b, int timeout_ms);
qs_status download_one(qs_batch b, int i, void* host);
qs_status probs_one(qs_batch b, int i, const int* qubits, int m, double* out);

// The wanted results of a finished run, written once per run.
qs_status deliver(qs_batch b)
{
    if (b->delivered) return QS_OK;
    std::vector<int> all;
    for (const auto& w : b->wants) {
        const int i = w.first, want = w.second.first;
        void* out = w.second.second;
        qs_status st = QS_OK;
        if (want == QS_WANT_STATE) {
            st = download_one(b, i, out);
        } else if (want == QS_WANT_PROBS) {
            all.resize((size_t)b->n[i]);
            for (int q = 0; q < b->n[i]; ++q) all[(size_t)q] = q;
            st = probs_one(b, i, all.data(), b->n[i], (double*)out);
        } else if (want == QS_WANT_NORM) {
            st = probs_one(b, i, nullptr, 0, (double*)out);
        }
        if (st != QS_OK) return st;
    }
    b->delivered = true;
    return QS_OK;
}

} // namespace

extern "C" {

qs_status qs_batch_wait(qs_batch b, int timeout_ms)
{
    qs_status st = wait_done(b, timeout_ms);
    if (st != QS_OK) return st;
    return deliver(b);
}

} // extern "C"

namespace {

qs_status wait_done(qs_batch b, int timeout_ms)
{
    if (!b) return set_err(QS_ERR_ARG, "null batch handle");
    if (b->failed) return set_err(QS_ERR_DEVICE, "batch is in the failed state");
    const auto t_end = std::chrono::steady_clock::now() + std::chrono::milliseconds(timeout_ms < 0 ? 0 : timeout_ms);
    for (;;) {
        bool all = true;
        for (hipEvent_t ev : b->done) {
            hipError_t e = hipEventQuery(ev);
            if (e == hipErrorNotReady) {
                all = false;
                (void)hipGetLastError();
            } else if (e != hipSuccess) {
                return bfail(b, e, "batch execution");
            }
        }
        if (all) break;
        if (timeout_ms >= 0 && std::chrono::steady_clock::now() >= t_end)
            return set_err(QS_ERR_TIMEOUT, "batch not finished after %d ms", timeout_ms);
        std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
    float ms = 0.f, best = 0.f;
    for (hipEvent_t ev : b->done)
        if (hipEventElapsedTime(&ms, b->t0, ev) == hipSuccess && ms > best) best = ms;
    b->stats.device_ms = best;
    for (int k = 0; k < 3; ++k)
        if (b->cls_done[k] && hipEventElapsedTime(&ms, b->t0, b->cls_done[k]) == hipSuccess) b->stats.class_ms[k] = ms;
    return QS_OK;
}

qs_status download_one(qs_batch b, int i, void* host)
{
    hipError_t e = hipMemcpy(host, b->arena + b->off[i], amp_bytes(b->dt) << b->n[i], hipMemcpyDeviceToHost);
    if (e != hipSuccess) return bfail(b, e, "batch download");
    return QS_OK;
}

qs_status probs_one(qs_batch b, int i, const int* qubits, int m, double* out)
{
    const int n = b->n[i];
    const uint64_t need = reduce_scratch_doubles(n, m) + (1ull << m);
    qs_status st;
    if (need > b->red_cap) {
        if (b->red) dev_free(b->red, b->red_cap * sizeof(double));
        b->red = nullptr;
        b->red_cap = 0;
        if ((st = dev_alloc((void**)&b->red, need * sizeof(double), "batch reduction scratch")) != QS_OK) return st;
        b->red_cap = need;
    }
    double* dout = b->red + reduce_scratch_doubles(n, m);
    hipStream_t s0 = b->st[0];
    hipError_t e = launch_probabilities(b->arena + b->off[i], b->dt, n, qubits, m, b->red, dout, s0);
    if (e == hipSuccess) e = hipMemcpyAsync(out, dout, sizeof(double) << m, hipMemcpyDeviceToHost, s0);
    if (e == hipSuccess) e = hipStreamSynchronize(s0);
    if (e != hipSuccess) return bfail(b, e, "batch probabilities");
    return QS_OK;
}

} // namespace

extern "C" {

qs_status qs_batch_state(qs_batch b, int i, void** dev_ptr, int* n)
{
    if (!b) return set_err(QS_ERR_ARG, "null batch handle");
    if (i < 0 || i >= b->count) return set_err(QS_ERR_ARG, "circuit index %d outside [0, %d)", i, b->count);
    if (dev_ptr) *dev_ptr = b->arena + b->off[i];
    if (n) *n = b->n[i];
    return QS_OK;
}

qs_status qs_batch_download(qs_batch b, int i, void* host)
{
    if (!b) return set_err(QS_ERR_ARG, "null batch handle");
    if (i < 0 || i >= b->count) return set_err(QS_ERR_ARG, "circuit index %d outside [0, %d)", i, b->count);
    if (!host) return set_err(QS_ERR_ARG, "null host buffer");
    qs_status st = wait_done(b, -1);
    if (st != QS_OK) return st;
    return download_one(b, i, host);
}

qs_status qs_batch_probabilities(qs_batch b, int i, const int* qubits, int m, double* out)
{
    if (!b) return set_err(QS_ERR_ARG, "null batch handle");
    if (i < 0 || i >= b->count) return set_err(QS_ERR_ARG, "circuit index %d outside [0, %d)", i, b->count);
    if (!out) return set_err(QS_ERR_ARG, "null output");
    const int n = b->n[i];
    if (m < 0 || m > 24 || m > n) return set_err(QS_ERR_ARG, "m=%d outside [0, min(24, n)]", m);
    if (m > 0 && !qubits) return set_err(QS_ERR_ARG, "null qubit list");
    uint64_t seen = 0;
    for (int j = 0; j < m; ++j) {
        if (qubits[j] < 0 || qubits[j] >= n) return set_err(QS_ERR_ARG, "qubit %d outside [0, %d)", qubits[j], n);
        if ((seen >> qubits[j]) & 1) return set_err(QS_ERR_ARG, "duplicate qubit %d", qubits[j]);
        seen |= 1ull << qubits[j];
    }
    qs_status st = wait_done(b, -1);
    if (st != QS_OK) return st;
    return probs_one(b, i, qubits, m, out);
}

qs_status qs_batch_norm(qs_batch b, int i, double* out) { return qs_batch_probabilities(b, i, nullptr, 0, out); }

qs_status qs_batch_get_stats(qs_batch b, qs_batch_stats* out)
{
    if (!b || !out) return set_err(QS_ERR_ARG, "null argument");
    *out = b->stats;
    return QS_OK;
}

qs_status qs_batch_release(qs_batch b)
{
    release(b);
    return QS_OK;
}

} // extern "C"

qs_status qs_batch_replay(qs_batch b)
{
    if (!b) return set_err(QS_ERR_ARG, "null batch handle");
    if (b->mode != 0) return set_err(QS_ERR_UNSUPPORTED, "replay needs a fused (mode 0) batch");
    qs_status st = wait_done(b, -1);
    if (st != QS_OK) return st;
    b->delivered = false;
    hipStream_t s0 = b->st[0];
    hipError_t e = hipEventRecord(b->t0, s0);
    if (e != hipSuccess) return bfail(b, e, "hipEventRecord");
    for (size_t i = 1; i < b->st.size(); ++i) (void)hipStreamWaitEvent(b->st[i], b->t0, 0);
    if (b->gexec) {
        e = hipGraphLaunch(b->gexec, s0);
        if (e != hipSuccess) return bfail(b, e, "hipGraphLaunch");
    } else if ((st = enqueue_fused(b, true)) != QS_OK) {
        return st;
    }
    for (size_t i = 0; i < b->st.size(); ++i) {
        e = hipEventRecord(b->done[i], b->st[i]);
        if (e != hipSuccess) return bfail(b, e, "hipEventRecord");
    }
    return QS_OK;
}

qs_status qs_batch_tune(const qs_circuit* sample, int count, qs_batch_opts* opts, qs_tune_entry* out, int max_out,
                        int* n_out)
{
    if (!sample || count <= 0 || !opts) return set_err(QS_ERR_ARG, "empty sample or null options");
    if (opts->mode != 0) return set_err(QS_ERR_ARG, "tuning needs mode 0 (fused)");
    const int dt = opts->dtype == 0 ? QS_C128 : opts->dtype;
    const int w0 = default_whole_max(dt), p0 = default_persist_max(dt);
    struct Cand {
        int m, f, w, p;
    };
    double best = -1.0;
    Cand bc{0, 0, w0, p0};
    int k = 0;
    auto time_one = [&](const Cand& c) -> qs_status {
        qs_batch_opts o = *opts;
        o.tile_qubits = c.m;
        o.fuse_k = c.f;
        o.whole_max = c.w;
        o.persist_max = c.p;
        o.graph = 0;
        qs_batch b = nullptr;
        qs_status st = qs_batch_submit(sample, count, &o, &b);
        if (st != QS_OK) return st;
        double t = -1.0;
        for (int rep = 0; rep < 3 && st == QS_OK; ++rep) {
            if (rep > 0) st = qs_batch_replay(b);
            if (st == QS_OK) st = qs_batch_wait(b, -1);
            if (st == QS_OK && rep > 0 && (t < 0 || b->stats.device_ms < t)) t = b->stats.device_ms;
        }
        qs_batch_release(b);
        if (st != QS_OK) return st;
        if (out && k < max_out) out[k] = qs_tune_entry{c.m, c.f, c.w, c.p, t};
        ++k;
        if (best < 0 || t < best) {
            best = t;
            bc = c;
        }
        return QS_OK;
    };
    // stage 1: tile size and fused width at the default classes
    for (int m = 10; m <= 12; ++m)
        for (int f : {0, 4, 5}) {
            qs_status st = time_one(Cand{m, f, w0, p0});
            if (st != QS_OK) return st;
        }
    // stage 2: workgroup classes around the defaults, at the best stage-1 setting
    const Cand s1 = bc;
    const Cand stage2[] = {{s1.m, s1.f, w0 - 1, p0}, {s1.m, s1.f, w0, p0 - 2}, {s1.m, s1.f, w0, p0 - 1},
                           {s1.m, s1.f, w0, p0 + 1}, {s1.m, s1.f, w0, p0 + 2}};
    for (const Cand& c : stage2) {
        qs_status st = time_one(c);
        if (st != QS_OK) return st;
    }
    opts->tile_qubits = bc.m;
    opts->fuse_k = bc.f;
    opts->whole_max = bc.w;
    opts->persist_max = bc.p;
    if (n_out) *n_out = k;
    return QS_OK;
}
