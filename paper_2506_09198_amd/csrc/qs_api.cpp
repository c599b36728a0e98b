// C ABI of the gate engine: handle lifetime, argument validation, stream
// ordering, matrix staging, tracing and error reporting.  Kernels live in the
// *.hip translation units; circuit planning in planner.cpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "qs_internal.h"
#include "runtime.h"

namespace qs {

int env_int(const char* name, int dflt)
{
    const char* v = std::getenv(name);
    if (!v || !*v) return dflt;
    return std::atoi(v);
}

static thread_local std::string g_err;

qs_status set_err(qs_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

// ------------------------------------------------------------ HBM budget

static std::atomic<uint64_t> g_allocated{0};

static uint64_t budget_bytes()
{
    const char* v = std::getenv("QS_HBM_BUDGET");
    if (!v || !*v) return ~0ull;
    return std::strtoull(v, nullptr, 10);
}

uint64_t allocated_bytes() { return g_allocated.load(); }

qs_status dev_alloc(void** p, uint64_t bytes, const char* what)
{
    const uint64_t cur = g_allocated.load();
    if (cur + bytes > budget_bytes())
        return set_err(QS_ERR_OOM, "%s: %llu bytes exceed the QS_HBM_BUDGET (%llu in use)", what,
                       (unsigned long long)bytes, (unsigned long long)cur);
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return set_err(QS_ERR_OOM, "%s: hipMalloc(%llu) failed: %s", what, (unsigned long long)bytes,
                       hipGetErrorString(e));
    }
    g_allocated += bytes;
    return QS_OK;
}

void dev_free(void* p, uint64_t bytes)
{
    if (!p) return;
    (void)hipFree(p);
    g_allocated -= bytes;
}

// ------------------------------------------------------------ fault injection

// QS_FAULT_INJECT=launch:N makes the N-th traced launch (1-based, counted over
// the process) report a device error, so failure handling can be exercised
// without a real GPU fault.
static std::atomic<long> g_launch_no{0};

bool inject_fault_now()
{
    static long target = [] {
        const char* v = std::getenv("QS_FAULT_INJECT");
        if (!v || std::strncmp(v, "launch:", 7) != 0) return -1L;
        return std::atol(v + 7);
    }();
    const long k = ++g_launch_no;
    return target > 0 && k == target;
}

// ------------------------------------------------------------ state helpers

qs_status fail_device(qs_state s, hipError_t e, const char* what)
{
    if (s) s->failed = true;
    (void)hipGetLastError();
    return set_err(QS_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

qs_status check_live(qs_state s)
{
    if (!s) return set_err(QS_ERR_ARG, "null state handle");
    if (s->failed) return set_err(QS_ERR_DEVICE, "state handle is in the failed state");
    int cur = -1;
    if (hipGetDevice(&cur) == hipSuccess && cur != s->dev) {
        hipError_t e = hipSetDevice(s->dev);
        if (e != hipSuccess) return fail_device(s, e, "hipSetDevice");
    }
    return QS_OK;
}

// Run `fn` (which enqueues one kernel launch and reports its class) with
// optional HIP-event timing on the state's stream.
qs_status traced_launch(qs_state s, qs_trace_rec rec, const std::function<hipError_t(int*)>& fn,
                        const char* what)
{
    if (inject_fault_now()) {
        s->failed = true;
        return set_err(QS_ERR_DEVICE, "%s: injected device fault (QS_FAULT_INJECT)", what);
    }
    hipEvent_t a = nullptr, b = nullptr;
    if (s->tracing) {
        if (s->ev_pool.size() < s->ev_used + 2) {
            hipEvent_t e1, e2;
            if (hipEventCreate(&e1) != hipSuccess || hipEventCreate(&e2) != hipSuccess)
                return fail_device(s, hipErrorOutOfMemory, "hipEventCreate");
            s->ev_pool.push_back(e1);
            s->ev_pool.push_back(e2);
        }
        a = s->ev_pool[s->ev_used++];
        b = s->ev_pool[s->ev_used++];
        hipError_t e = hipEventRecord(a, s->st);
        if (e != hipSuccess) return fail_device(s, e, "hipEventRecord");
    }
    int kind = -1;
    hipError_t e = fn(&kind);
    if (e != hipSuccess) return fail_device(s, e, what);
    if (s->tracing) {
        e = hipEventRecord(b, s->st);
        if (e != hipSuccess) return fail_device(s, e, "hipEventRecord");
        rec.kind = kind;
        s->trace.push_back({rec, a, b});
    }
    return QS_OK;
}

// Staging ring for small per-call device data (matrices, op tables): one
// device buffer with a pinned host mirror.  Regions are handed out in order;
// before the ring wraps (or grows) the stream is drained, so no queued kernel
// or copy can still be reading a region that is about to be rewritten.
static qs_status stage_reserve(qs_state s, uint64_t bytes, char** host, char** dev)
{
    bytes = (bytes + 255) & ~255ull;
    if (bytes > s->mat_cap) {
        hipError_t e = hipStreamSynchronize(s->st);
        if (e != hipSuccess) return fail_device(s, e, "hipStreamSynchronize");
        if (s->mat_dev) dev_free(s->mat_dev, s->mat_cap);
        if (s->mat_host) (void)hipHostFree(s->mat_host);
        s->mat_dev = nullptr;
        s->mat_host = nullptr;
        s->mat_cap = 0;
        uint64_t cap = 1ull << 20;
        while (cap < 2 * bytes) cap <<= 1;
        qs_status st = dev_alloc((void**)&s->mat_dev, cap, "staging ring");
        if (st != QS_OK) return st;
        e = hipHostMalloc((void**)&s->mat_host, cap, hipHostMallocDefault);
        if (e != hipSuccess) {
            dev_free(s->mat_dev, cap);
            s->mat_dev = nullptr;
            (void)hipGetLastError();
            return set_err(QS_ERR_OOM, "hipHostMalloc(%llu) failed", (unsigned long long)cap);
        }
        s->mat_cap = cap;
        s->mat_off = 0;
    }
    if (s->mat_off + bytes > s->mat_cap) {
        hipError_t e = hipStreamSynchronize(s->st);
        if (e != hipSuccess) return fail_device(s, e, "hipStreamSynchronize");
        s->mat_off = 0;
    }
    *host = s->mat_host + s->mat_off;
    *dev = s->mat_dev + s->mat_off;
    s->mat_off += bytes;
    return QS_OK;
}

qs_status stage_bytes(qs_state s, const void* src, uint64_t bytes, const void** dev_out)
{
    char *h = nullptr, *d = nullptr;
    qs_status st = stage_reserve(s, bytes, &h, &d);
    if (st != QS_OK) return st;
    std::memcpy(h, src, bytes);
    hipError_t e = hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, s->st);
    if (e != hipSuccess) return fail_device(s, e, "hipMemcpyAsync(staging)");
    *dev_out = d;
    return QS_OK;
}

// Stage `count` doubles of matrix data converted to the state's real type.
qs_status stage_matrices(qs_state s, const double* src, uint64_t count, const void** dev_out)
{
    const size_t es = s->dt == QS_C128 ? sizeof(double) : sizeof(float);
    char *h = nullptr, *d = nullptr;
    qs_status st = stage_reserve(s, count * es, &h, &d);
    if (st != QS_OK) return st;
    if (s->dt == QS_C128) {
        std::memcpy(h, src, count * sizeof(double));
    } else {
        float* f = (float*)h;
        for (uint64_t i = 0; i < count; ++i) f[i] = (float)src[i];
    }
    hipError_t e = hipMemcpyAsync(d, h, count * es, hipMemcpyHostToDevice, s->st);
    if (e != hipSuccess) return fail_device(s, e, "hipMemcpyAsync(matrix)");
    *dev_out = d;
    return QS_OK;
}

static uint64_t qubit_mask_ok(int n) { return n >= 64 ? ~0ull : ((1ull << n) - 1); }

qs_status validate_gate(int n, const int* t, int k, uint64_t cm, uint64_t cv)
{
    if (k < 1 || k > QS_MAX_FUSED) return set_err(QS_ERR_ARG, "target count %d outside [1, %d]", k, QS_MAX_FUSED);
    uint64_t tm = 0;
    for (int j = 0; j < k; ++j) {
        if (t[j] < 0 || t[j] >= n) return set_err(QS_ERR_ARG, "target %d outside [0, %d)", t[j], n);
        if ((tm >> t[j]) & 1) return set_err(QS_ERR_ARG, "duplicate target %d", t[j]);
        tm |= 1ull << t[j];
    }
    if (cm & ~qubit_mask_ok(n)) return set_err(QS_ERR_ARG, "control mask has qubits >= n=%d", n);
    if (cm & tm) return set_err(QS_ERR_ARG, "a target is also a control");
    if (cv & ~cm) return set_err(QS_ERR_ARG, "ctrl_vals has bits outside ctrl_mask");
    return QS_OK;
}

// With QS_CHECK_UNITARY=1 every gate matrix must satisfy max |(U^H U - I)_ij|
// <= 1e-10.  The switch is read once per API call (so a process can turn it
// on and off), the check itself is unconditional.
bool check_unitary_enabled() { return env_int("QS_CHECK_UNITARY", 0) != 0; }

qs_status check_unitary(const double* U, int k)
{
    const int D = 1 << k;
    double worst = 0.0;
    for (int i = 0; i < D; ++i)
        for (int j = 0; j < D; ++j) {
            double re = (i == j) ? -1.0 : 0.0, im = 0.0;
            for (int r = 0; r < D; ++r) { // (U^H U)_ij = sum_r conj(U_ri) U_rj
                const double ar = U[2 * (r * D + i)], ai = U[2 * (r * D + i) + 1];
                const double br = U[2 * (r * D + j)], bi = U[2 * (r * D + j) + 1];
                re += ar * br + ai * bi;
                im += ar * bi - ai * br;
            }
            worst = std::max(worst, std::hypot(re, im));
        }
    if (!(worst <= 1e-10)) return set_err(QS_ERR_ARG, "matrix is not unitary (max |U^H U - I| = %.3g)", worst);
    return QS_OK;
}

static qs_trace_rec make_rec(qs_state s, int t0, int t1, uint64_t cm)
{
    qs_trace_rec r;
    std::memset(&r, 0, sizeof r);
    r.n = s->n;
    r.t0 = t0;
    r.t1 = t1;
    r.nctrl = __builtin_popcountll(cm);
    r.dtype = s->dt;
    r.updates = 1ull << (s->n - r.nctrl);
    r.bytes = 2ull * amp_bytes(s->dt) * r.updates;
    return r;
}

qs_status apply_diag_internal(qs_state s, const DiagPlan& p, int t0, int t1, uint64_t cm)
{
    if (p.identity) return QS_OK;
    qs_trace_rec rec = make_rec(s, t0, t1, cm);
    rec.updates = diag_changed(p);
    rec.bytes = 2ull * amp_bytes(s->dt) * rec.updates;
    return traced_launch(
        s, rec,
        [&](int* kind) {
            *kind = QS_K_DIAG;
            return launch_diag(s->d, s->dt, p, s->st);
        },
        "diagonal gate launch");
}

qs_status apply_1q_internal(qs_state s, int target, const double* U, uint64_t cm, uint64_t cv)
{
    DiagPlan p;
    if (diag_plan_matrix(s->n, &target, 1, U, cm, cv, &p)) return apply_diag_internal(s, p, target, -1, cm);
    return traced_launch(
        s, make_rec(s, target, -1, cm),
        [&](int* kind) { return launch_apply_1q(s->d, s->dt, s->n, target, U, cm, cv, s->st, kind); },
        "apply_1q launch");
}

qs_status apply_2q_internal(qs_state s, int t0, int t1, const double* U, uint64_t cm, uint64_t cv)
{
    DiagPlan p;
    const int t[2] = {t0, t1};
    if (diag_plan_matrix(s->n, t, 2, U, cm, cv, &p)) return apply_diag_internal(s, p, t0, t1, cm);
    return traced_launch(
        s, make_rec(s, t0, t1, cm),
        [&](int* kind) { return launch_apply_2q(s->d, s->dt, s->n, t0, t1, U, cm, cv, s->st, kind); },
        "apply_2q launch");
}

qs_status apply_kq_dev_internal(qs_state s, const int* t, int k, const void* Ud, uint64_t cm, uint64_t cv)
{
    return traced_launch(
        s, make_rec(s, t[0], k > 1 ? t[1] : -1, cm),
        [&](int* kind) { return launch_apply_kq_dev(s->d, s->dt, s->n, t, k, Ud, cm, cv, s->st, kind); },
        "apply_fused launch");
}

} // namespace qs

using namespace qs;

// =================================================================== ABI

extern "C" {

int qs_version(void) { return (0 << 16) | 1; }

const char* qs_last_error(void) { return g_err.c_str(); }

int qs_device_count(void)
{
    int c = 0;
    if (hipGetDeviceCount(&c) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return c;
}

// Look up the no-allocation scratch of the state's device once, when a state
// is first created there, so that qs_probabilities_noalloc finds it resolved.
// A failure here is not the new state's: the entry point retries and reports.
static void resolve_noalloc_scratch(int dev)
{
    double* p = nullptr;
    uint64_t c = 0;
    if (noalloc_scratch(dev, &p, &c) != hipSuccess) (void)hipGetLastError();
}

static qs_status new_state(int n, qs_dtype dt, qs_state* out)
{
    if (!out) return set_err(QS_ERR_ARG, "null output pointer");
    *out = nullptr;
    if (n < 1 || n > QS_MAX_QUBITS) return set_err(QS_ERR_ARG, "n=%d outside [1, %d]", n, QS_MAX_QUBITS);
    if (dt != QS_C64 && dt != QS_C128) return set_err(QS_ERR_ARG, "unknown dtype %d", (int)dt);
    if (qs_device_count() < 1) return set_err(QS_ERR_DEVICE, "no HIP device available");
    return QS_OK;
}

qs_status qs_create(int n, qs_dtype dt, qs_state* out)
{
    qs_status st = new_state(n, dt, out);
    if (st != QS_OK) return st;
    qs_state s = new qs_state_s();
    s->n = n;
    s->dt = dt;
    s->bytes = (1ull << n) * amp_bytes(dt);
    (void)hipGetDevice(&s->dev);
    resolve_noalloc_scratch(s->dev);
    st = dev_alloc(&s->d, s->bytes, "state");
    if (st != QS_OK) {
        delete s;
        return st;
    }
    s->owned = true;
    hipError_t e = hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking);
    if (e != hipSuccess) {
        dev_free(s->d, s->bytes);
        delete s;
        (void)hipGetLastError();
        return set_err(QS_ERR_DEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
    }
    s->own_stream = true;
    st = traced_launch(s, make_rec(s, -1, -1, 0),
                       [&](int* kind) {
                           *kind = QS_K_INIT;
                           return launch_init_basis(s->d, s->dt, s->n, 0, s->st);
                       },
                       "init launch");
    if (st != QS_OK) {
        qs_destroy(s);
        return st;
    }
    *out = s;
    return QS_OK;
}

qs_status qs_create_external(int n, qs_dtype dt, void* dev_ptr, uint64_t bytes, void* stream, qs_state* out)
{
    qs_status st = new_state(n, dt, out);
    if (st != QS_OK) return st;
    const uint64_t need = (1ull << n) * amp_bytes(dt);
    if (!dev_ptr) return set_err(QS_ERR_ARG, "null device pointer");
    if (bytes < need) return set_err(QS_ERR_ARG, "buffer of %llu bytes < %llu needed", (unsigned long long)bytes,
                                     (unsigned long long)need);
    if (((uintptr_t)dev_ptr) & 255) return set_err(QS_ERR_ARG, "device pointer not 256-byte aligned");
    qs_state s = new qs_state_s();
    s->n = n;
    s->dt = dt;
    s->bytes = need;
    s->d = dev_ptr;
    s->owned = false;
    s->st = (hipStream_t)stream;
    s->own_stream = false;
    (void)hipGetDevice(&s->dev);
    resolve_noalloc_scratch(s->dev);
    *out = s;
    return QS_OK;
}

qs_status qs_destroy(qs_state s)
{
    if (!s) return QS_OK;
    if (!s->failed) (void)hipStreamSynchronize(s->st);
    for (hipEvent_t e : s->ev_pool) (void)hipEventDestroy(e);
    if (s->red_part) dev_free(s->red_part, s->red_cap * sizeof(double));
    if (s->mat_dev) dev_free(s->mat_dev, s->mat_cap);
    if (s->mat_host) (void)hipHostFree(s->mat_host);
    if (s->red_host) (void)hipHostFree(s->red_host);
    if (s->owned) dev_free(s->d, s->bytes);
    if (s->own_stream) (void)hipStreamDestroy(s->st);
    (void)hipGetLastError();
    delete s;
    return QS_OK;
}

qs_status qs_set_stream(qs_state s, void* stream)
{
    qs_status st = check_live(s);
    if (st != QS_OK) return st;
    hipError_t e = hipStreamSynchronize(s->st);
    if (e != hipSuccess) return fail_device(s, e, "hipStreamSynchronize");
    if (s->own_stream) (void)hipStreamDestroy(s->st);
    s->st = (hipStream_t)stream;
    s->own_stream = false;
    return QS_OK;
}

qs_status qs_get_info(qs_state s, int* n, int* dtype, void** dev_ptr)
{
    if (!s) return set_err(QS_ERR_ARG, "null state handle");
    if (n) *n = s->n;
    if (dtype) *dtype = s->dt;
    if (dev_ptr) *dev_ptr = s->d;
    return QS_OK;
}

qs_status qs_init_basis(qs_state s, uint64_t x)
{
    qs_status st = check_live(s);
    if (st != QS_OK) return st;
    if (x >= (1ull << s->n)) return set_err(QS_ERR_ARG, "basis index %llu >= 2^%d", (unsigned long long)x, s->n);
    return traced_launch(s, make_rec(s, -1, -1, 0),
                         [&](int* kind) {
                             *kind = QS_K_INIT;
                             return launch_init_basis(s->d, s->dt, s->n, x, s->st);
                         },
                         "init launch");
}

static qs_status range_ok(qs_state s, const void* host, uint64_t first, uint64_t count)
{
    if (!host && count) return set_err(QS_ERR_ARG, "null host buffer");
    const uint64_t N = 1ull << s->n;
    if (first > N || count > N - first) return set_err(QS_ERR_ARG, "amplitude range out of bounds");
    return QS_OK;
}

qs_status qs_upload(qs_state s, const void* host, uint64_t first, uint64_t count)
{
    qs_status st = check_live(s);
    if (st != QS_OK) return st;
    if ((st = range_ok(s, host, first, count)) != QS_OK) return st;
    const size_t es = amp_bytes(s->dt);
    hipError_t e = hipMemcpyAsync((char*)s->d + first * es, host, count * es, hipMemcpyHostToDevice, s->st);
    if (e == hipSuccess) e = hipStreamSynchronize(s->st);
    if (e != hipSuccess) return fail_device(s, e, "upload");
    return QS_OK;
}

qs_status qs_download(qs_state s, void* host, uint64_t first, uint64_t count)
{
    qs_status st = check_live(s);
    if (st != QS_OK) return st;
    if ((st = range_ok(s, host, first, count)) != QS_OK) return st;
    const size_t es = amp_bytes(s->dt);
    hipError_t e = hipMemcpyAsync(host, (const char*)s->d + first * es, count * es, hipMemcpyDeviceToHost, s->st);
    if (e == hipSuccess) e = hipStreamSynchronize(s->st);
    if (e != hipSuccess) return fail_device(s, e, "download");
    return QS_OK;
}

qs_status qs_apply_1q(qs_state s, int target, const double* U, uint64_t cm, uint64_t cv)
{
    qs_status st = check_live(s);
    if (st != QS_OK) return st;
    if (!U) return set_err(QS_ERR_ARG, "null matrix");
    if ((st = validate_gate(s->n, &target, 1, cm, cv)) != QS_OK) return st;
    if (check_unitary_enabled() && (st = check_unitary(U, 1)) != QS_OK) return st;
    return apply_1q_internal(s, target, U, cm, cv);
}

qs_status qs_apply_2q(qs_state s, int t0, int t1, const double* U, uint64_t cm, uint64_t cv)
{
    qs_status st = check_live(s);
    if (st != QS_OK) return st;
    if (!U) return set_err(QS_ERR_ARG, "null matrix");
    const int t[2] = {t0, t1};
    if ((st = validate_gate(s->n, t, 2, cm, cv)) != QS_OK) return st;
    if (check_unitary_enabled() && (st = check_unitary(U, 2)) != QS_OK) return st;
    return apply_2q_internal(s, t0, t1, U, cm, cv);
}

qs_status qs_apply_fused(qs_state s, const int* targets, int k, const double* U, uint64_t cm, uint64_t cv)
{
    qs_status st = check_live(s);
    if (st != QS_OK) return st;
    if (!U || !targets) return set_err(QS_ERR_ARG, "null matrix or target list");
    if ((st = validate_gate(s->n, targets, k, cm, cv)) != QS_OK) return st;
    if (check_unitary_enabled() && (st = check_unitary(U, k)) != QS_OK) return st;
    DiagPlan p;
    if (diag_plan_matrix(s->n, targets, k, U, cm, cv, &p))
        return apply_diag_internal(s, p, targets[0], k > 1 ? targets[1] : -1, cm);
    const void* Ud = nullptr;
    if ((st = stage_bytes(s, U, (2ull << (2 * k)) * sizeof(double), &Ud)) != QS_OK) return st;
    return apply_kq_dev_internal(s, targets, k, Ud, cm, cv);
}

qs_status qs_apply_diag(qs_state s, const int* targets, int k, const double* diag, uint64_t cm, uint64_t cv)
{
    qs_status st = check_live(s);
    if (st != QS_OK) return st;
    if (!diag || !targets) return set_err(QS_ERR_ARG, "null diagonal or target list");
    if ((st = validate_gate(s->n, targets, k, cm, cv)) != QS_OK) return st;
    for (int j = 0; j < (2 << k); ++j)
        if (!std::isfinite(diag[j])) return set_err(QS_ERR_ARG, "diagonal entry %d is not finite", j / 2);
    if (check_unitary_enabled())
        for (int j = 0; j < (1 << k); ++j)
            if (!(std::fabs(std::hypot(diag[2 * j], diag[2 * j + 1]) - 1.0) <= 1e-10))
                return set_err(QS_ERR_ARG, "diagonal entry %d does not have modulus 1", j);
    DiagPlan p;
    if (!diag_plan(s->n, targets, k, diag, cm, cv, &p)) return set_err(QS_ERR_ARG, "k=%d not supported", k);
    return apply_diag_internal(s, p, targets[0], k > 1 ? targets[1] : -1, cm);
}

static qs_status check_measured(qs_state s, const int* qubits, int m)
{
    if (m < 0 || m > 24 || m > s->n) return set_err(QS_ERR_ARG, "m=%d outside [0, min(24, n)]", m);
    if (m > 0 && !qubits) return set_err(QS_ERR_ARG, "null qubit list");
    uint64_t seen = 0;
    for (int j = 0; j < m; ++j) {
        if (qubits[j] < 0 || qubits[j] >= s->n) return set_err(QS_ERR_ARG, "qubit %d outside [0, %d)", qubits[j], s->n);
        if ((seen >> qubits[j]) & 1) return set_err(QS_ERR_ARG, "duplicate qubit %d", qubits[j]);
        seen |= 1ull << qubits[j];
    }
    return QS_OK;
}

qs_status qs_probabilities(qs_state s, const int* qubits, int m, double* out)
{
    qs_status st = check_live(s);
    if (st != QS_OK) return st;
    if (!out) return set_err(QS_ERR_ARG, "null output");
    if ((st = check_measured(s, qubits, m)) != QS_OK) return st;
    const uint64_t need = reduce_scratch_doubles(s->n, m) + (1ull << m);
    if (need > s->red_cap) {
        hipError_t e = hipStreamSynchronize(s->st);
        if (e != hipSuccess) return fail_device(s, e, "hipStreamSynchronize");
        if (s->red_part) dev_free(s->red_part, s->red_cap * sizeof(double));
        s->red_part = nullptr;
        s->red_cap = 0;
        if ((st = dev_alloc((void**)&s->red_part, need * sizeof(double), "reduction scratch")) != QS_OK) return st;
        s->red_cap = need;
    }
    double* part = s->red_part;
    double* dout = s->red_part + reduce_scratch_doubles(s->n, m);
    qs_trace_rec rec = make_rec(s, -1, -1, 0);
    rec.bytes = (1ull << s->n) * amp_bytes(s->dt);
    st = traced_launch(s, rec,
                       [&](int* kind) {
                           *kind = QS_K_REDUCE;
                           return launch_probabilities(s->d, s->dt, s->n, qubits, m, part, dout, s->st);
                       },
                       "probabilities launch");
    if (st != QS_OK) return st;
    hipError_t e = hipMemcpyAsync(out, dout, sizeof(double) << m, hipMemcpyDeviceToHost, s->st);
    if (e == hipSuccess) e = hipStreamSynchronize(s->st);
    if (e != hipSuccess) return fail_device(s, e, "probabilities download");
    return QS_OK;
}

qs_status qs_norm(qs_state s, double* out) { return qs_probabilities(s, nullptr, 0, out); }

qs_status qs_probabilities_noalloc(qs_state s, const int* qubits, int m, double* dev_out)
{
    qs_status st = check_live(s);
    if (st != QS_OK) return st;
    if (!dev_out) return set_err(QS_ERR_ARG, "null device output");
    if ((st = check_measured(s, qubits, m)) != QS_OK) return st;
    double* part = nullptr;
    uint64_t cap = 0;
    const hipError_t e0 = noalloc_scratch(s->dev, &part, &cap);
    if (e0 != hipSuccess) {
        (void)hipGetLastError();
        return set_err(QS_ERR_DEVICE, "no-allocation scratch lookup: %s", hipGetErrorString(e0));
    }
    const uint64_t need = reduce_scratch_doubles(s->n, m);
    if (need > cap)
        return set_err(QS_ERR_ARG, "n=%d, m=%d needs %llu doubles of scratch; the fixed scratch holds %llu", s->n, m,
                       (unsigned long long)need, (unsigned long long)cap);
    const hipError_t e = launch_probabilities(s->d, s->dt, s->n, qubits, m, part, dev_out, s->st);
    if (e != hipSuccess) return fail_device(s, e, "probabilities launch");
    return QS_OK;
}

qs_status qs_sync(qs_state s)
{
    qs_status st = check_live(s);
    if (st != QS_OK) return st;
    hipError_t e = hipStreamSynchronize(s->st);
    if (e != hipSuccess) return fail_device(s, e, "hipStreamSynchronize");
    return QS_OK;
}

qs_status qs_probe_inplace(qs_state s, int slots, int spread_log2)
{
    qs_status st = check_live(s);
    if (st != QS_OK) return st;
    if (slots != 1 && slots != 2 && slots != 4 && slots != 8)
        return set_err(QS_ERR_ARG, "slots=%d: expected 1, 2, 4 or 8", slots);
    if (spread_log2 < 8 || spread_log2 > 30) return set_err(QS_ERR_ARG, "spread_log2=%d outside [8, 30]", spread_log2);
    if (s->bytes % 16) return set_err(QS_ERR_ARG, "state of %llu bytes is not whole 16-byte words",
                                      (unsigned long long)s->bytes);
    qs_trace_rec rec = make_rec(s, -1, -1, 0);
    rec.bytes = 2 * s->bytes;
    rec.updates = 0;
    return traced_launch(
        s, rec,
        [&](int* kind) {
            *kind = QS_K_PROBE;
            return launch_probe_inplace(s->d, s->bytes, slots, spread_log2, 0, s->st);
        },
        "probe launch");
}

qs_status qs_trace_enable(qs_state s, int on)
{
    if (!s) return set_err(QS_ERR_ARG, "null state handle");
    if (!s->failed) (void)hipStreamSynchronize(s->st);
    s->trace.clear();
    s->ev_used = 0;
    s->tracing = on != 0;
    return QS_OK;
}

qs_status qs_trace_read(qs_state s, qs_trace_rec* out, int max, int* count)
{
    qs_status st = check_live(s);
    if (st != QS_OK) return st;
    if (!count || (max > 0 && !out)) return set_err(QS_ERR_ARG, "null output");
    hipError_t e = hipStreamSynchronize(s->st);
    if (e != hipSuccess) return fail_device(s, e, "hipStreamSynchronize");
    int c = 0;
    for (auto& it : s->trace) {
        if (c >= max) break;
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, it.a, it.b);
        if (e != hipSuccess) return fail_device(s, e, "hipEventElapsedTime");
        out[c] = it.rec;
        out[c].ms = ms;
        ++c;
    }
    *count = c;
    return QS_OK;
}

} // extern "C"
