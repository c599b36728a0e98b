// Run-time launch knobs: grid caps of the looping kernels, the per-gate
// memory schedule, restore-pass run length.  Each knob starts at its default,
// or at the value of its environment variable when that is set (read once, on
// first use), and can be changed at any time with qs_tunable_set; values are
// atomics, so a change from one thread is seen by launches on others (a launch
// already being set up may still use the old value).
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <utility>

#include "qs_internal.h"
#include "runtime.h"

namespace qs {

namespace {

struct TunDef {
    const char* name;
    const char* env;
    int64_t dflt;
    int64_t lo, hi;
};

// Order matches the Tun enum in qs_internal.h.
const TunDef kTun[T_COUNT] = {
    {"gate_grid_cap", "QS_GATE_GRID_CAP", 1 << 22, 1, 1 << 22},
    {"tile_grid_cap", "QS_TILE_GRID_CAP", 65536, 1, 1 << 22},
    {"round_grid_cap", "QS_ROUND_GRID_CAP", 65536, 1, 1 << 22},
    {"aux_grid_cap", "QS_GRID_CAP", 256 * 64, 1, 1 << 22},
    {"nontemporal", "QS_NT", 1, 0, 1},
    {"slot_spread_log2", "QS_SLOG", 11, 8, 16},
    {"slots_no_high", "QS_PPL_H0", 0, 0, 8},
    {"slots_one_high", "QS_PPL_H1", 0, 0, 8},
    {"slots_two_high", "QS_PPL_H2", 0, 0, 8},
    {"diag_spread_log2", "QS_DIAG_SLOG", 11, 8, 16},
    {"perm_run_log2", "QS_PERM_RUN", 0, 0, 6},
    {"gate_xcd_swizzle", "QS_GATE_XCD", 0, 0, 2},
    {"gate_wg_per_cu", "QS_GATE_WG_PER_CU", 0, 0, 32},
    {"gate_low_in_regs", "QS_GATE_LOW_HIGH", 1, 0, 2},
    {"diag_slots", "QS_DIAG_SLOTS", 0, 0, 8},
    {"tile_waves4", "QS_TILE_W4", 1, 0, 1},
    {"reduce_xcd_order", "QS_RED_XCD", 0, 0, 2},
};

std::atomic<int64_t> g_val[T_COUNT];
std::once_flag g_once;

int64_t from_env(int i)
{
    const char* v = std::getenv(kTun[i].env);
    if (!v || !*v) return kTun[i].dflt;
    const long long x = std::atoll(v);
    if (x < kTun[i].lo || x > kTun[i].hi) return kTun[i].dflt;
    return x;
}

void init_all()
{
    for (int i = 0; i < T_COUNT; ++i) g_val[i].store(from_env(i), std::memory_order_relaxed);
}

int find(const char* name)
{
    if (!name) return -1;
    for (int i = 0; i < T_COUNT; ++i)
        if (!std::strcmp(name, kTun[i].name)) return i;
    return -1;
}

} // namespace

int64_t tun(Tun id)
{
    std::call_once(g_once, init_all);
    return g_val[id].load(std::memory_order_relaxed);
}

hipError_t lds_optin(const void* fn, size_t bytes)
{
    if (bytes <= 65536) return hipSuccess;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    static std::mutex mu;
    static std::map<std::pair<const void*, int>, size_t> done;
    std::lock_guard<std::mutex> g(mu);
    size_t& have = done[{fn, dev}];
    if (have >= bytes) return hipSuccess;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess) have = bytes;
    return e;
}

} // namespace qs

using namespace qs;

extern "C" qs_status qs_tunable_set(const char* name, int64_t value)
{
    const int i = find(name);
    if (i < 0) return set_err(QS_ERR_ARG, "qs_tunable_set: unknown knob '%s'", name ? name : "(null)");
    std::call_once(g_once, init_all);
    if (value < 0) {
        g_val[i].store(from_env(i), std::memory_order_relaxed);
        return QS_OK;
    }
    if (value < kTun[i].lo || value > kTun[i].hi)
        return set_err(QS_ERR_ARG, "qs_tunable_set: %s = %lld outside [%lld, %lld]", name, (long long)value,
                       (long long)kTun[i].lo, (long long)kTun[i].hi);
    g_val[i].store(value, std::memory_order_relaxed);
    return QS_OK;
}

extern "C" qs_status qs_tunable_get(const char* name, int64_t* value)
{
    const int i = find(name);
    if (i < 0 || !value) return set_err(QS_ERR_ARG, "qs_tunable_get: unknown knob or NULL output");
    *value = tun((Tun)i);
    return QS_OK;
}
