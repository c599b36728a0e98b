// Per-gate schedule autotuner and its cache.
//
// The per-gate kernel's memory schedule (slots per lane, workgroups per CU,
// chunk order) comes from a built-in table measured on one part (gates.hip,
// gate_sched).  qs_tune_gates times candidate schedules on a caller's state
// for each gate class and installs the fastest as an override for that
// (amplitude type, qubit count, class); a cache file keeps the result keyed
// by (GPU architecture and CU count, type, n, class), so later processes load
// it instead of timing again.  Schedules change where and when amplitudes are
// read, never what is computed, so every schedule gives bitwise the same
// states (the GPU schedule tests check this).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cinttypes>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "runtime.h"

namespace qs {

namespace {

std::mutex g_mu;
std::map<std::tuple<int, int, int>, GateSchedOverride> g_over; // (dt, n, class)

// Representative gates of a class on an n-qubit state: target lists.  Class 0
// (members exchanged by shuffles) uses targets inside a 128-byte line; the
// others one or two targets at bit 6 or above, near and far.
std::vector<std::vector<int>> class_targets(int cls, int n, int dt)
{
    const int line = dt == QS_C128 ? 3 : 4;
    const int mid = n / 2;
    switch (cls) {
    case 0: return {{0}, {line - 1}, {0, 1}};
    case 1: return {{7}, {mid}, {n - 1}};
    case 2: return {{0, mid}, {1, n - 1}};
    default: return {{mid, mid + 1}, {n - 2, n - 1}, {8, n - 5}};
    }
}

std::string device_key(int dev, int dt, int n)
{
    hipDeviceProp_t p;
    std::memset(&p, 0, sizeof p);
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) {
        (void)hipGetLastError();
        return std::string();
    }
    std::string arch = p.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon); // gfx950 without feature flags
    char buf[160];
    std::snprintf(buf, sizeof buf, "%s/%dcu/%s/n%d", arch.c_str(), p.multiProcessorCount,
                  dt == QS_C128 ? "c128" : "c64", n);
    return buf;
}

// Cache lines: one JSON object per line,
//   {"key": "gfx950/256cu/c128/n30", "class": 1, "slots": 1, "wg_per_cu": 4, "xcd": 1, "gbs": 6412.3}
bool parse_line(const std::string& l, std::string* key, qs_gate_sched* r)
{
    const size_t k0 = l.find("\"key\"");
    if (k0 == std::string::npos) return false;
    const size_t q0 = l.find('"', l.find(':', k0) + 1);
    const size_t q1 = q0 == std::string::npos ? q0 : l.find('"', q0 + 1);
    if (q1 == std::string::npos) return false;
    *key = l.substr(q0 + 1, q1 - q0 - 1);
    auto num = [&](const char* name, double* v) {
        const size_t p = l.find(name);
        if (p == std::string::npos) return false;
        const size_t c = l.find(':', p);
        return c != std::string::npos && std::sscanf(l.c_str() + c + 1, "%lf", v) == 1;
    };
    double cls, slots, wg, xcd, gbs;
    if (!num("\"class\"", &cls) || !num("\"slots\"", &slots) || !num("\"wg_per_cu\"", &wg) ||
        !num("\"xcd\"", &xcd) || !num("\"gbs\"", &gbs))
        return false;
    r->cls = (int32_t)cls;
    r->slots = (int32_t)slots;
    r->wg_per_cu = (int32_t)wg;
    r->xcd = (int32_t)xcd;
    r->gbs = gbs;
    r->from_cache = 1;
    return r->cls >= 0 && r->cls < QS_GATE_CLASSES && (r->slots == 1 || r->slots == 2 || r->slots == 4 ||
                                                        r->slots == 8) &&
           r->wg_per_cu >= 0 && r->wg_per_cu <= 32 && (r->xcd == 0 || r->xcd == 1);
}

std::string format_line(const std::string& key, const qs_gate_sched& r)
{
    char buf[256];
    std::snprintf(buf, sizeof buf,
                  "{\"key\": \"%s\", \"class\": %d, \"slots\": %d, \"wg_per_cu\": %d, \"xcd\": %d, \"gbs\": %.1f}",
                  key.c_str(), r.cls, r.slots, r.wg_per_cu, r.xcd, r.gbs);
    return buf;
}

// Pauli X on each target as one 2^k x 2^k permutation matrix (FP64
// interleaved): applied twice it restores every amplitude.
std::vector<double> x_matrix(int k)
{
    const int d = 1 << k;
    std::vector<double> u(2 * d * d, 0.0);
    for (int r = 0; r < d; ++r) u[2 * (r * d + (r ^ (d - 1)))] = 1.0;
    return u;
}

} // namespace

bool gate_sched_override(int dt, int n, int cls, GateSchedOverride* o)
{
    std::lock_guard<std::mutex> g(g_mu);
    auto it = g_over.find(std::make_tuple(dt, n, cls));
    if (it == g_over.end()) return false;
    *o = it->second;
    return true;
}

} // namespace qs

using namespace qs;

extern "C" qs_status qs_tune_gates(qs_state s, const char* cache_path, qs_gate_sched* out, int max_out, int* n_out)
{
    qs_status st = check_live(s);
    if (st != QS_OK) return st;
    if (n_out) *n_out = 0;
    if (s->n < 12) return set_err(QS_ERR_ARG, "n=%d: tuning needs at least 12 qubits", s->n);
    const std::string key = device_key(s->dev, s->dt, s->n);
    if (key.empty()) return set_err(QS_ERR_DEVICE, "device properties unavailable");
    qs_gate_sched best[QS_GATE_CLASSES];
    bool have[QS_GATE_CLASSES] = {};
    std::vector<std::string> keep; // cache lines of other keys
    if (cache_path && *cache_path) {
        std::ifstream in(cache_path);
        std::string l;
        while (std::getline(in, l)) {
            std::string k;
            qs_gate_sched r;
            if (!parse_line(l, &k, &r)) continue;
            if (k == key) {
                best[r.cls] = r;
                have[r.cls] = true;
            } else {
                keep.push_back(l);
            }
        }
    }
    bool timed = false;
    for (int cls = 0; cls < QS_GATE_CLASSES; ++cls) {
        if (have[cls]) continue;
        timed = true;
        hipEvent_t e0, e1;
        if (hipEventCreate(&e0) != hipSuccess) return fail_device(s, hipErrorOutOfMemory, "hipEventCreate");
        if (hipEventCreate(&e1) != hipSuccess) {
            (void)hipEventDestroy(e0);
            return fail_device(s, hipErrorOutOfMemory, "hipEventCreate");
        }
        const auto gates = class_targets(cls, s->n, s->dt);
        const std::vector<double> u1 = x_matrix(1), u2 = x_matrix(2);
        // each gate applied twice, each application reading and writing the state
        const double bytes = (double)gates.size() * 2.0 * 2.0 * (double)s->bytes;
        best[cls] = qs_gate_sched{cls, 0, 0, 0, 0.0, 0};
        const int slot_opts[] = {1, 2, 4, 8};
        const int wg_opts[] = {0, 2, 3, 4, 6, 8};
        for (int slots : slot_opts) {
            if (slots == 8 && cls != 0) continue; // eight slots only for gates without register targets
            for (int wg : wg_opts)
                for (int xcd = 0; xcd <= 1 && st == QS_OK; ++xcd) {
                    {
                        std::lock_guard<std::mutex> g(g_mu);
                        g_over[std::make_tuple(s->dt, s->n, cls)] = GateSchedOverride{slots, wg, xcd};
                    }
                    float ms = 0.0f;
                    for (int rep = 0; rep < 2 && st == QS_OK; ++rep) { // rep 0 warms up
                        hipError_t e = hipEventRecord(e0, s->st);
                        for (const auto& t : gates)
                            for (int k = 0; k < 2 && st == QS_OK && e == hipSuccess; ++k)
                                st = t.size() == 1 ? apply_1q_internal(s, t[0], u1.data(), 0, 0)
                                                   : apply_2q_internal(s, t[0], t[1], u2.data(), 0, 0);
                        if (st != QS_OK) break;
                        if (e == hipSuccess) e = hipEventRecord(e1, s->st);
                        if (e == hipSuccess) e = hipEventSynchronize(e1);
                        if (e == hipSuccess && rep == 1) e = hipEventElapsedTime(&ms, e0, e1);
                        if (e != hipSuccess) st = fail_device(s, e, "gate tuning");
                    }
                    if (st != QS_OK) break;
                    const double gbs = bytes / (ms * 1e-3) / 1e9;
                    if (gbs > best[cls].gbs) best[cls] = qs_gate_sched{cls, slots, wg, xcd, gbs, 0};
                }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        std::lock_guard<std::mutex> g(g_mu);
        if (st != QS_OK) { // this class keeps the built-in schedule; the ones timed before keep theirs
            g_over.erase(std::make_tuple(s->dt, s->n, cls));
            return st;
        }
        g_over[std::make_tuple(s->dt, s->n, cls)] = GateSchedOverride{best[cls].slots, best[cls].wg_per_cu, best[cls].xcd};
    }
    {
        std::lock_guard<std::mutex> g(g_mu);
        for (int cls = 0; cls < QS_GATE_CLASSES; ++cls)
            g_over[std::make_tuple(s->dt, s->n, cls)] =
                GateSchedOverride{best[cls].slots, best[cls].wg_per_cu, best[cls].xcd};
    }
    if (timed && cache_path && *cache_path) {
        const std::string tmp = std::string(cache_path) + ".tmp";
        {
            std::ofstream o(tmp, std::ios::trunc);
            for (const auto& l : keep) o << l << "\n";
            for (int cls = 0; cls < QS_GATE_CLASSES; ++cls) o << format_line(key, best[cls]) << "\n";
            if (!o) return set_err(QS_ERR_ARG, "cannot write the tuning cache %s", tmp.c_str());
        }
        if (std::rename(tmp.c_str(), cache_path) != 0)
            return set_err(QS_ERR_ARG, "cannot replace the tuning cache %s", cache_path);
    }
    if (out)
        for (int cls = 0; cls < QS_GATE_CLASSES && cls < max_out; ++cls) out[cls] = best[cls];
    if (n_out) *n_out = std::max(0, std::min(max_out, QS_GATE_CLASSES));
    return QS_OK;
}

extern "C" qs_status qs_tune_gates_reset(void)
{
    std::lock_guard<std::mutex> g(g_mu);
    g_over.clear();
    return QS_OK;
}
