// Host-side runtime structures shared by qs_api.cpp and the circuit/batch
// executors.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <functional>
#include <vector>

#include "qs_internal.h"

struct qs_trace_item {
    qs_trace_rec rec;
    hipEvent_t a, b;
};

struct qs_state_s {
    int n = 0;
    int dt = QS_C128;
    void* d = nullptr;      // amplitudes
    uint64_t bytes = 0;     // bytes of amplitudes
    bool owned = false;     // library allocated d
    hipStream_t st = nullptr;
    bool own_stream = false;
    int dev = 0;
    bool failed = false;
    // reduction scratch (device): partial sums then the 2^m results
    double* red_part = nullptr;
    uint64_t red_cap = 0; // doubles
    double* red_host = nullptr;
    // matrix staging ring (device buffer + pinned host mirror)
    char* mat_dev = nullptr;
    char* mat_host = nullptr;
    uint64_t mat_cap = 0, mat_off = 0;
    // tracing
    bool tracing = false;
    std::vector<qs_trace_item> trace;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
};

namespace qs {

qs_status set_err(qs_status st, const char* fmt, ...);
qs_status fail_device(qs_state s, hipError_t e, const char* what);
qs_status check_live(qs_state s);
qs_status traced_launch(qs_state s, qs_trace_rec rec, const std::function<hipError_t(int*)>& fn,
                        const char* what);
qs_status stage_matrices(qs_state s, const double* src, uint64_t count, const void** dev_out);
qs_status stage_bytes(qs_state s, const void* src, uint64_t bytes, const void** dev_out);
qs_status validate_gate(int n, const int* t, int k, uint64_t cm, uint64_t cv);
qs_status dev_alloc(void** p, uint64_t bytes, const char* what);
void dev_free(void* p, uint64_t bytes);
uint64_t allocated_bytes();
// QS_FAULT_INJECT=launch:N: true exactly at the N-th launch of the process.
bool inject_fault_now();

qs_status apply_1q_internal(qs_state s, int target, const double* U, uint64_t cm, uint64_t cv);
qs_status apply_2q_internal(qs_state s, int t0, int t1, const double* U, uint64_t cm, uint64_t cv);
qs_status apply_kq_dev_internal(qs_state s, const int* t, int k, const void* Ud, uint64_t cm, uint64_t cv);
qs_status apply_diag_internal(qs_state s, const DiagPlan& p, int t0, int t1, uint64_t cm);
// QS_ERR_ARG unless U (2^k x 2^k, FP64 interleaved) is unitary to 1e-10;
// callers check only when check_unitary_enabled() (QS_CHECK_UNITARY=1).
bool check_unitary_enabled();
qs_status check_unitary(const double* U, int k);

} // namespace qs
