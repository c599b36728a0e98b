// Internal declarations shared by the runtime (qs_api.cpp, planner.cpp) and
// the kernel translation units (*.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/qs.h"

namespace qs {

// Zero bits inserted into a compact counter to form an amplitude index.  For
// sorted positions p_0 < p_1 < ..., inserting in ascending order turns the
// counter k (over the remaining bits) into the index with 0 at every p_j; the
// same walk as Alg. 1's block/offset split, for any number of fixed bits.
constexpr int kMaxIns = 36;
struct InsertPlan {
    int32_t n = 0;
    int32_t pad = 0;
    uint64_t low[kMaxIns]; // (1 << p_j) - 1, ascending
};

InsertPlan make_insert_plan(uint64_t positions_mask);

// Tile pass description (LDS-resident tiles of 2^m amplitudes).  Defined in
// tile.hip, built by the planner.
struct TileGate;
struct TilePass;

// Kernel launchers.  All return hipSuccess or the launch error; `kind`
// receives the QS_K_* class actually used (for tracing).
hipError_t launch_init_basis(void* psi, int dt, int n, uint64_t x, hipStream_t st);
hipError_t launch_apply_1q(void* psi, int dt, int n, int t, const double* U, uint64_t cm,
                           uint64_t cv, hipStream_t st, int* kind);
hipError_t launch_apply_2q(void* psi, int dt, int n, int t0, int t1, const double* U,
                           uint64_t cm, uint64_t cv, hipStream_t st, int* kind);
// Dense k-qubit gate; Ud is a device copy of U in the state's element type.
hipError_t launch_apply_kq_dev(void* psi, int dt, int n, const int* targets, int k, const void* Ud,
                               uint64_t cm, uint64_t cv, hipStream_t st, int* kind);

// Diagonal gates (phase-only kernel).  diag_plan folds the controls into the
// diagonal d (2^k complex entries, entry j bit b = target t[b]) and finds the
// fixed bits shared by every amplitude the gate changes; diag_plan_matrix
// does the same for a dense 2^k x 2^k matrix and returns false when it has a
// nonzero off-diagonal entry.
constexpr int kDiagMaxFree = 6;
struct DiagPlan {
    bool identity;          // every factor is exactly 1: nothing to launch
    int n, k, nctrl;
    uint64_t changed_per;   // diagonal entries that differ from 1
    uint64_t fixed_mask, fixed_val;
    int nfree;
    int fpos[kDiagMaxFree]; // qubit of free bit i
    int fbit[kDiagMaxFree]; // matrix bit of free bit i
    double tab[2 << kDiagMaxFree];
};
bool diag_plan(int n, const int* t, int k, const double* d, uint64_t cm, uint64_t cv, DiagPlan* p);
bool diag_plan_matrix(int n, const int* t, int k, const double* U, uint64_t cm, uint64_t cv, DiagPlan* p);
uint64_t diag_changed(const DiagPlan& p); // amplitudes the gate changes
hipError_t launch_diag(void* psi, int dt, const DiagPlan& p, hipStream_t st);

// Reductions.  `part` is device scratch of at least reduce_scratch_doubles()
// doubles.  Results land in `dev_out` (device, 2^m doubles).
// Pauli-string expectation: part needs pauli_scratch_doubles(n); dev_out
// receives (sum re, sum im) before the factor i^|x & z|.
uint64_t pauli_scratch_doubles(int n);
hipError_t launch_pauli_expect(const void* psi, int dt, int n, uint64_t x, uint64_t z, double* part,
                               double* dev_out, hipStream_t st);
// Sampling within chunks of min(4096, 2^n) amplitudes (the chunk sums come
// from launch_probabilities with m = 0, whose partials are per such chunk).
struct SampleReq {
    uint64_t chunk;
    double residual;
};
hipError_t launch_sample_chunks(const void* psi, int dt, int n, const SampleReq* req, int64_t shots, uint64_t* out,
                                hipStream_t st);
uint64_t reduce_scratch_doubles(int n, int m);
// The pass-1 partials of launch_probabilities (2^m outcomes x chunks, at the
// start of `part`); with m = 0 one per chunk of min(4096, 2^n) amplitudes.
uint64_t reduce_partials(int n, int m);
// The fixed per-device reduction scratch of the no-allocation entry points:
// its address on device `dev` (which must be current; resolved once per
// device, then cached) and its size in doubles.
hipError_t noalloc_scratch(int dev, double** ptr, uint64_t* doubles);
hipError_t launch_probabilities(const void* psi, int dt, int n, const int* qubits, int m,
                                double* part, double* dev_out, hipStream_t st);

// Tuned per-gate schedules (gate_tune.cpp): an override of the built-in
// table for (amplitude type, qubit count, gate class), if one is installed.
struct GateSchedOverride {
    int ppl, wg, xcd;
};
bool gate_sched_override(int dt, int n, int cls, GateSchedOverride* o);

// In-place read-modify-write of `bytes` (16-byte words, each XORed with
// `mask`): the memory ceiling probe.  slots 1/2/4/8, slog 8..30.
hipError_t launch_probe_inplace(void* dev, uint64_t bytes, int slots, int slog, uint64_t mask, hipStream_t st);

// Environment variable as an int (dflt when unset or empty).
int env_int(const char* name, int dflt);

// Launch knobs (tunables.cpp): default, else the environment variable read on
// first use, else the value last given to qs_tunable_set.
enum Tun {
    T_GATE_GRID_CAP,   // workgroups of a per-gate / diagonal launch (they loop beyond it)
    T_TILE_GRID_CAP,   // workgroups of a tile pass
    T_ROUND_GRID_CAP,  // workgroups of a batch / serving round
    T_AUX_GRID_CAP,    // workgroups of init, dense k-qubit and other grid-stride kernels
    T_NT,              // non-temporal loads/stores where whole lines are written
    T_SLOG,            // per-gate kernel: log2 of the counter distance between a lane's slots
    T_PPL_H0,          // per-gate kernel: slots per lane (0 = built-in table) without high targets,
    T_PPL_H1,          //   with one high target,
    T_PPL_H2,          //   with two
    T_DIAG_SLOG,       // diagonal kernel: log2 slot distance
    T_PERM_RUN,        // restore pass: log2 run length (0 = built-in choice)
    T_GATE_XCD,        // per-gate kernel chunk order: 0 rule, 1 workgroup order, 2 XCD-contiguous
    T_GATE_WG_PER_CU,  // per-gate kernel and probe: workgroups per CU (0 rule; 8 and up: no cap in effect)
    T_GATE_LOW_HIGH,   // per-gate kernel: targets below bit 6 held in registers (1: at or above the
                       //   128-byte line bit, 2: all) instead of exchanged by shuffles
    T_DIAG_SLOTS,      // diagonal kernel: slots per lane (0 = built-in: 4)
    T_TILE_W4,         // lean 2^11 tile passes held to 128 VGPRs (4 waves per SIMD)
    T_RED_XCD,         // reduction chunk order: 0 rule, 1 block order, 2 XCD-contiguous
    T_COUNT
};
int64_t tun(Tun id);
// Opt a kernel in to `bytes` of dynamic LDS on the current device (no-op up
// to 64 KiB; remembered per kernel and device; thread-safe).
hipError_t lds_optin(const void* fn, size_t bytes);
// Unused LDS bytes that cap a kernel at `wg` workgroups per CU (0: none).
size_t pad_for_wg_per_cu(int wg, size_t static_lds);

inline size_t amp_bytes(int dt) { return dt == QS_C128 ? 16 : 8; }

} // namespace qs
