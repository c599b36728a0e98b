// Circuit planner: groups a gate list into LDS tile passes (one HBM read and
// one write of the state per pass).  Not part of the public ABI.
#pragma once

#include <cstdint>
#include <vector>

#include "runtime.h"

namespace qs {

// One operation inside a tile pass (64 bytes, copied to device memory).
//   kind TK_DENSE1/2/K: dense gate on tile-local positions p[0..k); local
//       controls lcm/lcv are tile-local bit masks; global controls gcm/gcv are
//       bits outside the tile (a property of the whole tile).
//   kind TK_DIAG: diagonal gate on global target positions p[0..k) with global
//       controls gcm/gcv; it multiplies amplitude i by d[bits of i at p] and
//       never needs its qubits inside the tile.
//   kind TK_MFMA: dense k-qubit block applied with matrix cores.
enum { TK_DENSE1 = 0, TK_DENSE2 = 1, TK_DENSEK = 2, TK_DIAG = 3, TK_MFMA = 4 };

struct TileOp {
    int32_t kind;
    int32_t k;
    int32_t p[6];
    uint64_t lcm, lcv;
    uint64_t gcm, gcv;
    uint64_t moff; // offset, in reals, into the pass matrix pool
    // TK_DIAG only: tile-local position of each target (-1 outside the tile),
    // and the shape class the kernel folds per tile: DG_UNIFORM (no local bit:
    // one factor for the whole tile), DG_LTARGET (one local target, no local
    // control), DG_LCONTROL (no local target, one local control), DG_GENERAL.
    int8_t lp[6];
    int8_t dclass;
    int8_t dbit; // the local bit of DG_LTARGET / DG_LCONTROL
    int32_t dj;  // DG_LTARGET: which target is local
    int32_t rsv;
};
static_assert(sizeof(TileOp) == 88, "TileOp layout");
enum { DG_UNIFORM = 0, DG_LTARGET = 1, DG_LCONTROL = 2, DG_GENERAL = 3 };

struct PlanPass {
    int m = 0;                 // tile qubits
    int L = 0;                 // lowest L qubits are in the tile (contiguous runs)
    std::vector<int> Q;        // sorted tile qubits (size m)
    std::vector<TileOp> ops;
    uint64_t gates = 0;        // circuit gates absorbed
    uint64_t updates = 0;      // amplitude updates credited (sum over gates)
};

struct PlanOpts {
    int m = 12;       // tile qubits
    int L = 5;        // forced low qubits
    int fuse_k = 0;   // 0: no dense fusion; 4 or 5: matrix-core blocks (complex64)
    int fuse_min = 3; // dense gates a block must absorb to be worth a fused block
    int dt = QS_C128;
};

// Plan in FP64.  `mats_out` receives the pool the passes' moff index (FP64,
// interleaved complex); the executor converts it to the state's real type.
void plan_circuit(int n, const qs_op* ops, int64_t n_ops, const double* mats, const PlanOpts& po,
                  std::vector<PlanPass>& passes, std::vector<double>& mats_out);

qs_status run_planned(qs_state s, const qs_op* ops, int64_t n_ops, const double* mats, int64_t n_mats,
                      const qs_run_opts& o);

// Tile pass launcher (tile.hip).  `dops` and `dmats` are device copies.
hipError_t launch_tile_pass(void* psi, int dt, int n, const PlanPass& pass, const TileOp* dops,
                            const void* dmats, hipStream_t st);
size_t tile_lds_bytes(int dt, int m, int L);

} // namespace qs
