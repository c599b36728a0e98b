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
    // control), DG_LCONTROL (no local target, one local control), DG_CT (one
    // local target and one local control), DG_GENERAL.
    int8_t lp[6];
    int8_t dclass;
    int8_t dbit; // the local bit of DG_LTARGET / DG_LCONTROL
    int32_t dj;  // DG_LTARGET: which target is local
    int32_t rsv;
};
static_assert(sizeof(TileOp) == 88, "TileOp layout");
enum { DG_UNIFORM = 0, DG_LTARGET = 1, DG_LCONTROL = 2, DG_GENERAL = 3, DG_CT = 4 };

struct PlanPass {
    int m = 0;                 // tile qubits
    int L = 0;                 // lowest L qubits are in the tile (contiguous runs)
    std::vector<int> Q;        // sorted tile qubits (size m)
    std::vector<TileOp> ops;
    std::vector<int64_t> src;  // circuit index of each absorbed gate, in execution order
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

// ---------------------------------------------------------------- batches

// Pass descriptor in device memory (persistent batch kernels read it there).
struct BatchPass {
    int32_t m, L;
    int32_t q[QS_MAX_QUBITS];
    InsertPlan ip; // tile qubits, inserted into the tile counter
    int32_t op0, nops;
};

// Circuit descriptor in device memory.
struct BatchCirc {
    uint64_t psi_off; // byte offset of the state inside the batch arena
    uint64_t basis;   // initial basis state
    int32_t n;
    int32_t pass0, npass;
    int32_t rsv;
};

// One launch for `count` circuits listed in `list`: every circuit of n = M
// qubits runs whole in one block's LDS (initial basis state built in LDS; the
// final state written once).
hipError_t launch_batch_whole(int dt, int M, char* arena, const BatchCirc* circs, const int32_t* list, int count,
                              const BatchPass* passes, const TileOp* ops, const double* mats, bool mf,
                              hipStream_t st);
// One launch for `count` circuits whose passes all use tile size M: one block
// per circuit initialises its state and loops over its passes and tiles.
hipError_t launch_batch_persist(int dt, int M, char* arena, const BatchCirc* circs, const int32_t* list,
                                int count, const BatchPass* passes, const TileOp* ops, const double* mats, bool mf,
                                hipStream_t st);

// One entry of a pass-major round: blocks [first_block, first_block + 2^(n-m))
// of the round's launch process the tiles of pass `pass` of circuit `circ`.
struct RoundEntry {
    int32_t circ;
    int32_t pass;
    uint32_t first_block;
    uint32_t rsv;
};

// One launch covering the same pass index of many circuits (all with tile size M).
hipError_t launch_batch_round(int dt, int M, char* arena, const BatchCirc* circs, const BatchPass* passes,
                              const TileOp* ops, const double* mats, const RoundEntry* entries, int nentries,
                              uint32_t nblocks, bool mf, hipStream_t st);
// Zero `bytes` bytes of the arena and set each listed circuit's basis amplitude.
hipError_t launch_batch_init(int dt, char* arena, uint64_t bytes, const BatchCirc* circs, const int32_t* list,
                             int count, hipStream_t st);

// ---------------------------------------------------------------- serving

// One request's share of a serving round, with absolute device pointers.
// Round entries: blocks [first_block, first_block + 2^(n - M)) apply pass
// `pass` to the request's state.  Whole entries (n <= M): one block runs the
// request's single pass on a basis state built in LDS.
struct ServeEntry {
    void* psi;
    const BatchPass* pass;
    const TileOp* ops;     // base the pass's op0 indexes
    const double* mats;    // base the ops' moff index
    uint64_t basis;
    uint32_t first_block;
    int32_t n;
};

hipError_t launch_serve_round(int dt, int M, const ServeEntry* entries, int nentries, uint32_t nblocks, bool mf,
                              hipStream_t st);
hipError_t launch_serve_whole(int dt, int M, const ServeEntry* entries, int nentries, bool mf, hipStream_t st);

qs_status validate_circuit(int n, const qs_op* ops, int64_t n_ops, const double* mats, int64_t n_mats);
qs_status plan_opts_for(int dt, const qs_op* ops, int64_t n_ops, int fuse_k, int tile_qubits, PlanOpts& po);

qs_status run_planned(qs_state s, const qs_op* ops, int64_t n_ops, const double* mats, int64_t n_mats,
                      const qs_run_opts& o);

// Tile pass launcher (tile.hip).  `dops` and `dmats` are device copies.
hipError_t launch_tile_pass(void* psi, int dt, int n, const PlanPass& pass, const TileOp* dops,
                            const void* dmats, hipStream_t st);
size_t tile_lds_bytes(int dt, int m, int L);

} // namespace qs
