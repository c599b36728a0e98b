// Circuit planner: groups a gate list into LDS tile passes (one HBM read and
// one write of the state per pass).  Not part of the public ABI.
#pragma once

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <thread>
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
//   kind TK_SEG: header of a register segment: the next dj ops (TK_DENSE1,
//       TK_DENSE2, TK_DIAG) act only on the k tile-local positions p[0..k)
//       (ascending) as far as dense targets go, so each thread loads its 2^k
//       amplitudes from LDS once, applies all of them in registers and
//       stores them once.  Inside a segment the kernel reads 32-bit fields
//       only: a dense op's rsv holds the register bits of its targets
//       (target 0 | target 1 << 8, target 0 the lower) and dj its control
//       kinds (1: a control at a register position, 2: at a thread
//       position); diagonal members are described where the planner forms
//       them.
enum { TK_DENSE1 = 0, TK_DENSE2 = 1, TK_DENSEK = 2, TK_DIAG = 3, TK_MFMA = 4, TK_SEG = 5 };
// A diagonal segment member the planner could not put in register form
// (its dclass); the kernel gathers its factor per element.
enum { SD_GATHER = 7 };
// Segment member opcodes (rsv >> 16): dense 1q on register bit b (+4 with
// controls), dense 2q on register pair p (+6 with controls), diagonal forms.
// Register pairs (a < b < 4) are numbered 01, 02, 12, 03, 13, 23.
enum {
    SO_1Q = 0,    // 8 codes
    SO_2Q = 8,    // 12 codes
    SO_D0 = 20,   // 1
    SO_D1 = 21,   // 4: by rank
    SO_D2 = 25,   // 6: by pair
    SO_D1X = 31,  // 8: 2 rank + ri
    SO_D2X = 39,  // 24: 4 pair + ri
    SO_BLOCK = 63, // a fused 2^r x 2^r block on all register bits (row-major complex)
    SO_DG = 64,   // gather
    SO_DGROUP = 65, // several diagonal ops as one factor table (see the planner)
};
static_assert(SO_D2X + 4 * 6 <= SO_BLOCK, "segment opcode ranges overlap");

// Register qubits of a segment for tile size m (0: tiles below 2^10
// elements run op by op in LDS).  Every one of a block's 256 threads holds
// 2^r elements per loop step.  The tile kernels use the same formula.
inline int seg_reg_qubits(int dt, int m)
{
    (void)dt;
    if (m < 10) return 0;
    return m - 8 < 4 ? m - 8 : 4;
}

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

// The tile-kernel variant a pass's op list needs: 3 with a fused block in
// the FP32 matrix-core form (complex64), 2 with one in the FP64 form, else 1
// with any k >= 3 dense op or (tiles of >= 2^10 elements) any op outside a
// segment, else 0 (the lean kernel).  Each variant holds only what its passes
// need, which keeps the registers of the smaller ones low; a launch covering
// several passes takes the largest of their variants (a plan uses one form).
inline int ops_variant(const TileOp* ops, size_t n, int m)
{
    int v = 0;
    for (size_t i = 0; i < n; ++i) {
        const int k = ops[i].kind;
        if (k == TK_SEG) {
            i += (size_t)ops[i].dj;
            continue;
        }
        if (k == TK_MFMA) return ops[i].dclass == 1 ? 3 : 2;
        if (k == TK_DENSEK || m >= 10) v = 1;
    }
    return v;
}

struct PlanPass {
    int m = 0;                 // tile qubits
    int L = 0;                 // lowest L qubits are in the tile (contiguous runs)
    std::vector<int> Q;        // sorted tile qubits (size m)
    std::vector<TileOp> ops;
    std::vector<int64_t> src;   // per op: circuit index of the gate (-1: segment header or fused block)
    std::vector<int64_t> order; // circuit gates in execution order (fused blocks expanded)
    uint64_t gates = 0;        // circuit gates absorbed
    uint64_t updates = 0;      // amplitude updates credited (sum over gates)
};

struct PlanOpts {
    int m = 12;       // tile qubits
    int L = 5;        // forced low qubits
    int fuse_k = 0;   // 0: no dense fusion; 4 or 5: matrix-core blocks
    int fuse_min = 3; // dense gates a block must absorb to be worth a fused block
    bool fuse_fp32 = false; // complex64: FP32 matrix-core blocks (hi FP32 + lo bfloat16 parts)
    int dt = QS_C128;
    bool segments = true; // group ops into register segments (tiles of >= 2^10 elements)
};

// Plan in FP64.  `mats_out` receives the pool the passes' moff index (FP64,
// interleaved complex); the executor converts it to the state's real type.
// With encode = false the passes are partitioned but not encoded (no fused
// blocks or register segments): the pass count is the same, for comparing
// plans cheaply.
void plan_circuit(int n, const qs_op* ops, int64_t n_ops, const double* mats, const PlanOpts& po,
                  std::vector<PlanPass>& passes, std::vector<double>& mats_out, bool encode = true);

// Qubit relabeling.  An uncontrolled SWAP gate exchanges two qubits' values;
// instead of moving amplitudes, the planner can record that the two logical
// qubits now live at each other's bit positions and rewrite every later gate
// to the physical positions.  The state then ends with logical qubit q at
// position perm[q]; the restoring permutation of bit positions (position
// perm[q] -> q) is the product of at most two involutions tau[0], tau[1]
// (position maps, applied in that order), each one in-place pass.
struct Remap {
    std::vector<qs_op> ops;   // the circuit without its SWAP gates, on physical qubits
    std::vector<int64_t> src; // index of each in the original circuit
    int nrestore = 0;
    int tau[2][64];
};
// False (and r untouched) when the circuit has no uncontrolled SWAP gate.
bool remap_swaps(int n, const qs_op* ops, int64_t n_ops, const double* mats, Remap& r);
// Plan with relabeling when its tile passes plus half a pass per restoring
// involution are fewer than the plain plan's (remap = 0), or never (remap =
// 1).  r.nrestore = 0 when the plain plan is kept; P.src and P.order index the
// original circuit either way.
void plan_circuit_remap(int n, const qs_op* ops, int64_t n_ops, const double* mats, const PlanOpts& po, int remap,
                        std::vector<PlanPass>& passes, std::vector<double>& mats_out, Remap& r);
hipError_t launch_bit_involution(void* psi, int dt, int n, const int* tau, hipStream_t st);
uint64_t involution_moved(int n, const int* tau); // amplitudes one restoring pass moves

// Run fn(i) for i in [0, n) on up to 16 host threads (independent items,
// e.g. the circuits of a batch, which are planned one per call).
template <typename F>
void parallel_for(int n, F fn)
{
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int nt = (int)std::min<unsigned>(std::min(hw, 16u), (unsigned)std::max(1, n / 4));
    if (nt <= 1) {
        for (int i = 0; i < n; ++i) fn(i);
        return;
    }
    std::atomic<int> next{0};
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t)
        th.emplace_back([&]() {
            for (int i; (i = next.fetch_add(1)) < n;) fn(i);
        });
    for (auto& x : th) x.join();
}

// ---------------------------------------------------------------- batches

// Pass descriptor in device memory (persistent batch kernels read it there).
struct BatchPass {
    int32_t m, L;
    int32_t q[QS_MAX_QUBITS];
    InsertPlan ip; // tile qubits, inserted into the tile counter
    int32_t op0, nops;
};

// Circuit descriptor in device memory.
// BatchCirc / ServeEntry basis value meaning "the initial state is already in
// place" (copied in from the caller); a real basis index is below 2^34.
constexpr uint64_t kLoadInitial = ~0ull;

struct BatchCirc {
    uint64_t psi_off; // byte offset of the state inside the batch arena
    uint64_t basis;   // initial basis state, or kLoadInitial
    int32_t n;
    int32_t pass0, npass;
    int32_t rsv;
};

// One launch for `count` circuits listed in `list`: every circuit of n = M
// qubits runs whole in one block's LDS (initial basis state built in LDS; the
// final state written once).
hipError_t launch_batch_whole(int dt, int M, char* arena, const BatchCirc* circs, const int32_t* list, int count,
                              const BatchPass* passes, const TileOp* ops, const double* mats, int var,
                              hipStream_t st);
// One launch for `count` circuits whose passes all use tile size M: one block
// per circuit initialises its state and loops over its passes and tiles.
hipError_t launch_batch_persist(int dt, int M, char* arena, const BatchCirc* circs, const int32_t* list,
                                int count, const BatchPass* passes, const TileOp* ops, const double* mats, int var,
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
                              uint32_t nblocks, int var, hipStream_t st);
// Zero `bytes` bytes of the arena and set each listed circuit's basis amplitude.
hipError_t launch_batch_init(int dt, char* arena, uint64_t bytes, const BatchCirc* circs, const int32_t* list,
                             int count, hipStream_t st);

// ---------------------------------------------------------------- serving

// One request's share of a serving round, with absolute device pointers.
// Round entries: blocks [first_block, first_block + 2^(n - M)) apply pass
// `pass` to the request's state.  Whole entries (n <= M): one block runs the
// request's single pass on a basis state built in LDS.
// Byte offsets into the server's state pool (psi) and plan pool (the rest),
// which the kernels receive as restrict arguments: with the op tables
// reached from a restrict base the compiler keeps descriptor and matrix loads
// scalar, as in the single-circuit tile kernel (loading the pointers from the
// entry instead made every op a vector load and doubled the registers).
struct ServeEntry {
    uint64_t psi_off;
    uint64_t pass_off;     // UINT64_MAX: no pass (a whole circuit without gates)
    uint64_t ops_off;      // base the pass's op0 indexes
    uint64_t mats_off;     // base the ops' moff index
    uint64_t basis;        // initial basis state, or kLoadInitial
    uint32_t first_block;
    int32_t n;
};

hipError_t launch_serve_round(int dt, int M, char* pool, const char* plan, const ServeEntry* entries, int nentries,
                              uint32_t nblocks, int var, hipStream_t st);
hipError_t launch_serve_whole(int dt, int M, char* pool, const char* plan, const ServeEntry* entries, int nentries,
                              int var, hipStream_t st);

qs_status validate_circuit(int n, const qs_op* ops, int64_t n_ops, const double* mats, int64_t n_mats);
qs_status plan_opts_for(int dt, const qs_op* ops, int64_t n_ops, int fuse_k, int tile_qubits, PlanOpts& po);

qs_status run_planned(qs_state s, const qs_op* ops, int64_t n_ops, const double* mats, int64_t n_mats,
                      const qs_run_opts& o);

// Tile pass launcher (tile.hip).  `dops` and `dmats` are device copies.
// The `var` arguments of the launchers here are ops_variant values.
// max_blocks caps the launch's grid (0: the default cap); the blocks stride
// over the tiles.
hipError_t launch_tile_pass(void* psi, int dt, int n, const PlanPass& pass, const TileOp* dops,
                            const void* dmats, int max_blocks, hipStream_t st);
size_t tile_lds_bytes(int dt, int m, int L);

} // namespace qs
