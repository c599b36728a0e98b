/*
 * qs.h -- C ABI of the gfx950 state-vector gate engine (libqs.so).
 *
 * The engine applies gate matrices to a 2^n-amplitude complex state held in
 * device memory, the core operation of full state-vector simulation (the
 * paper's Section I; its kernels are the pair update of Alg. 1 and Alg. 9).
 *
 * Conventions used by every entry point
 * -------------------------------------
 * - State layout: 2^n complex amplitudes, interleaved (re, im) -- the
 *   array-of-structures layout of Section II-A.  QS_C128 stores two doubles
 *   (16 B) per amplitude, QS_C64 two floats (8 B).  The base address must be
 *   256-byte aligned.  This is exactly torch.complex128 / torch.complex64.
 * - Qubit q is bit q of the amplitude index.  A 1q gate on target t pairs
 *   index i (bit t clear) with i + 2^t (Alg. 1, Section II-C).
 * - Matrices are always FP64 at the ABI: 2^k x 2^k complex, row-major,
 *   interleaved (re, im).  For a gate on targets t[0..k), t[j] is bit j of the
 *   matrix row/column index (t[0] is the least significant).  QS_C64 states
 *   store FP32 amplitudes, but every update is computed in FP64 with the FP64
 *   matrices (fused products too, formed in FP64); each stored amplitude is
 *   rounded to FP32 once per write.  Matrices are not checked for unitarity
 *   unless the environment sets QS_CHECK_UNITARY=1: then every gate matrix
 *   with max |(U^H U - I)_ij| > 1e-10 (or a diagonal entry of modulus other
 *   than 1) is rejected with QS_ERR_ARG.
 * - Controls are a bitmask ctrl_mask with required values ctrl_vals (a subset
 *   of ctrl_mask; ctrl_vals == ctrl_mask means "control on 1").  A controlled
 *   gate updates only the amplitudes whose control bits match and leaves all
 *   others bitwise unchanged (Fig. control6q2, Section III-A).
 * - Ownership: the caller keeps every pointer it passes; matrices and op
 *   tables are copied before the call returns, so they may be freed at once.
 * - Asynchrony: qs_apply_* / qs_run_circuit / qs_init_basis enqueue work on the
 *   state's HIP stream and return.  qs_download, qs_probabilities, qs_norm and
 *   qs_sync block until the result is on the host.
 * - Errors: every call returns a qs_status; nothing aborts.  On QS_ERR_ARG the
 *   state is untouched.  A failing HIP call marks the state failed and every
 *   later call on it returns QS_ERR_DEVICE.  qs_last_error() gives a
 *   thread-local message for the last failure on the calling thread.
 * - Threads: one handle must not be used from two threads at once; distinct
 *   handles are independent.
 */
#ifndef QS_H
#define QS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QS_OK = 0,
    QS_ERR_ARG = 1,         /* invalid argument; nothing was changed */
    QS_ERR_OOM = 2,         /* device memory (or the configured budget) exhausted */
    QS_ERR_DEVICE = 3,      /* a HIP call failed; the handle is now failed */
    QS_ERR_BUSY = 4,        /* resource in use (e.g. batch not finished) */
    QS_ERR_UNSUPPORTED = 5, /* valid request the library does not handle */
    QS_ERR_CANCELLED = 6,
    QS_ERR_TIMEOUT = 7
} qs_status;

typedef enum { QS_C64 = 1, QS_C128 = 2 } qs_dtype;

#define QS_MAX_QUBITS 34   /* 2^34 complex64 amplitudes = 128 GiB */
#define QS_MAX_FUSED 6     /* largest k accepted by qs_apply_fused */

typedef struct qs_state_s* qs_state;

/* One gate of a circuit (64 bytes).  nt targets in t[0..nt) (t[0] is the least
 * significant bit of the matrix index), unused t[] entries are -1; controls as
 * described above; moff = offset, in doubles, of the gate's 2^nt x 2^nt complex
 * matrix inside the circuit's matrix pool. */
typedef struct {
    int32_t nt;
    int32_t t[6];
    uint32_t flags; /* must be 0 */
    uint64_t cmask;
    uint64_t cvals;
    uint64_t moff;
    uint64_t rsv; /* must be 0 */
} qs_op;

/* ------------------------------------------------------------------ basics */

/* Library version, (major << 16) | minor. */
int qs_version(void);

/* Message for the last failing call on this thread ("" if none).  The pointer
 * stays valid until the next qs_* call on the same thread. */
const char* qs_last_error(void);

/* Number of HIP devices visible (0 if none); never fails. */
int qs_device_count(void);

/* ------------------------------------------------------------------ states */

/* Allocate a state of n qubits (1 <= n <= QS_MAX_QUBITS) on the current HIP
 * device, initialised to |0..0>, with a library-created stream.  The library
 * owns the memory; qs_destroy frees it.  QS_ERR_OOM if it does not fit. */
qs_status qs_create(int n, qs_dtype dt, qs_state* out);

/* Wrap caller-owned device memory (e.g. a torch tensor's data_ptr) of `bytes`
 * bytes (>= 2^n * amplitude size, 256-byte aligned) as a state.  Contents are
 * used as they are.  `stream` is a hipStream_t (NULL = the null stream) on
 * which all of the state's work is enqueued.  qs_destroy does not free it. */
qs_status qs_create_external(int n, qs_dtype dt, void* dev_ptr, uint64_t bytes,
                             void* stream, qs_state* out);

/* Release the handle (waits for its pending work first).  NULL is accepted. */
qs_status qs_destroy(qs_state s);

/* Change the stream later work is enqueued on.  Work already enqueued on the
 * previous stream is ordered before new work (the library waits on it). */
qs_status qs_set_stream(qs_state s, void* stream);

/* Report n, dtype and the device pointer of the amplitudes. */
qs_status qs_get_info(qs_state s, int* n, int* dtype, void** dev_ptr);

/* Set the state to the basis state |x> (x < 2^n). */
qs_status qs_init_basis(qs_state s, uint64_t x);

/* Copy `count` amplitudes between host memory and amplitudes
 * [first, first + count) of the state.  The host buffer uses the state's own
 * element type (complex64 or complex128).  qs_upload is stream-ordered and
 * returns once the host buffer may be reused; qs_download blocks until the
 * data is on the host. */
qs_status qs_upload(qs_state s, const void* host, uint64_t first, uint64_t count);
qs_status qs_download(qs_state s, void* host, uint64_t first, uint64_t count);

/* ------------------------------------------------------------------ gates */

/* 1q gate: U is 2x2 complex (8 doubles).  Target and control qubits must be
 * distinct and < n; ctrl_vals must be a subset of ctrl_mask.  Pair update of
 * Alg. 1 with a general matrix, restricted to matching controls. */
qs_status qs_apply_1q(qs_state s, int target, const double* U,
                      uint64_t ctrl_mask, uint64_t ctrl_vals);

/* 2q gate on (t0, t1), t0 the least significant bit of the 4x4 matrix index:
 * for every index i with both target bits clear (and matching controls) the
 * quad psi[i + b0*2^t0 + b1*2^t1] (m = b0 + 2 b1) is replaced by U times it.
 * U is 4x4 complex (32 doubles). */
qs_status qs_apply_2q(qs_state s, int t0, int t1, const double* U,
                      uint64_t ctrl_mask, uint64_t ctrl_vals);

/* Dense gate on k distinct targets (1 <= k <= QS_MAX_FUSED), U 2^k x 2^k
 * complex: the same update for groups of 2^k amplitudes.  Typically U is the
 * product of several gates formed by the caller or by the planner (gate fusion,
 * Section I). */
qs_status qs_apply_fused(qs_state s, const int* targets, int k, const double* U,
                         uint64_t ctrl_mask, uint64_t ctrl_vals);

/* Diagonal gate on k distinct targets (1 <= k <= QS_MAX_FUSED): for every index
 * i whose control bits match, psi[i] *= d[j], where bit b of j is bit
 * targets[b] of i.  `diag` holds the 2^k complex entries (2^(k+1) doubles,
 * interleaved re, im; host memory, read before the call returns).  A 128-byte
 * line none of whose amplitudes has a factor other than exactly 1 is neither
 * read nor written (the memory access filtering that Section I mentions as
 * prior work); inside a touched line the unchanged amplitudes are written back
 * bit for bit.  CZ and CP(phi) with both qubits at bit 3 or above (complex128;
 * bit 4, complex64) touch a quarter of the state, a multi-controlled Z one
 * line; all factors 1 launches nothing.
 * qs_apply_1q, qs_apply_2q, qs_apply_fused and per-gate circuit runs take the
 * same kernel whenever their matrix has no nonzero off-diagonal entry. */
qs_status qs_apply_diag(qs_state s, const int* targets, int k, const double* diag,
                        uint64_t ctrl_mask, uint64_t ctrl_vals);

/* Execution options for qs_run_circuit.  Zero-initialised means defaults. */
typedef struct {
    int32_t mode;        /* 0 = auto (fused tile passes), 1 = one launch per gate */
    int32_t fuse_k;      /* 0 = default (no matrix-core blocks; register blocks only); 4 or 5 =
                            inside each tile pass, runs of gates on at most that many tile
                            qubits are multiplied (FP64, host) into one dense block applied
                            with FP64 matrix cores (both amplitude types; tiles of at least
                            fuse_k + 4 qubits).  With the environment variable
                            QS_FUSE_FP32=1 at planning time, complex64 blocks use FP32
                            matrix cores instead: the FP64 product split into an FP32 part
                            and a bfloat16 remainder, each with its own accumulator */
    int32_t tile_qubits; /* qubits held in LDS per tile; 0 = default */
    int32_t max_blocks;  /* cap on the workgroups of each tile-pass launch (they stride over
                            the tiles); 0 = default (65536).  A lower cap leaves compute units
                            to other streams, e.g. a serving loop beside a long run, at the
                            cost of this run's speed */
    int32_t remap;       /* 0 = auto: an uncontrolled SWAP gate becomes a relabeling of qubits
                            (later gates are rewritten to the swapped positions) when that saves
                            tile passes, and the qubit order is restored at the end by at most
                            two in-place passes (the swap-shifted QFT of Section III-B);
                            1 = never: SWAP gates run as 2q gates */
    int32_t rsv[3];
} qs_run_opts;

/* Apply a whole circuit (ops[0..n_ops), matrices in mats[0..n_mats)) in
 * order.  The result equals applying the gates one by one up to rounding; the
 * library may group gates into LDS tile passes and fused dense blocks.  The op
 * table and matrices are validated and copied before any work is enqueued. */
qs_status qs_run_circuit(qs_state s, const qs_op* ops, int64_t n_ops,
                         const double* mats, int64_t n_mats, const qs_run_opts* opts);

/* Plan a circuit for an n-qubit state of type dt without executing it (host
 * only; needs no GPU).  *n_passes receives the number of state read+write
 * sweeps qs_run_circuit would launch in mode 0 (LDS tile passes plus the
 * passes that restore the qubit order after SWAP relabeling), and *n_ops_out
 * the total operations inside the tile passes (a fused block counts once).
 * Same validation as qs_run_circuit. */
qs_status qs_plan_circuit(int n, qs_dtype dt, const qs_op* ops, int64_t n_ops, const double* mats,
                          int64_t n_mats, const qs_run_opts* opts, int64_t* n_passes, int64_t* n_ops_out);

/* The execution order qs_run_circuit (mode 0, no fused blocks, no SWAP
 * relabeling) gives the circuit's gates (host only; needs no GPU).  Gates that commute (neither
 * acts non-diagonally on a qubit the other touches; controls act
 * diagonally) may be reordered so that one tile pass absorbs more of them.
 * order[i] is the circuit index of the i-th gate executed and pass_of[i] its
 * pass (both n_ops long, caller-owned); tile_mask, if not NULL, receives each
 * pass's tile qubits as a bit mask (room for n_ops entries).  Same validation
 * as qs_run_circuit. */
qs_status qs_plan_order(int n, qs_dtype dt, const qs_op* ops, int64_t n_ops, const double* mats,
                        int64_t n_mats, const qs_run_opts* opts, int64_t* order, int32_t* pass_of,
                        uint64_t* tile_mask);

/* The tile passes qs_run_circuit (mode 0) would launch, for inspection and
 * for checking the planner on a host (host only; needs no GPU).  Their qubit
 * positions are physical: after SWAP relabeling, qs_plan_restore gives the
 * passes that follow them.  Call once
 * with pass_desc, ops_out and pool_out NULL to get *n_passes, *n_tile_ops
 * and *n_pool; then again with buffers of at least those sizes (the three
 * counts in, the actual counts out).  pass_desc: 36 int32 per pass: tile
 * qubits m, forced low qubits L, first op, op count, then the 32 tile qubit
 * positions ascending (-1 past m).  ops_out: *n_tile_ops records of
 * QS_TILE_OP_BYTES bytes in the library's internal op layout (kind, k,
 * p[6] as int32; lcm, lcv, gcm, gcv, moff as uint64; lp[6], dclass, dbit as
 * int8; dj, rsv as int32), which may change between versions.  pool_out:
 * the FP64 matrix pool the ops' moff index.  Same validation as
 * qs_run_circuit. */
#define QS_TILE_OP_BYTES 88
qs_status qs_plan_export(int n, qs_dtype dt, const qs_op* ops, int64_t n_ops, const double* mats,
                         int64_t n_mats, const qs_run_opts* opts, int32_t* pass_desc, int64_t* n_passes,
                         void* ops_out, int64_t* n_tile_ops, double* pool_out, int64_t* n_pool);

/* The passes qs_run_circuit (mode 0) launches after the tile passes to put the
 * qubits back in order when the planner relabeled SWAP gates (host only).
 * *n_restore (0, 1 or 2) passes; pass i is an involution of bit positions
 * given as tau[64 i + p] = the position that position p exchanges with (p
 * itself if unmoved, p < n); it swaps psi[y] with psi[y'] where y' is y with
 * the bits at each exchanged pair of positions swapped.  tau: room for 128
 * int32 (caller-owned).  Same validation as qs_run_circuit. */
qs_status qs_plan_restore(int n, qs_dtype dt, const qs_op* ops, int64_t n_ops, const double* mats,
                          int64_t n_mats, const qs_run_opts* opts, int32_t* tau, int32_t* n_restore);

/* ------------------------------------------------------------------ reductions */

/* Marginal probabilities over m distinct qubits (0 <= m <= 24): out[o] (2^m
 * doubles, host memory) = sum of |psi_i|^2 over indices i whose bits at
 * qubits[0..m) spell o (qubits[0] is bit 0 of o).  Accumulated in FP64 in a
 * fixed order, so repeated calls give bitwise equal results.  Blocking. */
qs_status qs_probabilities(qs_state s, const int* qubits, int m, double* out);

/* Squared norm sum |psi_i|^2 in FP64 (the m = 0 case).  Blocking. */
qs_status qs_norm(qs_state s, double* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * marginal probabilities of qs_probabilities -- same kernels, same summation
 * order, so bitwise the same numbers -- without any allocation.  dev_out:
 * DEVICE memory for 2^m doubles, caller-owned.  The work is enqueued on the
 * state's stream and the call returns at once (nothing is copied to the host
 * and nothing waits); read dev_out after that stream.  The partial sums live
 * in one fixed scratch array per GPU (2^22 + 2^12 doubles = 32 MiB + 32 KiB,
 * held by the library until the process ends), so the call calls no
 * hipMalloc/hipFree or allocating routine: QS_ERR_ARG when the reduction
 * would need more than that (2^(n-12) partial sums for m <= n - 12, else 2^m,
 * plus a 4096th of them for the second level of the final sum when an
 * outcome has more than 4096: every n <= 34 with m <= 22 fits), or for a
 * NULL dev_out or the qubit list errors of
 * qs_probabilities.  Every call on one GPU shares that array, and each call
 * overwrites all of it that it reads, so calls need no clearing between them;
 * calls that overlap on one GPU (different streams, or different threads)
 * race and must be ordered by the caller. */
qs_status qs_probabilities_noalloc(qs_state s, const int* qubits, int m, double* dev_out);

/* Expectation value <psi|P|psi> of the Pauli string P = i^w X^x Z^z with
 * w = popcount(x_mask & z_mask): X on the qubits of x_mask, Z on those of
 * z_mask, Y = iXZ on qubits in both.  Summed in FP64 in a fixed order as
 * i^w * sum_k conj(psi_{k ^ x}) psi_k (-1)^popcount(k & z); out[0] = real
 * part, out[1] = imaginary part (0 up to rounding, P being Hermitian).  The
 * state is not normalised first.  Blocking.  QS_ERR_ARG for mask bits at or
 * above n. */
qs_status qs_expect_pauli(qs_state s, uint64_t x_mask, uint64_t z_mask, double* out);

/* Sample basis-state indices from |psi_i|^2 / sum_j |psi_j|^2 by inverting
 * the cumulative distribution at the caller's uniforms u[0..shots), each in
 * [0, 1): out[k] is the smallest index whose cumulative probability exceeds
 * u[k] (FP64 chunk sums over min(4096, 2^n) amplitudes with a compensated
 * prefix, then a walk inside the chunk; results may differ from an exact
 * inversion only when u[k] lies within rounding of a boundary).  u and out
 * are host arrays of shots elements, owned by the caller.  Blocking.
 * QS_ERR_ARG for shots < 0 or a uniform outside [0, 1). */
qs_status qs_sample(qs_state s, const double* u, int64_t shots, uint64_t* out);

/* Wait for all work enqueued on the state. */
qs_status qs_sync(qs_state s);

/* ------------------------------------------------------------------ batches */

typedef struct qs_batch_s* qs_batch;

/* What a batch or served circuit writes to its `out` when it completes. */
enum {
    QS_WANT_NONE = 0,  /* nothing (results stay in the batch / server until read) */
    QS_WANT_STATE = 1, /* the final state: 2^n amplitudes in the batch / server dtype */
    QS_WANT_PROBS = 2, /* |psi_i|^2 for every index i: 2^n doubles (n <= 24) */
    QS_WANT_NORM = 3   /* sum of |psi_i|^2: one double */
};

/* One circuit of a batch or serving request: n qubits, its initial state, op
 * table and matrix pool exactly as for qs_run_circuit, and the result it
 * delivers on completion.
 * - Initial state: the basis state |init_basis>, or, when init_state is not
 *   NULL, the 2^n amplitudes at init_state: DEVICE memory on the batch's or
 *   server's GPU, in its dtype, caller-owned; it is read on the device, so
 *   it must stay valid and unchanged until qs_batch_wait returns (and for
 *   every qs_batch_replay) or until the served request has finished.
 *   init_basis is ignored then.
 * - Result: with want != QS_WANT_NONE, `out` (HOST memory, caller-owned, of
 *   the size QS_WANT_* names) receives the result: for a batch, each time
 *   qs_batch_wait returns QS_OK; for a served request, before qs_server_poll
 *   reports it finished.  The per-circuit queries (qs_batch_download,
 *   qs_batch_probabilities, qs_batch_norm, qs_server_download) stay
 *   available either way. */
typedef struct {
    int32_t n;
    int32_t want;           /* QS_WANT_* */
    uint64_t init_basis;
    const qs_op* ops;
    int64_t n_ops;
    const double* mats;
    int64_t n_mats;
    const void* init_state; /* NULL = start from |init_basis> */
    void* out;              /* host buffer for `want` (NULL when want == QS_WANT_NONE) */
} qs_circuit;

typedef struct {
    int32_t dtype;       /* QS_C64 or QS_C128 (0 = QS_C128) for every state of the batch */
    int32_t mode;        /* 0 = fused (LDS-resident / persistent / tile passes), 1 = one launch per gate */
    int32_t streams;     /* HIP streams the batch spreads over (0 = 8) */
    int32_t fuse_k;      /* as in qs_run_opts */
    int32_t tile_qubits; /* as in qs_run_opts */
    int32_t graph;       /* mode 0: 1 = capture the device work in a HIP graph (launched now and
                            by every qs_batch_replay) */
    int32_t whole_max;   /* mode 0: circuits with n <= whole_max run whole in one workgroup's LDS
                            (0 = 12 for complex128, 13 for complex64; at most those) */
    int32_t persist_max; /* mode 0: circuits with whole_max < n <= persist_max run their passes in
                            one persistent workgroup, larger ones pass-major (0 = 15 / 16; at
                            most 20) */
} qs_batch_opts;

typedef struct {
    uint64_t launches;   /* kernel launches enqueued */
    uint64_t passes;     /* tile passes planned (fused mode) */
    double device_ms;    /* first event to last completion, after qs_batch_wait */
    double class_ms[3];  /* fused mode: completion of the LDS-resident, persistent and
                            pass-major classes, from the same first event (0 if empty) */
    uint32_t class_circuits[3];
    uint32_t rsv;
    double submit_ms[4]; /* host time inside qs_batch_submit: device allocation, planning,
                            packing the plans into one descriptor buffer, upload and
                            enqueue */
} qs_batch_stats;

/* Run `count` independent circuits (the paper times one circuit at a time,
 * Section III).  All circuits are validated first (nothing
 * is enqueued if one is invalid), then one device arena is allocated for all
 * final states and the work is enqueued on the batch's own streams; the call
 * returns without waiting.  Each circuit's result equals running it alone with
 * qs_run_circuit (mode 0) or gate by gate (mode 1); it does not depend on the
 * other circuits of the batch.  The caller's tables may be freed on return. */
qs_status qs_batch_submit(const qs_circuit* circuits, int count, const qs_batch_opts* opts, qs_batch* out);

/* Wait until the batch is done (timeout_ms < 0: no limit).  QS_ERR_TIMEOUT if
 * it is still running after timeout_ms; the batch stays valid. */
qs_status qs_batch_wait(qs_batch b, int timeout_ms);

/* Device pointer and qubit count of circuit i's final state (owned by the
 * batch; valid until qs_batch_release; complete after qs_batch_wait). */
qs_status qs_batch_state(qs_batch b, int i, void** dev_ptr, int* n);

/* Copy circuit i's final state to host memory (2^n elements of the batch
 * dtype); waits for the batch first. */
qs_status qs_batch_download(qs_batch b, int i, void* host);

/* Marginal probabilities (as qs_probabilities: 0 <= m <= min(24, n), distinct
 * qubits, out[o] over the indices whose qubits[j] bits spell o, FP64 in a fixed
 * order) and squared norm of circuit i's final state, computed on the device
 * from the state in the batch arena; wait for the batch first and block until
 * out (host, 2^m doubles / one double) is filled.  Together with
 * qs_batch_download they give each circuit's result as a state, a distribution
 * or a norm.  Not thread-safe against other calls on the same batch. */
qs_status qs_batch_probabilities(qs_batch b, int i, const int* qubits, int m, double* out);
qs_status qs_batch_norm(qs_batch b, int i, double* out);

qs_status qs_batch_get_stats(qs_batch b, qs_batch_stats* out);

/* Run a fused (mode 0) batch again: the same circuits and plans, states
 * recomputed from their initial basis states, with no host planning or
 * upload (replaying the HIP graph if the batch was submitted with graph = 1).
 * Waits for the previous run first; returns without waiting for this one.
 * Results are bitwise those of the first run.  QS_ERR_UNSUPPORTED for
 * mode 1 batches. */
qs_status qs_batch_replay(qs_batch b);

/* One candidate configuration timed by qs_batch_tune. */
typedef struct {
    int32_t tile_qubits;
    int32_t fuse_k;
    int32_t whole_max;   /* class boundaries as in qs_batch_opts (never 0 here) */
    int32_t persist_max;
    double device_ms;    /* best device time of two replays of the sample */
} qs_tune_entry;

/* Autotune a batch configuration on a sample of circuits.  Stage 1 times
 * every tile size (10..12) and fused matrix-core width (0, 4, 5) with the
 * default class boundaries; stage 2 keeps the fastest of those and
 * times the workgroup classes around the defaults (whole-in-LDS limit one
 * lower; persistent limit two lower to two higher).  Each candidate is
 * planned, run, and replayed twice on the device; *opts (dtype and mode as
 * given, mode 0 only) gets the fastest tile_qubits, fuse_k, whole_max and
 * persist_max.  out[0..max_out) receives the timings (NULL allowed), *n_out
 * their number.  Allocates and frees device memory for the sample's states. */
qs_status qs_batch_tune(const qs_circuit* sample, int count, qs_batch_opts* opts, qs_tune_entry* out, int max_out,
                        int* n_out);

/* Wait for outstanding work and free the batch (NULL accepted). */
qs_status qs_batch_release(qs_batch b);

/* ------------------------------------------------------------------ serving */

typedef struct qs_server_s* qs_server;

typedef struct {
    int32_t dtype;        /* QS_C64 or QS_C128 (0 = QS_C128) */
    int32_t rounds_ahead; /* rounds enqueued ahead of completion (0 = 3, max 16) */
    uint64_t hbm_budget;  /* bytes of device memory for request states (0 = half the free memory) */
    uint64_t plan_budget; /* bytes of device memory for request plans (0 = 256 MiB) */
    int32_t tile_qubits;  /* tile size of the passes (0 = default; 9..13) */
    int32_t fuse_k;       /* as in qs_run_opts */
    int32_t rsv[4];
} qs_server_opts;

typedef struct {
    uint64_t id;
    int32_t status;       /* QS_OK, or why the request failed / was cancelled */
    int32_t n;
    double t_submit_ms;   /* milliseconds since qs_server_create, steady clock */
    double t_admit_ms;
    double t_done_ms;     /* when the server saw the last round of the request complete */
} qs_result;

typedef struct {
    uint64_t submitted, admitted, completed, failed, cancelled;
    uint64_t rounds, launches;
    uint64_t budget_bytes, used_bytes, peak_bytes;
    uint32_t queued, active;
} qs_server_stats;

/* Create a serving loop with its own stream and device pools (the paper runs
 * one circuit at a time).  Requests are admitted
 * in arrival order (later small ones may pass a large one that does not fit
 * yet, up to 64 times) while their state fits hbm_budget; admitted requests
 * advance together in rounds of one tile pass each, and requests arriving
 * while others run join the next round (continuous batching).  Each result is
 * bitwise the same as the request run alone. */
qs_status qs_server_create(const qs_server_opts* opts, qs_server* out);

/* Queue a request (validated and copied; the caller's tables may be freed).
 * QS_ERR_OOM at once if its state could never fit the budget.  A request
 * whose plan (passes, ops and fused matrices, known once it is planned at
 * admission) is larger than the whole plan_budget finishes with status
 * QS_ERR_ARG instead of waiting in the queue. */
qs_status qs_server_submit(qs_server s, const qs_circuit* c, uint64_t* id);

/* One scheduler tick: retire finished rounds, admit queued requests that fit,
 * enqueue up to rounds_ahead rounds, and return up to `max` newly finished
 * requests (*count of them).  Never blocks on the GPU. */
qs_status qs_server_poll(qs_server s, qs_result* out, int max, int* count);

/* A finished request's state: device pointer (owned by the server) and n;
 * QS_ERR_BUSY while it is queued or running. */
qs_status qs_server_state(qs_server s, uint64_t id, void** dev_ptr, int* n);
qs_status qs_server_download(qs_server s, uint64_t id, void* host);

/* Free a finished (or failed / cancelled) request and its state. */
qs_status qs_server_release(qs_server s, uint64_t id);

/* Cancel a request that is still queued (QS_ERR_BUSY otherwise). */
qs_status qs_server_cancel(qs_server s, uint64_t id);

qs_status qs_server_get_stats(qs_server s, qs_server_stats* out);

/* Wait for outstanding rounds and free the server and every state it holds. */
qs_status qs_server_destroy(qs_server s);

/* ------------------------------------------------------------------ tracing */

/* One traced kernel launch. */
typedef struct {
    int32_t kind;       /* QS_K_* below */
    int32_t n;
    int32_t t0, t1;     /* first two targets (-1 if unused) */
    int32_t nctrl;
    int32_t dtype;
    uint64_t bytes;     /* algorithmic HBM bytes: 2 * S * amplitudes touched */
    uint64_t updates;   /* amplitude updates credited to the launch */
    float ms;           /* duration between HIP events around the launch */
    int32_t rsv;
} qs_trace_rec;

enum {
    QS_K_INIT = 0, QS_K_1Q_HI = 1, QS_K_1Q_LO = 2, QS_K_2Q = 3, QS_K_KQ = 4,
    QS_K_TILE = 5, QS_K_MFMA = 6, QS_K_REDUCE = 7, QS_K_DIAG = 8, QS_K_PERM = 9,
    QS_K_PROBE = 10, QS_K_SAMPLE = 11
};

/* Start (on != 0) or stop recording HIP events around every launch on the
 * state's stream.  Starting clears earlier records. */
qs_status qs_trace_enable(qs_state s, int on);

/* Wait for traced work and copy up to `max` records; *count = records copied. */
qs_status qs_trace_read(qs_state s, qs_trace_rec* out, int max, int* count);

/* Measurement helper, not a step of the method: the memory ceiling that every
 * gate pass is bounded by.  Reads every 16-byte word of the state's amplitude
 * buffer and writes it back in place, unchanged (bitwise, whatever the
 * buffer holds), enqueued on the state's stream like a gate (a traced launch
 * of class QS_K_PROBE with bytes = 2 x the buffer).  The schedule is the
 * per-gate kernel's: a workgroup of 256 lanes per chunk of 256 x `slots`
 * words, a lane's slots 2^spread_log2 words apart (slots 1, 2, 4 or 8;
 * spread_log2 8..30), non-temporal loads and stores; the per-gate kernel's
 * occupancy and chunk-order knobs (gate_wg_per_cu, gate_xcd_swizzle) apply.
 * QS_ERR_ARG for other values. */
qs_status qs_probe_inplace(qs_state s, int slots, int spread_log2);

/* ------------------------------------------------------------------ schedule autotuner */

/* Gate classes of the per-gate kernel's memory schedule: 0 = every target
 * inside a 128-byte line (members exchanged by shuffles), 1 = one-qubit gate
 * on a target at bit 6 or above, 2 = two-qubit gate with one such target, 3 =
 * two-qubit gate with both. */
#define QS_GATE_CLASSES 4

/* A tuned schedule: slots per lane (1, 2, 4 or 8), workgroups per CU (0 = as
 * many as fit), chunk order (1 = each of the 8 XCDs walks a contiguous
 * eighth), and the rate the timing measured (GB/s of bytes read and written
 * by the class's representative gates). */
typedef struct {
    int32_t cls;
    int32_t slots;
    int32_t wg_per_cu;
    int32_t xcd;
    double gbs;
    int32_t from_cache; /* 1 = read from the cache file, 0 = timed by this call */
} qs_gate_sched;

/* Autotune the per-gate kernel's memory schedule for the state's amplitude
 * type and qubit count (the paper's counterpart is choosing its kernel
 * variants per machine, Section II).  For each class,
 * every candidate (slots 1/2/4, and 8 for class 0; 0, 2, 3, 4, 6 or 8
 * workgroups per CU; either chunk order) is timed on `s` with Pauli X gates on
 * representative targets, each applied twice, so every amplitude ends as it
 * started (only the sign of an exactly zero amplitude may change).  The
 * fastest becomes the process-wide schedule for gates of that class on states
 * of this type and size; explicit launch knobs (qs_tunable_set) still take
 * precedence.  With `cache_path` (host path, may be NULL): classes found
 * there under this device's key (architecture, CU count, type, n) are loaded
 * instead of timed, and newly timed ones are written back, one JSON object
 * per line, the file replaced atomically.  out[0..max_out) receives the
 * schedules by class (NULL allowed), *n_out their number.  Blocking; takes a
 * few seconds per class at 30 qubits.  QS_ERR_ARG for n < 12 or an
 * unwritable cache file.  Schedules never change results (bitwise). */
qs_status qs_tune_gates(qs_state s, const char* cache_path, qs_gate_sched* out, int max_out, int* n_out);

/* Drop every tuned schedule: gates use the built-in table again. */
qs_status qs_tune_gates_reset(void);

/* ------------------------------------------------------------------ launch knobs */

/* Launch knobs that change how work is spread over the GPU, never what is
 * computed: every setting gives bitwise the same results.  Each starts at its
 * built-in default, or at its environment variable (in brackets) when that is
 * set when the library first reads a knob.
 *   gate_grid_cap     [QS_GATE_GRID_CAP]  workgroups of one per-gate or diagonal
 *                                         launch, 1..2^22 (default 2^22); the
 *                                         workgroups loop over the rest
 *   tile_grid_cap     [QS_TILE_GRID_CAP]  workgroups of a tile pass (65536)
 *   round_grid_cap    [QS_ROUND_GRID_CAP] workgroups of a batch / serving round (65536)
 *   aux_grid_cap      [QS_GRID_CAP]       workgroups of init and dense k-qubit kernels (16384)
 *   nontemporal       [QS_NT]             1 = streaming loads/stores where whole lines are written
 *   slot_spread_log2  [QS_SLOG]           per-gate kernel: counter distance of a lane's slots (11)
 *   slots_no_high, slots_one_high, slots_two_high  [QS_PPL_H0/H1/H2]
 *                                         per-gate kernel: slots per lane for gates with 0, 1 or
 *                                         2 targets at bit 6 or above (1, 2, 4 or 8; 0 = built-in
 *                                         table)
 *   diag_spread_log2  [QS_DIAG_SLOG]      diagonal kernel slot distance (11)
 *   perm_run_log2     [QS_PERM_RUN]       restore pass run length (0 = built-in)
 *   gate_xcd_swizzle  [QS_GATE_XCD]       per-gate kernel chunk order: 0 = built-in rule,
 *                                         1 = workgroup order, 2 = each of the 8 XCDs walks a
 *                                         contiguous eighth of the chunks
 *   gate_wg_per_cu    [QS_GATE_WG_PER_CU] per-gate kernel (and qs_probe_inplace): workgroups
 *                                         per CU, capped through unused LDS (0 = built-in rule
 *                                         for gates, no cap for the probe; 8 and more: no cap
 *                                         in effect)
 *   diag_slots        [QS_DIAG_SLOTS]     diagonal kernel: slots per lane (1, 2, 4 or 8; 0 =
 *                                         built-in); gate_wg_per_cu and gate_xcd_swizzle apply
 *                                         to the diagonal kernel too
 *   gate_low_in_regs  [QS_GATE_LOW_HIGH]  per-gate kernel: targets below bit 6 held in a lane's
 *                                         registers instead of exchanged by shuffles (0 none,
 *                                         1 = default: those at or above the 128-byte line,
 *                                         2 all)
 *   tile_waves4       [QS_TILE_W4]        tile passes of 2^11 amplitudes without k >= 3 ops:
 *                                         1 (default) = the kernel held to 4 waves per SIMD,
 *                                         0 = the kernel the compiler sizes (3 waves)
 *   reduce_xcd_order  [QS_RED_XCD]        chunk order of the norm, marginal and Pauli reductions:
 *                                         0 = built-in rule (XCD-contiguous for the norm, sampling
 *                                         and Pauli strings on states of 512 MiB and more, workgroup
 *                                         order for marginals), 1 = workgroup order, 2 = each of
 *                                         the 8 XCDs reads a contiguous eighth of the chunks
 * qs_tunable_set stores `value` (value < 0: back to the default / environment
 * value); QS_ERR_ARG for an unknown name or a value outside the knob's range.
 * Knobs are process-wide and may be changed from any thread; a launch being
 * set up concurrently may still use the old value. */
qs_status qs_tunable_set(const char* name, int64_t value);
qs_status qs_tunable_get(const char* name, int64_t* value);

#ifdef __cplusplus
}
#endif

#endif /* QS_H */
