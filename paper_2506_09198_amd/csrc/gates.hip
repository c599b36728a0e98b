// Per-gate kernels for gfx950 (wave64).
//
//   k_init_basis   zero the state and set one amplitude to 1.
//   k_gate         1q and 2q gates: the pair update of Alg. 1 for a general
//                  matrix (and its 4x4 analogue), controls as in
//                  Fig. control6q2.  Targets at bit 6 and above are reached by
//                  bit-inserted indexing (each lane holds the group members in
//                  registers); targets below bit 6 by cross-lane shuffles, so
//                  every memory instruction of a wave covers 64 consecutive
//                  amplitudes whatever the targets.
//   k_kq_lds       dense gate on k <= 6 targets: groups of 2^k amplitudes are
//                  staged through LDS with the matrix, one output per lane.
#include <algorithm>
#include <cstring>
#include <type_traits>

#include "device_common.h"

namespace qs {

InsertPlan make_insert_plan(uint64_t mask)
{
    InsertPlan p;
    p.n = 0;
    for (int b = 0; b < 64 && p.n < kMaxIns; ++b)
        if ((mask >> b) & 1) p.low[p.n++] = (b == 63) ? ~0ull >> 1 : ((1ull << b) - 1);
    return p;
}

static uint64_t grid_cap() { return (uint64_t)tun(T_AUX_GRID_CAP); }

static unsigned blocks_for(uint64_t items, uint64_t per_block)
{
    uint64_t b = (items + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > grid_cap()) b = grid_cap();
    return (unsigned)b;
}

// ---------------------------------------------------------------- K0 init

template <typename V>
__global__ void __launch_bounds__(256) k_init_basis(V* __restrict__ psi, uint64_t namps, uint64_t x)
{
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < namps; i += stride) {
        V v;
        v.x = (i == x) ? 1 : 0;
        v.y = 0;
        psi[i] = v;
    }
}

hipError_t launch_init_basis(void* psi, int dt, int n, uint64_t x, hipStream_t st)
{
    const uint64_t N = 1ull << n;
    const unsigned g = blocks_for(N, 256 * 4);
    if (dt == QS_C128)
        hipLaunchKernelGGL(k_init_basis<double2>, dim3(g), dim3(256), 0, st, (double2*)psi, N, x);
    else
        hipLaunchKernelGGL(k_init_basis<float2>, dim3(g), dim3(256), 0, st, (float2*)psi, N, x);
    return hipGetLastError();
}

// ---------------------------------------------------------------- K1-K3

// One kernel family for 1q and 2q gates.  Let K be the number of targets and
// NH of them lie at bit 6 or above ("high"); the other NL = K - NH are "low"
// (inside a 64-amplitude run).  A compact counter k enumerates the amplitudes
// whose high-target bits are 0 and whose high control bits match; its low 6
// bits are the lane, so every load and store instruction of a wave covers 64
// consecutive amplitudes.  A lane holds, per slot, the 2^NH amplitudes that
// differ in the high-target bits (registers); the partners along low targets
// sit in other lanes of the same wave and arrive by cross-lane shuffles.  Each
// lane then forms its own outputs from the 2^K group members.  Controls below
// bit 6 are tested per amplitude (the whole wave still takes part in the
// shuffles); controls at bit 6 or above are inserted into the counter.
//
// Memory schedule (measured on MI355X for in-place read-modify-write; see
// gate_sched below): one counter chunk per block (no grid-stride loop), a
// lane's PPL slots spread S = 2^11 counter steps apart, non-temporal loads
// and stores when every store instruction writes whole lines, occupancy
// capped through unused LDS, and an optional XCD-contiguous chunk order.
// Targets below bit 6 but at or above the 128-byte line are held in
// registers like high ones (each load instruction then still covers whole
// lines); only targets inside a line are exchanged by shuffles.
struct GateArgs {
    uint64_t C;          // counter range
    uint64_t cv_hi;      // control values at positions >= 6
    uint64_t nblocks;    // counter chunks (blocks loop when the grid is capped)
    uint32_t cm_lo, cv_lo;
    uint32_t lowmask;    // lane bits of the low targets
    int32_t slog;        // log2 of the slot spread S
    int32_t xcd;         // chunk order: 0 = block order, 1 = each XCD a contiguous eighth
    int32_t skip_fail;   // lanes whose in-line controls fail skip their stores (64-byte pieces)
    uint64_t roff[4];    // register r -> index offset (high-target bits of r)
    int32_t srcl[4];     // member m -> lane bits of its low targets
    int32_t hreg[4];     // member m -> register holding it
    int32_t tlow[2];     // target j is low?
    int32_t tbit[2];     // target j: lane bit (low) or register bit (high)
    double U[32];        // 2^K x 2^K complex, row-major
    InsertPlan ip;       // high targets and high controls, inserted into k
};

// Register r of a lane's slot, chosen with selects (r is a runtime value).
template <int NR>
__device__ __forceinline__ double2 pick(const double2 (&x)[NR], int r)
{
    double2 v = x[0];
#pragma unroll
    for (int i = 1; i < NR; ++i)
        if (r == i) v = x[i];
    return v;
}

template <typename R, int K, int NH, int PPL, bool NT>
__global__ void __launch_bounds__(256) k_gate(typename CT<R>::V* __restrict__ psi, GateArgs ga)
{
    using V = typename CT<R>::V;
    constexpr int D = 1 << K;
    constexpr int NR = 1 << NH;
    __shared__ double su[2 * D * D];
    if (threadIdx.x < 2 * D * D) su[threadIdx.x] = ga.U[threadIdx.x];
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t S = 1ull << ga.slog;
    const uint64_t spb = S >> 8;
    for (uint64_t bb = blockIdx.x; bb < ga.nblocks; bb += gridDim.x) {
    // Workgroups are dispatched to the 8 XCDs round-robin; with xcd set the
    // chunk of workgroup bb is (bb mod 8) * nblocks/8 + bb/8 (nblocks is a
    // multiple of 8 then), a bijection on the chunks.
    const uint64_t b = ga.xcd ? (bb & 7) * (ga.nblocks >> 3) + (bb >> 3) : bb;
    const uint64_t base = (b / spb) * (S * PPL) + (b % spb) * 256 + threadIdx.x;

    // Controls inside a 128-byte line are tested per lane.  A lane whose
    // control bits fail stores its amplitudes back unchanged, bit for bit, so
    // every store instruction still writes whole lines, unless the changed
    // amplitudes come in aligned 64-byte halves of lines (skip_fail): measured
    // on MI355X, lines written in 16- or 32-byte pieces cost 10-18 % more than
    // whole lines, 64-byte halves about 3 % less.
    const uint32_t myctl = lane & ga.cm_lo;
    const bool cok = myctl == ga.cv_lo;
    double2 x[PPL][NR];
    uint64_t idx[PPL];
    bool live[PPL];
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        const uint64_t k = base + (uint64_t)p * S;
        live[p] = k < ga.C;
        idx[p] = ins_bits(k, ga.ip) | ga.cv_hi;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if (live[p])
                x[p][r] = ld2(gld<NT>(psi + (idx[p] | ga.roff[r])));
            else
                x[p][r] = make_double2(0.0, 0.0);
        }
    }
    // row of the matrix each register of this lane computes
    int rr[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        int v = 0;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int bit = ga.tlow[j] ? (int)((lane >> ga.tbit[j]) & 1) : ((r >> ga.tbit[j]) & 1);
            v |= bit << j;
        }
        rr[r] = v;
    }
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        double2 mem[D];
#pragma unroll
        for (int m = 0; m < D; ++m) {
            // all-high gates keep member m in register m (targets in order)
            const double2 v = (NH == K) ? x[p][m & (NR - 1)] : pick<NR>(x[p], ga.hreg[m]);
            if (NH == K) {
                mem[m] = v; // no low targets: every member is in this lane
            } else {
                const int src = (int)((lane & ~ga.lowmask) | (uint32_t)ga.srcl[m]);
                mem[m].x = __shfl(v.x, src, 64);
                mem[m].y = __shfl(v.y, src, 64);
            }
        }
        if (live[p]) {
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                double sr = 0.0, si = 0.0;
#pragma unroll
                for (int m = 0; m < D; ++m) {
                    const double ur = su[2 * (rr[r] * D + m)], ui = su[2 * (rr[r] * D + m) + 1];
                    sr += ur * mem[m].x - ui * mem[m].y;
                    si += ur * mem[m].y + ui * mem[m].x;
                }
                // plain double selects (a select of double2 values is lowered
                // through a per-lane indexed stack copy)
                const double ox = cok ? sr : x[p][r].x, oy = cok ? si : x[p][r].y;
                if (cok || !ga.skip_fail) gst<NT>(psi + (idx[p] | ga.roff[r]), st2<V>(make_double2(ox, oy)));
            }
        }
    }
    }
}

// LDS bytes a workgroup must hold so that at most `wg` fit on one CU (160 KiB
// of LDS per CU on gfx950): just over a (wg+1)-th of it, so wg + 1 do not fit
// and wg do.  The unused part caps the kernel's occupancy.
size_t pad_for_wg_per_cu(int wg, size_t static_lds)
{
    if (wg <= 0) return 0;
    const size_t per = 163840 / ((size_t)wg + 1) + 64;
    return per > static_lds ? per - static_lds : 0;
}

template <typename R, int K, int NH, int PPL>
static hipError_t launch_gate_p(void* psi, const GateArgs& ga, bool nt, int wg_per_cu, hipStream_t st)
{
    using V = typename CT<R>::V;
    // One block per counter chunk up to the cap (at most 2^22: 2^32 threads
    // would overflow the dispatch size); beyond it the blocks loop over the
    // remaining chunks.
    const uint64_t cap = (uint64_t)tun(T_GATE_GRID_CAP);
    const unsigned g = (unsigned)(ga.nblocks < cap ? ga.nblocks : cap);
    constexpr size_t kStatic = 2 * (1 << K) * (1 << K) * sizeof(double); // the matrix in LDS
    const size_t pad = pad_for_wg_per_cu(wg_per_cu, kStatic);
    const void* fn = nt ? (const void*)k_gate<R, K, NH, PPL, true> : (const void*)k_gate<R, K, NH, PPL, false>;
    hipError_t e = lds_optin(fn, pad);
    if (e != hipSuccess) return e;
    if (nt)
        hipLaunchKernelGGL((k_gate<R, K, NH, PPL, true>), dim3(g), dim3(256), pad, st, (V*)psi, ga);
    else
        hipLaunchKernelGGL((k_gate<R, K, NH, PPL, false>), dim3(g), dim3(256), pad, st, (V*)psi, ga);
    return hipGetLastError();
}

// The memory schedule of one gate: slots per lane, workgroups per CU (0 = as
// many as fit) and chunk order.  Measured on MI355X at n=30 (16 GiB complex128
// and 8 GiB complex64 states) over every target, in-place:
// - the bytes of loads in flight per CU, not occupancy as such, set the rate
//   of the streaming cases: about 32 KiB per CU for two-stream gates (one
//   high target) and 48 KiB for four-stream ones (two high targets) give
//   6.1-6.8 TB/s, while full occupancy keeps two to three times that in
//   flight and thrashes DRAM pages (5.4-6.1 TB/s for complex128; complex64
//   at the complex128 workgroup counts drops to 3-4.4 TB/s, half the bytes in
//   flight).  Gates whose members are exchanged by shuffles (a target inside
//   a 128-byte line) are bound by the shuffle latency instead and want more
//   waves: 3 workgroups of 8 slots (complex128), as many as fit (complex64).
//   Complex128 / complex64 workgroups per CU: one high target 4 / 8, two
//   high targets 3 / 6, shuffled 3 / 8;
// - every XCD walking its own contiguous eighth of the chunks beats
//   workgroup order on most target distances (by up to 25 % for pairs 8-32
//   MiB apart); which order wins for a given distance varies between boxes
//   (the physical placement of the buffer differs), so XCD order is taken
//   whenever a target is held in registers;
// - states that fit the 256 MB Infinity Cache keep full occupancy and
//   workgroup order (their traffic does not reach the DRAM pages).
// The slots_*, gate_wg_per_cu and gate_xcd_swizzle knobs override the rule.
struct GateSched {
    int ppl, wg, xcd;
};

template <typename R, int K, int NH>
static GateSched gate_sched(uint64_t state_bytes)
{
    constexpr bool C128 = sizeof(R) == 8;
    GateSched g;
    if (NH == 0)
        g = {8, C128 ? 3 : 8, 0};
    else if (NH == 1 && K == 2) // the other target is exchanged by shuffles
        g = {2, C128 ? 3 : 8, 1};
    else if (NH == 1)
        g = {1, C128 ? 4 : 8, 1};
    else
        g = {1, C128 ? 3 : 6, 1};
    if (state_bytes < (512ull << 20)) {
        g.wg = 0;
        g.xcd = 0;
    }
    // a schedule tuned for this type, size and class (qs_tune_gates)
    constexpr int cls = NH == 0 ? 0 : (NH == 1 ? (K == 1 ? 1 : 2) : 3);
    GateSchedOverride o;
    const int n = 63 - __builtin_clzll(state_bytes / (2 * sizeof(R)));
    if (gate_sched_override(C128 ? QS_C128 : QS_C64, n, cls, &o)) {
        g.ppl = o.ppl;
        g.wg = o.wg;
        g.xcd = o.xcd;
    }
    const int ppl_k = (int)tun(NH == 0 ? T_PPL_H0 : (NH == 1 ? T_PPL_H1 : T_PPL_H2));
    if (ppl_k > 0) g.ppl = ppl_k;
    const int wg_k = (int)tun(T_GATE_WG_PER_CU);
    if (wg_k > 0) g.wg = wg_k;
    const int xcd_k = (int)tun(T_GATE_XCD);
    if (xcd_k > 0) g.xcd = xcd_k - 1;
    return g;
}

template <typename R, int K, int NH>
static hipError_t launch_gate_k(void* psi, GateArgs& ga, bool nt, uint64_t state_bytes, hipStream_t st)
{
    const GateSched gs = gate_sched<R, K, NH>(state_bytes);
    auto go = [&](auto pplc) {
        constexpr int P = decltype(pplc)::value;
        const int sl = (int)tun(T_SLOG);
        ga.slog = (ga.C >= ((1ull << sl) * P)) ? sl : 8;
        ga.nblocks = (ga.C + 256 * P - 1) / (256 * P);
        ga.xcd = (gs.xcd && ga.nblocks % 8 == 0) ? 1 : 0;
        return launch_gate_p<R, K, NH, P>(psi, ga, nt, gs.wg, st);
    };
    if (gs.ppl == 1) return go(std::integral_constant<int, 1>());
    if (gs.ppl == 2) return go(std::integral_constant<int, 2>());
    if constexpr (NH == 0)
        if (gs.ppl >= 8) return go(std::integral_constant<int, 8>());
    return go(std::integral_constant<int, 4>());
}

template <typename R>
static hipError_t apply_gate_t(void* psi, int n, int K, const int* t, const double* U, uint64_t cm, uint64_t cv,
                               hipStream_t st)
{
    // Amplitudes per 128-byte line: controls at or above this bit select whole
    // lines and are inserted into the counter (only needed lines are read);
    // controls below it are tested per amplitude.
    constexpr int LINE_BITS = sizeof(R) == 8 ? 3 : 4;
    GateArgs ga;
    std::memset(&ga, 0, sizeof ga);
    const int D = 1 << K;
    for (int i = 0; i < 2 * D * D; ++i) ga.U[i] = U[i];
    const uint64_t linemask = (1ull << LINE_BITS) - 1;
    const uint64_t cm_ins = cm & ~linemask;
    // lane bits: the lowest 6 positions not taken by inserted controls (or,
    // with the low-in-registers knob, by targets held in registers)
    // With targets moved into registers, every other target at or above the
    // line is kept out of the lane bits too (it would otherwise slide into
    // the six lane positions and be exchanged by shuffles).
    const int lowhigh = (int)tun(T_GATE_LOW_HIGH);
    uint64_t reg_low = 0, not_lane = 0;
    if (lowhigh)
        for (int j = 0; j < K; ++j) {
            if (t[j] < 6 && (lowhigh == 2 || t[j] >= LINE_BITS)) reg_low |= 1ull << t[j];
            if (lowhigh == 2 || t[j] >= LINE_BITS) not_lane |= 1ull << t[j];
        }
    int lanepos[6];
    int nl = 0;
    for (int q = 0; q < 64 && nl < 6; ++q)
        if (!(((cm_ins | not_lane) >> q) & 1)) lanepos[nl++] = q;
    uint64_t himask = 0;
    int nh = 0;
    uint32_t lowmask = 0;
    for (int j = 0; j < K; ++j) {
        int lb = -1;
        for (int l = 0; l < 6; ++l)
            if (lanepos[l] == t[j]) lb = l;
        if (lb < 0) {
            ga.tlow[j] = 0;
            ga.tbit[j] = nh++;
            himask |= 1ull << t[j];
        } else {
            ga.tlow[j] = 1;
            ga.tbit[j] = lb;
            lowmask |= 1u << lb;
        }
    }
    ga.lowmask = lowmask;
    for (int r = 0; r < (1 << nh); ++r) {
        uint64_t off = 0;
        for (int j = 0; j < K; ++j)
            if (!ga.tlow[j] && ((r >> ga.tbit[j]) & 1)) off |= 1ull << t[j];
        ga.roff[r] = off;
    }
    for (int m = 0; m < D; ++m) {
        int sl = 0, hr = 0;
        for (int j = 0; j < K; ++j)
            if ((m >> j) & 1) {
                if (ga.tlow[j])
                    sl |= 1 << ga.tbit[j];
                else
                    hr |= 1 << ga.tbit[j];
            }
        ga.srcl[m] = sl;
        ga.hreg[m] = hr;
    }
    // Controls below LINE_BITS are tested per lane: control position q sits at
    // the lane bit l with lanepos[l] == q (q < 4 is never inserted, and at
    // most two targets below it are, so it is among the six lane positions).
    ga.cm_lo = ga.cv_lo = 0;
    for (int l = 0; l < 6; ++l) {
        const int q = lanepos[l];
        if (q < LINE_BITS && ((cm >> q) & 1)) {
            ga.cm_lo |= 1u << l;
            if ((cv >> q) & 1) ga.cv_lo |= 1u << l;
        }
    }
    ga.cv_hi = cv & ~linemask;
    ga.ip = make_insert_plan(himask | cm_ins);
    const int nins = nh + __builtin_popcountll(cm_ins);
    ga.C = 1ull << (n - nins);
    // Lanes whose in-line controls fail skip their stores only when every
    // such control leaves aligned runs of at least 64 bytes (the lowest
    // in-line control at or above bit log2(64 / sizeof amplitude)); otherwise
    // they store their values back and every line is written whole.
    {
        const uint64_t cm_line = cm & linemask;
        const int min_run_bit = sizeof(R) == 8 ? 2 : 3; // 64-byte runs
        ga.skip_fail = (cm_line != 0 && __builtin_ctzll(cm_line) >= min_run_bit) ? 1 : 0;
    }
    // Non-temporal stores only when each store instruction writes whole lines:
    // no register target inside a line, no skipped stores, and full waves.
    const bool nt = tun(T_NT) && (reg_low & linemask) == 0 && !ga.skip_fail && ga.C >= 64;
    const uint64_t sb = (1ull << n) * sizeof(R) * 2;
    if (K == 1)
        return nh == 0 ? launch_gate_k<R, 1, 0>(psi, ga, nt, sb, st) : launch_gate_k<R, 1, 1>(psi, ga, nt, sb, st);
    if (nh == 0) return launch_gate_k<R, 2, 0>(psi, ga, nt, sb, st);
    if (nh == 1) return launch_gate_k<R, 2, 1>(psi, ga, nt, sb, st);
    return launch_gate_k<R, 2, 2>(psi, ga, nt, sb, st);
}

hipError_t launch_apply_1q(void* psi, int dt, int n, int t, const double* U, uint64_t cm, uint64_t cv,
                           hipStream_t st, int* kind)
{
    if (kind) *kind = t >= 6 ? QS_K_1Q_HI : QS_K_1Q_LO; // class by target only (tracing)
    return dt == QS_C128 ? apply_gate_t<double>(psi, n, 1, &t, U, cm, cv, st)
                         : apply_gate_t<float>(psi, n, 1, &t, U, cm, cv, st);
}

hipError_t launch_apply_2q(void* psi, int dt, int n, int t0, int t1, const double* U, uint64_t cm,
                           uint64_t cv, hipStream_t st, int* kind)
{
    if (kind) *kind = QS_K_2Q;
    const int t[2] = {t0, t1};
    return dt == QS_C128 ? apply_gate_t<double>(psi, n, 2, t, U, cm, cv, st)
                         : apply_gate_t<float>(psi, n, 2, t, U, cm, cv, st);
}

// ---------------------------------------------------------------- generic k

// Dense k-qubit gate.  The block stages G = 256 / D groups of D = 2^k
// amplitudes in LDS together with U (D x D); lane j then produces output row
// r = j % D of group j / D.
template <typename R, int K>
__global__ void __launch_bounds__(256)
k_kq_lds(typename CT<R>::V* __restrict__ psi, uint64_t ngroups, uint64_t cvals, InsertPlan ip,
         const double2* __restrict__ Ud, uint64_t tbits_packed_lo, uint64_t tbits_packed_hi)
{
    using V = typename CT<R>::V;
    constexpr int D = 1 << K;
    constexpr int G = 256 / D;
    // U goes to LDS when it fits in 32 KiB; the c128 6-qubit matrix (64 KiB) is
    // read through the caches instead.
    constexpr bool kUL = D * D * sizeof(double2) <= 32768;
    __shared__ double2 su[kUL ? D * D : 1];
    __shared__ V sx[256];
    __shared__ uint64_t soff[D];
    if (kUL)
        for (int j = threadIdx.x; j < D * D; j += 256) su[j] = Ud[j];
    if (threadIdx.x < D) {
        // targets are packed 6 bits each: t[0..4] in lo (bits 0..59), t[5] in hi
        uint64_t off = 0;
        for (int b = 0; b < K; ++b) {
            const int tb = b < 5 ? (int)((tbits_packed_lo >> (6 * b)) & 63) : (int)(tbits_packed_hi & 63);
            if ((threadIdx.x >> b) & 1) off |= 1ull << tb;
        }
        soff[threadIdx.x] = off;
    }
    __syncthreads();
    const int lg = threadIdx.x % G, lm = threadIdx.x / G; // load mapping: consecutive lanes, groups
    const int cg = threadIdx.x / D, cr = threadIdx.x % D; // compute mapping
    const uint64_t stride = (uint64_t)gridDim.x * G;
    for (uint64_t g0 = (uint64_t)blockIdx.x * G; g0 < ngroups; g0 += stride) {
        {
            const uint64_t gi = g0 + lg;
            if (gi < ngroups) sx[lg * D + lm] = psi[(ins_bits(gi, ip) | cvals) | soff[lm]];
        }
        __syncthreads();
        const uint64_t gi = g0 + cg;
        if (gi < ngroups) {
            double sr = 0, si = 0;
#pragma unroll 4
            for (int m = 0; m < D; ++m) {
                const double2 a = kUL ? su[cr * D + m] : Ud[cr * D + m];
                const double2 x = ld2(sx[cg * D + m]);
                sr += a.x * x.x - a.y * x.y;
                si += a.x * x.y + a.y * x.x;
            }
            psi[(ins_bits(gi, ip) | cvals) | soff[cr]] = st2<V>(make_double2(sr, si));
        }
        __syncthreads();
    }
}

template <typename R, int K>
static void launch_kq_k(void* psi, int n, uint64_t tmask, uint64_t cm, uint64_t cv, const void* Ud,
                        uint64_t plo, uint64_t phi, hipStream_t st)
{
    using V = typename CT<R>::V;
    constexpr int D = 1 << K;
    constexpr int G = 256 / D;
    const int nc = __builtin_popcountll(cm);
    const uint64_t ng = 1ull << (n - K - nc);
    InsertPlan ip = make_insert_plan(cm | tmask);
    const unsigned g = blocks_for(ng, G * 4);
    hipLaunchKernelGGL((k_kq_lds<R, K>), dim3(g), dim3(256), 0, st, (V*)psi, ng, cv, ip, (const double2*)Ud, plo,
                       phi);
}

// Ud: device copy of the FP64 matrix.
hipError_t launch_apply_kq_dev(void* psi, int dt, int n, const int* targets, int k, const void* Ud,
                               uint64_t cm, uint64_t cv, hipStream_t st, int* kind)
{
    uint64_t tmask = 0, plo = 0, phi = 0;
    for (int j = 0; j < k; ++j) {
        tmask |= 1ull << targets[j];
        if (j < 5)
            plo |= (uint64_t)targets[j] << (6 * j);
        else
            phi = (uint64_t)targets[j];
    }
    const bool d = dt == QS_C128;
    switch (k) {
    case 1: d ? launch_kq_k<double, 1>(psi, n, tmask, cm, cv, Ud, plo, phi, st)
              : launch_kq_k<float, 1>(psi, n, tmask, cm, cv, Ud, plo, phi, st); break;
    case 2: d ? launch_kq_k<double, 2>(psi, n, tmask, cm, cv, Ud, plo, phi, st)
              : launch_kq_k<float, 2>(psi, n, tmask, cm, cv, Ud, plo, phi, st); break;
    case 3: d ? launch_kq_k<double, 3>(psi, n, tmask, cm, cv, Ud, plo, phi, st)
              : launch_kq_k<float, 3>(psi, n, tmask, cm, cv, Ud, plo, phi, st); break;
    case 4: d ? launch_kq_k<double, 4>(psi, n, tmask, cm, cv, Ud, plo, phi, st)
              : launch_kq_k<float, 4>(psi, n, tmask, cm, cv, Ud, plo, phi, st); break;
    case 5: d ? launch_kq_k<double, 5>(psi, n, tmask, cm, cv, Ud, plo, phi, st)
              : launch_kq_k<float, 5>(psi, n, tmask, cm, cv, Ud, plo, phi, st); break;
    case 6: d ? launch_kq_k<double, 6>(psi, n, tmask, cm, cv, Ud, plo, phi, st)
              : launch_kq_k<float, 6>(psi, n, tmask, cm, cv, Ud, plo, phi, st); break;
    default: return hipErrorInvalidValue;
    }
    if (kind) *kind = QS_K_KQ;
    return hipGetLastError();
}

} // namespace qs
