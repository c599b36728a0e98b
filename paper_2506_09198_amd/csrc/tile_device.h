// Device code of the LDS tile passes, shared by the single-circuit pass
// (tile.hip), the batch kernels (tile_batch.hip) and the serving rounds
// (tile_serve.hip).
#pragma once
//
// K4: LDS tile passes.
//
// A pass owns a set Q of M tile qubits (sorted; the lowest L qubits are always
// in Q so a tile is made of contiguous runs of 2^L amplitudes).  The state
// splits into 2^(n-M) tiles, one per setting of the qubits outside Q.  A block
// loads a tile into LDS (tile element e holds amplitude base | dep_Q(e)),
// applies the pass's operation list in order with a barrier after each, and
// writes the tile back: one HBM read and one write per pass however many
// gates the pass absorbed (gate fusion / cache blocking, Section I; here the
// "cache" is the 160 KiB LDS of a CDNA4 compute unit).
//
// Operations (TileOp): dense 1q / 2q / k-qubit gates whose targets are in Q,
// with controls split into tile-local and per-tile parts; diagonal gates act
// elementwise from the global index and need not lie in Q.
#include <type_traits>

#include "device_common.h"
#include "planner.h"

namespace qs {

namespace {

struct QList {
    int32_t m, L;
    int32_t q[QS_MAX_QUBITS];
};

// LDS placement of tile element e.  Each G-bit group of e above the lowest
// is XORed into the lowest G bits (G = 4 for 16-byte, 5 for 8-byte
// amplitudes: one 256-byte row of banks), so lanes whose elements lie a
// power of two apart -- a register segment over low positions, a fused
// block's column gather -- land in different banks.  A bijection on
// [0, 2^M): the high bits are kept.
template <int ES>
__device__ __forceinline__ uint32_t swz(uint32_t e)
{
    constexpr int G = ES == 16 ? 4 : 5;
    constexpr uint32_t MK = (1u << G) - 1;
    uint32_t r = e;
#pragma unroll
    for (int s = G; s < 13; s += G) r ^= (e >> s) & MK;
    return r;
}
#define QS_SW(e) swz<(int)sizeof(V)>(e)

// Fused dense block on K = 4 or 5 tile-local qubits with FP64 matrix cores
// (both amplitude types).  The complex 2^K x 2^K matrix acts as its real
// embedding [[Ur, -Ui], [Ui, Ur]] (interleaved rows/columns, 2^(K+1) square)
// on the tile's 2^(M-K) groups ("columns"), with v_mfma_f64_16x16x4f64: lane
// l holds A[l%16][l/16], B[l/16][l%16] and D[l/16 + 4v][l%16].  Tile values
// enter exactly (FP32 widens to FP64 without rounding) and each result is
// rounded once, to nearest, when it is stored.  An FP32 form would need the
// matrix as hi + lo FP32 parts (a matrix rounded to FP32 repeats its
// rounding coherently at every application) with the lo products kept out of
// the hi accumulator, where they fall below its last bit; two FP32 MFMAs
// cost what one FP64 MFMA costs.  The A fragments come
// pre-arranged by the planner ([q][lane][2] doubles, q*2+j = rb*KS + ks), so
// a wave loads them with 16-byte coalesced loads.  Each wave owns whole
// column blocks of 16 groups, so its in-place writes never race another wave.
typedef double d4_t __attribute__((ext_vector_type(4)));
typedef double d2_t __attribute__((ext_vector_type(2)));

template <typename R, int K, int M>
__device__ __forceinline__ void mfma_block(typename CT<R>::V* tile, const TileOp& d, const double* mats, int tid)
{
    using V = typename CT<R>::V;
    constexpr int DR = 2 << K;     // real dimension
    constexpr int RB = DR / 16;    // 16-row blocks
    constexpr int KS = DR / 4;     // k steps of 4
    constexpr int NF = RB * KS;    // A fragments per lane
    constexpr int C = 1 << (M - K);
    constexpr int CB = C / 16;
    static_assert(CB >= 1, "tile too small for a fused block");
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const d2_t* frag = (const d2_t*)(mats + d.moff);
    double a[NF];
#pragma unroll
    for (int q = 0; q < NF / 2; ++q) {
        const d2_t v = frag[q * 64 + lane];
        a[2 * q] = v[0];
        a[2 * q + 1] = v[1];
    }
    uint32_t tm = 0;
    int pos[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        pos[j] = d.p[j];
        tm |= 1u << pos[j];
    }
    R* tr = (R*)tile; // component c of element e at 2 * swz(e) + c
    for (int cb = wave; cb < CB; cb += 4) {
        const uint32_t col = cb * 16 + li;
        uint32_t gb = col; // insert zeros at the block qubits (ascending)
        for (int b = 0; b < M; ++b)
            if ((tm >> b) & 1) gb = ins0_32(gb, b);
        d4_t acc[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) acc[rb] = d4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int mm = 2 * ks + (lk >> 1); // group member of real row 4ks + lk
            uint32_t e = gb;
#pragma unroll
            for (int j = 0; j < K; ++j)
                if ((mm >> j) & 1) e |= 1u << pos[j];
            const double bv = (double)tr[2 * QS_SW(e) + (lk & 1)];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
                acc[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rb * KS + ks], bv, acc[rb], 0, 0, 0);
        }
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                // real row 16rb + lk + 4v = component (lk & 1) of member 8rb + 2v + lk/2
                const int mm = 8 * rb + 2 * v + (lk >> 1);
                uint32_t e = gb;
#pragma unroll
                for (int j = 0; j < K; ++j)
                    if ((mm >> j) & 1) e |= 1u << pos[j];
                tr[2 * QS_SW(e) + (lk & 1)] = (R)acc[rb][v];
            }
        }
    }
}

// The same block on FP32 matrix cores (complex64 tiles, planner option
// QS_FUSE_FP32).  The FP64 product A is split into hi = fl32(A) and lo =
// bf16(A - hi): hi enters v_mfma_f32_16x16x4f32 (lane l: A[l%16][l/16],
// B[l/16][l%16]) and lo, whose products are about 2^-24 of hi's, a separate
// accumulator through v_mfma_f32_16x16x16bf16 (lane l: A[l%16][4(l/16)+j],
// B[4(l/16)+j][l%16], j < 4) with the amplitudes rounded to bfloat16; both
// accumulate rows D[4(l/16)+v][l%16] and are added once at the end.  Keeping
// lo out of the hi accumulator matters: added there, each lo product falls
// below the accumulator's last bit and the block acts as the FP32-rounded
// matrix, whose rounding repeats at every application.  The bfloat16 part
// costs about 1/16 of the FP32 part, so a block takes about half the time of
// the FP64 form.
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef short s4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short bf16_rne_dev(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

template <int K, int M>
__device__ __forceinline__ void mfma_block32(float2* tile, const TileOp& d, const double* mats, int tid)
{
    constexpr int DR = 2 << K;  // real dimension
    constexpr int RB = DR / 16; // 16-row blocks
    constexpr int KS = DR / 4;  // FP32 k steps of 4
    constexpr int KB = KS / 4;  // bfloat16 k steps of 16
    constexpr int NF = RB * KS;
    constexpr int NG = 4;       // hi accumulators (over quarters of the k steps)
    constexpr int C = 1 << (M - K);
    constexpr int CB = C / 16;
    static_assert(CB >= 1, "tile too small for a fused block");
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    // fragments stay in memory (read once per row block, coalesced): holding
    // them all in registers left one wave per SIMD
    const float* fh = (const float*)(mats + d.moff);                          // [rb * KS + ks][lane]
    const s4_t* fl = (const s4_t*)((const char*)(mats + d.moff) + sizeof(float) * NF * 64); // [rb * KB + kb][lane]
    uint32_t tm = 0;
    int pos[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        pos[j] = d.p[j];
        tm |= 1u << pos[j];
    }
    float* tf = (float*)tile; // component c of element e at 2 * swz(e) + c
    for (int cb = wave; cb < CB; cb += 4) {
        const uint32_t col = cb * 16 + li;
        uint32_t gb = col; // insert zeros at the block qubits (ascending)
        for (int b = 0; b < M; ++b)
            if ((tm >> b) & 1) gb = ins0_32(gb, b);
        auto elem = [&](int mm) {
            uint32_t e = gb;
#pragma unroll
            for (int j = 0; j < K; ++j)
                if ((mm >> j) & 1) e |= 1u << pos[j];
            return e;
        };
        // NG accumulators over consecutive quarters of the k steps, summed in
        // FP64 at the end: each sees 16 (K = 5) sequentially rounded products
        // instead of 64, which keeps the rounding of structured inputs (a
        // Grover state's equal amplitudes add up the same rounding error at
        // every step) from accumulating.  Row blocks run one after another;
        // their results are held until every row block has read the column.
        float out[RB][4];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            f4_t acc[NG], accl = f4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int g = 0; g < NG; ++g) acc[g] = f4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                // real row 4ks + lk = component (lk & 1) of member 2ks + lk/2
                const float bv = tf[2 * swz<8>(elem(2 * ks + (lk >> 1))) + (lk & 1)];
                constexpr int per = KS / NG;
                acc[ks / per] = __builtin_amdgcn_mfma_f32_16x16x4f32(fh[(rb * KS + ks) * 64 + lane], bv,
                                                                     acc[ks / per], 0, 0, 0);
            }
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
                // real rows 16kb + 4lk + j: members 8kb + 2lk (j = 0, 1) and + 1 (j = 2, 3)
                const float2 x0 = tile[swz<8>(elem(8 * kb + 2 * lk))];
                const float2 x1 = tile[swz<8>(elem(8 * kb + 2 * lk + 1))];
                const s4_t bl = {bf16_rne_dev(x0.x), bf16_rne_dev(x0.y), bf16_rne_dev(x1.x), bf16_rne_dev(x1.y)};
                accl = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(fl[(rb * KB + kb) * 64 + lane], bl, accl, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                double s = (double)accl[v];
#pragma unroll
                for (int g = 0; g < NG; ++g) s += (double)acc[g][v];
                out[rb][v] = (float)s;
            }
        }
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int h = 0; h < 2; ++h) // real rows 16rb + 4lk + 2h (+1) = (re, im) of member 8rb + 2lk + h
                tile[swz<8>(elem(8 * rb + 2 * lk + h))] = make_float2(out[rb][2 * h], out[rb][2 * h + 1]);
    }
}

// ------------------------------------------------------------ segments
//
// A segment (TK_SEG header + dj member ops) acts on r register positions of
// the tile.  Thread t holds, per loop step l, the 2^r elements whose other
// bits spell t | l << 8 (deposited into the non-register positions in
// ascending order): it loads them from LDS once, widened to FP64, applies
// every member op with compile-time register indices, and rounds and stores
// them once.  Every wave64 VALU instruction costs the same issue time here
// (FP64 included), so the code keeps per-element work to the arithmetic
// itself: a condition or factor index splits into a per-thread part
// (non-register bits, evaluated once per op) and a per-register part (the
// register bits, uniform across the wave, so it becomes a scalar branch).
template <typename R, int M>
struct Seg {
    static constexpr int RMAX = 4;
    static constexpr int RR = (M - 8 < RMAX) ? (M - 8) : RMAX; // register qubits (M >= 10)
    static constexpr int NR = 1 << RR;
    static constexpr int TB = M - RR;                           // thread + loop bits (>= 8)
    static constexpr int LI = 1 << (TB - 8);                    // loop steps
};

// Keep `old` where this thread's controls fail (plain double selects: a
// select of double2 values is lowered through a per-lane indexed stack copy).
__device__ __forceinline__ double2 keep_if(bool tok, double2 nw, double2 old)
{
    double2 r;
    r.x = tok ? nw.x : old.x;
    r.y = tok ? nw.y : old.y;
    return r;
}

// Dense 1q op on register bit B.  With CTL the op has controls: rcm/rcv are
// control bits at register positions (uniform, tested per pair) and tok
// says whether this thread's own bits pass the others (if not its values
// are kept bit for bit).  The matrix stays uniform either way (scalar
// operands), so controls cost a select per result, not per-lane matrices.
// Without CTL the loop has no branch at all.
template <int NR, int B, bool CTL>
__device__ __forceinline__ void seg_1q(double2 (&reg)[NR], const uint32_t (&roff)[NR], uint32_t rcm, uint32_t rcv,
                                       bool tok, const double* __restrict__ u)
{
    double m[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) m[i] = u[i];
    constexpr int S = 1 << B;
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        if (j & S) continue;
        if constexpr (CTL)
            if ((roff[j] & rcm) != rcv) continue;
        const double2 a = reg[j], b = reg[j + S];
        const double2 na = cmad2<double2, double>(m[0], m[1], a, m[2], m[3], b);
        const double2 nb = cmad2<double2, double>(m[4], m[5], a, m[6], m[7], b);
        reg[j] = CTL ? keep_if(tok, na, a) : na;
        reg[j + S] = CTL ? keep_if(tok, nb, b) : nb;
    }
}

template <int NR, int B0, int B1, bool CTL>
__device__ __forceinline__ void seg_2q(double2 (&reg)[NR], const uint32_t (&roff)[NR], uint32_t rcm, uint32_t rcv,
                                       bool tok, const double* __restrict__ u)
{
    constexpr int S0 = 1 << B0, S1 = 1 << B1;
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        if (j & (S0 | S1)) continue;
        if constexpr (CTL)
            if ((roff[j] & rcm) != rcv) continue;
        const double2 v0 = reg[j], v1 = reg[j + S0], v2 = reg[j + S1], v3 = reg[j + S0 + S1];
        double2 o[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double* m = u + 8 * r;
            const double2 s1 = cmad2<double2, double>(m[0], m[1], v0, m[2], m[3], v1);
            const double2 s2 = cmad2<double2, double>(m[4], m[5], v2, m[6], m[7], v3);
            o[r].x = s1.x + s2.x;
            o[r].y = s1.y + s2.y;
        }
        reg[j] = CTL ? keep_if(tok, o[0], v0) : o[0];
        reg[j + S0] = CTL ? keep_if(tok, o[1], v1) : o[1];
        reg[j + S1] = CTL ? keep_if(tok, o[2], v2) : o[2];
        reg[j + S0 + S1] = CTL ? keep_if(tok, o[3], v3) : o[3];
    }
}

// Diagonal bodies: multiply each register by its factor F[ri], ri spelled
// by the register's bits at ranks B0 (and B1); the X forms multiply only the
// registers whose combination is RI (the others have factor 1).
template <int NR, int B0>
__device__ __forceinline__ void diag_r1(double2 (&reg)[NR], const double2 (&F)[4])
{
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        const int ri = (j >> B0) & 1;
        reg[j] = cmul<double2, double>(F[ri].x, F[ri].y, reg[j]);
    }
}

template <int NR, int B0, int B1>
__device__ __forceinline__ void diag_r2(double2 (&reg)[NR], const double2 (&F)[4])
{
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        const int ri = ((j >> B0) & 1) | (((j >> B1) & 1) << 1);
        reg[j] = cmul<double2, double>(F[ri].x, F[ri].y, reg[j]);
    }
}

template <int NR, int B0, int RI>
__device__ __forceinline__ void diag_r1x(double2 (&reg)[NR], const double2 (&F)[4])
{
#pragma unroll
    for (int j = 0; j < NR; ++j)
        if (((j >> B0) & 1) == RI) reg[j] = cmul<double2, double>(F[RI].x, F[RI].y, reg[j]);
}

template <int NR, int B0, int B1, int RI>
__device__ __forceinline__ void diag_r2x(double2 (&reg)[NR], const double2 (&F)[4])
{
#pragma unroll
    for (int j = 0; j < NR; ++j)
        if ((((j >> B0) & 1) | (((j >> B1) & 1) << 1)) == RI)
            reg[j] = cmul<double2, double>(F[RI].x, F[RI].y, reg[j]);
}

// Per-thread factors of a diagonal member (register form): F[ri] for each
// combination ri of its register targets, selected by the thread's own bits
// among uniform loads of the factor table.
__device__ __forceinline__ void diag_factors(double2 (&F)[4], const TileOp& g, uint64_t base, uint32_t eb,
                                             const double* __restrict__ dd)
{
    const int kr = g.dj & 15, kt = (g.dj >> 4) & 15, k = g.k;
    uint32_t gi = 0; // uniform: targets outside the tile
    for (int j = kr + kt; j < k; ++j) gi |= (uint32_t)((base >> g.p[j]) & 1) << j;
    const bool t0 = kt > 0 && ((eb >> g.p[kr]) & 1);
    const bool t1 = kt > 1 && ((eb >> g.p[kr + 1]) & 1);
#pragma unroll
    for (int ri = 0; ri < 4; ++ri) {
        // plain double selects: a select of double2 values is lowered through
        // a per-lane indexed stack copy
        double fx = 1.0, fy = 0.0;
        if (ri < (1 << kr)) {
            const uint32_t i0 = gi | (uint32_t)ri;
            const uint32_t s0 = 1u << kr, s1 = 2u << kr;
            fx = dd[2 * i0];
            fy = dd[2 * i0 + 1];
            if (kt > 0) {
                const double ax = dd[2 * (i0 | s0)], ay = dd[2 * (i0 | s0) + 1];
                if (kt > 1) {
                    const double bx = dd[2 * (i0 | s1)], by = dd[2 * (i0 | s1) + 1];
                    const double cx = dd[2 * (i0 | s0 | s1)], cy = dd[2 * (i0 | s0 | s1) + 1];
                    const double lox = t0 ? ax : fx, loy = t0 ? ay : fy;
                    const double hix = t0 ? cx : bx, hiy = t0 ? cy : by;
                    fx = t1 ? hix : lox;
                    fy = t1 ? hiy : loy;
                } else {
                    fx = t0 ? ax : fx;
                    fy = t0 ? ay : fy;
                }
            }
        }
        F[ri].x = fx;
        F[ri].y = fy;
    }
}

// A diagonal member the planner left in general form: factor gathered per
// element from its local bits (controls tested per element).
template <int NR>
__device__ __forceinline__ void diag_gather(double2 (&reg)[NR], const uint32_t (&roff)[NR], uint32_t rmask,
                                            uint32_t eb, const TileOp& g, uint64_t base,
                                            const double* __restrict__ dd)
{
    const uint32_t lcm = (uint32_t)g.lcm, lcv = (uint32_t)g.lcv;
    const uint32_t tcm = lcm & ~rmask, rcm = lcm & rmask, rcv = lcv & rcm;
    if ((eb & tcm) != (lcv & tcm)) return;
    uint32_t tidx = 0;
    for (int t = 0; t < g.k; ++t) {
        const int q = g.lp[t];
        if (q < 0) tidx |= (uint32_t)((base >> g.p[t]) & 1) << t;
        else if (!((rmask >> q) & 1)) tidx |= ((eb >> q) & 1) << t;
    }
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        if ((roff[j] & rcm) != rcv) continue;
        uint32_t idx = tidx;
        for (int t = 0; t < g.k; ++t) {
            const int q = g.lp[t];
            if (q >= 0 && ((rmask >> q) & 1)) idx |= ((roff[j] >> q) & 1) << t;
        }
        reg[j] = cmul<double2, double>(dd[2 * idx], dd[2 * idx + 1], reg[j]);
    }
}

// A fused block: the registers are multiplied by a 2^r x 2^r complex matrix
// (row-major, FP64) that the planner formed from a run of register-only ops.
template <int NR>
__device__ __forceinline__ void seg_block(double2 (&reg)[NR], const double* __restrict__ u)
{
    double2 o[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        double sr = 0.0, si = 0.0;
#pragma unroll
        for (int c = 0; c < NR; ++c) {
            const double ar = u[2 * (r * NR + c)], ai = u[2 * (r * NR + c) + 1];
            sr = fma(ar, reg[c].x, sr);
            sr = fma(-ai, reg[c].y, sr);
            si = fma(ar, reg[c].y, si);
            si = fma(ai, reg[c].x, si);
        }
        o[r].x = sr;
        o[r].y = si;
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) reg[r] = o[r];
}

// A diagonal group's factors for one thread: f holds one factor per
// combination of the register bits in RD (compressed, ascending), so the
// thread loads 2^|RD| factors instead of one per register.
constexpr int pext_c(int j, int m)
{
    int r = 0, b = 0;
    for (int q = 0; q < 4; ++q)
        if ((m >> q) & 1) r |= ((j >> q) & 1) << b++;
    return r;
}

template <int NR, int RD>
__device__ __forceinline__ void dgroup_mul(double2 (&reg)[NR], const double2* __restrict__ f)
{
    constexpr int C = 1 << __builtin_popcount(RD);
    double2 F[C];
#pragma unroll
    for (int c = 0; c < C; ++c) F[c] = f[c];
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        const int c = pext_c(j, RD);
        reg[j] = cmul<double2, double>(F[c].x, F[c].y, reg[j]);
    }
}

template <int NR>
__device__ __forceinline__ void dgroup_apply(double2 (&reg)[NR], const double2* __restrict__ f, int rd)
{
    switch (rd) {
#define QS_G(RD_)                                                                                    \
    case RD_:                                                                                        \
        if constexpr (RD_ < NR) dgroup_mul<NR, RD_>(reg, f);                                         \
        break;
        QS_G(0) QS_G(1) QS_G(2) QS_G(3) QS_G(4) QS_G(5) QS_G(6) QS_G(7)
        QS_G(8) QS_G(9) QS_G(10) QS_G(11) QS_G(12) QS_G(13) QS_G(14) QS_G(15)
#undef QS_G
    default: break;
    }
}

// One segment member, dispatched by its opcode in a single switch so the
// register array has one join per op.
template <int RR, int NR>
__device__ __forceinline__ void seg_op(double2 (&reg)[NR], const uint32_t (&roff)[NR], uint32_t rmask, uint32_t eb,
                                       const TileOp& d, uint64_t base, const double* __restrict__ mats)
{
    const int opc = d.rsv >> 16;
    const double* u = mats + d.moff;
    if (opc == SO_BLOCK) {
        seg_block<NR>(reg, u);
        return;
    }
    if (opc < SO_D0) {
        const uint32_t lcm = (uint32_t)d.lcm, lcv = (uint32_t)d.lcv;
        const uint32_t rcm = lcm & rmask, rcv = lcv & rcm, tcm = lcm & ~rmask;
        const bool tok = (eb & tcm) == (lcv & tcm); // controls at thread positions
        switch (opc) {
#define QS_C1(B_)                                                                                    \
    case SO_1Q + B_:                                                                                 \
        if constexpr (B_ < RR) seg_1q<NR, B_, false>(reg, roff, 0, 0, true, u);                            \
        break;                                                                                       \
    case SO_1Q + 4 + B_:                                                                             \
        if constexpr (B_ < RR) seg_1q<NR, B_, true>(reg, roff, rcm, rcv, tok, u);                         \
        break;
        QS_C1(0) QS_C1(1) QS_C1(2) QS_C1(3)
#undef QS_C1
#define QS_C2(P_, A_, B_)                                                                            \
    case SO_2Q + P_:                                                                                 \
        if constexpr (B_ < RR) seg_2q<NR, A_, B_, false>(reg, roff, 0, 0, true, u);                        \
        break;                                                                                       \
    case SO_2Q + 6 + P_:                                                                             \
        if constexpr (B_ < RR) seg_2q<NR, A_, B_, true>(reg, roff, rcm, rcv, tok, u);                     \
        break;
        QS_C2(0, 0, 1) QS_C2(1, 0, 2) QS_C2(2, 1, 2) QS_C2(3, 0, 3) QS_C2(4, 1, 3) QS_C2(5, 2, 3)
#undef QS_C2
        default: break;
        }
        return;
    }
    if (opc == SO_DG) {
        diag_gather<NR>(reg, roff, rmask, eb, d, base, u);
        return;
    }
    if (opc == SO_DGROUP) {
        // factor table index: the register bits the factors depend on (mask
        // RD, compressed), then the thread positions in lcm, then the
        // positions outside the tile in lcv
        const uint32_t tpm = (uint32_t)d.lcm;
        const uint64_t gpm = d.lcv;
        uint32_t ti = 0, gi = 0;
        int b = 0;
        for (uint64_t m = gpm; m; m &= m - 1) gi |= (uint32_t)((base >> __builtin_ctzll(m)) & 1) << b++;
        const int kt = d.dj & 255, rd = (d.dj >> 16) & 15;
        if (kt == 0) {
            // no thread positions: every thread of the tile multiplies by the
            // same factors, read with uniform (scalar) loads -- a call site of
            // its own, so the pointer stays uniform
            dgroup_apply<NR>(reg, (const double2*)u + ((uint64_t)gi << __builtin_popcount(rd)), rd);
            return;
        }
        b = 0;
        for (uint32_t m = tpm; m; m &= m - 1) ti |= ((eb >> __builtin_ctz(m)) & 1) << b++;
        dgroup_apply<NR>(reg, (const double2*)u + ((((uint64_t)gi << kt) | ti) << __builtin_popcount(rd)), rd);
        return;
    }
    double2 F[4];
    diag_factors(F, d, base, eb, u);
    switch (opc) {
    case SO_D0:
#pragma unroll
        for (int j = 0; j < NR; ++j) reg[j] = cmul<double2, double>(F[0].x, F[0].y, reg[j]);
        break;
#define QS_D1(B_)                                                                                    \
    case SO_D1 + B_:                                                                                 \
        if constexpr (B_ < RR) diag_r1<NR, B_>(reg, F);                                              \
        break;                                                                                       \
    case SO_D1X + 2 * B_:                                                                            \
        if constexpr (B_ < RR) diag_r1x<NR, B_, 0>(reg, F);                                          \
        break;                                                                                       \
    case SO_D1X + 2 * B_ + 1:                                                                        \
        if constexpr (B_ < RR) diag_r1x<NR, B_, 1>(reg, F);                                          \
        break;
        QS_D1(0) QS_D1(1) QS_D1(2) QS_D1(3)
#undef QS_D1
#define QS_D2(P_, A_, B_)                                                                            \
    case SO_D2 + P_:                                                                                 \
        if constexpr (B_ < RR) diag_r2<NR, A_, B_>(reg, F);                                          \
        break;                                                                                       \
    case SO_D2X + 4 * P_:                                                                            \
        if constexpr (B_ < RR) diag_r2x<NR, A_, B_, 0>(reg, F);                                      \
        break;                                                                                       \
    case SO_D2X + 4 * P_ + 1:                                                                        \
        if constexpr (B_ < RR) diag_r2x<NR, A_, B_, 1>(reg, F);                                      \
        break;                                                                                       \
    case SO_D2X + 4 * P_ + 2:                                                                        \
        if constexpr (B_ < RR) diag_r2x<NR, A_, B_, 2>(reg, F);                                      \
        break;                                                                                       \
    case SO_D2X + 4 * P_ + 3:                                                                        \
        if constexpr (B_ < RR) diag_r2x<NR, A_, B_, 3>(reg, F);                                      \
        break;
        QS_D2(0, 0, 1) QS_D2(1, 0, 2) QS_D2(2, 1, 2) QS_D2(3, 0, 3) QS_D2(4, 1, 3) QS_D2(5, 2, 3)
#undef QS_D2
    default: break;
    }
}

template <typename R, int M>
__device__ __forceinline__ void run_segment(typename CT<R>::V* tile, uint64_t base, const TileOp* __restrict__ hdr,
                                            const double* __restrict__ mats, int tid)
{
    using V = typename CT<R>::V;
    using S = Seg<R, M>;
    constexpr int RR = S::RR, NR = S::NR;
    const int nmem = hdr->dj;
    uint32_t rmask = 0;
    int rp[RR];
#pragma unroll
    for (int b = 0; b < RR; ++b) {
        rp[b] = hdr->p[b];
        rmask |= 1u << rp[b];
    }
    uint32_t roff[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        uint32_t o = 0;
#pragma unroll
        for (int b = 0; b < RR; ++b)
            if ((j >> b) & 1) o |= 1u << rp[b];
        roff[j] = o;
    }
    // The swizzle is linear over XOR, and eb and roff[j] share no bits, so
    // swz(eb | roff[j]) = swz(eb) ^ swz(roff[j]): the register offsets are
    // swizzled once per segment (uniform), each element address is one XOR.
    uint32_t sroff[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) sroff[j] = QS_SW(roff[j]);
    int rs[RR]; // register positions, ascending, for zero insertion
#pragma unroll
    for (int b = 0; b < RR; ++b) rs[b] = rp[b];
#pragma unroll
    for (int b = 1; b < RR; ++b)
#pragma unroll
        for (int c = RR - 1; c >= b; --c)
            if (rs[c - 1] > rs[c]) {
                const int t = rs[c - 1];
                rs[c - 1] = rs[c];
                rs[c] = t;
            }
    for (int li = 0; li < S::LI; ++li) {
        // the thread's element bits: tid | li << 8 with zeros inserted at the
        // register positions (ascending)
        uint32_t eb = (uint32_t)tid | ((uint32_t)li << 8);
#pragma unroll
        for (int b = 0; b < RR; ++b) eb = ins0_32(eb, rs[b]);
        const uint32_t seb = QS_SW(eb);
        double2 reg[NR];
#pragma unroll
        for (int j = 0; j < NR; ++j) reg[j] = ld2(tile[seb ^ sroff[j]]);
        for (int o = 1; o <= nmem; ++o) {
            const TileOp& d = hdr[o];
            if ((base & d.gcm) == d.gcv) seg_op<RR, NR>(reg, roff, rmask, eb, d, base, mats);
        }
#pragma unroll
        for (int j = 0; j < NR; ++j) tile[seb ^ sroff[j]] = st2<V>(reg[j]);
    }
}

// Apply a pass's operation list to the tile held in LDS (all lanes of the
// block call this; it ends with the tile complete in LDS).  `base` is the
// global index of tile element 0 (tile bits zero).  VAR selects what the
// kernel holds (the host launches the variant a pass needs, ops_variant):
// 0 = segments only for tiles of >= 2^10 (every op for smaller tiles),
// 1 = every op but fused matrix-core blocks, 2 = every op with blocks in the
// FP64 form, 3 = every op with blocks in the FP32 form (complex64; the
// fragments of either form would otherwise cost every other pass registers).
template <typename R, int M, int VAR>
__device__ __forceinline__ void tile_ops(typename CT<R>::V* tile, uint64_t base, const TileOp* __restrict__ ops,
                                         int nops, const double* __restrict__ mats)
{
    using V = typename CT<R>::V;
    constexpr uint32_t E = 1u << M;
    constexpr int PER = (E + 255) / 256; // tile elements per lane
    const int tid = threadIdx.x;
    // element e = tid + 256 s sits at swz(tid) ^ swz(256 s) (the swizzle is linear over XOR)
    const uint32_t stid = QS_SW((uint32_t)tid);
    for (int o = 0; o < nops; ++o) {
        const TileOp& d = ops[o];
        const int kind = d.kind;
        if (kind == TK_SEG) {
            if constexpr (M >= 10) run_segment<R, M>(tile, base, ops + o, mats, tid);
            o += d.dj;
            __syncthreads();
            continue;
        }
        // the lean kernel of a large tile holds segments only (the host
        // launches the full kernel for any other op)
        if constexpr (VAR == 0 && M >= 10) continue;
        if (kind != TK_DIAG && (base & d.gcm) != d.gcv) continue; // tile fails the outside controls
        const double* u = mats + d.moff;
        const uint32_t lcm = (uint32_t)d.lcm, lcv = (uint32_t)d.lcv;
        if (kind == TK_DENSE1) {
            const int p = d.p[0];
            const uint32_t hm = ~((1u << p) - 1); // pair k -> e0 = k + (k & hm) (zero inserted at p)
            const uint32_t pb = 1u << p;
            const double u0 = u[0], u1 = u[1], u2 = u[2], u3 = u[3], u4 = u[4], u5 = u[5], u6 = u[6],
                         u7 = u[7];
            if (lcm == 0) {
#pragma unroll 4
                for (int s = 0; s < (PER + 1) / 2; ++s) {
                    const uint32_t k = tid + 256 * s;
                    if (E >= 512 || k < E / 2) {
                        const uint32_t e0 = k + (k & hm), e1 = e0 + pb;
                        const double2 a = ld2(tile[QS_SW(e0)]), b = ld2(tile[QS_SW(e1)]);
                        tile[QS_SW(e0)] = st2<V>(cmad2<double2, double>(u0, u1, a, u2, u3, b));
                        tile[QS_SW(e1)] = st2<V>(cmad2<double2, double>(u4, u5, a, u6, u7, b));
                    }
                }
            } else {
#pragma unroll 4
                for (int s = 0; s < (PER + 1) / 2; ++s) {
                    const uint32_t k = tid + 256 * s;
                    if (E >= 512 || k < E / 2) {
                        const uint32_t e0 = k + (k & hm), e1 = e0 + pb;
                        if ((e0 & lcm) == lcv) {
                            const double2 a = ld2(tile[QS_SW(e0)]), b = ld2(tile[QS_SW(e1)]);
                            tile[QS_SW(e0)] = st2<V>(cmad2<double2, double>(u0, u1, a, u2, u3, b));
                            tile[QS_SW(e1)] = st2<V>(cmad2<double2, double>(u4, u5, a, u6, u7, b));
                        }
                    }
                }
            }
        } else if (kind == TK_DENSE2) {
            const int p0 = d.p[0], p1 = d.p[1];
            const int lo = p0 < p1 ? p0 : p1, hi = p0 < p1 ? p1 : p0;
            const uint32_t b0 = 1u << p0, b1 = 1u << p1;
#pragma unroll 2
            for (int s = 0; s < (PER + 3) / 4; ++s) {
                const uint32_t k = tid + 256 * s;
                if (k < E / 4) {
                    const uint32_t e = ins0_32(ins0_32(k, lo), hi);
                    if ((e & lcm) == lcv) {
                        const double2 v0 = ld2(tile[QS_SW(e)]), v1 = ld2(tile[QS_SW(e | b0)]), v2 = ld2(tile[QS_SW(e | b1)]),
                                      v3 = ld2(tile[QS_SW(e | b0 | b1)]);
                        double2 out[4];
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const double* ur = u + 8 * r;
                            const double2 s1 = cmad2<double2, double>(ur[0], ur[1], v0, ur[2], ur[3], v1);
                            const double2 s2 = cmad2<double2, double>(ur[4], ur[5], v2, ur[6], ur[7], v3);
                            out[r].x = s1.x + s2.x;
                            out[r].y = s1.y + s2.y;
                        }
                        tile[QS_SW(e)] = st2<V>(out[0]);
                        tile[QS_SW(e | b0)] = st2<V>(out[1]);
                        tile[QS_SW(e | b1)] = st2<V>(out[2]);
                        tile[QS_SW(e | b0 | b1)] = st2<V>(out[3]);
                    }
                }
            }
        } else if (kind == TK_DENSEK) {
            if constexpr (VAR == 0) continue;
            // Rounds of 256 slots; a round holds whole groups (D <= 64
            // divides 256), so every lane reads its group, all wait, and
            // all write: no group is overwritten while still being read.
            const int k = d.k;
            const uint32_t D = 1u << k;
            uint32_t tm = 0;
            for (int j = 0; j < k; ++j) tm |= 1u << d.p[j];
            for (uint32_t r0 = 0; r0 < E; r0 += 256) {
                const uint32_t slot = r0 + tid;
                bool act = false;
                uint32_t eo = 0;
                double2 res;
                if (slot < E) {
                    const uint32_t g = slot >> k, r = slot & (D - 1);
                    uint32_t gb = g; // insert zeros at the target positions (ascending)
                    for (int b = 0; b < M; ++b)
                        if ((tm >> b) & 1) gb = ins0_32(gb, b);
                    if ((gb & lcm) == lcv) {
                        act = true;
                        double sr = 0, si = 0;
#pragma unroll 4
                        for (uint32_t mm = 0; mm < D; ++mm) {
                            uint32_t ei = gb;
                            for (int j = 0; j < k; ++j)
                                if ((mm >> j) & 1) ei |= 1u << d.p[j];
                            const double2 x = ld2(tile[QS_SW(ei)]);
                            const double ar = u[2 * (r * D + mm)], ai = u[2 * (r * D + mm) + 1];
                            sr += ar * x.x - ai * x.y;
                            si += ar * x.y + ai * x.x;
                        }
                        eo = gb;
                        for (int j = 0; j < k; ++j)
                            if ((r >> j) & 1) eo |= 1u << d.p[j];
                        res.x = sr;
                        res.y = si;
                    }
                }
                __syncthreads();
                if (act) tile[QS_SW(eo)] = st2<V>(res);
                __syncthreads();
            }
        } else if (kind == TK_MFMA) {
            if constexpr (VAR == 3 && sizeof(R) == 4 && M >= 8) { // FP32 form (complex64)
                if (d.k == 5) {
                    if constexpr (M >= 9) mfma_block32<5, M>((float2*)tile, d, mats, tid);
                } else {
                    mfma_block32<4, M>((float2*)tile, d, mats, tid);
                }
            } else if constexpr (VAR >= 2 && M >= 8) {
                if (d.k == 5) {
                    if constexpr (M >= 9) mfma_block<R, 5, M>(tile, d, mats, tid);
                } else {
                    mfma_block<R, 4, M>(tile, d, mats, tid);
                }
            }
        } else if (kind == TK_DIAG) {
            // A run of diagonal gates [o, o2) is applied in one sweep with
            // the lane's elements in registers.  Per tile the gates' bits
            // outside the tile are fixed, so most gates reduce to a factor
            // on one local bit (or to one factor for the whole tile); such
            // factors are multiplied together in uniform (scalar) code and
            // reach each element as one complex multiply per local bit.
            int o2 = o + 1;
            while (o2 < nops && ops[o2].kind == TK_DIAG) ++o2;
            // Every lane touches only its own elements (e = tid + 256 s) during
            // the run, so the run needs no barrier until its end; values stay
            // in LDS (no per-lane register copy of the tile).
            double cr = 1.0, ci = 0.0;              // whole-tile factor
            int abit = -1;                          // pending one-bit factor
            double a0r = 1.0, a0i = 0.0, a1r = 1.0, a1i = 0.0;
            auto flush = [&]() {
                if (abit < 0) return;
#pragma unroll 4
                for (int s = 0; s < PER; ++s) {
                    const uint32_t e = tid + 256 * s;
                    if (E >= 256 || e < E) {
                        const bool one = (e >> abit) & 1;
                        tile[(stid ^ QS_SW(256u * s))] = st2<V>(cmul<double2, double>(one ? a1r : a0r, one ? a1i : a0i, ld2(tile[(stid ^ QS_SW(256u * s))])));
                    }
                }
                abit = -1;
            };
            auto merge = [&](int bit, double f0r, double f0i, double f1r, double f1i) {
                if (bit != abit) {
                    flush();
                    abit = bit;
                    a0r = f0r; a0i = f0i; a1r = f1r; a1i = f1i;
                } else {
                    const double t0r = a0r * f0r - a0i * f0i, t0i = a0r * f0i + a0i * f0r;
                    const double t1r = a1r * f1r - a1i * f1i, t1i = a1r * f1i + a1i * f1r;
                    a0r = t0r; a0i = t0i; a1r = t1r; a1i = t1i;
                }
            };
            for (int q = o; q < o2; ++q) {
                const TileOp& g = ops[q];
                if ((base & g.gcm) != g.gcv) continue;
                const double* dd = mats + g.moff;
                uint32_t gidx = 0; // index bits contributed by targets outside the tile
                for (int j = 0; j < g.k; ++j)
                    if (g.lp[j] < 0) gidx |= (uint32_t)((base >> g.p[j]) & 1) << j;
                const int cls = g.dclass;
                if (cls == DG_UNIFORM) {
                    const double fr = dd[2 * gidx], fi = dd[2 * gidx + 1];
                    const double tr = cr * fr - ci * fi, ti = cr * fi + ci * fr;
                    cr = tr; ci = ti;
                } else if (cls == DG_LTARGET) {
                    const uint32_t i1 = gidx | (1u << g.dj);
                    merge(g.dbit, dd[2 * gidx], dd[2 * gidx + 1], dd[2 * i1], dd[2 * i1 + 1]);
                } else if (cls == DG_LCONTROL) {
                    const double fr = dd[2 * gidx], fi = dd[2 * gidx + 1];
                    if (g.lcv) merge(g.dbit, 1.0, 0.0, fr, fi);
                    else merge(g.dbit, fr, fi, 1.0, 0.0);
                } else if (cls == DG_CT) {
                    // one local target bit and one local control bit (CZ, CP)
                    flush();
                    const int tb = g.dbit, cb = (int)__builtin_ctzll(g.lcm);
                    const uint32_t cv = g.lcv ? 1u : 0u;
                    const uint32_t i1 = gidx | (1u << g.dj);
                    const double f0r = dd[2 * gidx], f0i = dd[2 * gidx + 1], f1r = dd[2 * i1], f1i = dd[2 * i1 + 1];
#pragma unroll 4
                    for (int s = 0; s < PER; ++s) {
                        const uint32_t e = tid + 256 * s;
                        if ((E >= 256 || e < E) && ((e >> cb) & 1) == cv) {
                            const bool one = (e >> tb) & 1;
                            tile[(stid ^ QS_SW(256u * s))] = st2<V>(cmul<double2, double>(one ? f1r : f0r, one ? f1i : f0i, ld2(tile[(stid ^ QS_SW(256u * s))])));
                        }
                    }
                } else {
                    flush();
                    const uint32_t lc = (uint32_t)g.lcm, lv = (uint32_t)g.lcv;
#pragma unroll 4
                    for (int s = 0; s < PER; ++s) {
                        const uint32_t e = tid + 256 * s;
                        if ((E >= 256 || e < E) && (e & lc) == lv) {
                            uint32_t idx = gidx;
                            for (int j = 0; j < g.k; ++j)
                                if (g.lp[j] >= 0) idx |= ((e >> g.lp[j]) & 1) << j;
                            tile[(stid ^ QS_SW(256u * s))] = st2<V>(cmul<double2, double>(dd[2 * idx], dd[2 * idx + 1], ld2(tile[(stid ^ QS_SW(256u * s))])));
                        }
                    }
                }
            }
            if (abit >= 0) {
                const double t0r = a0r * cr - a0i * ci, t0i = a0r * ci + a0i * cr;
                const double t1r = a1r * cr - a1i * ci, t1i = a1r * ci + a1i * cr;
                a0r = t0r; a0i = t0i; a1r = t1r; a1i = t1i;
                flush();
            } else if (cr != 1.0 || ci != 0.0) {
#pragma unroll 4
                for (int s = 0; s < PER; ++s) {
                    const uint32_t e = tid + 256 * s;
                    if (E >= 256 || e < E) tile[(stid ^ QS_SW(256u * s))] = st2<V>(cmul<double2, double>(cr, ci, ld2(tile[(stid ^ QS_SW(256u * s))])));
                }
            }
            o = o2 - 1;
        }
        __syncthreads();
    }
}

// Tile element e <-> amplitude base | (e & lowm) | (hoff[e >> L] << L).
template <typename R, int M>
__device__ __forceinline__ void tile_load(const typename CT<R>::V* __restrict__ psi, uint64_t base, int L,
                                          const uint32_t* hoff, typename CT<R>::V* tile, int nt)
{
    using V = typename CT<R>::V;
    constexpr uint32_t E = 1u << M;
    constexpr int PER = (E + 255) / 256;
    const uint32_t lowm = (1u << L) - 1;
    const int tid = threadIdx.x;
    // all loads of the tile are issued before the first LDS write
    R rx[PER], ry[PER];
#pragma unroll
    for (int s = 0; s < PER; ++s) {
        const uint32_t e = tid + 256 * s;
        if (E >= 256 || e < E) {
            const V* a = psi + (base | (e & lowm) | ((uint64_t)hoff[e >> L] << L));
            const V v = nt ? gld<true>(a) : gld<false>(a);
            rx[s] = v.x;
            ry[s] = v.y;
        }
    }
    // swz(tid + 256 s) = swz(tid) ^ swz(256 s): the swizzle is linear over XOR
    const uint32_t st = QS_SW((uint32_t)tid);
#pragma unroll
    for (int s = 0; s < PER; ++s) {
        const uint32_t e = tid + 256 * s;
        if (E >= 256 || e < E) {
            V v;
            v.x = rx[s];
            v.y = ry[s];
            tile[st ^ QS_SW(256u * s)] = v;
        }
    }
}

template <typename R, int M>
__device__ __forceinline__ void tile_store(typename CT<R>::V* __restrict__ psi, uint64_t base, int L,
                                           const uint32_t* hoff, const typename CT<R>::V* tile, int nt)
{
    using V = typename CT<R>::V;
    constexpr uint32_t E = 1u << M;
    constexpr int PER = (E + 255) / 256;
    const uint32_t lowm = (1u << L) - 1;
    const int tid = threadIdx.x;
    const uint32_t st = QS_SW((uint32_t)tid); // as in tile_load
#pragma unroll
    for (int s = 0; s < PER; ++s) {
        const uint32_t e = tid + 256 * s;
        if (e < E) {
            V* a = psi + (base | (e & lowm) | ((uint64_t)hoff[e >> L] << L));
            const V v = tile[st ^ QS_SW(256u * s)];
            if (nt)
                gst<true>(a, v);
            else
                gst<false>(a, v);
        }
    }
}

// hoff[h] = dep_Q of the tile bits above L, shifted right by L.
__device__ __forceinline__ void build_hoff(uint32_t* hoff, int M, int L, const int32_t* q)
{
    const uint32_t H = 1u << (M - L);
    for (uint32_t h = threadIdx.x; h < H; h += 256) {
        uint64_t off = 0;
        for (int j = L; j < M; ++j)
            if ((h >> (j - L)) & 1) off |= 1ull << q[j];
        hoff[h] = (uint32_t)(off >> L);
    }
}

// Host: call f(RTag<R>, integral_constant<int, VAR>) for the amplitude type
// dt and the tile-kernel variant var (an ops_variant value).
template <typename R>
struct RTag {
    using type = R;
};

template <typename F>
inline hipError_t dispatch_var(int dt, int var, F&& f)
{
    auto by_r = [&](auto r) {
        if constexpr (std::is_same<typename decltype(r)::type, float>::value)
            if (var >= 3) return f(r, std::integral_constant<int, 3>());
        if (var >= 2) return f(r, std::integral_constant<int, 2>());
        if (var == 1) return f(r, std::integral_constant<int, 1>());
        return f(r, std::integral_constant<int, 0>());
    };
    return dt == QS_C128 ? by_r(RTag<double>()) : by_r(RTag<float>());
}

} // namespace
} // namespace qs
