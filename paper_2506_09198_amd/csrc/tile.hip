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
#include "device_common.h"
#include "planner.h"

namespace qs {

namespace {

struct QList {
    int32_t m, L;
    int32_t q[QS_MAX_QUBITS];
};

// Fused dense block on K = 4 or 5 tile-local qubits with FP64 matrix cores
// (complex64 tiles).  The complex 2^K x 2^K matrix acts as its real embedding
// [[Ur, -Ui], [Ui, Ur]] (interleaved rows/columns, 2^(K+1) square) on the
// tile's 2^(M-K) groups ("columns"), with v_mfma_f64_16x16x4f64: lane l holds
// A[l%16][l/16], B[l/16][l%16] and D[l/16 + 4v][l%16].  The FP32 amplitudes
// convert to FP64 exactly and the result is rounded once, to nearest, when it
// is stored; FP32 matrix-core accumulation instead shrinks the norm by a
// one-signed ~1e-8 per block, which adds up over a deep circuit.  One FP64
// MFMA costs as much as the two FP32 ones an exact (hi + lo) matrix would
// need.  The A fragments come pre-arranged by the planner ([q][lane][2]
// doubles, q*2+j = rb*KS + ks), so a wave loads them with 16-byte coalesced
// loads.  Each wave owns whole column blocks of 16 groups, so its in-place
// writes never race another wave.
typedef double d4_t __attribute__((ext_vector_type(4)));
typedef double d2_t __attribute__((ext_vector_type(2)));

template <int K, int M>
__device__ __forceinline__ void mfma_block(float2* tile, const TileOp& d, const double* mats, int tid)
{
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
    float* tf = (float*)tile;
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
            const double bv = (double)tf[2 * e + (lk & 1)];
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
                tf[2 * e + (lk & 1)] = (float)acc[rb][v];
            }
        }
    }
}

// Apply a pass's operation list to the tile held in LDS (all lanes of the
// block call this; it ends with the tile complete in LDS).  `base` is the
// global index of tile element 0 (tile bits zero).
template <typename R, int M, bool MF>
__device__ __forceinline__ void tile_ops(typename CT<R>::V* tile, uint64_t base, const TileOp* __restrict__ ops,
                                         int nops, const double* __restrict__ mats)
{
    using V = typename CT<R>::V;
    constexpr uint32_t E = 1u << M;
    constexpr int PER = (E + 255) / 256; // tile elements per lane
    const int tid = threadIdx.x;
    for (int o = 0; o < nops; ++o) {
        const TileOp& d = ops[o];
        const int kind = d.kind;
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
                        const double2 a = ld2(tile[e0]), b = ld2(tile[e1]);
                        tile[e0] = st2<V>(cmad2<double2, double>(u0, u1, a, u2, u3, b));
                        tile[e1] = st2<V>(cmad2<double2, double>(u4, u5, a, u6, u7, b));
                    }
                }
            } else {
#pragma unroll 4
                for (int s = 0; s < (PER + 1) / 2; ++s) {
                    const uint32_t k = tid + 256 * s;
                    if (E >= 512 || k < E / 2) {
                        const uint32_t e0 = k + (k & hm), e1 = e0 + pb;
                        if ((e0 & lcm) == lcv) {
                            const double2 a = ld2(tile[e0]), b = ld2(tile[e1]);
                            tile[e0] = st2<V>(cmad2<double2, double>(u0, u1, a, u2, u3, b));
                            tile[e1] = st2<V>(cmad2<double2, double>(u4, u5, a, u6, u7, b));
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
                        const double2 v0 = ld2(tile[e]), v1 = ld2(tile[e | b0]), v2 = ld2(tile[e | b1]),
                                      v3 = ld2(tile[e | b0 | b1]);
                        double2 out[4];
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const double* ur = u + 8 * r;
                            const double2 s1 = cmad2<double2, double>(ur[0], ur[1], v0, ur[2], ur[3], v1);
                            const double2 s2 = cmad2<double2, double>(ur[4], ur[5], v2, ur[6], ur[7], v3);
                            out[r].x = s1.x + s2.x;
                            out[r].y = s1.y + s2.y;
                        }
                        tile[e] = st2<V>(out[0]);
                        tile[e | b0] = st2<V>(out[1]);
                        tile[e | b1] = st2<V>(out[2]);
                        tile[e | b0 | b1] = st2<V>(out[3]);
                    }
                }
            }
        } else if (kind == TK_DENSEK) {
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
                            const double2 x = ld2(tile[ei]);
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
                if (act) tile[eo] = st2<V>(res);
                __syncthreads();
            }
        } else if (kind == TK_MFMA) {
            if constexpr (sizeof(R) == 4 && M >= 8) {
                if (d.k == 5) {
                    if constexpr (M >= 9) mfma_block<5, M>((float2*)tile, d, mats, tid);
                } else {
                    mfma_block<4, M>((float2*)tile, d, mats, tid);
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
                        tile[e] = st2<V>(cmul<double2, double>(one ? a1r : a0r, one ? a1i : a0i, ld2(tile[e])));
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
                            tile[e] = st2<V>(cmul<double2, double>(one ? f1r : f0r, one ? f1i : f0i, ld2(tile[e])));
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
                            tile[e] = st2<V>(cmul<double2, double>(dd[2 * idx], dd[2 * idx + 1], ld2(tile[e])));
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
                    if (E >= 256 || e < E) tile[e] = st2<V>(cmul<double2, double>(cr, ci, ld2(tile[e])));
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
#pragma unroll
    for (int s = 0; s < PER; ++s) {
        const uint32_t e = tid + 256 * s;
        if (E >= 256 || e < E) {
            V v;
            v.x = rx[s];
            v.y = ry[s];
            tile[e] = v;
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
#pragma unroll
    for (int s = 0; s < PER; ++s) {
        const uint32_t e = tid + 256 * s;
        if (e < E) {
            V* a = psi + (base | (e & lowm) | ((uint64_t)hoff[e >> L] << L));
            if (nt)
                gst<true>(a, tile[e]);
            else
                gst<false>(a, tile[e]);
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

template <typename R, int M, bool MF>
__global__ void __launch_bounds__(256)
k_tile(typename CT<R>::V* __restrict__ psi, uint64_t ntiles, QList ql, InsertPlan ipQ,
       const TileOp* __restrict__ ops, int nops, const double* __restrict__ mats, int nt)
{
    using V = typename CT<R>::V;
    constexpr uint32_t E = 1u << M;
    extern __shared__ __align__(16) unsigned char smem[];
    V* tile = (V*)smem;
    uint32_t* hoff = (uint32_t*)(smem + sizeof(V) * E);
    build_hoff(hoff, M, ql.L, ql.q);
    __syncthreads();
    for (uint64_t tau = blockIdx.x; tau < ntiles; tau += gridDim.x) {
        const uint64_t base = ins_bits(tau, ipQ);
        tile_load<R, M>(psi, base, ql.L, hoff, tile, nt);
        __syncthreads();
        tile_ops<R, M, MF>(tile, base, ops, nops, mats);
        tile_store<R, M>(psi, base, ql.L, hoff, tile, nt);
        __syncthreads();
    }
}

// ---------------------------------------------------------------- batches

template <typename R, int M, bool MF>
__global__ void __launch_bounds__(256)
k_batch_whole(char* __restrict__ arena, const BatchCirc* __restrict__ circs, const int32_t* __restrict__ list,
              const BatchPass* __restrict__ passes, const TileOp* __restrict__ ops,
              const double* __restrict__ mats)
{
    using V = typename CT<R>::V;
    constexpr uint32_t E = 1u << M;
    extern __shared__ __align__(16) unsigned char smem[];
    V* tile = (V*)smem;
    uint32_t* hoff = (uint32_t*)(smem + sizeof(V) * E);
    const BatchCirc& c = circs[list[blockIdx.x]];
    V* psi = (V*)(arena + c.psi_off);
    for (uint32_t e = threadIdx.x; e < E; e += 256) {
        V v;
        v.x = (e == c.basis) ? (R)1 : (R)0;
        v.y = 0;
        tile[e] = v;
    }
    if (threadIdx.x == 0) hoff[0] = 0;
    __syncthreads();
    for (int p = 0; p < c.npass; ++p) {
        const BatchPass& bp = passes[c.pass0 + p];
        tile_ops<R, M, MF>(tile, 0, ops + bp.op0, bp.nops, mats);
    }
    tile_store<R, M>(psi, 0, M, hoff, tile, M >= 4 ? 1 : 0);
}

template <typename R, int M, bool MF>
__global__ void __launch_bounds__(256)
k_batch_persist(char* __restrict__ arena, const BatchCirc* __restrict__ circs, const int32_t* __restrict__ list,
                const BatchPass* __restrict__ passes, const TileOp* __restrict__ ops,
                const double* __restrict__ mats)
{
    using V = typename CT<R>::V;
    constexpr uint32_t E = 1u << M;
    extern __shared__ __align__(16) unsigned char smem[];
    V* tile = (V*)smem;
    uint32_t* hoff = (uint32_t*)(smem + sizeof(V) * E);
    const BatchCirc& c = circs[list[blockIdx.x]];
    V* psi = (V*)(arena + c.psi_off);
    const uint64_t N = 1ull << c.n;
    for (uint64_t i = threadIdx.x; i < N; i += 256) {
        V v;
        v.x = (i == c.basis) ? (R)1 : (R)0;
        v.y = 0;
        psi[i] = v;
    }
    __syncthreads(); // global writes of this block are visible to its own later loads
    const uint64_t ntiles = 1ull << (c.n - M);
    for (int p = 0; p < c.npass; ++p) {
        const BatchPass& bp = passes[c.pass0 + p];
        build_hoff(hoff, M, bp.L, bp.q);
        __syncthreads();
        for (uint64_t tau = 0; tau < ntiles; ++tau) {
            const uint64_t base = ins_bits(tau, bp.ip);
            tile_load<R, M>(psi, base, bp.L, hoff, tile, 0);
            __syncthreads();
            tile_ops<R, M, MF>(tile, base, ops + bp.op0, bp.nops, mats);
            tile_store<R, M>(psi, base, bp.L, hoff, tile, 0);
            __syncthreads();
        }
    }
}

template <typename R, int M, bool MF>
__global__ void __launch_bounds__(256)
k_batch_round(char* __restrict__ arena, const BatchCirc* __restrict__ circs, const BatchPass* __restrict__ passes,
              const TileOp* __restrict__ ops, const double* __restrict__ mats,
              const RoundEntry* __restrict__ entries, int nentries)
{
    using V = typename CT<R>::V;
    constexpr uint32_t E = 1u << M;
    extern __shared__ __align__(16) unsigned char smem[];
    V* tile = (V*)smem;
    uint32_t* hoff = (uint32_t*)(smem + sizeof(V) * E);
    // the entry owning this block: last one with first_block <= blockIdx.x
    int lo = 0, hi = nentries - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (entries[mid].first_block <= blockIdx.x)
            lo = mid;
        else
            hi = mid - 1;
    }
    const RoundEntry& en = entries[lo];
    const BatchCirc& c = circs[en.circ];
    const BatchPass& bp = passes[en.pass];
    V* psi = (V*)(arena + c.psi_off);
    build_hoff(hoff, M, bp.L, bp.q);
    __syncthreads();
    const uint64_t base = ins_bits((uint64_t)(blockIdx.x - en.first_block), bp.ip);
    const int nt = bp.L >= (sizeof(R) == 8 ? 3 : 4) ? 1 : 0;
    tile_load<R, M>(psi, base, bp.L, hoff, tile, nt);
    __syncthreads();
    tile_ops<R, M, MF>(tile, base, ops + bp.op0, bp.nops, mats);
    tile_store<R, M>(psi, base, bp.L, hoff, tile, nt);
}

template <typename V>
__global__ void __launch_bounds__(256)
k_batch_init(char* __restrict__ arena, uint64_t n16, const BatchCirc* __restrict__ circs,
             const int32_t* __restrict__ list, int count)
{
    // zero the arena with 16-byte stores, then (last block) the basis amplitudes
    uint4* z = (uint4*)arena;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += (uint64_t)gridDim.x * 256)
        z[i] = make_uint4(0, 0, 0, 0);
}

template <typename V>
__global__ void __launch_bounds__(256)
k_batch_basis(char* __restrict__ arena, const BatchCirc* __restrict__ circs, const int32_t* __restrict__ list,
              int count)
{
    for (int i = blockIdx.x * 256 + threadIdx.x; i < count; i += gridDim.x * 256) {
        const BatchCirc& c = circs[list[i]];
        V v;
        v.x = 1;
        v.y = 0;
        ((V*)(arena + c.psi_off))[c.basis] = v;
    }
}

template <typename R, int M, bool MF>
static hipError_t launch_round_m(char* arena, const BatchCirc* circs, const BatchPass* passes, const TileOp* ops,
                                 const double* mats, const RoundEntry* entries, int nentries, uint32_t nblocks,
                                 hipStream_t st)
{
    const size_t lds_max = tile_lds_bytes(sizeof(R) == 8 ? QS_C128 : QS_C64, M, 0);
    const size_t lds = lds_max > 163840 ? 163840 : lds_max;
    if (lds > 65536) {
        static bool set = false;
        if (!set) {
            hipError_t e = hipFuncSetAttribute((const void*)k_batch_round<R, M, MF>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
            set = true;
        }
    }
    hipLaunchKernelGGL((k_batch_round<R, M, MF>), dim3(nblocks), dim3(256), lds, st, arena, circs, passes, ops, mats,
                       entries, nentries);
    return hipGetLastError();
}

template <typename R, int M, bool MF>
__global__ void __launch_bounds__(256)
k_serve_round(const ServeEntry* __restrict__ entries, int nentries)
{
    using V = typename CT<R>::V;
    constexpr uint32_t E = 1u << M;
    extern __shared__ __align__(16) unsigned char smem[];
    V* tile = (V*)smem;
    uint32_t* hoff = (uint32_t*)(smem + sizeof(V) * E);
    int lo = 0, hi = nentries - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (entries[mid].first_block <= blockIdx.x)
            lo = mid;
        else
            hi = mid - 1;
    }
    const ServeEntry& en = entries[lo];
    const BatchPass& bp = *en.pass;
    V* psi = (V*)en.psi;
    build_hoff(hoff, M, bp.L, bp.q);
    __syncthreads();
    const uint64_t base = ins_bits((uint64_t)(blockIdx.x - en.first_block), bp.ip);
    const int nt = bp.L >= (sizeof(R) == 8 ? 3 : 4) ? 1 : 0;
    tile_load<R, M>(psi, base, bp.L, hoff, tile, nt);
    __syncthreads();
    tile_ops<R, M, MF>(tile, base, en.ops + bp.op0, bp.nops, en.mats);
    tile_store<R, M>(psi, base, bp.L, hoff, tile, nt);
}

template <typename R, int M, bool MF>
__global__ void __launch_bounds__(256)
k_serve_whole(const ServeEntry* __restrict__ entries)
{
    using V = typename CT<R>::V;
    constexpr uint32_t E = 1u << M;
    extern __shared__ __align__(16) unsigned char smem[];
    V* tile = (V*)smem;
    uint32_t* hoff = (uint32_t*)(smem + sizeof(V) * E);
    const ServeEntry& en = entries[blockIdx.x];
    for (uint32_t e = threadIdx.x; e < E; e += 256) {
        V v;
        v.x = (e == en.basis) ? (R)1 : (R)0;
        v.y = 0;
        tile[e] = v;
    }
    if (threadIdx.x == 0) hoff[0] = 0;
    __syncthreads();
    if (en.pass) tile_ops<R, M, MF>(tile, 0, en.ops + en.pass->op0, en.pass->nops, en.mats);
    tile_store<R, M>((V*)en.psi, 0, M, hoff, tile, M >= 4 ? 1 : 0);
}

template <typename R, int M, bool MF>
static hipError_t launch_serve_round_m(const ServeEntry* entries, int nentries, uint32_t nblocks, hipStream_t st)
{
    const size_t lds_max = tile_lds_bytes(sizeof(R) == 8 ? QS_C128 : QS_C64, M, 0);
    const size_t lds = lds_max > 163840 ? 163840 : lds_max;
    if (lds > 65536) {
        static bool set = false;
        if (!set) {
            hipError_t e = hipFuncSetAttribute((const void*)k_serve_round<R, M, MF>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
            set = true;
        }
    }
    hipLaunchKernelGGL((k_serve_round<R, M, MF>), dim3(nblocks), dim3(256), lds, st, entries, nentries);
    return hipGetLastError();
}

template <typename R, int M, bool MF>
static hipError_t launch_serve_whole_m(const ServeEntry* entries, int nentries, hipStream_t st)
{
    const size_t lds = sizeof(typename CT<R>::V) * (1ull << M) + 16;
    if (lds > 65536) {
        static bool set = false;
        if (!set) {
            hipError_t e = hipFuncSetAttribute((const void*)k_serve_whole<R, M, MF>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
            set = true;
        }
    }
    hipLaunchKernelGGL((k_serve_whole<R, M, MF>), dim3(nentries), dim3(256), lds, st, entries);
    return hipGetLastError();
}

template <typename R, int M, bool MF>
static hipError_t launch_whole_m(char* arena, const BatchCirc* circs, const int32_t* list, int count,
                                 const BatchPass* passes, const TileOp* ops, const double* mats, hipStream_t st)
{
    const size_t lds = sizeof(typename CT<R>::V) * (1ull << M) + 16;
    if (lds > 65536) {
        static bool set = false;
        if (!set) {
            hipError_t e = hipFuncSetAttribute((const void*)k_batch_whole<R, M, MF>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
            set = true;
        }
    }
    hipLaunchKernelGGL((k_batch_whole<R, M, MF>), dim3(count), dim3(256), lds, st, arena, circs, list, passes, ops, mats);
    return hipGetLastError();
}

template <typename R, int M, bool MF>
static hipError_t launch_persist_m(char* arena, const BatchCirc* circs, const int32_t* list, int count,
                                   const BatchPass* passes, const TileOp* ops, const double* mats, hipStream_t st)
{
    const size_t lds_max = tile_lds_bytes(sizeof(R) == 8 ? QS_C128 : QS_C64, M, 0);
    if (lds_max > 65536) {
        static bool set = false;
        if (!set) {
            const int lim = lds_max > 163840 ? 163840 : (int)lds_max;
            hipError_t e = hipFuncSetAttribute((const void*)k_batch_persist<R, M, MF>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, lim);
            if (e != hipSuccess) return e;
            set = true;
        }
    }
    // LDS for the smallest L any pass may have
    const size_t lds = lds_max > 163840 ? 163840 : lds_max;
    hipLaunchKernelGGL((k_batch_persist<R, M, MF>), dim3(count), dim3(256), lds, st, arena, circs, list, passes, ops,
                       mats);
    return hipGetLastError();
}

template <typename R, int M>
hipError_t launch_m(void* psi, int n, const PlanPass& pass, const TileOp* dops, const void* dmats,
                    hipStream_t st)
{
    using V = typename CT<R>::V;
    QList ql;
    ql.m = pass.m;
    ql.L = pass.L;
    uint64_t qmask = 0;
    for (int j = 0; j < pass.m; ++j) {
        ql.q[j] = pass.Q[j];
        qmask |= 1ull << pass.Q[j];
    }
    InsertPlan ip = make_insert_plan(qmask);
    const uint64_t ntiles = 1ull << (n - M);
    const size_t lds = tile_lds_bytes(sizeof(R) == 8 ? QS_C128 : QS_C64, M, pass.L);
    // Opt in once per instantiation to the largest LDS any pass of this tile
    // size can ask for (L = 0), so later passes never exceed the attribute.
    static bool attr_set = false;
    const size_t lds_max = tile_lds_bytes(sizeof(R) == 8 ? QS_C128 : QS_C64, M, 0);
    if (!attr_set && lds_max > 65536) {
        const int lim = lds_max > 163840 ? 163840 : (int)lds_max;
        hipError_t e = hipFuncSetAttribute((const void*)k_tile<R, M, false>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lim);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void*)k_tile<R, M, true>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    if (lds > 163840) return hipErrorInvalidValue;
    static int cap = env_int("QS_TILE_GRID_CAP", 256 * 8);
    const unsigned g = (unsigned)(ntiles < (uint64_t)cap ? ntiles : (uint64_t)cap);
    // non-temporal when each contiguous run covers whole 128-byte lines
    const int line_bits = sizeof(R) == 8 ? 3 : 4;
    static int nt_env = env_int("QS_NT", 1);
    const int nt = (nt_env && pass.L >= line_bits) ? 1 : 0;
    // the matrix-core variant only when the pass holds a fused block (its
    // fragments would otherwise cost every pass registers)
    bool mf = false;
    for (const TileOp& t : pass.ops) mf |= t.kind == TK_MFMA;
    if (mf)
        hipLaunchKernelGGL((k_tile<R, M, true>), dim3(g), dim3(256), lds, st, (V*)psi, ntiles, ql, ip, dops,
                           (int)pass.ops.size(), (const double*)dmats, nt);
    else
        hipLaunchKernelGGL((k_tile<R, M, false>), dim3(g), dim3(256), lds, st, (V*)psi, ntiles, ql, ip, dops,
                           (int)pass.ops.size(), (const double*)dmats, nt);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_r(void* psi, int n, const PlanPass& pass, const TileOp* dops, const void* dmats,
                    hipStream_t st)
{
    switch (pass.m) {
#define QS_TILE_CASE(MM) \
    case MM: return launch_m<R, MM>(psi, n, pass, dops, dmats, st);
        QS_TILE_CASE(1) QS_TILE_CASE(2) QS_TILE_CASE(3) QS_TILE_CASE(4) QS_TILE_CASE(5) QS_TILE_CASE(6)
        QS_TILE_CASE(7) QS_TILE_CASE(8) QS_TILE_CASE(9) QS_TILE_CASE(10) QS_TILE_CASE(11) QS_TILE_CASE(12)
        QS_TILE_CASE(13)
#undef QS_TILE_CASE
    default: return hipErrorInvalidValue;
    }
}

template <typename R, bool MF>
static hipError_t batch_whole_r(int M, char* arena, const BatchCirc* circs, const int32_t* list, int count,
                                const BatchPass* passes, const TileOp* ops, const double* mats, hipStream_t st)
{
    switch (M) {
#define QS_WCASE(MM) \
    case MM: return launch_whole_m<R, MM, MF>(arena, circs, list, count, passes, ops, mats, st);
        QS_WCASE(1) QS_WCASE(2) QS_WCASE(3) QS_WCASE(4) QS_WCASE(5) QS_WCASE(6) QS_WCASE(7) QS_WCASE(8)
        QS_WCASE(9) QS_WCASE(10) QS_WCASE(11) QS_WCASE(12) QS_WCASE(13)
#undef QS_WCASE
    default: return hipErrorInvalidValue;
    }
}

template <typename R, bool MF>
static hipError_t batch_persist_r(int M, char* arena, const BatchCirc* circs, const int32_t* list, int count,
                                  const BatchPass* passes, const TileOp* ops, const double* mats, hipStream_t st)
{
    switch (M) {
#define QS_PCASE(MM) \
    case MM: return launch_persist_m<R, MM, MF>(arena, circs, list, count, passes, ops, mats, st);
        QS_PCASE(9) QS_PCASE(10) QS_PCASE(11) QS_PCASE(12) QS_PCASE(13)
#undef QS_PCASE
    default: return hipErrorInvalidValue;
    }
}

} // namespace

size_t tile_lds_bytes(int dt, int m, int L)
{
    return amp_bytes(dt) * (1ull << m) + 4ull * (1ull << (m - L));
}

hipError_t launch_batch_whole(int dt, int M, char* arena, const BatchCirc* circs, const int32_t* list, int count,
                              const BatchPass* passes, const TileOp* ops, const double* mats, bool mf,
                              hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    if (dt == QS_C128) return batch_whole_r<double, false>(M, arena, circs, list, count, passes, ops, mats, st);
    return mf ? batch_whole_r<float, true>(M, arena, circs, list, count, passes, ops, mats, st)
              : batch_whole_r<float, false>(M, arena, circs, list, count, passes, ops, mats, st);
}

hipError_t launch_batch_persist(int dt, int M, char* arena, const BatchCirc* circs, const int32_t* list,
                                int count, const BatchPass* passes, const TileOp* ops, const double* mats, bool mf,
                                hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    if (dt == QS_C128) return batch_persist_r<double, false>(M, arena, circs, list, count, passes, ops, mats, st);
    return mf ? batch_persist_r<float, true>(M, arena, circs, list, count, passes, ops, mats, st)
              : batch_persist_r<float, false>(M, arena, circs, list, count, passes, ops, mats, st);
}

template <typename R, bool MF>
static hipError_t batch_round_r(int M, char* arena, const BatchCirc* circs, const BatchPass* passes,
                                const TileOp* ops, const double* mats, const RoundEntry* entries, int nentries,
                                uint32_t nblocks, hipStream_t st)
{
    switch (M) {
#define QS_RCASE(MM) \
    case MM: return launch_round_m<R, MM, MF>(arena, circs, passes, ops, mats, entries, nentries, nblocks, st);
        QS_RCASE(9) QS_RCASE(10) QS_RCASE(11) QS_RCASE(12) QS_RCASE(13)
#undef QS_RCASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batch_round(int dt, int M, char* arena, const BatchCirc* circs, const BatchPass* passes,
                              const TileOp* ops, const double* mats, const RoundEntry* entries, int nentries,
                              uint32_t nblocks, bool mf, hipStream_t st)
{
    if (nentries <= 0 || nblocks == 0) return hipSuccess;
    if (dt == QS_C128)
        return batch_round_r<double, false>(M, arena, circs, passes, ops, mats, entries, nentries, nblocks, st);
    return mf ? batch_round_r<float, true>(M, arena, circs, passes, ops, mats, entries, nentries, nblocks, st)
              : batch_round_r<float, false>(M, arena, circs, passes, ops, mats, entries, nentries, nblocks, st);
}

hipError_t launch_batch_init(int dt, char* arena, uint64_t bytes, const BatchCirc* circs, const int32_t* list,
                             int count, hipStream_t st)
{
    const uint64_t n16 = bytes / 16;
    uint64_t g = (n16 + 255) / 256;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_batch_init<double2>, dim3((unsigned)g), dim3(256), 0, st, arena, n16, circs, list, count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || count <= 0) return e;
    const unsigned gb = (unsigned)((count + 255) / 256);
    if (dt == QS_C128)
        hipLaunchKernelGGL(k_batch_basis<double2>, dim3(gb), dim3(256), 0, st, arena, circs, list, count);
    else
        hipLaunchKernelGGL(k_batch_basis<float2>, dim3(gb), dim3(256), 0, st, arena, circs, list, count);
    return hipGetLastError();
}

template <typename R, bool MF>
static hipError_t serve_round_r(int M, const ServeEntry* entries, int nentries, uint32_t nblocks, hipStream_t st)
{
    switch (M) {
#define QS_SRCASE(MM) \
    case MM: return launch_serve_round_m<R, MM, MF>(entries, nentries, nblocks, st);
        QS_SRCASE(9) QS_SRCASE(10) QS_SRCASE(11) QS_SRCASE(12) QS_SRCASE(13)
#undef QS_SRCASE
    default: return hipErrorInvalidValue;
    }
}

template <typename R, bool MF>
static hipError_t serve_whole_r(int M, const ServeEntry* entries, int nentries, hipStream_t st)
{
    switch (M) {
#define QS_SWCASE(MM) \
    case MM: return launch_serve_whole_m<R, MM, MF>(entries, nentries, st);
        QS_SWCASE(1) QS_SWCASE(2) QS_SWCASE(3) QS_SWCASE(4) QS_SWCASE(5) QS_SWCASE(6) QS_SWCASE(7)
        QS_SWCASE(8) QS_SWCASE(9) QS_SWCASE(10) QS_SWCASE(11) QS_SWCASE(12) QS_SWCASE(13)
#undef QS_SWCASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_serve_round(int dt, int M, const ServeEntry* entries, int nentries, uint32_t nblocks, bool mf,
                              hipStream_t st)
{
    if (nentries <= 0 || nblocks == 0) return hipSuccess;
    if (dt == QS_C128) return serve_round_r<double, false>(M, entries, nentries, nblocks, st);
    return mf ? serve_round_r<float, true>(M, entries, nentries, nblocks, st)
              : serve_round_r<float, false>(M, entries, nentries, nblocks, st);
}

hipError_t launch_serve_whole(int dt, int M, const ServeEntry* entries, int nentries, bool mf, hipStream_t st)
{
    if (nentries <= 0) return hipSuccess;
    if (dt == QS_C128) return serve_whole_r<double, false>(M, entries, nentries, st);
    return mf ? serve_whole_r<float, true>(M, entries, nentries, st)
              : serve_whole_r<float, false>(M, entries, nentries, st);
}

hipError_t launch_tile_pass(void* psi, int dt, int n, const PlanPass& pass, const TileOp* dops,
                            const void* dmats, hipStream_t st)
{
    if (pass.m < 1 || pass.m > 13 || pass.m > n || pass.L > pass.m) return hipErrorInvalidValue;
    return dt == QS_C128 ? launch_r<double>(psi, n, pass, dops, dmats, st)
                         : launch_r<float>(psi, n, pass, dops, dmats, st);
}

} // namespace qs
