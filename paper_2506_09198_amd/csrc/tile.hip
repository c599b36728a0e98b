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

template <typename R, int M>
__global__ void __launch_bounds__(256)
k_tile(typename CT<R>::V* __restrict__ psi, uint64_t ntiles, QList ql, InsertPlan ipQ,
       const TileOp* __restrict__ ops, int nops, const double* __restrict__ mats)
{
    using V = typename CT<R>::V;
    constexpr uint32_t E = 1u << M;
    constexpr int PER = (E + 255) / 256; // tile elements per lane
    extern __shared__ __align__(16) unsigned char smem[];
    V* tile = (V*)smem;
    uint32_t* hoff = (uint32_t*)(smem + sizeof(V) * E); // dep_Q of the upper tile bits, >> L
    const int L = ql.L;
    const uint32_t H = 1u << (M - L);
    for (uint32_t h = threadIdx.x; h < H; h += 256) {
        uint64_t off = 0;
        for (int j = L; j < M; ++j)
            if ((h >> (j - L)) & 1) off |= 1ull << ql.q[j];
        hoff[h] = (uint32_t)(off >> L);
    }
    __syncthreads();
    const uint32_t lowm = (1u << L) - 1;
    const int tid = threadIdx.x;
    for (uint64_t tau = blockIdx.x; tau < ntiles; tau += gridDim.x) {
        const uint64_t base = ins_bits(tau, ipQ);
        {
            // all loads of the tile are issued before the first LDS write
            R rx[PER], ry[PER];
#pragma unroll
            for (int s = 0; s < PER; ++s) {
                const uint32_t e = tid + 256 * s;
                if (E >= 256 || e < E) {
                    const V v = psi[base | (e & lowm) | ((uint64_t)hoff[e >> L] << L)];
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
        __syncthreads();
        for (int o = 0; o < nops; ++o) {
            const TileOp& d = ops[o];
            const int kind = d.kind;
            if ((base & d.gcm) != d.gcv) continue; // whole tile fails the outside controls
            const double* u = mats + d.moff;
            const uint32_t lcm = (uint32_t)d.lcm, lcv = (uint32_t)d.lcv;
            if (kind == TK_DENSE1) {
                const int p = d.p[0];
                const double u0 = u[0], u1 = u[1], u2 = u[2], u3 = u[3], u4 = u[4], u5 = u[5], u6 = u[6],
                             u7 = u[7];
#pragma unroll
                for (int s = 0; s < (PER + 1) / 2; ++s) {
                    const uint32_t k = tid + 256 * s;
                    if (k < E / 2) {
                        const uint32_t e0 = ins0_32(k, p), e1 = e0 | (1u << p);
                        if ((e0 & lcm) == lcv) {
                            const double2 a = ld2(tile[e0]), b = ld2(tile[e1]);
                            tile[e0] = st2<V>(cmad2<double2, double>(u0, u1, a, u2, u3, b));
                            tile[e1] = st2<V>(cmad2<double2, double>(u4, u5, a, u6, u7, b));
                        }
                    }
                }
            } else if (kind == TK_DENSE2) {
                const int p0 = d.p[0], p1 = d.p[1];
                const int lo = p0 < p1 ? p0 : p1, hi = p0 < p1 ? p1 : p0;
                const uint32_t b0 = 1u << p0, b1 = 1u << p1;
#pragma unroll
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
            } else if (kind == TK_DIAG) {
                const int k = d.k;
#pragma unroll
                for (int s = 0; s < PER; ++s) {
                    const uint32_t e = tid + 256 * s;
                    if (e < E && (e & lcm) == lcv) {
                        const uint64_t g = base | (e & lowm) | ((uint64_t)hoff[e >> L] << L);
                        uint32_t idx = 0;
                        for (int j = 0; j < k; ++j) idx |= (uint32_t)((g >> d.p[j]) & 1) << j;
                        tile[e] = st2<V>(cmul<double2, double>(u[2 * idx], u[2 * idx + 1], ld2(tile[e])));
                    }
                }
            }
            __syncthreads();
        }
        {
#pragma unroll
            for (int s = 0; s < PER; ++s) {
                const uint32_t e = tid + 256 * s;
                if (e < E) psi[base | (e & lowm) | ((uint64_t)hoff[e >> L] << L)] = tile[e];
            }
        }
        __syncthreads();
    }
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
        hipError_t e = hipFuncSetAttribute((const void*)k_tile<R, M>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           lim);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    if (lds > 163840) return hipErrorInvalidValue;
    static int cap = env_int("QS_TILE_GRID_CAP", 256 * 8);
    const unsigned g = (unsigned)(ntiles < (uint64_t)cap ? ntiles : (uint64_t)cap);
    hipLaunchKernelGGL((k_tile<R, M>), dim3(g), dim3(256), lds, st, (V*)psi, ntiles, ql, ip, dops,
                       (int)pass.ops.size(), (const double*)dmats);
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

} // namespace

size_t tile_lds_bytes(int dt, int m, int L)
{
    return amp_bytes(dt) * (1ull << m) + 4ull * (1ull << (m - L));
}

hipError_t launch_tile_pass(void* psi, int dt, int n, const PlanPass& pass, const TileOp* dops,
                            const void* dmats, hipStream_t st)
{
    if (pass.m < 1 || pass.m > 13 || pass.m > n || pass.L > pass.m) return hipErrorInvalidValue;
    return dt == QS_C128 ? launch_r<double>(psi, n, pass, dops, dmats, st)
                         : launch_r<float>(psi, n, pass, dops, dmats, st);
}

} // namespace qs
