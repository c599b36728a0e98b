// K4 launcher: the single-circuit LDS tile pass (device code in tile_device.h).
#include "tile_device.h"

namespace qs {

namespace {

template <typename R, int M, int VAR>
__device__ __forceinline__ void tile_pass(typename CT<R>::V* __restrict__ psi, uint64_t ntiles, const QList& ql,
                                          const InsertPlan& ipQ, const TileOp* __restrict__ ops, int nops,
                                          const double* __restrict__ mats, int nt)
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
        tile_ops<R, M, VAR>(tile, base, ops, nops, mats);
        tile_store<R, M>(psi, base, ql.L, hoff, tile, nt);
        __syncthreads();
    }
}

template <typename R, int M, int VAR>
__global__ void __launch_bounds__(256)
k_tile(typename CT<R>::V* __restrict__ psi, uint64_t ntiles, QList ql, InsertPlan ipQ,
       const TileOp* __restrict__ ops, int nops, const double* __restrict__ mats, int nt)
{
    tile_pass<R, M, VAR>(psi, ntiles, ql, ipQ, ops, nops, mats, nt);
}

// The same pass held to 128 VGPRs (4 waves per SIMD instead of 3): for tiles
// of 2^11 the compiler then keeps a few values in scratch (12 bytes per lane
// for the lean kernel); larger tiles would spill heavily and keep k_tile.
template <typename R, int M, int VAR>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k_tile_w4(typename CT<R>::V* __restrict__ psi, uint64_t ntiles, QList ql, InsertPlan ipQ,
          const TileOp* __restrict__ ops, int nops, const double* __restrict__ mats, int nt)
{
    tile_pass<R, M, VAR>(psi, ntiles, ql, ipQ, ops, nops, mats, nt);
}

template <typename R, int M>
hipError_t launch_m(void* psi, int n, const PlanPass& pass, const TileOp* dops, const void* dmats,
                    int max_blocks, hipStream_t st)
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
    const size_t lds_max = tile_lds_bytes(sizeof(R) == 8 ? QS_C128 : QS_C64, M, 0);
    {
        const size_t lim = lds_max > 163840 ? 163840 : lds_max;
        hipError_t e = lds_optin((const void*)k_tile<R, M, 0>, lim);
        if (e == hipSuccess) e = lds_optin((const void*)k_tile<R, M, 1>, lim);
        if constexpr (M >= 8)
            if (e == hipSuccess) e = lds_optin((const void*)k_tile<R, M, 2>, lim);
        if constexpr (M >= 8 && sizeof(R) == 4)
            if (e == hipSuccess) e = lds_optin((const void*)k_tile<R, M, 3>, lim);
        if constexpr (M == 11)
            if (e == hipSuccess) e = lds_optin((const void*)k_tile_w4<R, M, 0>, lim);
        if (e != hipSuccess) return e;
    }
    if (lds > 163840) return hipErrorInvalidValue;
    // Blocks loop over tiles.  Measured on 30- and 32-qubit circuits: 65536
    // blocks (8-32 tiles each) beat 2048 by 9-12 % and one tile per block;
    // blocks that start and finish at different times keep more of them in
    // different phases (loading, computing, storing) on each CU.
    const uint64_t cap = max_blocks > 0 ? (uint64_t)max_blocks : (uint64_t)tun(T_TILE_GRID_CAP);
    const unsigned g = (unsigned)(ntiles < cap ? ntiles : cap);
    // non-temporal when each contiguous run covers whole 128-byte lines
    const int line_bits = sizeof(R) == 8 ? 3 : 4;
    const int nt = (tun(T_NT) && pass.L >= line_bits) ? 1 : 0;
    // the variant the pass needs (k >= 3 ops, fused blocks or ops outside
    // segments would otherwise cost every pass registers)
    const int var = ops_variant(pass.ops.data(), pass.ops.size(), pass.m);
    const int nops = (int)pass.ops.size();
    if constexpr (M >= 8 && sizeof(R) == 4) {
        if (var == 3) { // FP32 matrix-core blocks
            hipLaunchKernelGGL((k_tile<R, M, 3>), dim3(g), dim3(256), lds, st, (V*)psi, ntiles, ql, ip, dops, nops,
                               (const double*)dmats, nt);
            return hipGetLastError();
        }
    }
    if constexpr (M >= 8) {
        if (var >= 2) {
            hipLaunchKernelGGL((k_tile<R, M, 2>), dim3(g), dim3(256), lds, st, (V*)psi, ntiles, ql, ip, dops, nops,
                               (const double*)dmats, nt);
            return hipGetLastError();
        }
    }
    if (var >= 1) {
        hipLaunchKernelGGL((k_tile<R, M, 1>), dim3(g), dim3(256), lds, st, (V*)psi, ntiles, ql, ip, dops, nops,
                           (const double*)dmats, nt);
        return hipGetLastError();
    }
    if constexpr (M == 11) {
        if (tun(T_TILE_W4)) {
            hipLaunchKernelGGL((k_tile_w4<R, M, 0>), dim3(g), dim3(256), lds, st, (V*)psi, ntiles, ql, ip, dops, nops,
                               (const double*)dmats, nt);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((k_tile<R, M, 0>), dim3(g), dim3(256), lds, st, (V*)psi, ntiles, ql, ip, dops, nops,
                       (const double*)dmats, nt);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_r(void* psi, int n, const PlanPass& pass, const TileOp* dops, const void* dmats,
                    int max_blocks, hipStream_t st)
{
    switch (pass.m) {
#define QS_TILE_CASE(MM) \
    case MM: return launch_m<R, MM>(psi, n, pass, dops, dmats, max_blocks, st);
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
                            const void* dmats, int max_blocks, hipStream_t st)
{
    if (pass.m < 1 || pass.m > 13 || pass.m > n || pass.L > pass.m) return hipErrorInvalidValue;
    return dt == QS_C128 ? launch_r<double>(psi, n, pass, dops, dmats, max_blocks, st)
                         : launch_r<float>(psi, n, pass, dops, dmats, max_blocks, st);
}

} // namespace qs
