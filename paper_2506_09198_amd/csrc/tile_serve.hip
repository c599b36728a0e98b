// Serving-loop kernels: rounds of one tile pass of every active request, and
// whole small requests in one workgroup (device code in tile_device.h).
#include "tile_device.h"

namespace qs {

namespace {

// Grid of the round kernels: blocks loop over tiles, as in the single-circuit
// tile pass (65536 blocks measured best there).
static inline unsigned round_grid(uint32_t ntiles)
{
    const uint32_t c = (uint32_t)tun(T_ROUND_GRID_CAP);
    return ntiles < c ? ntiles : c;
}

template <typename R, int M, int VAR>
__global__ void __launch_bounds__(256)
k_serve_round(char* __restrict__ pool, const char* __restrict__ plan, const ServeEntry* __restrict__ entries,
              int nentries, uint32_t ntiles)
{
    using V = typename CT<R>::V;
    constexpr uint32_t E = 1u << M;
    extern __shared__ __align__(16) unsigned char smem[];
    V* tile = (V*)smem;
    uint32_t* hoff = (uint32_t*)(smem + sizeof(V) * E);
    for (uint32_t g = blockIdx.x; g < ntiles; g += gridDim.x) {
        int lo = 0, hi = nentries - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (entries[mid].first_block <= g)
                lo = mid;
            else
                hi = mid - 1;
        }
        const ServeEntry& en = entries[lo];
        const BatchPass& bp = *(const BatchPass*)(plan + en.pass_off);
        V* psi = (V*)(pool + en.psi_off);
        build_hoff(hoff, M, bp.L, bp.q);
        __syncthreads();
        const uint64_t base = ins_bits((uint64_t)(g - en.first_block), bp.ip);
        const int nt = bp.L >= (sizeof(R) == 8 ? 3 : 4) ? 1 : 0;
        tile_load<R, M>(psi, base, bp.L, hoff, tile, nt);
        __syncthreads();
        tile_ops<R, M, VAR>(tile, base, (const TileOp*)(plan + en.ops_off) + bp.op0, bp.nops,
                             (const double*)(plan + en.mats_off));
        tile_store<R, M>(psi, base, bp.L, hoff, tile, nt);
        __syncthreads(); // the next tile rewrites hoff and the tile
    }
}

template <typename R, int M, int VAR>
__global__ void __launch_bounds__(256)
k_serve_whole(char* __restrict__ pool, const char* __restrict__ plan, const ServeEntry* __restrict__ entries)
{
    using V = typename CT<R>::V;
    constexpr uint32_t E = 1u << M;
    extern __shared__ __align__(16) unsigned char smem[];
    V* tile = (V*)smem;
    uint32_t* hoff = (uint32_t*)(smem + sizeof(V) * E);
    const ServeEntry& en = entries[blockIdx.x];
    if (threadIdx.x == 0) hoff[0] = 0;
    if (en.basis == kLoadInitial) { // the caller's initial state, copied into the pool
        __syncthreads();
        tile_load<R, M>((const V*)(pool + en.psi_off), 0, M, hoff, tile, 0);
    } else {
        for (uint32_t e = threadIdx.x; e < E; e += 256) {
            V v;
            v.x = (e == en.basis) ? (R)1 : (R)0;
            v.y = 0;
            tile[QS_SW(e)] = v;
        }
    }
    __syncthreads();
    if (en.pass_off != ~0ull) {
        const BatchPass& bp = *(const BatchPass*)(plan + en.pass_off);
        tile_ops<R, M, VAR>(tile, 0, (const TileOp*)(plan + en.ops_off) + bp.op0, bp.nops,
                             (const double*)(plan + en.mats_off));
    }
    tile_store<R, M>((V*)(pool + en.psi_off), 0, M, hoff, tile, M >= 4 ? 1 : 0);
}

template <typename R, int M, int VAR>
static hipError_t launch_serve_round_m(char* pool, const char* plan, const ServeEntry* entries, int nentries,
                                       uint32_t nblocks, hipStream_t st)
{
    const size_t lds_max = tile_lds_bytes(sizeof(R) == 8 ? QS_C128 : QS_C64, M, 0);
    const size_t lds = lds_max > 163840 ? 163840 : lds_max;
    {
        const hipError_t e = lds_optin((const void*)k_serve_round<R, M, VAR>, lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_serve_round<R, M, VAR>), dim3(round_grid(nblocks)), dim3(256), lds, st, pool, plan, entries,
                       nentries, nblocks);
    return hipGetLastError();
}

template <typename R, int M, int VAR>
static hipError_t launch_serve_whole_m(char* pool, const char* plan, const ServeEntry* entries, int nentries,
                                       hipStream_t st)
{
    const size_t lds = sizeof(typename CT<R>::V) * (1ull << M) + 16;
    {
        const hipError_t e = lds_optin((const void*)k_serve_whole<R, M, VAR>, lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_serve_whole<R, M, VAR>), dim3(nentries), dim3(256), lds, st, pool, plan, entries);
    return hipGetLastError();
}

template <typename R, int VAR>
static hipError_t serve_round_r(int M, char* pool, const char* plan, const ServeEntry* entries, int nentries,
                                uint32_t nblocks, hipStream_t st)
{
    switch (M) {
#define QS_SRCASE(MM) \
    case MM: return launch_serve_round_m<R, MM, (VAR >= 2 && MM < 8 ? 1 : VAR)>(pool, plan, entries, nentries, nblocks, st);
        QS_SRCASE(9) QS_SRCASE(10) QS_SRCASE(11) QS_SRCASE(12) QS_SRCASE(13)
#undef QS_SRCASE
    default: return hipErrorInvalidValue;
    }
}

template <typename R, int VAR>
static hipError_t serve_whole_r(int M, char* pool, const char* plan, const ServeEntry* entries, int nentries,
                                hipStream_t st)
{
    switch (M) {
#define QS_SWCASE(MM) \
    case MM: return launch_serve_whole_m<R, MM, (VAR >= 2 && MM < 8 ? 1 : VAR)>(pool, plan, entries, nentries, st);
        QS_SWCASE(1) QS_SWCASE(2) QS_SWCASE(3) QS_SWCASE(4) QS_SWCASE(5) QS_SWCASE(6) QS_SWCASE(7)
        QS_SWCASE(8) QS_SWCASE(9) QS_SWCASE(10) QS_SWCASE(11) QS_SWCASE(12) QS_SWCASE(13)
#undef QS_SWCASE
    default: return hipErrorInvalidValue;
    }
}

} // namespace

hipError_t launch_serve_round(int dt, int M, char* pool, const char* plan, const ServeEntry* entries, int nentries,
                              uint32_t nblocks, int var, hipStream_t st)
{
    if (nentries <= 0 || nblocks == 0) return hipSuccess;
    return dispatch_var(dt, var, [&](auto r, auto v) {
        return serve_round_r<typename decltype(r)::type, decltype(v)::value>(M, pool, plan, entries, nentries, nblocks,
                                                                             st);
    });
}

hipError_t launch_serve_whole(int dt, int M, char* pool, const char* plan, const ServeEntry* entries, int nentries,
                              int var, hipStream_t st)
{
    if (nentries <= 0) return hipSuccess;
    return dispatch_var(dt, var, [&](auto r, auto v) {
        return serve_whole_r<typename decltype(r)::type, decltype(v)::value>(M, pool, plan, entries, nentries, st);
    });
}

} // namespace qs
