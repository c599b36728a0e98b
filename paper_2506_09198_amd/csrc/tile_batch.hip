// Batch kernels: whole circuits in one workgroup's LDS, persistent
// single-workgroup passes, and pass-major rounds (device code in
// tile_device.h).
#include "tile_device.h"

namespace qs {

namespace {

// ---------------------------------------------------------------- batches

template <typename R, int M, int VAR>
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
    if (threadIdx.x == 0) hoff[0] = 0;
    if (c.basis == kLoadInitial) { // the caller's initial state, copied into the arena
        __syncthreads();
        tile_load<R, M>(psi, 0, M, hoff, tile, 0);
    } else {
        for (uint32_t e = threadIdx.x; e < E; e += 256) {
            V v;
            v.x = (e == c.basis) ? (R)1 : (R)0;
            v.y = 0;
            tile[QS_SW(e)] = v;
        }
    }
    __syncthreads();
    for (int p = 0; p < c.npass; ++p) {
        const BatchPass& bp = passes[c.pass0 + p];
        tile_ops<R, M, VAR>(tile, 0, ops + bp.op0, bp.nops, mats);
    }
    tile_store<R, M>(psi, 0, M, hoff, tile, M >= 4 ? 1 : 0);
}

template <typename R, int M, int VAR>
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
    if (c.basis != kLoadInitial) // else the caller's initial state is in place
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
            tile_ops<R, M, VAR>(tile, base, ops + bp.op0, bp.nops, mats);
            tile_store<R, M>(psi, base, bp.L, hoff, tile, 0);
            __syncthreads();
        }
    }
}

template <typename R, int M, int VAR>
__global__ void __launch_bounds__(256)
k_batch_round(char* __restrict__ arena, const BatchCirc* __restrict__ circs, const BatchPass* __restrict__ passes,
              const TileOp* __restrict__ ops, const double* __restrict__ mats,
              const RoundEntry* __restrict__ entries, int nentries, uint32_t ntiles)
{
    using V = typename CT<R>::V;
    constexpr uint32_t E = 1u << M;
    extern __shared__ __align__(16) unsigned char smem[];
    V* tile = (V*)smem;
    uint32_t* hoff = (uint32_t*)(smem + sizeof(V) * E);
    // blocks loop over the round's tiles (numbered across its entries)
    for (uint32_t g = blockIdx.x; g < ntiles; g += gridDim.x) {
        // the entry owning tile g: last one with first_block <= g
        int lo = 0, hi = nentries - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (entries[mid].first_block <= g)
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
        const uint64_t base = ins_bits((uint64_t)(g - en.first_block), bp.ip);
        const int nt = bp.L >= (sizeof(R) == 8 ? 3 : 4) ? 1 : 0;
        tile_load<R, M>(psi, base, bp.L, hoff, tile, nt);
        __syncthreads();
        tile_ops<R, M, VAR>(tile, base, ops + bp.op0, bp.nops, mats);
        tile_store<R, M>(psi, base, bp.L, hoff, tile, nt);
        __syncthreads(); // the next tile rewrites hoff and the tile
    }
}

// Grid of the round kernels: blocks loop over tiles, as in the single-circuit
// tile pass (65536 blocks measured best there).
static inline unsigned round_grid(uint32_t ntiles)
{
    const uint32_t c = (uint32_t)tun(T_ROUND_GRID_CAP);
    return ntiles < c ? ntiles : c;
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
        if (c.basis == kLoadInitial) continue; // copied in after this kernel
        V v;
        v.x = 1;
        v.y = 0;
        ((V*)(arena + c.psi_off))[c.basis] = v;
    }
}

template <typename R, int M, int VAR>
static hipError_t launch_round_m(char* arena, const BatchCirc* circs, const BatchPass* passes, const TileOp* ops,
                                 const double* mats, const RoundEntry* entries, int nentries, uint32_t nblocks,
                                 hipStream_t st)
{
    const size_t lds_max = tile_lds_bytes(sizeof(R) == 8 ? QS_C128 : QS_C64, M, 0);
    const size_t lds = lds_max > 163840 ? 163840 : lds_max;
    {
        const hipError_t e = lds_optin((const void*)k_batch_round<R, M, VAR>, lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_batch_round<R, M, VAR>), dim3(round_grid(nblocks)), dim3(256), lds, st, arena, circs, passes,
                       ops, mats, entries, nentries, nblocks);
    return hipGetLastError();
}

template <typename R, int M, int VAR>
static hipError_t launch_whole_m(char* arena, const BatchCirc* circs, const int32_t* list, int count,
                                 const BatchPass* passes, const TileOp* ops, const double* mats, hipStream_t st)
{
    const size_t lds = sizeof(typename CT<R>::V) * (1ull << M) + 16;
    {
        const hipError_t e = lds_optin((const void*)k_batch_whole<R, M, VAR>, lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_batch_whole<R, M, VAR>), dim3(count), dim3(256), lds, st, arena, circs, list, passes, ops, mats);
    return hipGetLastError();
}

template <typename R, int M, int VAR>
static hipError_t launch_persist_m(char* arena, const BatchCirc* circs, const int32_t* list, int count,
                                   const BatchPass* passes, const TileOp* ops, const double* mats, hipStream_t st)
{
    const size_t lds_max = tile_lds_bytes(sizeof(R) == 8 ? QS_C128 : QS_C64, M, 0);
    {
        const hipError_t e = lds_optin((const void*)k_batch_persist<R, M, VAR>, lds_max > 163840 ? 163840 : lds_max);
        if (e != hipSuccess) return e;
    }
    // LDS for the smallest L any pass may have
    const size_t lds = lds_max > 163840 ? 163840 : lds_max;
    hipLaunchKernelGGL((k_batch_persist<R, M, VAR>), dim3(count), dim3(256), lds, st, arena, circs, list, passes, ops,
                       mats);
    return hipGetLastError();
}

template <typename R, int VAR>
static hipError_t batch_whole_r(int M, char* arena, const BatchCirc* circs, const int32_t* list, int count,
                                const BatchPass* passes, const TileOp* ops, const double* mats, hipStream_t st)
{
    switch (M) {
#define QS_WCASE(MM) \
    case MM: return launch_whole_m<R, MM, (VAR >= 2 && MM < 8 ? 1 : VAR)>(arena, circs, list, count, passes, ops, mats, st);
        QS_WCASE(1) QS_WCASE(2) QS_WCASE(3) QS_WCASE(4) QS_WCASE(5) QS_WCASE(6) QS_WCASE(7) QS_WCASE(8)
        QS_WCASE(9) QS_WCASE(10) QS_WCASE(11) QS_WCASE(12) QS_WCASE(13)
#undef QS_WCASE
    default: return hipErrorInvalidValue;
    }
}

template <typename R, int VAR>
static hipError_t batch_persist_r(int M, char* arena, const BatchCirc* circs, const int32_t* list, int count,
                                  const BatchPass* passes, const TileOp* ops, const double* mats, hipStream_t st)
{
    switch (M) {
#define QS_PCASE(MM) \
    case MM: return launch_persist_m<R, MM, (VAR >= 2 && MM < 8 ? 1 : VAR)>(arena, circs, list, count, passes, ops, mats, st);
        QS_PCASE(9) QS_PCASE(10) QS_PCASE(11) QS_PCASE(12) QS_PCASE(13)
#undef QS_PCASE
    default: return hipErrorInvalidValue;
    }
}

} // namespace

hipError_t launch_batch_whole(int dt, int M, char* arena, const BatchCirc* circs, const int32_t* list, int count,
                              const BatchPass* passes, const TileOp* ops, const double* mats, int var,
                              hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    return dispatch_var(dt, var, [&](auto r, auto v) {
        return batch_whole_r<typename decltype(r)::type, decltype(v)::value>(M, arena, circs, list, count, passes, ops,
                                                                             mats, st);
    });
}

hipError_t launch_batch_persist(int dt, int M, char* arena, const BatchCirc* circs, const int32_t* list,
                                int count, const BatchPass* passes, const TileOp* ops, const double* mats, int var,
                                hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    return dispatch_var(dt, var, [&](auto r, auto v) {
        return batch_persist_r<typename decltype(r)::type, decltype(v)::value>(M, arena, circs, list, count, passes,
                                                                               ops, mats, st);
    });
}

template <typename R, int VAR>
static hipError_t batch_round_r(int M, char* arena, const BatchCirc* circs, const BatchPass* passes,
                                const TileOp* ops, const double* mats, const RoundEntry* entries, int nentries,
                                uint32_t nblocks, hipStream_t st)
{
    switch (M) {
#define QS_RCASE(MM) \
    case MM: return launch_round_m<R, MM, (VAR >= 2 && MM < 8 ? 1 : VAR)>(arena, circs, passes, ops, mats, entries, nentries, nblocks, st);
        QS_RCASE(9) QS_RCASE(10) QS_RCASE(11) QS_RCASE(12) QS_RCASE(13)
#undef QS_RCASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batch_round(int dt, int M, char* arena, const BatchCirc* circs, const BatchPass* passes,
                              const TileOp* ops, const double* mats, const RoundEntry* entries, int nentries,
                              uint32_t nblocks, int var, hipStream_t st)
{
    if (nentries <= 0 || nblocks == 0) return hipSuccess;
    return dispatch_var(dt, var, [&](auto r, auto v) {
        return batch_round_r<typename decltype(r)::type, decltype(v)::value>(M, arena, circs, passes, ops, mats,
                                                                             entries, nentries, nblocks, st);
    });
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

} // namespace qs
