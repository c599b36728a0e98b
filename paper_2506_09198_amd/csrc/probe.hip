// Memory ceiling probe: in-place read-modify-write of a device buffer.
//
// Every gate pass reads each amplitude it changes and writes it back in place,
// so the fastest such pass over plain contiguous data is the ceiling the gate
// kernels are measured against (beside the published HBM peak).  The probe
// uses the per-gate kernel's schedule family: 16-byte words, one chunk of
// 256 x SLOTS words per workgroup, a lane's slots 2^spread_log2 words apart,
// non-temporal loads and stores.  Each word is XORed with a run-time mask (0
// leaves the buffer bitwise unchanged, whatever it holds).
#include "device_common.h"

namespace qs {

namespace {

typedef unsigned long long u2v_t __attribute__((ext_vector_type(2)));

template <int SLOTS>
__global__ void __launch_bounds__(256)
k_probe_rmw(ulonglong2* __restrict__ p, uint64_t n16, uint64_t nblocks, int slog, int xcd, uint64_t mask)
{
    const uint64_t S = 1ull << slog;
    const uint64_t spb = S >> 8;
    for (uint64_t bb = blockIdx.x; bb < nblocks; bb += gridDim.x) {
        // xcd: chunk (bb mod 8) * nblocks/8 + bb/8 (as the per-gate kernel)
        const uint64_t b = xcd ? (bb & 7) * (nblocks >> 3) + (bb >> 3) : bb;
        const uint64_t base = (b / spb) * (S * SLOTS) + (b % spb) * 256 + threadIdx.x;
        u2v_t x[SLOTS];
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            const uint64_t i = base + (uint64_t)s * S;
            if (i < n16) x[s] = __builtin_nontemporal_load((const u2v_t*)(p + i));
        }
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            const uint64_t i = base + (uint64_t)s * S;
            if (i < n16) {
                u2v_t y = x[s];
                y.x ^= mask;
                y.y ^= mask;
                __builtin_nontemporal_store(y, (u2v_t*)(p + i));
            }
        }
    }
}

template <int SLOTS>
hipError_t launch_probe_k(void* dev, uint64_t n16, int slog, uint64_t mask, hipStream_t st)
{
    const uint64_t nblocks = (n16 + 256 * SLOTS - 1) / (256 * SLOTS);
    const uint64_t cap = (uint64_t)tun(T_GATE_GRID_CAP);
    const unsigned g = (unsigned)(nblocks < cap ? nblocks : cap);
    // the per-gate kernel's occupancy knob applies (unused LDS: fewer workgroups per CU)
    const size_t pad = pad_for_wg_per_cu((int)tun(T_GATE_WG_PER_CU), 0);
    hipError_t e = lds_optin((const void*)k_probe_rmw<SLOTS>, pad);
    if (e != hipSuccess) return e;
    const int xcd = (tun(T_GATE_XCD) == 2 && nblocks % 8 == 0) ? 1 : 0;
    hipLaunchKernelGGL(k_probe_rmw<SLOTS>, dim3(g), dim3(256), pad, st, (ulonglong2*)dev, n16, nblocks, slog, xcd,
                       mask);
    return hipGetLastError();
}

} // namespace

hipError_t launch_probe_inplace(void* dev, uint64_t bytes, int slots, int slog, uint64_t mask, hipStream_t st)
{
    const uint64_t n16 = bytes / 16;
    switch (slots) {
    case 1: return launch_probe_k<1>(dev, n16, slog, mask, st);
    case 2: return launch_probe_k<2>(dev, n16, slog, mask, st);
    case 4: return launch_probe_k<4>(dev, n16, slog, mask, st);
    case 8: return launch_probe_k<8>(dev, n16, slog, mask, st);
    default: return hipErrorInvalidValue;
    }
}

} // namespace qs
