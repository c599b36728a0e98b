// In-place permutation of qubit positions by an involution.
//
// When the planner turns SWAP gates into a relabeling of qubits (the
// swap-shifted form of the blocked QFT, Section III-B), the state ends with
// its qubits at permuted bit positions.  Any permutation of bit positions is
// the product of two involutions, and an involution tau (disjoint pairs of
// positions) induces an involution on amplitude indices: sigma(y) exchanges
// the bits of y at each pair.  One pass per involution restores the order.
//
// Pairing a low bit with a high one (QFT pairs bit 0 with bit n-1) would
// scatter a wave's partner accesses over the whole state, so the pass works
// on tiles.  T = {0..K-1} together with the partners of those bits is closed
// under tau; a tile holds the 2^|T| amplitudes that share their bits outside
// T.  The pairs outside T map tile t to tile t' = sigma_out(t), the pairs
// inside permute within a tile: new[t', sigma_in(u)] = old[t, u].  A
// workgroup loads tiles t and t' (runs of 2^K consecutive amplitudes) into
// LDS and writes each back permuted into the other, so every access is
// coalesced and each amplitude is read and written once.
#include <algorithm>
#include <cstring>

#include "device_common.h"

namespace qs {

namespace {

constexpr int kMaxRun = 6;            // K <= 6: runs of up to 64 consecutive amplitudes
constexpr int kMaxT = 2 * kMaxRun;    // |T| <= 2K
constexpr int kMaxPairs = 32;

struct InvArgs {
    uint64_t ntiles;                  // 2^(n - |T|)
    int32_t nt;                       // |T|
    int32_t tpos[kMaxT];              // positions of T, ascending (the first K are 0..K-1)
    int32_t sin_[kMaxT];              // compact bit j of a tile index -> compact bit sin_[j]
    int32_t np;                       // pairs outside T
    int32_t pa[kMaxPairs], pb[kMaxPairs];
    InsertPlan ip;                    // the positions of T, inserted into the tile counter
};

template <typename V, int K>
__global__ void __launch_bounds__(256) k_bit_involution(V* __restrict__ psi, InvArgs a)
{
    __shared__ V la[1 << (2 * K)], lb[1 << (2 * K)];
    constexpr int PT = ((1 << (2 * K)) + 255) / 256; // elements per thread at most (|T| <= 2K)
    const int E = 1 << a.nt;
    auto deposit = [&](int u) {
        uint64_t off = (uint64_t)(u & ((1 << K) - 1)) & (((uint64_t)1 << a.nt) - 1);
        for (int j = K; j < a.nt; ++j) off |= (uint64_t)((u >> j) & 1) << a.tpos[j];
        return off;
    };
    auto sigma_in = [&](int u) {
        int v = 0;
        for (int j = 0; j < a.nt; ++j) v |= ((u >> j) & 1) << a.sin_[j];
        return v;
    };
    for (uint64_t b = blockIdx.x; b < a.ntiles; b += gridDim.x) {
        const uint64_t t = ins_bits(b, a.ip);
        uint64_t t2 = t;
        for (int i = 0; i < a.np; ++i)
            if (((t >> a.pa[i]) ^ (t >> a.pb[i])) & 1) t2 ^= (1ull << a.pa[i]) | (1ull << a.pb[i]);
        if (t2 < t) continue; // the block of tile t2 does this pair (same decision for the whole block)
        // every load of the pair is issued before the first LDS store, so a
        // thread keeps all its reads in flight at once; each amplitude is
        // read and written once, so loads and stores bypass the caches
        V ra[PT], rb[PT];
#pragma unroll
        for (int i = 0; i < PT; ++i) {
            const int u = threadIdx.x + 256 * i;
            if (u < E) {
                const uint64_t off = deposit(u);
                ra[i] = gld<true>(psi + (t | off));
                if (t2 != t) rb[i] = gld<true>(psi + (t2 | off));
            }
        }
#pragma unroll
        for (int i = 0; i < PT; ++i) {
            const int u = threadIdx.x + 256 * i;
            if (u < E) {
                la[u] = ra[i];
                if (t2 != t) lb[u] = rb[i];
            }
        }
        __syncthreads();
        for (int u = threadIdx.x; u < E; u += 256) {
            const uint64_t off = deposit(u);
            const int su = sigma_in(u);
            gst<true>(psi + (t2 | off), la[su]);
            if (t2 != t) gst<true>(psi + (t | off), lb[su]);
        }
        __syncthreads();
    }
}

template <typename V, int K>
hipError_t launch_inv(V* psi, const InvArgs& a, unsigned g, int wg, hipStream_t st)
{
    const size_t pad = pad_for_wg_per_cu(wg, 2 * sizeof(V) << (2 * K)); // the two tiles in LDS
    hipError_t e = lds_optin((const void*)k_bit_involution<V, K>, pad);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_bit_involution<V, K>), dim3(g), dim3(256), pad, st, psi, a);
    return hipGetLastError();
}

} // namespace

uint64_t involution_moved(int n, const int* tau)
{
    int np = 0;
    for (int p = 0; p < n; ++p)
        if (tau[p] > p) ++np;
    return (1ull << n) - (1ull << (n - np)); // indices whose bits differ at some pair
}

hipError_t launch_bit_involution(void* psi, int dt, int n, const int* tau, hipStream_t st)
{
    for (int p = 0; p < n; ++p)
        if (tau[p] < 0 || tau[p] >= n || tau[tau[p]] != p) return hipErrorInvalidValue;
    bool id = true;
    for (int p = 0; p < n; ++p) id &= tau[p] == p;
    if (id) return hipSuccess;
    InvArgs a;
    std::memset(&a, 0, sizeof a);
    // Runs of 2^Kr amplitudes; both tiles of a pair sit in LDS.  Measured at
    // 30 qubits (QFT restore), with the batched non-temporal loads and stores:
    // Kr = 5 for both types -- complex64 3.2 TB/s (256-byte runs; Kr = 6 needs
    // 64 KiB of LDS per block and drops to 1.7), complex128 4.0 TB/s (512-byte
    // runs; 3.4 at Kr = 4; with cached accesses Kr = 5 fell to 1.9).  Issuing
    // the stores in one burst as well (LDS reads first) lost 10 %.
    const int kenv = (int)tun(T_PERM_RUN);
    const int Kr = (kenv >= 4 && kenv <= (dt == QS_C128 ? 5 : 6)) ? kenv : 5;
    const int K = n < Kr ? n : Kr;
    uint64_t T = 0;
    for (int p = 0; p < K; ++p) T |= (1ull << p) | (1ull << tau[p]);
    int pos_to_j[64];
    for (int p = 0; p < n; ++p)
        if ((T >> p) & 1) {
            pos_to_j[p] = a.nt;
            a.tpos[a.nt++] = p;
        }
    for (int j = 0; j < a.nt; ++j) a.sin_[j] = pos_to_j[tau[a.tpos[j]]];
    for (int p = 0; p < n; ++p)
        if (!((T >> p) & 1) && tau[p] > p) {
            a.pa[a.np] = p;
            a.pb[a.np] = tau[p];
            a.np++;
        }
    a.ip = make_insert_plan(T);
    a.ntiles = 1ull << (n - a.nt);
    // up to 2^20 workgroups (fewer with a lower gate_grid_cap); they loop over the tile pairs
    const uint64_t cap = std::min<uint64_t>(1ull << 20, (uint64_t)tun(T_GATE_GRID_CAP));
    const unsigned g = (unsigned)(a.ntiles < cap ? a.ntiles : cap);
    // workgroups per CU: the per-gate kernel's occupancy knob applies (0 = no cap)
    const int wg = (int)tun(T_GATE_WG_PER_CU);
    if (dt == QS_C128)
        return Kr == 4 ? launch_inv<double2, 4>((double2*)psi, a, g, wg, st)
                       : launch_inv<double2, 5>((double2*)psi, a, g, wg, st);
    if (Kr == 4) return launch_inv<float2, 4>((float2*)psi, a, g, wg, st);
    if (Kr == 5) return launch_inv<float2, 5>((float2*)psi, a, g, wg, st);
    return launch_inv<float2, 6>((float2*)psi, a, g, wg, st);
}

} // namespace qs
