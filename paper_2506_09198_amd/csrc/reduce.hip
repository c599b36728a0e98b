// FP64 reductions: marginal probabilities over m qubits and the squared norm
// (m = 0).  Amplitudes of a complex64 state are widened to double on load.
//
// Order is fixed by construction, so a given (n, m, qubits) always sums the
// same numbers in the same order, whatever the grid size:
//   pass 1: measured qubits at bit 6 or above select, per block, one pattern
//           oh of their bits; the remaining indices (measured low bits
//           included) are cut into chunks of CH = 4096 x 2^(low measured)
//           consecutive ones, which the block's lanes read contiguously (each
//           lane a fixed strided subsequence, so its amplitudes all share the
//           low six index bits: a lane belongs to one low-bit outcome).  A
//           fixed LDS tree folds the lanes of each low outcome, and the block
//           writes part[o * nch + chunk] for the 2^(low) outcomes o of oh.
//           Blocks are numbered chunk-major (the patterns oh of one chunk are
//           consecutive blocks);
//   pass 2: one block per outcome sums part[o * nch .. + nch) the same way;
//           with more than 4096 partials per outcome, blocks first sum
//           consecutive runs of 4096 of them (a level of 2^m x nch / 4096
//           partials after the first level), and one block per outcome sums
//           those.
#include <cstring>
#include <mutex>

#include "device_common.h"

namespace qs {

// Device scratch for callers that cannot allocate (qs_probabilities_noalloc):
// the per-chunk partial sums of one reduction go here instead of into a
// buffer the library allocates.  2^22 + 2^12 doubles (32 MiB + 32 KiB: the
// chunk partials and the second level of the final sum) cover every state
// the library takes (n <= 34) for m <= 22 measured qubits.  Each GPU holds its own
// copy until the process ends; calls that overlap on one GPU share it and race.
constexpr uint64_t kNoAllocScratchDoubles = (1ull << 22) + (1ull << 12);
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

constexpr int kRT = 256;        // threads per reduction block
constexpr int kChunkLog2 = 12;  // CH = 4096 rest indices per block
constexpr int kU = 8;           // loads a lane issues before summing them
constexpr int kSegLog2 = 12;    // partials one block of the final sum reads at most

// Measured qubits split by position: those at bit 6 or above ("high") are
// fixed per block (inserted into the counter), those below ("low") are lane
// bits -- every amplitude a lane reads has the same low bits, so the lanes
// read contiguous amplitudes and the block folds its lanes per low outcome.
struct MeasQubits {
    int32_t m, mh, nl;
    uint32_t lmask;  // lane bits of the low measured qubits
    int32_t hq[24];  // position of high measured qubit i
    int32_t hj[24];  // its bit in the outcome index
    int32_t lq[6];   // position (= lane bit) of low measured qubit i
    int32_t lj[6];   // its bit in the outcome index
};

// Logical block of workgroup bb.  Workgroups go to the 8 XCDs round-robin;
// with xcd set (grid a multiple of 8) XCD j takes the j-th contiguous eighth
// of the logical blocks, so each XCD streams its own part of the state.
// Which data a logical block reads and where its partials go do not change.
__device__ __forceinline__ uint64_t xcd_block(uint64_t bb, uint64_t grid, int xcd)
{
    return xcd ? (bb & 7) * (grid >> 3) + (bb >> 3) : bb;
}

// XCD-contiguous order for grids that are a multiple of 8, by default for
// streams over the whole state in index order (norm, sampling chunk sums,
// Pauli strings) that do not fit the 256 MB Infinity Cache.  Measured at 30
// qubits (complex128): 6.3 -> 6.5 TB/s for the norm, 6.1 -> 6.5 for Pauli
// strings, but 0.1-0.3 TB/s slower for marginals over measured qubits, whose
// consecutive blocks read different outcome patterns (block order there).
static int red_xcd(uint64_t grid, uint64_t state_bytes, bool stream)
{
    const int k = (int)tun(T_RED_XCD);
    const bool on = k == 2 || (k == 0 && stream && state_bytes >= (512ull << 20));
    return on && grid % 8 == 0 ? 1 : 0;
}

__device__ __forceinline__ double block_tree_sum(double v, double* sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = kRT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

template <typename V>
__global__ void __launch_bounds__(kRT)
k_prob_chunks(const V* __restrict__ psi, uint64_t rest_per_outcome, uint64_t ch, uint64_t nch,
              InsertPlan ip, MeasQubits mq, double* __restrict__ part, int xcd)
{
    __shared__ double sh[kRT];
    const uint32_t tid = threadIdx.x;
    const uint64_t noh = (uint64_t)1 << mq.mh;
    const uint64_t b = xcd_block(blockIdx.x, gridDim.x, xcd);
    const uint64_t oh = b % noh, chunk = b / noh;
    uint64_t obits = 0, ohout = 0; // high qubits: their index bits and outcome bits
    for (int i = 0; i < mq.mh; ++i)
        if ((oh >> i) & 1) {
            obits |= 1ull << mq.hq[i];
            ohout |= 1ull << mq.hj[i];
        }
    // kU loads in flight per lane before they are summed, in the same order
    // (r = tid, tid + kRT, ...) as one at a time; missing elements add +0
    double acc = 0.0;
    const uint64_t r0 = chunk * ch;
    for (uint64_t r = tid; r < ch; r += (uint64_t)kRT * kU) {
        V a[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const uint64_t ru = r + (uint64_t)u * kRT;
            if (ru < ch && r0 + ru < rest_per_outcome) {
                a[u] = psi[ins_bits(r0 + ru, ip) | obits];
            } else {
                a[u].x = 0;
                a[u].y = 0;
            }
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const double x = (double)a[u].x, y = (double)a[u].y;
            acc += x * x + y * y;
        }
    }
    // Fold the other thread bits, highest first, so thread t with those bits
    // zero holds the sum over the threads sharing its low-qubit lane bits.
    sh[tid] = acc;
    uint32_t done = 0;
    for (int b = 7; b >= 0; --b) {
        if ((mq.lmask >> b) & 1) continue;
        __syncthreads();
        if (!(tid & (done | (1u << b)))) sh[tid] += sh[tid | (1u << b)];
        done |= 1u << b;
    }
    __syncthreads();
    if (!(tid & done)) {
        uint64_t o = ohout;
        for (int i = 0; i < mq.nl; ++i)
            if ((tid >> mq.lq[i]) & 1) o |= 1ull << mq.lj[i];
        part[o * nch + chunk] = sh[tid];
    }
}

// Block o sums part[o * nch .. + nch): lane t the partials t, t + kRT, ...
// in order (kU loads in flight), then a fixed tree over the lanes.
__global__ void __launch_bounds__(kRT)
k_prob_final(const double* __restrict__ part, uint64_t nch, double* __restrict__ out)
{
    __shared__ double sh[kRT];
    const uint64_t o = blockIdx.x;
    double acc = 0.0;
    for (uint64_t c = threadIdx.x; c < nch; c += (uint64_t)kRT * kU) {
        double v[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const uint64_t cu = c + (uint64_t)u * kRT;
            v[u] = cu < nch ? part[o * nch + cu] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) acc += v[u];
    }
    const double s = block_tree_sum(acc, sh);
    if (threadIdx.x == 0) out[o] = s;
}

// The final sum of `groups` runs of nch partials each (part[g * nch ..]) into
// out[g]: one block per run, or, for runs longer than 2^kSegLog2, one block
// per 2^kSegLog2-partial segment into lvl (groups x nch / 2^kSegLog2
// doubles), then one block per run over its segments.
hipError_t final_sums(const double* part, uint64_t groups, uint64_t nch, double* lvl, double* out, hipStream_t st)
{
    const uint64_t seg = 1ull << kSegLog2;
    if (nch <= seg) {
        hipLaunchKernelGGL(k_prob_final, dim3((unsigned)groups), dim3(kRT), 0, st, part, nch, out);
        return hipGetLastError();
    }
    const uint64_t per = nch / seg; // nch is a power of two
    hipLaunchKernelGGL(k_prob_final, dim3((unsigned)(groups * per)), dim3(kRT), 0, st, part, seg, lvl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_prob_final, dim3((unsigned)groups), dim3(kRT), 0, st, (const double*)lvl, per, out);
    return hipGetLastError();
}

// Doubles of the second level for `groups` runs of nch partials.
uint64_t level_doubles(uint64_t groups, uint64_t nch)
{
    return nch > (1ull << kSegLog2) ? groups * (nch >> kSegLog2) : 0;
}

// Pauli-string expectation, pass 1.  Terms (x != 0): pairs (k0, k1 = k0 ^ x)
// with bit b = highest bit of x clear in k0, term = conj(psi_k1) psi_k0 s(k0)
// + conj(psi_k0) psi_k1 s(k1), s(k) = (-1)^{|k & z|}; (x == 0): |psi_k|^2 s(k).
// Chunks of CH consecutive terms per block, fixed lane order and tree;
// part[chunk] = real sum, part[nch + chunk] = imaginary sum.
template <typename V>
__global__ void __launch_bounds__(kRT)
k_pauli_chunks(const V* __restrict__ psi, uint64_t nterms, uint64_t ch, uint64_t nch, uint64_t x, uint64_t z,
               int b, double* __restrict__ part, int xcd)
{
    __shared__ double sh[kRT];
    const uint64_t chunk = xcd_block(blockIdx.x, gridDim.x, xcd);
    const uint64_t lowm = (1ull << b) - 1;
    // kU terms' loads in flight per lane, summed in the order r = tid,
    // tid + kRT, ... as one at a time (missing terms add zeros)
    double ar = 0.0, ai = 0.0;
    for (uint64_t r = threadIdx.x; r < ch; r += (uint64_t)kRT * kU) {
        if (x == 0) {
            V a[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const uint64_t t = chunk * ch + r + (uint64_t)u * kRT;
                if (r + (uint64_t)u * kRT < ch && t < nterms) {
                    a[u] = psi[t];
                } else {
                    a[u].x = 0;
                    a[u].y = 0;
                }
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const uint64_t t = chunk * ch + r + (uint64_t)u * kRT;
                const double p = (double)a[u].x * (double)a[u].x + (double)a[u].y * (double)a[u].y;
                ar += (__popcll(t & z) & 1) ? -p : p;
            }
        } else {
            V a0[kU], a1[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const uint64_t t = chunk * ch + r + (uint64_t)u * kRT;
                if (r + (uint64_t)u * kRT < ch && t < nterms) {
                    const uint64_t k0 = ((t >> b) << (b + 1)) | (t & lowm);
                    a0[u] = psi[k0];
                    a1[u] = psi[k0 ^ x];
                } else {
                    a0[u].x = 0;
                    a0[u].y = 0;
                    a1[u] = a0[u];
                }
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const uint64_t t = chunk * ch + r + (uint64_t)u * kRT;
                const uint64_t k0 = ((t >> b) << (b + 1)) | (t & lowm), k1 = k0 ^ x;
                const double x0 = a0[u].x, y0 = a0[u].y, x1 = a1[u].x, y1 = a1[u].y;
                // conj(a1) a0 and conj(a0) a1 = conj of the first
                const double pr = x1 * x0 + y1 * y0, pi = x1 * y0 - y1 * x0;
                const double s0 = (__popcll(k0 & z) & 1) ? -1.0 : 1.0, s1 = (__popcll(k1 & z) & 1) ? -1.0 : 1.0;
                ar += s0 * pr + s1 * pr;
                ai += s0 * pi - s1 * pi;
            }
        }
    }
    const double sr = block_tree_sum(ar, sh);
    const double si = block_tree_sum(ai, sh);
    if (threadIdx.x == 0) {
        part[chunk] = sr;
        part[nch + chunk] = si;
    }
}

// Sampling, within a chunk: one wave per shot.  Lane l holds the (up to) 64
// consecutive amplitudes [64 l, 64 l + 64) of the shot's chunk of csize
// (4096, or the whole state when it is smaller); lane
// sums, an ordered prefix over the lanes, then the chosen lane walks its 64
// probabilities in order to the first cumulative sum above the residual.  If
// rounding leaves the residual at or above the chunk's total, the last index
// with nonzero probability is taken.
template <typename V>
__global__ void __launch_bounds__(kRT)
k_sample_chunk(const V* __restrict__ psi, uint32_t csize, const SampleReq* __restrict__ req, int64_t shots,
               uint64_t* __restrict__ out)
{
    const int lane = threadIdx.x & 63;
    const int64_t shot = (int64_t)blockIdx.x * (kRT / 64) + (threadIdx.x >> 6);
    if (shot >= shots) return;
    const SampleReq q = req[shot];
    const uint32_t first = 64u * (uint32_t)lane;              // this lane's run inside the chunk
    const int len = first >= csize ? 0 : (csize - first < 64u ? (int)(csize - first) : 64);
    const uint64_t base = q.chunk * csize + first;
    double ls = 0.0;
    int lastnz = -1;
    for (int j = 0; j < len; ++j) {
        const V a = psi[base + j];
        const double p = (double)a.x * (double)a.x + (double)a.y * (double)a.y;
        ls += p;
        if (p > 0.0) lastnz = j;
    }
    // ordered exclusive prefix of the lane sums (lane 0 first)
    double excl = 0.0, incl = 0.0;
    for (int l = 0; l < 64; ++l) {
        const double v = __shfl(ls, l);
        if (l < lane) excl += v;
    }
    incl = excl + ls;
    const unsigned long long hit = __ballot(incl > q.residual);
    int pick = hit ? __ffsll(hit) - 1 : -1;
    if (pick < 0) { // residual not reached: last nonzero probability of the chunk
        const unsigned long long nz = __ballot(lastnz >= 0);
        const int l = nz ? 63 - __clzll(nz) : 0;
        const int j = __shfl(lastnz, l);
        if (lane == 0) out[shot] = q.chunk * csize + 64 * (uint64_t)l + (uint64_t)(j < 0 ? 0 : j);
        return;
    }
    if (lane == pick) {
        double c = excl;
        uint64_t idx = base + (len > 0 ? len - 1 : 0);
        for (int j = 0; j < len; ++j) {
            const V a = psi[base + j];
            c += (double)a.x * (double)a.x + (double)a.y * (double)a.y;
            if (c > q.residual) {
                idx = base + j;
                break;
            }
        }
        out[shot] = idx;
    }
}

} // namespace

hipError_t launch_pauli_expect(const void* psi, int dt, int n, uint64_t x, uint64_t z, double* part,
                               double* dev_out, hipStream_t st)
{
    // pairs (k0, k0 ^ x) with the highest bit of x clear in k0: k0 runs over
    // whole lines and k0 ^ x permutes within lines, so both reads coalesce
    const uint64_t nterms = x == 0 ? (1ull << n) : (1ull << (n - 1));
    const int b = x == 0 ? 0 : 63 - __builtin_clzll(x);
    const uint64_t ch = 1ull << kChunkLog2;
    const uint64_t nch = (nterms + ch - 1) / ch;
    if (nch > 0x7fffffffull) return hipErrorInvalidValue;
    const int xo = red_xcd(nch, (uint64_t)amp_bytes(dt) << n, true);
    if (dt == QS_C128)
        hipLaunchKernelGGL(k_pauli_chunks<double2>, dim3((unsigned)nch), dim3(kRT), 0, st, (const double2*)psi,
                           nterms, ch, nch, x, z, b, part, xo);
    else
        hipLaunchKernelGGL(k_pauli_chunks<float2>, dim3((unsigned)nch), dim3(kRT), 0, st, (const float2*)psi,
                           nterms, ch, nch, x, z, b, part, xo);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // real sums part[0, nch), imaginary part[nch, 2 nch); second level after them
    return final_sums(part, 2, nch, part + 2 * nch, dev_out, st);
}

uint64_t pauli_scratch_doubles(int n)
{
    const uint64_t nch = ((1ull << n) + 4095) / 4096; // the most any Pauli string needs
    return 2 * nch + level_doubles(2, nch) + 2;
}

hipError_t launch_sample_chunks(const void* psi, int dt, int n, const SampleReq* req, int64_t shots, uint64_t* out,
                                hipStream_t st)
{
    if (shots <= 0) return hipSuccess;
    const uint32_t csize = 1u << (n < kChunkLog2 ? n : kChunkLog2);
    const int64_t g = (shots + kRT / 64 - 1) / (kRT / 64);
    if (g > 0x7fffffffll) return hipErrorInvalidValue;
    if (dt == QS_C128)
        hipLaunchKernelGGL(k_sample_chunk<double2>, dim3((unsigned)g), dim3(kRT), 0, st, (const double2*)psi, csize,
                           req, shots, out);
    else
        hipLaunchKernelGGL(k_sample_chunk<float2>, dim3((unsigned)g), dim3(kRT), 0, st, (const float2*)psi, csize,
                           req, shots, out);
    return hipGetLastError();
}

hipError_t noalloc_scratch(int dev, double** ptr, uint64_t* doubles)
{
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        // The array's name is a host-side handle; its address on this
        // device comes from the runtime (the caller made `dev` current).
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_dev[dev] = p;
    }
    *ptr = (double*)g_scratch_dev[dev];
    *doubles = kNoAllocScratchDoubles;
    return hipSuccess;
}

// Chunks per outcome of launch_probabilities (its pass-1 partials are 2^m x
// this many, chunk-major within each outcome).
static uint64_t chunks_per_outcome(int n, int m)
{
    const int rest = n - m;
    const int chl = rest < kChunkLog2 ? rest : kChunkLog2;
    return 1ull << (rest - chl);
}

uint64_t reduce_partials(int n, int m) { return (1ull << m) * chunks_per_outcome(n, m); }

uint64_t reduce_scratch_doubles(int n, int m)
{
    return reduce_partials(n, m) + level_doubles(1ull << m, chunks_per_outcome(n, m));
}

hipError_t launch_probabilities(const void* psi, int dt, int n, const int* qubits, int m, double* part,
                                double* dev_out, hipStream_t st)
{
    if (m > 24) return hipErrorInvalidValue;
    MeasQubits mq;
    std::memset(&mq, 0, sizeof mq);
    mq.m = m;
    uint64_t mask = 0; // high measured qubits, inserted into the counter
    for (int j = 0; j < m; ++j) {
        if (qubits[j] >= 6) {
            mq.hq[mq.mh] = qubits[j];
            mq.hj[mq.mh++] = j;
            mask |= 1ull << qubits[j];
        } else {
            mq.lq[mq.nl] = qubits[j];
            mq.lj[mq.nl++] = j;
            mq.lmask |= 1u << qubits[j];
        }
    }
    InsertPlan ip = make_insert_plan(mask);
    // a block reads 4096 x 2^nl rest indices (or all of them) and writes one
    // partial per low outcome: 2^m x nch partials, as reduce_scratch_doubles
    const int rest = n - mq.mh;
    const int chl = rest < kChunkLog2 + mq.nl ? rest : kChunkLog2 + mq.nl;
    const uint64_t ch = 1ull << chl;
    const uint64_t nch = 1ull << (rest - chl);
    const uint64_t nblk = (1ull << mq.mh) * nch;
    if (nblk > 0x7fffffffull) return hipErrorInvalidValue;
    const int xo = red_xcd(nblk, (uint64_t)amp_bytes(dt) << n, m == 0);
    if (dt == QS_C128)
        hipLaunchKernelGGL(k_prob_chunks<double2>, dim3((unsigned)nblk), dim3(kRT), 0, st, (const double2*)psi,
                           1ull << rest, ch, nch, ip, mq, part, xo);
    else
        hipLaunchKernelGGL(k_prob_chunks<float2>, dim3((unsigned)nblk), dim3(kRT), 0, st, (const float2*)psi,
                           1ull << rest, ch, nch, ip, mq, part, xo);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // second level after the 2^m x nch partials, as reduce_scratch_doubles
    return final_sums(part, 1ull << m, nch, part + (1ull << m) * nch, dev_out, st);
}

} // namespace qs
