// FP64 reductions: marginal probabilities over m qubits and the squared norm
// (m = 0).  Amplitudes of a complex64 state are widened to double on load.
//
// Order is fixed by construction, so a given (n, m, qubits) always sums the
// same numbers in the same order, whatever the grid size:
//   pass 1: the 2^(n-m) "rest" indices of each outcome o are cut into chunks of
//           CH consecutive rest indices; block (o, chunk) sums its chunk (each
//           lane a fixed strided subsequence, then a fixed LDS tree) into
//           part[o * nch + chunk];
//   pass 2: one block per outcome sums part[o * nch .. + nch) the same way.
#include "device_common.h"

namespace qs {

namespace {

constexpr int kRT = 256;        // threads per reduction block
constexpr int kChunkLog2 = 12;  // CH = 4096 rest indices per block

struct MeasQubits {
    int32_t m;
    int32_t q[24];
};

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
              InsertPlan ip, MeasQubits mq, double* __restrict__ part)
{
    __shared__ double sh[kRT];
    const uint64_t blk = blockIdx.x;
    const uint64_t o = blk / nch, chunk = blk % nch;
    uint64_t obits = 0;
    for (int j = 0; j < mq.m; ++j)
        if ((o >> j) & 1) obits |= 1ull << mq.q[j];
    double acc = 0.0;
    const uint64_t r0 = chunk * ch;
    for (uint64_t r = threadIdx.x; r < ch; r += kRT) {
        const uint64_t rr = r0 + r;
        if (rr < rest_per_outcome) {
            const V a = psi[ins_bits(rr, ip) | obits];
            const double x = (double)a.x, y = (double)a.y;
            acc += x * x + y * y;
        }
    }
    const double s = block_tree_sum(acc, sh);
    if (threadIdx.x == 0) part[blk] = s;
}

__global__ void __launch_bounds__(kRT)
k_prob_final(const double* __restrict__ part, uint64_t nch, double* __restrict__ out)
{
    __shared__ double sh[kRT];
    const uint64_t o = blockIdx.x;
    double acc = 0.0;
    for (uint64_t c = threadIdx.x; c < nch; c += kRT) acc += part[o * nch + c];
    const double s = block_tree_sum(acc, sh);
    if (threadIdx.x == 0) out[o] = s;
}

} // namespace

uint64_t reduce_scratch_doubles(int n, int m)
{
    const int rest = n - m;
    const int chl = rest < kChunkLog2 ? rest : kChunkLog2;
    const uint64_t nch = 1ull << (rest - chl);
    return (1ull << m) * nch;
}

hipError_t launch_probabilities(const void* psi, int dt, int n, const int* qubits, int m, double* part,
                                double* dev_out, hipStream_t st)
{
    if (m > 24) return hipErrorInvalidValue;
    MeasQubits mq;
    mq.m = m;
    uint64_t mask = 0;
    for (int j = 0; j < m; ++j) {
        mq.q[j] = qubits[j];
        mask |= 1ull << qubits[j];
    }
    InsertPlan ip = make_insert_plan(mask);
    const int rest = n - m;
    const int chl = rest < kChunkLog2 ? rest : kChunkLog2;
    const uint64_t ch = 1ull << chl;
    const uint64_t nch = 1ull << (rest - chl);
    const uint64_t nblk = (1ull << m) * nch;
    if (nblk > 0x7fffffffull) return hipErrorInvalidValue;
    if (dt == QS_C128)
        hipLaunchKernelGGL(k_prob_chunks<double2>, dim3((unsigned)nblk), dim3(kRT), 0, st, (const double2*)psi,
                           1ull << rest, ch, nch, ip, mq, part);
    else
        hipLaunchKernelGGL(k_prob_chunks<float2>, dim3((unsigned)nblk), dim3(kRT), 0, st, (const float2*)psi,
                           1ull << rest, ch, nch, ip, mq, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_prob_final, dim3(1u << m), dim3(kRT), 0, st, part, nch, dev_out);
    return hipGetLastError();
}

} // namespace qs
