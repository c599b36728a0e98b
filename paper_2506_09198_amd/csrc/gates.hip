// Per-gate kernels for gfx950 (wave64).
//
//   k_init_basis   zero the state and set one amplitude to 1.
//   k_1q_pairs     1q gate, pair walk over a compact counter with the target
//                  and control bits inserted (the pair update of Alg. 1 for a
//                  general 2x2 matrix; controls as fixed inserted bits, so no
//                  branch skips work as in Fig. control6q2).  Consecutive lanes
//                  take consecutive pairs, so for targets >= 7 (c128) / 8 (c64)
//                  every load and store instruction covers whole 128-byte lines.
//   k_1q_wave      1q gate on a low target: each wave loads one contiguous
//                  chunk (64 lanes x A amplitudes); the partner amplitude is in
//                  the lane's own registers (t < log2 A) or in lane
//                  (lane ^ 2^(t - log2 A)) of the same wave, fetched with a
//                  cross-lane shuffle.  All HBM traffic stays fully coalesced.
//   k_2q_quads     2q gate on any (t0, t1): 4x4 complex matvec per quad.
//   k_kq_lds       dense gate on k <= 6 targets: groups of 2^k amplitudes are
//                  staged through LDS with the matrix, one output per lane.
#include "device_common.h"

namespace qs {

struct M2 { double m[8]; };
struct M4 { double m[32]; };

InsertPlan make_insert_plan(uint64_t mask)
{
    InsertPlan p;
    p.n = 0;
    for (int b = 0; b < 64 && p.n < kMaxIns; ++b)
        if ((mask >> b) & 1) p.low[p.n++] = (b == 63) ? ~0ull >> 1 : ((1ull << b) - 1);
    return p;
}

static int grid_cap()
{
    static int cap = env_int("QS_GRID_CAP", 256 * 64);
    return cap;
}

static unsigned blocks_for(uint64_t items, uint64_t per_block)
{
    uint64_t b = (items + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > (uint64_t)grid_cap()) b = grid_cap();
    return (unsigned)b;
}

// ---------------------------------------------------------------- K0 init

template <typename V>
__global__ void __launch_bounds__(256) k_init_basis(V* __restrict__ psi, uint64_t namps, uint64_t x)
{
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < namps; i += stride) {
        V v;
        v.x = (i == x) ? 1 : 0;
        v.y = 0;
        psi[i] = v;
    }
}

hipError_t launch_init_basis(void* psi, int dt, int n, uint64_t x, hipStream_t st)
{
    const uint64_t N = 1ull << n;
    const unsigned g = blocks_for(N, 256 * 4);
    if (dt == QS_C128)
        hipLaunchKernelGGL(k_init_basis<double2>, dim3(g), dim3(256), 0, st, (double2*)psi, N, x);
    else
        hipLaunchKernelGGL(k_init_basis<float2>, dim3(g), dim3(256), 0, st, (float2*)psi, N, x);
    return hipGetLastError();
}

// ---------------------------------------------------------------- K1 pairs

template <typename R, int PPL>
__global__ void __launch_bounds__(256)
k_1q_pairs(typename CT<R>::V* __restrict__ psi, uint64_t npairs, uint64_t half, uint64_t cvals,
           InsertPlan ip, M2 u)
{
    using V = typename CT<R>::V;
    const uint64_t stride = (uint64_t)gridDim.x * (256 * PPL);
    for (uint64_t k0 = (uint64_t)blockIdx.x * (256 * PPL) + threadIdx.x; k0 < npairs; k0 += stride) {
        V a[PPL], b[PPL];
        uint64_t ia[PPL];
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            const uint64_t k = k0 + (uint64_t)p * 256;
            ia[p] = ins_bits(k, ip) | cvals;
            if (k < npairs) {
                a[p] = psi[ia[p]];
                b[p] = psi[ia[p] + half];
            }
        }
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            const uint64_t k = k0 + (uint64_t)p * 256;
            if (k < npairs) {
                const double2 x = ld2(a[p]), y = ld2(b[p]);
                psi[ia[p]] = st2<V>(cmad2<double2, double>(u.m[0], u.m[1], x, u.m[2], u.m[3], y));
                psi[ia[p] + half] = st2<V>(cmad2<double2, double>(u.m[4], u.m[5], x, u.m[6], u.m[7], y));
            }
        }
    }
}

// ---------------------------------------------------------------- K2 wave

template <typename V>
__device__ __forceinline__ V shfl_xor_v(V v, int d)
{
    V r;
    r.x = __shfl_xor(v.x, d, 64);
    r.y = __shfl_xor(v.y, d, 64);
    return r;
}

template <int A, int D>
__device__ __forceinline__ void inlane_pairs(const double2 (&x)[A], double2 (&y)[A], const M2& u)
{
#pragma unroll
    for (int j = 0; j < A; ++j) {
        if (j & D) continue;
        if (j + D >= A) continue;
        const double2 a = x[j], b = x[j + D];
        y[j] = cmad2<double2, double>(u.m[0], u.m[1], a, u.m[2], u.m[3], b);
        y[j + D] = cmad2<double2, double>(u.m[4], u.m[5], a, u.m[6], u.m[7], b);
    }
}

// A amplitudes per lane (LA = log2 A); a wave covers W = 6 + LA index bits.
template <typename R, int LA>
__global__ void __launch_bounds__(256)
k_1q_wave(typename CT<R>::V* __restrict__ psi, uint64_t nchunks, uint64_t namps, int t,
          uint64_t cm_lo, uint64_t cv_lo, uint64_t cv_hi, InsertPlan ip_hi, M2 u)
{
    using V = typename CT<R>::V;
    constexpr int A = 1 << LA;
    constexpr int W = 6 + LA;
    const int lane = threadIdx.x & 63;
    const uint64_t nw = (uint64_t)gridDim.x * 4;
    for (uint64_t c = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6); c < nchunks; c += nw) {
        const uint64_t i0 = ((ins_bits(c, ip_hi) << W) | cv_hi) + (uint64_t)lane * A;
        double2 x[A], y[A];
#pragma unroll
        for (int j = 0; j < A; ++j) {
            if (i0 + j < namps) {
                x[j] = ld2(psi[i0 + j]);
            } else {
                x[j].x = 0;
                x[j].y = 0;
            }
        }
        if (t < LA) {
            // partner in the lane's own registers; t is 0 or 1, unrolled
            // separately so every register index is a constant
            if (t == 0)
                inlane_pairs<A, 1>(x, y, u);
            else
                inlane_pairs<A, 2>(x, y, u);
        } else {
            const int d = 1 << (t - LA);
            const bool upper = (lane & d) == 0;
            // upper lane (bit clear): u00*x + u01*partner; lower: u10*partner + u11*x
            const double ar = upper ? u.m[0] : u.m[6], ai = upper ? u.m[1] : u.m[7];
            const double br = upper ? u.m[2] : u.m[4], bi = upper ? u.m[3] : u.m[5];
#pragma unroll
            for (int j = 0; j < A; ++j) {
                const double2 p = shfl_xor_v(x[j], d);
                y[j] = cmad2<double2, double>(ar, ai, x[j], br, bi, p);
            }
        }
#pragma unroll
        for (int j = 0; j < A; ++j) {
            const uint64_t i = i0 + j;
            if (i < namps && ((i & cm_lo) == cv_lo)) psi[i] = st2<V>(y[j]);
        }
    }
}

template <typename R>
static hipError_t apply_1q_t(void* psiv, int n, int t, const double* U, uint64_t cm, uint64_t cv,
                             hipStream_t st, int* kind)
{
    using V = typename CT<R>::V;
    V* psi = (V*)psiv;
    M2 u;
    for (int i = 0; i < 8; ++i) u.m[i] = U[i];
    constexpr int LA = sizeof(R) == 8 ? 1 : 2; // 32 bytes of amplitudes per lane
    constexpr int W = 6 + LA;
    if (t < W) {
        const uint64_t lo_mask = (W >= 64) ? ~0ull : ((1ull << W) - 1);
        const uint64_t cm_lo = cm & lo_mask, cv_lo = cv & lo_mask;
        const uint64_t cm_hi = cm & ~lo_mask, cv_hi = cv & ~lo_mask;
        const int nhi = __builtin_popcountll(cm_hi);
        const uint64_t nchunks = (n > W) ? (1ull << (n - W - nhi)) : 1;
        InsertPlan ip = make_insert_plan(cm_hi >> W);
        const unsigned g = blocks_for(nchunks, 4);
        hipLaunchKernelGGL((k_1q_wave<R, LA>), dim3(g), dim3(256), 0, st, psi, nchunks, 1ull << n, t,
                           cm_lo, cv_lo, cv_hi, ip, u);
        if (kind) *kind = QS_K_1Q_LO;
    } else {
        const int nc = __builtin_popcountll(cm);
        const uint64_t npairs = 1ull << (n - 1 - nc);
        InsertPlan ip = make_insert_plan(cm | (1ull << t));
        constexpr int PPL = 2;
        const unsigned g = blocks_for(npairs, 256 * PPL);
        hipLaunchKernelGGL((k_1q_pairs<R, PPL>), dim3(g), dim3(256), 0, st, psi, npairs, 1ull << t, cv, ip,
                           u);
        if (kind) *kind = QS_K_1Q_HI;
    }
    return hipGetLastError();
}

hipError_t launch_apply_1q(void* psi, int dt, int n, int t, const double* U, uint64_t cm, uint64_t cv,
                           hipStream_t st, int* kind)
{
    return dt == QS_C128 ? apply_1q_t<double>(psi, n, t, U, cm, cv, st, kind)
                         : apply_1q_t<float>(psi, n, t, U, cm, cv, st, kind);
}

// ---------------------------------------------------------------- K3 quads

template <typename R, int PPL>
__global__ void __launch_bounds__(256)
k_2q_quads(typename CT<R>::V* __restrict__ psi, uint64_t nquads, uint64_t b0, uint64_t b1, uint64_t cvals,
           InsertPlan ip, M4 u)
{
    using V = typename CT<R>::V;
    const uint64_t stride = (uint64_t)gridDim.x * (256 * PPL);
    for (uint64_t k0 = (uint64_t)blockIdx.x * (256 * PPL) + threadIdx.x; k0 < nquads; k0 += stride) {
        V v[PPL][4];
        uint64_t ia[PPL];
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            const uint64_t k = k0 + (uint64_t)p * 256;
            ia[p] = ins_bits(k, ip) | cvals;
            if (k < nquads) {
                v[p][0] = psi[ia[p]];
                v[p][1] = psi[ia[p] | b0];
                v[p][2] = psi[ia[p] | b1];
                v[p][3] = psi[ia[p] | b0 | b1];
            }
        }
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            const uint64_t k = k0 + (uint64_t)p * 256;
            if (k < nquads) {
                double2 o[4];
                const double2 w0 = ld2(v[p][0]), w1 = ld2(v[p][1]), w2 = ld2(v[p][2]), w3 = ld2(v[p][3]);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const double* ur = &u.m[8 * r];
                    const double2 s = cmad2<double2, double>(ur[0], ur[1], w0, ur[2], ur[3], w1);
                    const double2 s2 = cmad2<double2, double>(ur[4], ur[5], w2, ur[6], ur[7], w3);
                    o[r].x = s.x + s2.x;
                    o[r].y = s.y + s2.y;
                }
                psi[ia[p]] = st2<V>(o[0]);
                psi[ia[p] | b0] = st2<V>(o[1]);
                psi[ia[p] | b1] = st2<V>(o[2]);
                psi[ia[p] | b0 | b1] = st2<V>(o[3]);
            }
        }
    }
}

template <typename R>
static hipError_t apply_2q_t(void* psiv, int n, int t0, int t1, const double* U, uint64_t cm, uint64_t cv,
                             hipStream_t st, int* kind)
{
    using V = typename CT<R>::V;
    M4 u;
    for (int i = 0; i < 32; ++i) u.m[i] = U[i];
    const int nc = __builtin_popcountll(cm);
    const uint64_t nq = 1ull << (n - 2 - nc);
    InsertPlan ip = make_insert_plan(cm | (1ull << t0) | (1ull << t1));
    constexpr int PPL = 2;
    const unsigned g = blocks_for(nq, 256 * PPL);
    hipLaunchKernelGGL((k_2q_quads<R, PPL>), dim3(g), dim3(256), 0, st, (V*)psiv, nq, 1ull << t0, 1ull << t1,
                       cv, ip, u);
    if (kind) *kind = QS_K_2Q;
    return hipGetLastError();
}

hipError_t launch_apply_2q(void* psi, int dt, int n, int t0, int t1, const double* U, uint64_t cm,
                           uint64_t cv, hipStream_t st, int* kind)
{
    return dt == QS_C128 ? apply_2q_t<double>(psi, n, t0, t1, U, cm, cv, st, kind)
                         : apply_2q_t<float>(psi, n, t0, t1, U, cm, cv, st, kind);
}

// ---------------------------------------------------------------- generic k

// Dense k-qubit gate.  The block stages G = 256 / D groups of D = 2^k
// amplitudes in LDS together with U (D x D); lane j then produces output row
// r = j % D of group j / D.
template <typename R, int K>
__global__ void __launch_bounds__(256)
k_kq_lds(typename CT<R>::V* __restrict__ psi, uint64_t ngroups, uint64_t cvals, InsertPlan ip,
         const double2* __restrict__ Ud, uint64_t tbits_packed_lo, uint64_t tbits_packed_hi)
{
    using V = typename CT<R>::V;
    constexpr int D = 1 << K;
    constexpr int G = 256 / D;
    // U goes to LDS when it fits in 32 KiB; the c128 6-qubit matrix (64 KiB) is
    // read through the caches instead.
    constexpr bool kUL = D * D * sizeof(double2) <= 32768;
    __shared__ double2 su[kUL ? D * D : 1];
    __shared__ V sx[256];
    __shared__ uint64_t soff[D];
    if (kUL)
        for (int j = threadIdx.x; j < D * D; j += 256) su[j] = Ud[j];
    if (threadIdx.x < D) {
        // targets are packed 6 bits each: t[0..4] in lo (bits 0..59), t[5] in hi
        uint64_t off = 0;
        for (int b = 0; b < K; ++b) {
            const int tb = b < 5 ? (int)((tbits_packed_lo >> (6 * b)) & 63) : (int)(tbits_packed_hi & 63);
            if ((threadIdx.x >> b) & 1) off |= 1ull << tb;
        }
        soff[threadIdx.x] = off;
    }
    __syncthreads();
    const int lg = threadIdx.x % G, lm = threadIdx.x / G; // load mapping: consecutive lanes, groups
    const int cg = threadIdx.x / D, cr = threadIdx.x % D; // compute mapping
    const uint64_t stride = (uint64_t)gridDim.x * G;
    for (uint64_t g0 = (uint64_t)blockIdx.x * G; g0 < ngroups; g0 += stride) {
        {
            const uint64_t gi = g0 + lg;
            if (gi < ngroups) sx[lg * D + lm] = psi[(ins_bits(gi, ip) | cvals) | soff[lm]];
        }
        __syncthreads();
        const uint64_t gi = g0 + cg;
        if (gi < ngroups) {
            double sr = 0, si = 0;
#pragma unroll 4
            for (int m = 0; m < D; ++m) {
                const double2 a = kUL ? su[cr * D + m] : Ud[cr * D + m];
                const double2 x = ld2(sx[cg * D + m]);
                sr += a.x * x.x - a.y * x.y;
                si += a.x * x.y + a.y * x.x;
            }
            psi[(ins_bits(gi, ip) | cvals) | soff[cr]] = st2<V>(make_double2(sr, si));
        }
        __syncthreads();
    }
}

template <typename R, int K>
static void launch_kq_k(void* psi, int n, uint64_t tmask, uint64_t cm, uint64_t cv, const void* Ud,
                        uint64_t plo, uint64_t phi, hipStream_t st)
{
    using V = typename CT<R>::V;
    constexpr int D = 1 << K;
    constexpr int G = 256 / D;
    const int nc = __builtin_popcountll(cm);
    const uint64_t ng = 1ull << (n - K - nc);
    InsertPlan ip = make_insert_plan(cm | tmask);
    const unsigned g = blocks_for(ng, G * 4);
    hipLaunchKernelGGL((k_kq_lds<R, K>), dim3(g), dim3(256), 0, st, (V*)psi, ng, cv, ip, (const double2*)Ud, plo,
                       phi);
}

// Ud: device copy of the FP64 matrix.
hipError_t launch_apply_kq_dev(void* psi, int dt, int n, const int* targets, int k, const void* Ud,
                               uint64_t cm, uint64_t cv, hipStream_t st, int* kind)
{
    uint64_t tmask = 0, plo = 0, phi = 0;
    for (int j = 0; j < k; ++j) {
        tmask |= 1ull << targets[j];
        if (j < 5)
            plo |= (uint64_t)targets[j] << (6 * j);
        else
            phi = (uint64_t)targets[j];
    }
    const bool d = dt == QS_C128;
    switch (k) {
    case 1: d ? launch_kq_k<double, 1>(psi, n, tmask, cm, cv, Ud, plo, phi, st)
              : launch_kq_k<float, 1>(psi, n, tmask, cm, cv, Ud, plo, phi, st); break;
    case 2: d ? launch_kq_k<double, 2>(psi, n, tmask, cm, cv, Ud, plo, phi, st)
              : launch_kq_k<float, 2>(psi, n, tmask, cm, cv, Ud, plo, phi, st); break;
    case 3: d ? launch_kq_k<double, 3>(psi, n, tmask, cm, cv, Ud, plo, phi, st)
              : launch_kq_k<float, 3>(psi, n, tmask, cm, cv, Ud, plo, phi, st); break;
    case 4: d ? launch_kq_k<double, 4>(psi, n, tmask, cm, cv, Ud, plo, phi, st)
              : launch_kq_k<float, 4>(psi, n, tmask, cm, cv, Ud, plo, phi, st); break;
    case 5: d ? launch_kq_k<double, 5>(psi, n, tmask, cm, cv, Ud, plo, phi, st)
              : launch_kq_k<float, 5>(psi, n, tmask, cm, cv, Ud, plo, phi, st); break;
    case 6: d ? launch_kq_k<double, 6>(psi, n, tmask, cm, cv, Ud, plo, phi, st)
              : launch_kq_k<float, 6>(psi, n, tmask, cm, cv, Ud, plo, phi, st); break;
    default: return hipErrorInvalidValue;
    }
    if (kind) *kind = QS_K_KQ;
    return hipGetLastError();
}

} // namespace qs
