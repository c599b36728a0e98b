// Diagonal (phase-only) gates for gfx950.
//
// A diagonal gate multiplies each amplitude by a factor that depends only on
// its index, so an amplitude whose factor is exactly 1 need not be read at
// all -- the memory access filtering that Section I mentions for gates that
// leave most of the state unchanged.  Controls fold into the diagonal (factor
// 1 where a control bit does not match), and every qubit whose bit is the
// same in all amplitudes the gate changes becomes a fixed bit:
//
//   CZ, CP(phi)        two fixed bits: 2^(n-2) amplitudes touched
//   Z / phase on t     one fixed bit:  2^(n-1)
//   multi-controlled Z every bit fixed: one amplitude (one 128-byte line)
//   RZ                 no fixed bit, one free bit (a 2-entry factor table)
//
// Fixed bits at or above the 128-byte line boundary are inserted into the
// counter (those lines are never fetched); fixed bits below it are tested per
// amplitude, and every lane stores (unchanged amplitudes are written back bit
// for bit) so each line is written whole.  Measured on MI355X: reading half of
// every 128-byte line takes as long as reading all of it, and writing halves
// is slower, so 64-byte granularity gains nothing.  The remaining target bits
// index a factor table of at most 2^6 entries held in LDS.
#include <cstring>

#include "device_common.h"

namespace qs {

namespace {

struct DiagArgs {
    uint64_t C;         // counter range: amplitudes read
    uint64_t fv_hi;     // values of the inserted fixed bits
    uint64_t nblocks;   // counter chunks of 256 * PPL
    uint32_t fm_lo, fv_lo;
    int32_t slog;       // log2 of the slot spread
    int32_t xcd;        // chunk order: 1 = each XCD a contiguous eighth (as the per-gate kernel)
    int32_t nfree;
    int32_t fpos[kDiagMaxFree];
    double tab[2 << kDiagMaxFree];
    InsertPlan ip;
};

template <typename R, int PPL, bool NT>
__global__ void __launch_bounds__(256) k_diag(typename CT<R>::V* __restrict__ psi, DiagArgs a)
{
    using V = typename CT<R>::V;
    __shared__ double stab[2 << kDiagMaxFree];
    if (threadIdx.x < (2u << a.nfree)) stab[threadIdx.x] = a.tab[threadIdx.x];
    __syncthreads();
    const uint64_t S = 1ull << a.slog;
    const uint64_t spb = S >> 8;
    for (uint64_t bb = blockIdx.x; bb < a.nblocks; bb += gridDim.x) {
        const uint64_t b = a.xcd ? (bb & 7) * (a.nblocks >> 3) + (bb >> 3) : bb;
        const uint64_t base = (b / spb) * (S * PPL) + (b % spb) * 256 + threadIdx.x;
        V x[PPL];
        uint64_t idx[PPL];
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            const uint64_t k = base + (uint64_t)p * S;
            idx[p] = ins_bits(k, a.ip) | a.fv_hi;
            if (k < a.C) x[p] = gld<NT>(psi + idx[p]);
        }
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            if (base + (uint64_t)p * S >= a.C) continue;
            int j = 0;
            for (int f = 0; f < a.nfree; ++f) j |= (int)((idx[p] >> a.fpos[f]) & 1) << f;
            const double fr = stab[2 * j], fi = stab[2 * j + 1];
            const double2 v = ld2(x[p]);
            const bool m = ((uint32_t)idx[p] & a.fm_lo) == a.fv_lo;
            double2 w;
            w.x = m ? fr * v.x - fi * v.y : v.x;
            w.y = m ? fr * v.y + fi * v.x : v.y;
            gst<NT>(psi + idx[p], st2<V>(w));
        }
    }
}

template <typename R, int PPL>
hipError_t launch_diag_t(void* psi, DiagArgs& a, int wg, int xcd, hipStream_t st)
{
    using V = typename CT<R>::V;
    const int sl = (int)tun(T_DIAG_SLOG);
    a.slog = a.C >= ((1ull << sl) * PPL) ? sl : 8;
    a.nblocks = (a.C + 256 * PPL - 1) / (256 * PPL);
    a.xcd = (xcd && a.nblocks % 8 == 0) ? 1 : 0;
    const uint64_t cap = (uint64_t)tun(T_GATE_GRID_CAP);
    const unsigned g = (unsigned)(a.nblocks < cap ? a.nblocks : cap);
    const size_t pad = pad_for_wg_per_cu(wg, sizeof(double) * (2 << kDiagMaxFree));
    const bool nt = a.C >= 64;
    hipError_t e = lds_optin(nt ? (const void*)k_diag<R, PPL, true> : (const void*)k_diag<R, PPL, false>, pad);
    if (e != hipSuccess) return e;
    if (nt)
        hipLaunchKernelGGL((k_diag<R, PPL, true>), dim3(g), dim3(256), pad, st, (V*)psi, a);
    else
        hipLaunchKernelGGL((k_diag<R, PPL, false>), dim3(g), dim3(256), pad, st, (V*)psi, a);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_diag_r(void* psi, DiagArgs& a, uint64_t state_bytes, hipStream_t st)
{
    // Memory schedule (the per-gate kernel's knobs apply).  Measured on
    // MI355X at n=30 over CZ on neighbouring pairs and CP with random controls:
    // each XCD walking its own contiguous eighth of the chunks (+3 % complex64,
    // +18 % complex128, where pairs 1-64 MiB apart gain the most) and, for
    // complex128, one slot per lane (the reads skip lines, so the streams are
    // already many); unlike the dense per-gate kernel, capping occupancy only
    // loses here.  States that fit the Infinity Cache keep workgroup order.
    int ppl = (int)tun(T_DIAG_SLOTS), wg = 0, xcd = 1;
    if (ppl == 0) ppl = sizeof(R) == 8 ? 1 : 4;
    const int wg_k = (int)tun(T_GATE_WG_PER_CU), xcd_k = (int)tun(T_GATE_XCD);
    if (state_bytes < (512ull << 20)) xcd = 0;
    if (wg_k > 0) wg = wg_k;
    if (xcd_k > 0) xcd = xcd_k - 1;
    switch (ppl) {
    case 1: return launch_diag_t<R, 1>(psi, a, wg, xcd, st);
    case 2: return launch_diag_t<R, 2>(psi, a, wg, xcd, st);
    case 8: return launch_diag_t<R, 8>(psi, a, wg, xcd, st);
    default: return launch_diag_t<R, 4>(psi, a, wg, xcd, st);
    }
}

} // namespace

bool diag_plan(int n, const int* t, int k, const double* d, uint64_t cm, uint64_t cv, DiagPlan* p)
{
    std::memset(p, 0, sizeof *p);
    if (k < 1 || k > kDiagMaxFree) return false;
    const int D = 1 << k;
    // entries that change an amplitude, and the target bits they all share
    int nchg = 0;
    uint32_t all1 = (uint32_t)D - 1, all0 = (uint32_t)D - 1; // bits equal to 1 / 0 in every changing entry
    for (int j = 0; j < D; ++j) {
        if (d[2 * j] == 1.0 && d[2 * j + 1] == 0.0) continue;
        ++nchg;
        all1 &= (uint32_t)j;
        all0 &= ~(uint32_t)j;
    }
    p->changed_per = (uint64_t)nchg;
    p->n = n;
    p->k = k;
    p->nctrl = __builtin_popcountll(cm);
    if (nchg == 0) {
        p->identity = true;
        return true;
    }
    uint64_t fm = cm, fv = cv;
    int fixed_t = 0; // matrix bits of the fixed targets
    for (int b = 0; b < k; ++b) {
        const uint64_t q = 1ull << t[b];
        if ((all1 >> b) & 1) {
            fm |= q;
            fv |= q;
            fixed_t |= 1 << b;
        } else if ((all0 >> b) & 1) {
            fm |= q;
            fixed_t |= 1 << b;
        } else {
            p->fpos[p->nfree] = t[b];
            p->fbit[p->nfree] = b;
            p->nfree++;
        }
    }
    p->fixed_mask = fm;
    p->fixed_val = fv;
    // factor per pattern of the free bits (fixed target bits at their values)
    int jfix = 0;
    for (int b = 0; b < k; ++b)
        if (((fixed_t >> b) & 1) && ((fv >> t[b]) & 1)) jfix |= 1 << b;
    for (int f = 0; f < (1 << p->nfree); ++f) {
        int j = jfix;
        for (int i = 0; i < p->nfree; ++i)
            if ((f >> i) & 1) j |= 1 << p->fbit[i];
        p->tab[2 * f] = d[2 * j];
        p->tab[2 * f + 1] = d[2 * j + 1];
    }
    return true;
}

bool diag_plan_matrix(int n, const int* t, int k, const double* U, uint64_t cm, uint64_t cv, DiagPlan* p)
{
    if (k < 1 || k > kDiagMaxFree) return false;
    const int D = 1 << k;
    double d[2 << kDiagMaxFree];
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c) {
            const double re = U[2 * (r * D + c)], im = U[2 * (r * D + c) + 1];
            if (r == c) {
                d[2 * r] = re;
                d[2 * r + 1] = im;
            } else if (re != 0.0 || im != 0.0) {
                return false;
            }
        }
    return diag_plan(n, t, k, d, cm, cv, p);
}

uint64_t diag_changed(const DiagPlan& p)
{
    return p.changed_per << (p.n - p.k - p.nctrl);
}

hipError_t launch_diag(void* psi, int dt, const DiagPlan& p, hipStream_t st)
{
    if (p.identity) return hipSuccess;
    // fixed bits inside a 128-byte line are tested per amplitude
    const int line_bits = dt == QS_C128 ? 3 : 4;
    const uint64_t lo = (1ull << line_bits) - 1;
    DiagArgs a;
    std::memset(&a, 0, sizeof a);
    const uint64_t hi = p.fixed_mask & ~lo;
    a.fm_lo = (uint32_t)(p.fixed_mask & lo);
    a.fv_lo = (uint32_t)(p.fixed_val & lo);
    a.fv_hi = p.fixed_val & hi;
    a.ip = make_insert_plan(hi);
    a.C = 1ull << (p.n - __builtin_popcountll(hi));
    a.nfree = p.nfree;
    for (int i = 0; i < p.nfree; ++i) a.fpos[i] = p.fpos[i];
    for (int i = 0; i < (2 << p.nfree); ++i) a.tab[i] = p.tab[i];
    const uint64_t sb = (1ull << p.n) * amp_bytes(dt);
    return dt == QS_C128 ? launch_diag_r<double>(psi, a, sb, st) : launch_diag_r<float>(psi, a, sb, st);
}

} // namespace qs
