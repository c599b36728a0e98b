// Device helpers shared by the kernel translation units.
#pragma once

#include "qs_internal.h"

namespace qs {

template <typename R> struct CT;
template <> struct CT<double> { using V = double2; };
template <> struct CT<float> { using V = float2; };

// Insert a zero bit at every position listed in `p` (ascending), turning a
// compact counter into an amplitude index.
__device__ __forceinline__ uint64_t ins_bits(uint64_t k, const InsertPlan& p)
{
    for (int j = 0; j < p.n; ++j) {
        const uint64_t lo = p.low[j];
        k = (k & lo) | ((k & ~lo) << 1);
    }
    return k;
}

__device__ __forceinline__ uint32_t ins0_32(uint32_t k, int p)
{
    const uint32_t lo = (1u << p) - 1;
    return (k & lo) | ((k & ~lo) << 1);
}

// a*x + b*y for complex scalars a=(ar,ai), b=(br,bi) and complex vectors x, y.
template <typename V, typename R>
__device__ __forceinline__ V cmad2(R ar, R ai, V x, R br, R bi, V y)
{
    V r;
    r.x = ar * x.x - ai * x.y + br * y.x - bi * y.y;
    r.y = ar * x.y + ai * x.x + br * y.y + bi * y.x;
    return r;
}

template <typename V, typename R>
__device__ __forceinline__ V cmul(R ar, R ai, V x)
{
    V r;
    r.x = ar * x.x - ai * x.y;
    r.y = ar * x.y + ai * x.x;
    return r;
}

// Amplitudes are stored as R (float or double) but every gate is computed in
// FP64 with FP64 matrices: a complex64 state is rounded once per stored
// result, and gate matrices are never rounded to FP32 (rounding 1/sqrt2 to FP32
// would shrink the norm by the same factor at every Hadamard).
__device__ __forceinline__ double2 ld2(float2 v) { return make_double2(v.x, v.y); }
__device__ __forceinline__ double2 ld2(double2 v) { return v; }
template <typename V> __device__ __forceinline__ V st2(double2 v);
template <> __device__ __forceinline__ float2 st2<float2>(double2 v) { return make_float2((float)v.x, (float)v.y); }
template <> __device__ __forceinline__ double2 st2<double2>(double2 v) { return v; }

// Global loads/stores, optionally non-temporal (streamed past the caches:
// a gate pass touches every amplitude once, so nothing is reused).
typedef double d2v_t __attribute__((ext_vector_type(2)));
typedef float f2v_t __attribute__((ext_vector_type(2)));
template <bool NT> __device__ __forceinline__ double2 gld(const double2* p)
{
    if (NT) {
        const d2v_t v = __builtin_nontemporal_load((const d2v_t*)p);
        return make_double2(v.x, v.y);
    }
    return *p;
}
template <bool NT> __device__ __forceinline__ float2 gld(const float2* p)
{
    if (NT) {
        const f2v_t v = __builtin_nontemporal_load((const f2v_t*)p);
        return make_float2(v.x, v.y);
    }
    return *p;
}
template <bool NT> __device__ __forceinline__ void gst(double2* p, double2 v)
{
    if (NT) {
        d2v_t w = {v.x, v.y};
        __builtin_nontemporal_store(w, (d2v_t*)p);
    } else {
        *p = v;
    }
}
template <bool NT> __device__ __forceinline__ void gst(float2* p, float2 v)
{
    if (NT) {
        f2v_t w = {v.x, v.y};
        __builtin_nontemporal_store(w, (f2v_t*)p);
    } else {
        *p = v;
    }
}

} // namespace qs
