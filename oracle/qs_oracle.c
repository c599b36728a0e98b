/*
 * qs_oracle.c -- plain FP64 CPU state-vector simulator.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness oracle for the GPU
 * gate engine.  Only the test suite, the smoke check and the bench's CPU
 * baseline may load it; the GPU product path never links or calls it, and it
 * shares no code, headers or tables with that path (it parses the same circuit
 * IR, which is plain data).
 *
 * What it computes: the state after applying the circuit's gate operators in
 * order.  A gate on target set T with matrix U (2^|T| x 2^|T|) and control
 * condition (i & cmask) == cvals is the operator that, for every index i with
 * all target bits 0 that satisfies the control condition, replaces the 2^|T|
 * amplitudes psi[i | bits(m)] (m = 0 .. 2^|T|-1, target T[j] holding bit j of
 * m) by U times them, and leaves every other amplitude unchanged.  This is the
 * paper's pair update (Alg. 1: indices i and i + 2^t, Section II-C) for a general
 * 2x2 matrix, extended to several targets, with the control semantics of
 * Fig. control6q2 (only amplitudes whose control bits are 1 are updated;
 * Section III-A).
 *
 * Plainness rules: FP64 throughout, complex products written out as explicit
 * real arithmetic, built with -ffp-contract=off and without fast-math, no gate
 * fusion, no blocking.  Iterations of one gate touch disjoint amplitude groups,
 * so the OpenMP loops give results bitwise equal to the serial loop.
 *
 * Layout: psi is 2^n complex numbers stored interleaved (re, im), the
 * array-of-structures layout of Section II-A.  Qubit q is bit q of the index.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t nt;
    int32_t t[6];
    uint32_t flags;
    uint64_t cmask;
    uint64_t cvals;
    uint64_t moff;
    uint64_t rsv;
} orc_op; /* 64-byte record of the circuit IR */

int orc_op_size(void) { return (int)sizeof(orc_op); }

void orc_init_basis(int n, double* psi, uint64_t x)
{
    uint64_t N = (uint64_t)1 << n;
    memset(psi, 0, (size_t)(2 * N) * sizeof(double));
    psi[2 * x] = 1.0;
}

/* One 1q gate.  U is 2x2 complex, row-major, interleaved (8 doubles).  Same
 * walk as Alg. 1 (each index with the target bit 0 is the upper member of a
 * pair whose lower member is 2^t above it), with the Hadamard's constants
 * replaced by a general U and the control test of Fig. control6q2. */
void orc_apply_1q(int n, double* psi, int t, const double* U, uint64_t cmask, uint64_t cvals)
{
    const int64_t N = (int64_t)1 << n;
    const int64_t half = (int64_t)1 << t;
    const double u00r = U[0], u00i = U[1], u01r = U[2], u01i = U[3];
    const double u10r = U[4], u10i = U[5], u11r = U[6], u11i = U[7];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        if (i & half) continue;
        if (((uint64_t)i & cmask) != cvals) continue;
        int64_t j = i + half;
        double ar = psi[2 * i], ai = psi[2 * i + 1];
        double br = psi[2 * j], bi = psi[2 * j + 1];
        psi[2 * i]     = (u00r * ar - u00i * ai) + (u01r * br - u01i * bi);
        psi[2 * i + 1] = (u00r * ai + u00i * ar) + (u01r * bi + u01i * br);
        psi[2 * j]     = (u10r * ar - u10i * ai) + (u11r * br - u11i * bi);
        psi[2 * j + 1] = (u10r * ai + u10i * ar) + (u11r * bi + u11i * br);
    }
}

/* A gate on k = nt targets (1..6).  U is 2^k x 2^k complex, row-major. */
void orc_apply_kq(int n, double* psi, int nt, const int32_t* t, const double* U,
                  uint64_t cmask, uint64_t cvals)
{
    const int64_t N = (int64_t)1 << n;
    const int d = 1 << nt;
    uint64_t tmask = 0;
    for (int j = 0; j < nt; ++j) tmask |= (uint64_t)1 << t[j];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        if ((uint64_t)i & tmask) continue;
        if (((uint64_t)i & cmask) != cvals) continue;
        int64_t idx[64];
        double vr[64], vi[64];
        for (int m = 0; m < d; ++m) {
            uint64_t a = (uint64_t)i;
            for (int j = 0; j < nt; ++j)
                if ((m >> j) & 1) a |= (uint64_t)1 << t[j];
            idx[m] = (int64_t)a;
            vr[m] = psi[2 * a];
            vi[m] = psi[2 * a + 1];
        }
        for (int r = 0; r < d; ++r) {
            double sr = 0.0, si = 0.0;
            for (int m = 0; m < d; ++m) {
                double ur = U[2 * (r * d + m)], ui = U[2 * (r * d + m) + 1];
                sr += ur * vr[m] - ui * vi[m];
                si += ur * vi[m] + ui * vr[m];
            }
            psi[2 * idx[r]] = sr;
            psi[2 * idx[r] + 1] = si;
        }
    }
}

void orc_apply_op(int n, double* psi, const orc_op* op, const double* mats)
{
    const double* U = mats + op->moff;
    if (op->nt == 1)
        orc_apply_1q(n, psi, op->t[0], U, op->cmask, op->cvals);
    else
        orc_apply_kq(n, psi, op->nt, op->t, U, op->cmask, op->cvals);
}

void orc_run(int n, double* psi, const orc_op* ops, int64_t nops, const double* mats)
{
    for (int64_t g = 0; g < nops; ++g) orc_apply_op(n, psi, &ops[g], mats);
}

/* Neumaier compensated sum step. */
static inline void nsum(double* s, double* c, double x)
{
    double t = *s + x;
    if (fabs(*s) >= fabs(x))
        *c += (*s - t) + x;
    else
        *c += (x - t) + *s;
    *s = t;
}

/* Marginal probabilities: out[o] = sum of |psi_i|^2 over i whose bits at
 * qubits[0..m) spell o (qubits[0] is bit 0 of o).  Serial, compensated. */
void orc_probabilities(int n, const double* psi, const int32_t* qubits, int m, double* out)
{
    const int64_t N = (int64_t)1 << n;
    const int64_t M = (int64_t)1 << m;
    double* comp = (double*)calloc((size_t)M, sizeof(double));
    for (int64_t o = 0; o < M; ++o) out[o] = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        int64_t o = 0;
        for (int j = 0; j < m; ++j) o |= (((i >> qubits[j]) & 1) << j);
        double p = psi[2 * i] * psi[2 * i] + psi[2 * i + 1] * psi[2 * i + 1];
        nsum(&out[o], &comp[o], p);
    }
    for (int64_t o = 0; o < M; ++o) out[o] += comp[o];
    free(comp);
}

double orc_norm2(int n, const double* psi)
{
    double out;
    orc_probabilities(n, psi, NULL, 0, &out);
    return out;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for the parallel loops that follow (timing only: the loops split
 * disjoint groups, so the result does not depend on it). */
void orc_set_threads(int t)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* Expectation value of a Pauli string.  P = i^w X^x Z^z with w = |x & z|
 * (X on the bits of x, Z on the bits of z, Y = iXZ on bits in both), so
 * P|k> = i^w (-1)^{|k & z|} |k ^ x> and
 *   <psi|P|psi> = i^w * sum_k conj(psi_{k^x}) psi_k (-1)^{|k & z|}.
 * Serial, compensated sums of the real and imaginary parts; out = (re, im). */
void orc_expect_pauli(int n, const double* psi, uint64_t x, uint64_t z, double* out)
{
    const int64_t N = (int64_t)1 << n;
    double sr = 0.0, cr = 0.0, si = 0.0, ci = 0.0;
    for (int64_t k = 0; k < N; ++k) {
        const int64_t j = k ^ (int64_t)x;
        const double ar = psi[2 * j], ai = -psi[2 * j + 1]; /* conj(psi_j) */
        const double br = psi[2 * k], bi = psi[2 * k + 1];
        double pr = ar * br - ai * bi, pi = ar * bi + ai * br;
        if (__builtin_popcountll((uint64_t)k & z) & 1) {
            pr = -pr;
            pi = -pi;
        }
        nsum(&sr, &cr, pr);
        nsum(&si, &ci, pi);
    }
    double re = sr + cr, im = si + ci;
    /* multiply by i^w */
    for (int w = __builtin_popcountll(x & z) & 3; w > 0; --w) {
        const double t = re;
        re = -im;
        im = t;
    }
    out[0] = re;
    out[1] = im;
}

/* Sampling by inversion of the cumulative distribution: for each uniform
 * u[s] in [0, 1), out[s] is the smallest index i with
 *   sum_{j <= i} |psi_j|^2 > u[s] * sum_j |psi_j|^2
 * (cumulative sums in FP64 in index order, compensated); a target at or
 * above the total gives the last index with nonzero probability. */
void orc_sample(int n, const double* psi, const double* u, int64_t shots, uint64_t* out)
{
    const int64_t N = (int64_t)1 << n;
    double* C = (double*)malloc((size_t)N * sizeof(double));
    double s = 0.0, c = 0.0;
    int64_t last = 0;
    for (int64_t i = 0; i < N; ++i) {
        const double p = psi[2 * i] * psi[2 * i] + psi[2 * i + 1] * psi[2 * i + 1];
        nsum(&s, &c, p);
        C[i] = s + c;
        if (p > 0.0) last = i;
    }
    const double total = C[N - 1];
    for (int64_t k = 0; k < shots; ++k) {
        const double t = u[k] * total;
        int64_t lo = 0, hi = N; /* first i with C[i] > t */
        while (lo < hi) {
            const int64_t mid = lo + (hi - lo) / 2;
            if (C[mid] > t)
                hi = mid;
            else
                lo = mid + 1;
        }
        out[k] = (uint64_t)(lo < N ? lo : last);
    }
    free(C);
}
