// Measurement on a state: Pauli-string expectation values and sampling.
//
// qs_expect_pauli: <psi|P|psi> for P = i^|x & z| X^x Z^z, FP64 partial sums
// over fixed chunks of pair terms, then a fixed-order final sum on the device.
// qs_sample: inversion of the cumulative distribution at caller-given
// uniforms: per-chunk probabilities on the device (the same chunks as
// qs_probabilities), a compensated prefix and a binary search per shot on
// the host, then one wave per shot walks its chunk on the device.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "qs_internal.h"
#include "runtime.h"

using namespace qs;

namespace {

// Grow the state's reduction scratch to `need` doubles.
qs_status scratch(qs_state s, uint64_t need)
{
    if (need <= s->red_cap) return QS_OK;
    hipError_t e = hipStreamSynchronize(s->st);
    if (e != hipSuccess) return fail_device(s, e, "hipStreamSynchronize");
    if (s->red_part) dev_free(s->red_part, s->red_cap * sizeof(double));
    s->red_part = nullptr;
    s->red_cap = 0;
    qs_status st = dev_alloc((void**)&s->red_part, need * sizeof(double), "reduction scratch");
    if (st != QS_OK) return st;
    s->red_cap = need;
    return QS_OK;
}

// Trace record of a read-only pass over `amps` amplitudes of the state.
qs_trace_rec read_rec(qs_state s, uint64_t amps)
{
    qs_trace_rec r;
    std::memset(&r, 0, sizeof r);
    r.n = s->n;
    r.t0 = r.t1 = -1;
    r.dtype = s->dt;
    r.bytes = amps * amp_bytes(s->dt);
    return r;
}

} // namespace

extern "C" qs_status qs_expect_pauli(qs_state s, uint64_t x_mask, uint64_t z_mask, double* out)
{
    qs_status st = check_live(s);
    if (st != QS_OK) return st;
    if (!out) return set_err(QS_ERR_ARG, "null output");
    const uint64_t all = s->n >= 64 ? ~0ull : ((1ull << s->n) - 1);
    if ((x_mask | z_mask) & ~all) return set_err(QS_ERR_ARG, "Pauli mask has bits at or above n=%d", s->n);
    const uint64_t need = pauli_scratch_doubles(s->n);
    if ((st = scratch(s, need)) != QS_OK) return st;
    double* part = s->red_part;
    double* dout = s->red_part + need - 2;
    st = traced_launch(s, read_rec(s, 1ull << s->n),
                       [&](int* kind) {
                           *kind = QS_K_REDUCE;
                           return launch_pauli_expect(s->d, s->dt, s->n, x_mask, z_mask, part, dout, s->st);
                       },
                       "Pauli expectation launch");
    if (st != QS_OK) return st;
    double sum[2];
    hipError_t e = hipMemcpyAsync(sum, dout, sizeof sum, hipMemcpyDeviceToHost, s->st);
    if (e == hipSuccess) e = hipStreamSynchronize(s->st);
    if (e != hipSuccess) return fail_device(s, e, "Pauli expectation download");
    double re = sum[0], im = sum[1];
    for (int w = __builtin_popcountll(x_mask & z_mask) & 3; w > 0; --w) { // times i^w
        const double t = re;
        re = -im;
        im = t;
    }
    out[0] = re;
    out[1] = im;
    return QS_OK;
}

extern "C" qs_status qs_sample(qs_state s, const double* u, int64_t shots, uint64_t* out)
{
    qs_status st = check_live(s);
    if (st != QS_OK) return st;
    if (shots < 0) return set_err(QS_ERR_ARG, "shots=%lld < 0", (long long)shots);
    if (shots == 0) return QS_OK;
    if (!u || !out) return set_err(QS_ERR_ARG, "null uniforms or output");
    for (int64_t k = 0; k < shots; ++k)
        if (!(u[k] >= 0.0 && u[k] < 1.0)) return set_err(QS_ERR_ARG, "u[%lld] outside [0, 1)", (long long)k);
    const uint64_t nch = reduce_partials(s->n, 0);  // chunk sums
    const uint64_t red = reduce_scratch_doubles(s->n, 0);
    if ((st = scratch(s, red + 1)) != QS_OK) return st;
    double* part = s->red_part;
    st = traced_launch(s, read_rec(s, 1ull << s->n),
                       [&](int* kind) {
                           *kind = QS_K_REDUCE;
                           return launch_probabilities(s->d, s->dt, s->n, nullptr, 0, part, part + red, s->st);
                       },
                       "sampling chunk sums");
    if (st != QS_OK) return st;
    std::vector<double> ch(nch);
    hipError_t e = hipMemcpyAsync(ch.data(), part, nch * sizeof(double), hipMemcpyDeviceToHost, s->st);
    if (e == hipSuccess) e = hipStreamSynchronize(s->st);
    if (e != hipSuccess) return fail_device(s, e, "sampling chunk download");
    // compensated inclusive prefix over the chunks
    std::vector<double> incl(nch);
    double sum = 0.0, comp = 0.0;
    uint64_t lastnz = 0;
    for (uint64_t c = 0; c < nch; ++c) {
        const double x = ch[c];
        const double t = sum + x;
        comp += std::fabs(sum) >= std::fabs(x) ? (sum - t) + x : (x - t) + sum;
        sum = t;
        incl[c] = sum + comp;
        if (x > 0.0) lastnz = c;
    }
    const double total = incl[nch - 1];
    std::vector<SampleReq> req((size_t)shots);
    for (int64_t k = 0; k < shots; ++k) {
        const double t = u[k] * total;
        const uint64_t c = (uint64_t)(std::upper_bound(incl.begin(), incl.end(), t) - incl.begin());
        if (c >= nch) { // at or above the total (rounding): the last nonzero probability
            req[k].chunk = lastnz;
            req[k].residual = INFINITY;
        } else {
            req[k].chunk = c;
            req[k].residual = t - (c > 0 ? incl[c - 1] : 0.0);
        }
    }
    SampleReq* dreq = nullptr;
    uint64_t* dout = nullptr;
    const uint64_t rb = (uint64_t)shots * sizeof(SampleReq), ob = (uint64_t)shots * sizeof(uint64_t);
    if ((st = dev_alloc((void**)&dreq, rb, "sampling requests")) != QS_OK) return st;
    if ((st = dev_alloc((void**)&dout, ob, "sampling output")) != QS_OK) {
        dev_free(dreq, rb);
        return st;
    }
    e = hipMemcpyAsync(dreq, req.data(), rb, hipMemcpyHostToDevice, s->st);
    if (e == hipSuccess) {
        // one wave per shot reads its chunk: min(4096, 2^n) amplitudes per shot
        const uint64_t csize = s->n < 12 ? (1ull << s->n) : 4096;
        st = traced_launch(s, read_rec(s, csize * (uint64_t)shots),
                           [&](int* kind) {
                               *kind = QS_K_SAMPLE;
                               return launch_sample_chunks(s->d, s->dt, s->n, dreq, shots, dout, s->st);
                           },
                           "sampling launch");
        if (st != QS_OK) {
            (void)hipStreamSynchronize(s->st);
            dev_free(dreq, rb);
            dev_free(dout, ob);
            return st;
        }
    }
    if (e == hipSuccess) e = hipMemcpyAsync(out, dout, ob, hipMemcpyDeviceToHost, s->st);
    if (e == hipSuccess) e = hipStreamSynchronize(s->st);
    dev_free(dreq, rb);
    dev_free(dout, ob);
    if (e != hipSuccess) return fail_device(s, e, "sampling");
    return QS_OK;
}
