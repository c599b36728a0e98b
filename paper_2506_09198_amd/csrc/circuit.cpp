// qs_run_circuit: validate a whole circuit, then execute it either one launch
// per gate or through the planner's tile passes.
#include <cstring>
#include <vector>

#include "planner.h"
#include "runtime.h"

using namespace qs;

namespace qs {

qs_status validate_circuit(int n, const qs_op* ops, int64_t n_ops, const double* mats, int64_t n_mats)
{
    if (n_ops < 0 || n_mats < 0) return set_err(QS_ERR_ARG, "negative op or matrix count");
    if (n_ops > 0 && !ops) return set_err(QS_ERR_ARG, "null op table");
    if (n_mats > 0 && !mats) return set_err(QS_ERR_ARG, "null matrix pool");
    const bool chk = check_unitary_enabled();
    for (int64_t g = 0; g < n_ops; ++g) {
        const qs_op& o = ops[g];
        if (o.flags != 0 || o.rsv != 0) return set_err(QS_ERR_ARG, "op %lld: flags/rsv must be 0", (long long)g);
        qs_status st = validate_gate(n, o.t, o.nt, o.cmask, o.cvals);
        if (st != QS_OK) return set_err(st, "op %lld: %s", (long long)g, qs_last_error());
        const uint64_t need = 2ull << (2 * o.nt);
        if (o.moff > (uint64_t)n_mats || need > (uint64_t)n_mats - o.moff)
            return set_err(QS_ERR_ARG, "op %lld: matrix range outside the pool", (long long)g);
        if (chk && (st = check_unitary(mats + o.moff, o.nt)) != QS_OK)
            return set_err(st, "op %lld: %s", (long long)g, qs_last_error());
    }
    return QS_OK;
}

qs_status run_per_gate(qs_state s, const qs_op* ops, int64_t n_ops, const double* mats, int64_t n_mats)
{
    const void* dpool = nullptr;
    bool need_pool = false;
    for (int64_t g = 0; g < n_ops; ++g) need_pool |= ops[g].nt > 2;
    if (need_pool) {
        qs_status st = stage_bytes(s, mats, (uint64_t)n_mats * sizeof(double), &dpool);
        if (st != QS_OK) return st;
    }
    const size_t es = sizeof(double);
    for (int64_t g = 0; g < n_ops; ++g) {
        const qs_op& o = ops[g];
        const double* U = mats + o.moff;
        qs_status st;
        if (o.nt == 1)
            st = apply_1q_internal(s, o.t[0], U, o.cmask, o.cvals);
        else if (o.nt == 2)
            st = apply_2q_internal(s, o.t[0], o.t[1], U, o.cmask, o.cvals);
        else {
            DiagPlan p;
            if (diag_plan_matrix(s->n, o.t, o.nt, U, o.cmask, o.cvals, &p))
                st = apply_diag_internal(s, p, o.t[0], o.t[1], o.cmask);
            else
                st = apply_kq_dev_internal(s, o.t, o.nt, (const char*)dpool + o.moff * es, o.cmask, o.cvals);
        }
        if (st != QS_OK) return st;
    }
    return QS_OK;
}

} // namespace qs

extern "C" qs_status qs_run_circuit(qs_state s, const qs_op* ops, int64_t n_ops, const double* mats,
                                   int64_t n_mats, const qs_run_opts* opts)
{
    qs_status st = check_live(s);
    if (st != QS_OK) return st;
    if ((st = validate_circuit(s->n, ops, n_ops, mats, n_mats)) != QS_OK) return st;
    qs_run_opts o;
    std::memset(&o, 0, sizeof o);
    if (opts) o = *opts;
    if (o.max_blocks < 0) return set_err(QS_ERR_ARG, "max_blocks=%d < 0", o.max_blocks);
    if (o.mode == 1) return run_per_gate(s, ops, n_ops, mats, n_mats);
    if (o.mode != 0) return set_err(QS_ERR_ARG, "unknown run mode %d", o.mode);
    return run_planned(s, ops, n_ops, mats, n_mats, o);
}
