// checkpoint.cpp -- long exhaustive solves in slices, resumable from a file.
//
// The search space splits into independent segments whose local minima
// reduce to the global one (the map-reduce scheme of Sec. III-C; Sec. IV-C
// uses it to go past the kernel's size limit).  Here a segment is a range of
// the plan's walk items: item c covers the contiguous index block
// [g(c) 2^(L+B), (g(c)+1) 2^(L+B)), g(c) = c ^ (c >> 1), so a range of items
// fixes the outer prefix bits of Sec. III-C.1 to a run of Gray values.  The
// solve walks the items in slices, reduces each slice's (E, index) into the
// running lexicographic minimum and, after every slice, rewrites a small
// text checkpoint (written beside the target and renamed over it, so a
// reader never sees half a file).  A later call with the same input resumes
// after the last finished slice.
#include <algorithm>
#include <cerrno>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "hostio.h"
#include "plan.h"
#include "runtime.h"

namespace {

using qhost::Ckpt;
using qhost::input_hash;
using qhost::read_ckpt;
using qhost::write_ckpt;

void to_result(const Ckpt &c, uint64_t states_done, double total_ms, qubo_result_t *out)
{
    std::memset(out, 0, sizeof *out);
    out->best.energy_i = c.energy_i;
    out->best.energy = c.energy;
    out->best.index = c.index;
    out->tol = c.tol;
    out->p = c.p;
    out->A = c.A;
    out->B = c.B;
    out->L = c.L;
    out->tier = c.tier;
    out->vgpr_levels = c.vgpr_levels;
    out->states = states_done;
    out->kernel_ms = c.walk_ms;
    out->total_ms = total_ms;
}

bool lex_less(int64_t e0, uint64_t i0, int64_t e1, uint64_t i1)
{
    return e0 < e1 || (e0 == e1 && i0 < i1);
}

qubo_status_t run(const void *Q, int n, qubo_dtype_t dtype, const qubo_options_t *opt,
                  uint64_t items_per_slice, int max_slices, const char *path, qubo_result_t *out)
{
    const auto t0 = std::chrono::steady_clock::now();
    if (!Q || !path || !*path || !out || max_slices < 0) {
        qrt::set_error("null Q, path or output, or negative max_slices");
        return QUBO_EINVAL;
    }
    if (opt && (opt->item_first || opt->item_count)) {
        qrt::set_error("a checkpointed solve walks every item: item_first and item_count must be 0");
        return QUBO_EINVAL;
    }
    qrt::tune_autoload();
    std::string msg;
    qplan::Plan P;
    qubo_status_t st = qplan::make_plan(Q, n, dtype, opt, &P, &msg);
    if (st != QUBO_OK) {
        qrt::set_error(msg);
        return st;
    }
    const uint64_t qhash = input_hash(Q, n, dtype);

    Ckpt c;
    int have = read_ckpt(path, &c, &msg);
    if (have < 0) {
        qrt::set_error(msg);
        return QUBO_EINVAL;
    }
    if (have) {
        if (c.n != n || c.dtype != int(dtype) || c.qhash != qhash) {
            qrt::set_error(std::string("checkpoint ") + path + " belongs to another input");
            return QUBO_EINVAL;
        }
        // The checkpoint's plan wins (a tuning table may have changed since),
        // unless the caller forces a different one.
        if (opt && ((opt->B && opt->B != c.B) || (opt->L && opt->L != c.L) ||
                    (opt->tier && opt->tier != c.tier) ||
                    (opt->vgpr_levels && opt->vgpr_levels != c.vgpr_levels))) {
            qrt::set_error(std::string("checkpoint ") + path + " was written with another plan");
            return QUBO_EINVAL;
        }
    } else {
        c.n = n;
        c.dtype = int(dtype);
        c.qhash = qhash;
        c.A = P.A;
        c.B = P.direct ? 0 : P.B;
        c.L = P.direct ? 0 : P.L;
        c.tier = P.tier;
        c.vgpr_levels = P.direct ? 0 : P.vgpr_levels;
        c.items = P.direct ? 1 : P.items;
        c.p = P.p;
        c.tol = dtype == QUBO_FP32 ? 2.0 * P.eps_q : 0.0;
    }
    if (c.items > uint64_t(INT_MAX)) {
        qrt::set_error("plan has more work items than a slice can address");
        return QUBO_EINVAL;
    }

    qubo_options_t o{};
    if (opt) o.waves_per_cu = opt->waves_per_cu;
    if (c.B) {          // walked plan: every slice runs exactly the recorded plan
        o.B = c.B;
        o.L = c.L;
        o.tier = c.tier;
        o.vgpr_levels = c.vgpr_levels;
    }
    const uint64_t slice = items_per_slice ? items_per_slice : c.items;
    const double states_per_item = std::ldexp(1.0, n) / double(c.items);
    int slices = 0;
    while (c.next_item < c.items) {
        if (max_slices && slices == max_slices) return QUBO_EAGAIN;
        qubo_result_t r{};
        if (c.B) {
            const uint64_t cnt = std::min<uint64_t>(slice, c.items - c.next_item);
            o.item_first = int(c.next_item);
            o.item_count = int(cnt);
            st = qubo_solve_ex(Q, n, dtype, 1, &o, &r, nullptr);
            if (st != QUBO_OK) return st;
            if (r.A != c.A || r.B != c.B || r.L != c.L || r.p != c.p) {
                qrt::set_error(std::string("checkpoint ") + path + ": plan does not reproduce");
                return QUBO_EINVAL;
            }
            c.next_item += cnt;
        } else {
            st = qubo_solve_ex(Q, n, dtype, 1, nullptr, &r, nullptr);   // direct: one slice
            if (st != QUBO_OK) return st;
            c.next_item = c.items;
        }
        if (!c.found || lex_less(r.best.energy_i, r.best.index, c.energy_i, c.index)) {
            c.found = 1;
            c.energy_i = r.best.energy_i;
            c.energy = r.best.energy;
            c.index = r.best.index;
        }
        c.walk_ms += r.kernel_ms;
        ++slices;
        if (!write_ckpt(path, c, &msg)) {
            qrt::set_error(msg);
            return QUBO_EINVAL;
        }
    }
    const double ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    to_result(c, uint64_t(states_per_item * double(c.next_item)), ms, out);
    return QUBO_OK;
}

}  // namespace

extern "C" {

qubo_status_t qubo_solve_checkpointed(const void *Q, int n, qubo_dtype_t dtype,
                                      const qubo_options_t *opt, uint64_t items_per_slice,
                                      int max_slices, const char *path, qubo_result_t *out)
{
    try {
        qrt::set_error("");
        return run(Q, n, dtype, opt, items_per_slice, max_slices, path, out);
    } catch (const std::bad_alloc &) {
        qrt::set_error("host allocation failed");
        return QUBO_ENOMEM;
    } catch (...) {
        qrt::set_error("unexpected exception");
        return QUBO_EINTERNAL;
    }
}

qubo_status_t qubo_checkpoint_info(const char *path, qubo_checkpoint_t *info)
{
    try {
        qrt::set_error("");
        if (!path || !info) {
            qrt::set_error("null path or info");
            return QUBO_EINVAL;
        }
        Ckpt c;
        std::string msg;
        int have = read_ckpt(path, &c, &msg);
        if (have <= 0) {
            qrt::set_error(have == 0 ? std::string("no checkpoint at ") + path : msg);
            return QUBO_EINVAL;
        }
        std::memset(info, 0, sizeof *info);
        info->n = c.n;
        info->dtype = qubo_dtype_t(c.dtype);
        info->A = c.A;
        info->B = c.B;
        info->L = c.L;
        info->tier = c.tier;
        info->vgpr_levels = c.vgpr_levels;
        info->q_hash = c.qhash;
        info->items = c.items;
        info->next_item = c.next_item;
        info->found = c.found;
        info->best.energy_i = c.energy_i;
        info->best.energy = c.energy;
        info->best.index = c.index;
        info->p = c.p;
        info->tol = c.tol;
        info->walk_ms = c.walk_ms;
        return QUBO_OK;
    } catch (...) {
        qrt::set_error("unexpected exception");
        return QUBO_EINTERNAL;
    }
}

}  // extern "C"
