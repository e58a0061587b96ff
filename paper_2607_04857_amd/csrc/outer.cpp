// outer.cpp -- outer-bit reduction of a QUBO (Sec. III-C.1, the
// straightforward parallelisation): fixing the first k variables x_f leaves
// a QUBO of the other n - k variables, Q' = T_rr + diag(x_f T_fr), with the
// constant c(x_f) = E_ff(x_f); the 2^k reduced instances are solved as one
// batch and the global answer is the lexicographic minimum of
// (c(x_f) + E'_min, x_f 2^(n-k) + index').  Host code; the batch runs the
// usual kernels.
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/qubo.h"
#include "runtime.h"

namespace {

constexpr int kMaxOuterBits = 12;   // at most 4096 reduced instances (one batch)
constexpr int kMaxOuterN = 64;      // indices are 64-bit

// Folded upper-triangular T of an int32 Q, in int64.
std::vector<int64_t> fold_int(const int32_t *Q, int n)
{
    std::vector<int64_t> T(size_t(n) * n, 0);
    for (int i = 0; i < n; i++)
        for (int j = i; j < n; j++)
            T[size_t(i) * n + j] = i == j ? int64_t(Q[size_t(i) * n + i])
                                          : int64_t(Q[size_t(i) * n + j]) + int64_t(Q[size_t(j) * n + i]);
    return T;
}

// The reduced instance for the outer bits xf (variable i < k is bit k-1-i):
// Qr (m x m, m = n - k, upper-triangular) and c.  False if an entry leaves int32.
bool reduce(const std::vector<int64_t> &T, int n, int k, uint64_t xf, int32_t *Qr, int64_t *c)
{
    const int m = n - k;
    auto bit = [&](int i) { return int((xf >> (k - 1 - i)) & 1u); };
    int64_t cc = 0;
    for (int i = 0; i < k; i++) {
        if (!bit(i)) continue;
        for (int j = i; j < k; j++)
            if (bit(j)) cc += T[size_t(i) * n + j];
    }
    for (int r = 0; r < m; r++) {
        for (int s = 0; s < m; s++) {
            int64_t v = 0;
            if (s > r) {
                v = T[size_t(k + r) * n + k + s];
            } else if (s == r) {
                v = T[size_t(k + r) * n + k + r];
                for (int f = 0; f < k; f++)
                    if (bit(f)) v += T[size_t(f) * n + k + r];   // x_f T_fr on the diagonal
            }
            if (v < INT32_MIN || v > INT32_MAX) return false;
            Qr[size_t(r) * m + s] = int32_t(v);
        }
    }
    *c = cc;
    return true;
}

}  // namespace

extern "C" {

qubo_status_t qubo_reduce_outer(const int32_t *Q, int n, int k, uint64_t xf, int32_t *Qr, int64_t *c)
{
    try {
        qrt::set_error("");
        if (!Q || !Qr || !c || n < 2 || n > kMaxOuterN || k < 1 || k >= n || k > 63 ||
            (xf >> k) != 0) {
            qrt::set_error("need Q, Qr, c, 2 <= n <= 64, 1 <= k < n and xf < 2^k");
            return QUBO_EINVAL;
        }
        const std::vector<int64_t> T = fold_int(Q, n);
        if (!reduce(T, n, k, xf, Qr, c)) {
            qrt::set_error("a reduced entry leaves int32");
            return QUBO_EOVERFLOW;
        }
        return QUBO_OK;
    } catch (const std::bad_alloc &) {
        qrt::set_error("host allocation failed");
        return QUBO_ENOMEM;
    }
}

qubo_status_t qubo_solve_outer(const void *Q, int n, qubo_dtype_t dtype, int k, qubo_result_t *out)
{
    using clock = std::chrono::steady_clock;
    const auto t0 = clock::now();
    try {
        qrt::set_error("");
        if (!Q || !out) {
            qrt::set_error("null argument");
            return QUBO_EINVAL;
        }
        if (dtype != QUBO_INT32) {
            qrt::set_error("outer reduction takes int32 input (its constants and diagonals stay exact)");
            return QUBO_EINVAL;
        }
        if (n < 2 || n > kMaxOuterN || k < 1 || k > kMaxOuterBits || n - k < 1 || n - k > 60) {
            qrt::set_error("need 2 <= n <= 64, 1 <= k <= 12 and 1 <= n - k <= 60");
            return QUBO_EINVAL;
        }
        const int m = n - k;
        const size_t count = size_t(1) << k;
        const std::vector<int64_t> T = fold_int(static_cast<const int32_t *>(Q), n);
        std::vector<int32_t> mats(count * size_t(m) * size_t(m));
        std::vector<int64_t> cs(count);
        std::vector<const void *> ptrs(count);
        std::vector<int> ns(count, m);
        std::vector<qubo_dtype_t> dts(count, QUBO_INT32);
        for (size_t x = 0; x < count; x++) {
            int32_t *Qr = mats.data() + x * size_t(m) * size_t(m);
            if (!reduce(T, n, k, uint64_t(x), Qr, &cs[x])) {
                qrt::set_error("a reduced entry leaves int32");
                return QUBO_EOVERFLOW;
            }
            ptrs[x] = Qr;
        }
        qubo_batch_t *b = nullptr;
        qubo_status_t st = qubo_batch_create(int(count), ptrs.data(), ns.data(), dts.data(), nullptr, &b);
        if (st != QUBO_OK) return st;
        std::vector<qubo_result_t> res(count);
        double states = 0.0, kms = 0.0;
        st = qubo_batch_run(b, nullptr);
        if (st == QUBO_OK) st = qubo_batch_results(b, res.data());
        if (st == QUBO_OK) st = qubo_batch_stats(b, &states, &kms);
        qubo_batch_destroy(b);
        if (st != QUBO_OK) return st;
        // lexicographic minimum of (E, index); x_f are the index's top bits
        size_t best = 0;
        int64_t bestE = INT64_MAX;
        uint64_t bestI = ~0ull;
        for (size_t x = 0; x < count; x++) {
            const int64_t e = cs[x] + res[x].best.energy_i;
            const uint64_t idx = (uint64_t(x) << m) | res[x].best.index;
            if (e < bestE || (e == bestE && idx < bestI)) {
                bestE = e;
                bestI = idx;
                best = x;
            }
        }
        *out = res[best];
        out->best.energy_i = bestE;
        out->best.energy = double(bestE);
        out->best.index = bestI;
        out->states = n >= 64 ? ~0ull : (1ull << n);
        out->kernel_ms = kms;
        out->total_ms = std::chrono::duration<double, std::milli>(clock::now() - t0).count();
        return QUBO_OK;
    } catch (const std::bad_alloc &) {
        qrt::set_error("host allocation failed");
        return QUBO_ENOMEM;
    }
}

}  // extern "C"
