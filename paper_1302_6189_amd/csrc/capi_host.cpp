// capi_host.cpp -- the host-only half of the C ABI (include/fftrw.h):
// decomposition maps, communication amounts, transpose orders, comparison
// models.  No HIP calls here, so these work on a machine without a GPU.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <thread>
#include <vector>

#include "../../include/fftrw.h"
#include "decomp.hpp"
#include "errors.hpp"

using namespace fftrw;

namespace fftrw {

thread_local std::string g_last_error;

int log_level()
{
    static const int level = [] {
        const char *v = std::getenv("FFTRW_LOG");
        return v ? std::max(0, std::min(3, std::atoi(v))) : 0;
    }();
    return level;
}

void log_line(int level, const char *fmt, ...)
{
    if (log_level() < level) return;
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    std::fprintf(stderr, "fftrw: %s\n", buf);
}

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    log_line(1, "error %d: %s", code, msg.c_str());
    return code;
}

int fail(const Status &s) { return fail(s.code, s.msg); }

}  // namespace fftrw

namespace {

// Calls f(index, perm_idx[M]) for every valid order in canonical order, where
// perm_idx[t] indexes all_perms(M).
template <class F>
void enumerate_orders(int M, const std::vector<std::vector<int8_t>> &perms, F &&f)
{
    int idx[kMaxHostDims];
    idx[0] = 0;  // identity is the first permutation in lexicographic order
    bool used[kMaxHostDims] = {};
    used[M - 1] = true;
    i64 counter = 0;
    auto rec = [&](auto &&self, int s) -> void {
        if (s == M) {
            f(counter++, idx);
            return;
        }
        for (size_t i = 0; i < perms.size(); ++i) {
            int last = perms[i][M - 1];
            if (used[last]) continue;
            used[last] = true;
            idx[s] = (int)i;
            self(self, s + 1);
            used[last] = false;
        }
    };
    rec(rec, 1);
}

struct PairTable {
    int M;
    i64 P;
    const i64 *dims;
    int ownership;
    const std::vector<std::vector<int8_t>> &perms;
    std::vector<Layout> layouts;
    std::vector<i64> vol;  // perms x perms, -1 = not computed
    Status status;

    PairTable(int M_, const i64 *dims_, i64 P_, int own, const std::vector<std::vector<int8_t>> &pr)
        : M(M_), P(P_), dims(dims_), ownership(own), perms(pr)
    {
        layouts.resize(perms.size());
        for (size_t i = 0; i < perms.size(); ++i) {
            Status s = make_layout(M, dims, P, perms[i].data(), &layouts[i]);
            if (!s && status.code == 0) status = s;
        }
        vol.assign(perms.size() * perms.size(), -1);
    }
    // Computes the listed pairs on several host threads (the amounts are
    // independent; each entry is written by one thread).
    void fill(const std::vector<std::pair<int, int>> &pairs)
    {
        const size_t nt = std::max<size_t>(1, std::min<size_t>(16, std::thread::hardware_concurrency()));
        std::vector<Status> st(nt);
        std::vector<std::thread> th;
        for (size_t w = 0; w < nt; ++w)
            th.emplace_back([&, w] {
                for (size_t i = w; i < pairs.size(); i += nt) {
                    const int a = pairs[i].first, b = pairs[i].second;
                    i64 moved = 0;
                    Status s = transpose_amount(layouts[a], layouts[b], ownership, &moved, nullptr);
                    if (!s) {
                        st[w] = s;
                        return;
                    }
                    vol[(size_t)a * perms.size() + b] = moved;
                }
            });
        for (auto &t : th) t.join();
        for (const Status &s : st)
            if (!s && status.code == 0) status = s;
    }
    i64 get(int a, int b)
    {
        i64 &v = vol[(size_t)a * perms.size() + b];
        if (v < 0) {
            i64 moved = 0;
            Status s = transpose_amount(layouts[a], layouts[b], ownership, &moved, nullptr);
            if (!s && status.code == 0) status = s;
            v = moved;
        }
        return v;
    }
};

// Best and worst orders by dynamic programming.  The amount of an order is a
// sum over its consecutive decompositions, so the optimum over all
// (M-1)!^M orders follows from the optimal completion of each state: the
// current decomposition a and the set U of axes already transformed (a bit
// mask).  A completion of (a, U) continues with any b whose last axis is not
// in U.  The number of optimal orders adds up over the same recursion.  The
// canonical enumeration is lexicographic in permutation indices, so the
// lowest-index optimal order is found by walking forward and taking, at each
// step, the smallest b whose completion attains the optimum.
struct OrderSearch {
    int M = 0;
    size_t np = 0;
    std::vector<int> last;
    std::vector<i64> val[2], cnt[2];  // [0] least, [1] largest completion amount; index a << M | U

    // needed pairs: the identity (index 0) only starts an order, and no later
    // decomposition ends with the identity's last axis
    static std::vector<std::pair<int, int>> pairs(int M, const std::vector<std::vector<int8_t>> &perms)
    {
        std::vector<std::pair<int, int>> out;
        for (size_t a = 0; a < perms.size(); ++a) {
            if (a != 0 && perms[a][M - 1] == M - 1) continue;
            for (size_t b = 1; b < perms.size(); ++b)
                if (perms[b][M - 1] != M - 1 && perms[b][M - 1] != perms[a][M - 1]) out.push_back({(int)a, (int)b});
        }
        return out;
    }

    void run(int M_, const std::vector<std::vector<int8_t>> &perms, PairTable &tab)
    {
        M = M_;
        np = perms.size();
        const int full = (1 << M) - 1;
        last.resize(np);
        for (size_t a = 0; a < np; ++a) last[a] = perms[a][M - 1];
        for (int k = 0; k < 2; ++k) {
            val[k].assign(np << M, -1);
            cnt[k].assign(np << M, 0);
        }
        // masks with more bits first: every completion refers to a larger mask
        std::vector<int> masks;
        for (int U = 1; U <= full; ++U)
            if (U & (1 << (M - 1))) masks.push_back(U);
        std::sort(masks.begin(), masks.end(),
                  [](int x, int y) { return __builtin_popcount(x) > __builtin_popcount(y); });
        for (int U : masks) {
            for (size_t a = 0; a < np; ++a) {
                if (!(U & (1 << last[a]))) continue;
                if (last[a] == M - 1 && (a != 0 || U != (1 << (M - 1)))) continue;
                const size_t s = (a << M) | (size_t)U;
                if (U == full) {
                    for (int k = 0; k < 2; ++k) {
                        val[k][s] = 0;
                        cnt[k][s] = 1;
                    }
                    continue;
                }
                for (size_t b = 0; b < np; ++b) {
                    if (U & (1 << last[b])) continue;
                    const size_t nx = (b << M) | (size_t)(U | (1 << last[b]));
                    const i64 v = tab.get((int)a, (int)b) + val[0][nx];
                    const i64 w = tab.get((int)a, (int)b) + val[1][nx];
                    if (val[0][s] < 0 || v < val[0][s]) {
                        val[0][s] = v;
                        cnt[0][s] = cnt[0][nx];
                    } else if (v == val[0][s]) {
                        cnt[0][s] += cnt[0][nx];
                    }
                    if (val[1][s] < 0 || w > val[1][s]) {
                        val[1][s] = w;
                        cnt[1][s] = cnt[1][nx];
                    } else if (w == val[1][s]) {
                        cnt[1][s] += cnt[1][nx];
                    }
                }
            }
        }
    }

    // the lowest-index order attaining optimum k, as permutation indices
    std::vector<int> walk(int k, PairTable &tab) const
    {
        std::vector<int> seq{0};
        int U = 1 << (M - 1);
        size_t a = 0;
        for (int t = 1; t < M; ++t) {
            const i64 want = val[k][(a << M) | (size_t)U];
            for (size_t b = 0; b < np; ++b) {
                if (U & (1 << last[b])) continue;
                const size_t nx = (b << M) | (size_t)(U | (1 << last[b]));
                if (tab.get((int)a, (int)b) + val[k][nx] == want) {
                    seq.push_back((int)b);
                    U |= 1 << last[b];
                    a = b;
                    break;
                }
            }
        }
        return seq;
    }
    i64 optimum(int k) const { return val[k][(size_t)1 << (M - 1)]; }
    i64 ties(int k) const { return cnt[k][(size_t)1 << (M - 1)]; }
};

}  // namespace

extern "C" {

const char *fft_last_error(void) { return g_last_error.c_str(); }

const char *fft_version(void) { return "fftrw 0.2.0 (gfx950)"; }

int fft_decomp(int M, const int64_t *dims, int64_t P, const int8_t *perm, int64_t myid, int *level,
               int64_t *xs, int64_t *xe, int64_t *start, int64_t *end)
{
    g_last_error.clear();
    if (!level || !xs || !xe) return fail(FFTRW_E_ARG, "level, xs and xe must not be null");
    Layout L;
    Status s = make_layout(M, dims, P, perm, &L);
    if (!s) return fail(s);
    if (myid < 0 || myid >= P) return fail(FFTRW_E_ARG, "myid must be in [0, P)");
    *level = L.k;
    range_of(L, myid, xs, xe, start, end);
    return FFTRW_OK;
}

int fft_comm_volume(int M, const int64_t *dims, int64_t P, const int8_t *order, int ownership,
                    int64_t *per_step, int64_t *total, int64_t *return_volume)
{
    g_last_error.clear();
    if (!total) return fail(FFTRW_E_ARG, "total must not be null");
    Status s = check_dims(M, dims);
    if (!s) return fail(s);
    s = check_order(M, order);
    if (!s) return fail(s);
    if (ownership != FFTRW_OWN_LITERAL && ownership != FFTRW_OWN_MATCHED)
        return fail(FFTRW_E_ARG, "unknown ownership reading");
    std::vector<Layout> L(M + 1);
    bool split = false;
    for (int t = 0; t < M; ++t) {
        s = make_layout(M, dims, P, order + t * M, &L[t]);
        if (!s) return fail(s);
        split = split || L[t].row_split();
    }
    int8_t ident[kMaxHostDims];
    for (int i = 0; i < M; ++i) ident[i] = (int8_t)i;
    s = make_layout(M, dims, P, ident, &L[M]);
    if (!s) return fail(s);
    i64 sum = 0;
    for (int t = 0; t + 1 < M; ++t) {
        i64 v = 0;
        s = transpose_amount(L[t], L[t + 1], ownership, &v, nullptr);
        if (!s) return fail(s);
        if (per_step) per_step[t] = v;
        sum += v;
    }
    *total = sum;
    if (return_volume) {
        i64 v = 0;
        s = transpose_amount(L[M - 1], L[M], ownership, &v, nullptr);
        if (!s) return fail(s);
        *return_volume = v;
    }
    if (split) return fail(FFTRW_E_ROWSPLIT, "some step splits rows along its FFT axis (level M)");
    return FFTRW_OK;
}

int fft_rowsplit_volume(int M, const int64_t *dims, int64_t P, const int8_t *order, int64_t *per_step,
                        int64_t *total)
{
    g_last_error.clear();
    if (!total) return fail(FFTRW_E_ARG, "total must not be null");
    Status s = check_dims(M, dims);
    if (!s) return fail(s);
    s = check_order(M, order);
    if (!s) return fail(s);
    // stages of a binary exchange over c processes: ceil(log2 c)
    auto stages = [](i64 c) {
        int n = 0;
        while (((i64)1 << n) < c) ++n;
        return (i64)n;
    };
    i64 sum = 0;
    for (int t = 0; t < M; ++t) {
        Layout L;
        s = make_layout(M, dims, P, order + t * M, &L);
        if (!s) return fail(s);
        i64 v = 0;
        if (L.row_split()) {
            // a row of the FFT axis holds 1 + (boundaries strictly inside it)
            // processes: walk the process boundaries, not the rows
            const i64 N = L.pd[M - 1];
            i64 row = -1, inside = 0;
            for (i64 p = 1; p < P; ++p) {
                const i64 b = L.boundary(p);
                if (b % N == 0) continue;
                if (b / N != row) {
                    if (row >= 0) v += N * stages(inside + 1);
                    row = b / N;
                    inside = 0;
                }
                ++inside;
            }
            if (row >= 0) v += N * stages(inside + 1);
        }
        if (per_step) per_step[t] = v;
        sum += v;
    }
    *total = sum;
    return FFTRW_OK;
}

int fft_pair_counts(int M, const int64_t *dims, int64_t P, const int8_t *perm_a, const int8_t *perm_b,
                    int64_t *C)
{
    g_last_error.clear();
    if (!C) return fail(FFTRW_E_ARG, "C must not be null");
    if (P > 4096) return fail(FFTRW_E_ARG, "P too large for a dense matrix");
    Layout a, b;
    Status s = make_layout(M, dims, P, perm_a, &a);
    if (!s) return fail(s);
    s = make_layout(M, dims, P, perm_b, &b);
    if (!s) return fail(s);
    std::memset(C, 0, sizeof(int64_t) * (size_t)(P * P));
    for (const PairCount &e : pair_counts(a, b)) C[e.p * P + e.q] = e.n;
    return FFTRW_OK;
}

int64_t fft_order_count(int M) { return order_count(M); }

int fft_order_at(int M, int64_t index, int8_t *order)
{
    g_last_error.clear();
    Status s = order_at(M, index, order);
    return s ? FFTRW_OK : fail(s);
}

int fft_order_index(int M, const int8_t *order, int64_t *index)
{
    g_last_error.clear();
    if (!index) return fail(FFTRW_E_ARG, "index must not be null");
    Status s = order_index(M, order, index);
    return s ? FFTRW_OK : fail(s);
}

int fft_order_volumes(int M, const int64_t *dims, int64_t P, int ownership, int64_t *volumes)
{
    g_last_error.clear();
    if (!volumes) return fail(FFTRW_E_ARG, "volumes must not be null");
    Status s = check_dims(M, dims);
    if (!s) return fail(s);
    if (M > 5) return fail(FFTRW_E_UNSUPPORTED, "one amount per order needs M <= 5 (use fft_order_search)");
    if (ownership != FFTRW_OWN_LITERAL && ownership != FFTRW_OWN_MATCHED)
        return fail(FFTRW_E_ARG, "unknown ownership reading");
    auto perms = all_perms(M);
    PairTable tab(M, dims, P, ownership, perms);
    if (!tab.status) return fail(tab.status);
    enumerate_orders(M, perms, [&](i64 n, const int *idx) {
        i64 v = 0;
        for (int t = 0; t + 1 < M; ++t) v += tab.get(idx[t], idx[t + 1]);
        volumes[n] = v;
    });
    if (!tab.status) return fail(tab.status);
    return FFTRW_OK;
}

int fft_transpose_volumes(int M, const int64_t *dims, int64_t P, int ownership, int64_t *table)
{
    g_last_error.clear();
    if (!table) return fail(FFTRW_E_ARG, "table must not be null");
    Status s = check_dims(M, dims);
    if (!s) return fail(s);
    if (ownership != FFTRW_OWN_LITERAL && ownership != FFTRW_OWN_MATCHED)
        return fail(FFTRW_E_ARG, "unknown ownership reading");
    auto perms = all_perms(M);
    PairTable tab(M, dims, P, ownership, perms);
    if (!tab.status) return fail(tab.status);
    tab.fill(OrderSearch::pairs(M, perms));
    if (!tab.status) return fail(tab.status);
    std::memcpy(table, tab.vol.data(), sizeof(int64_t) * tab.vol.size());
    return FFTRW_OK;
}

int fft_order_search(int M, const int64_t *dims, int64_t P, int ownership, int64_t *best_index,
                     int64_t *best_volume, int64_t *n_best, int64_t *worst_index, int64_t *worst_volume,
                     int64_t *n_worst, int8_t *best_order, int8_t *worst_order)
{
    g_last_error.clear();
    Status s = check_dims(M, dims);
    if (!s) return fail(s);
    if (ownership != FFTRW_OWN_LITERAL && ownership != FFTRW_OWN_MATCHED)
        return fail(FFTRW_E_ARG, "unknown ownership reading");
    auto perms = all_perms(M);
    PairTable tab(M, dims, P, ownership, perms);
    if (!tab.status) return fail(tab.status);
    tab.fill(OrderSearch::pairs(M, perms));
    if (!tab.status) return fail(tab.status);
    OrderSearch dp;
    dp.run(M, perms, tab);
    log_line(2, "order search M=%d P=%lld ownership=%d: least %lld (%lld orders), largest %lld (%lld orders)", M,
             (long long)P, ownership, (long long)dp.optimum(0), (long long)dp.ties(0), (long long)dp.optimum(1),
             (long long)dp.ties(1));
    int8_t ord[kMaxHostDims * kMaxHostDims];
    for (int k = 0; k < 2; ++k) {
        const std::vector<int> seq = dp.walk(k, tab);
        for (int t = 0; t < M; ++t) std::memcpy(ord + t * M, perms[seq[t]].data(), (size_t)M);
        i64 idx = 0;
        s = order_index(M, ord, &idx);
        if (!s) return fail(s);
        if (k == 0) {
            if (best_index) *best_index = idx;
            if (best_volume) *best_volume = dp.optimum(0);
            if (n_best) *n_best = dp.ties(0);
            if (best_order) std::memcpy(best_order, ord, (size_t)(M * M));
        } else {
            if (worst_index) *worst_index = idx;
            if (worst_volume) *worst_volume = dp.optimum(1);
            if (n_worst) *n_worst = dp.ties(1);
            if (worst_order) std::memcpy(worst_order, ord, (size_t)(M * M));
        }
    }
    return FFTRW_OK;
}

int fft_compare_models(double N, double P, double *out)
{
    g_last_error.clear();
    if (!out || !(N > 0) || !(P > 0)) return fail(FFTRW_E_ARG, "N and P must be positive, out non-null");
    // Eqs. (21)-(25), as printed
    out[0] = std::pow(N, 3) - std::pow(N, 3) / P;
    out[1] = 2 * std::pow(N, 3) - 2 * P * std::pow(N * N / P, 1.5);
    out[2] = 3 * std::pow(N, 3) * (N / std::cbrt(std::pow(N, 3) / P) - 1);
    out[3] = 4 * std::pow(N, 4) * (N / std::pow(std::pow(N, 4) / P, 0.25) - 1);
    out[4] = 5 * std::pow(N, 5) * (N / std::pow(std::pow(N, 5) / P, 0.2) - 1);
    return FFTRW_OK;
}

}  // extern "C"
