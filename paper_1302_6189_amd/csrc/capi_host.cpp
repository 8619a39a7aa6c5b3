// capi_host.cpp -- the host-only half of the C ABI (include/fftrw.h):
// decomposition maps, communication amounts, transpose orders, comparison
// models.  No HIP calls here, so these work on a machine without a GPU.
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/fftrw.h"
#include "decomp.hpp"
#include "errors.hpp"

using namespace fftrw;

namespace fftrw {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
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
    int idx[kMaxDims];
    idx[0] = 0;  // identity is the first permutation in lexicographic order
    bool used[kMaxDims] = {};
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

}  // namespace

extern "C" {

const char *fft_last_error(void) { return g_last_error.c_str(); }

const char *fft_version(void) { return "fftrw 0.1.0 (gfx950)"; }

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
    int8_t ident[kMaxDims];
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
    i64 bi = -1, bv = 0, nb = 0, wi = -1, wv = 0, nw = 0;
    enumerate_orders(M, perms, [&](i64 n, const int *idx) {
        i64 v = 0;
        for (int t = 0; t + 1 < M; ++t) v += tab.get(idx[t], idx[t + 1]);
        if (bi < 0 || v < bv) {
            bi = n;
            bv = v;
            nb = 1;
        } else if (v == bv) {
            ++nb;
        }
        if (wi < 0 || v > wv) {
            wi = n;
            wv = v;
            nw = 1;
        } else if (v == wv) {
            ++nw;
        }
    });
    if (!tab.status) return fail(tab.status);
    if (best_index) *best_index = bi;
    if (best_volume) *best_volume = bv;
    if (n_best) *n_best = nb;
    if (worst_index) *worst_index = wi;
    if (worst_volume) *worst_volume = wv;
    if (n_worst) *n_worst = nw;
    if (best_order) order_at(M, bi, best_order);
    if (worst_order) order_at(M, wi, worst_order);
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
