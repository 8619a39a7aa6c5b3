// decomp.cpp -- host integer model of the row-wise adaptive decomposition.
//
// Section 3 of Duy & Ozaki: each process owns the contiguous 1-D range
// [f(myid), f(myid+1) - 1] of Eqs. (13)-(15) in the current axis order; a
// transpose re-decomposes in the next order.  The amount of a transpose is
// the number of points whose owner changes.  Here it is counted analytically:
// a process's range is a union of at most 2k-1 axis-aligned boxes, so the
// kept points are box intersections instead of a walk over every point.
#include "decomp.hpp"

#include <algorithm>
#include <cstring>
#include <limits>
#include <numeric>
#include <queue>

namespace fftrw {

i64 box_volume(const Box &b, int M)
{
    i64 v = 1;
    for (int d = 0; d < M; ++d) {
        if (b.hi[d] < b.lo[d]) return 0;
        v *= b.hi[d] - b.lo[d] + 1;
    }
    return v;
}

bool box_intersect(const Box &a, const Box &b, int M, Box *out)
{
    for (int d = 0; d < M; ++d) {
        i64 lo = std::max(a.lo[d], b.lo[d]);
        i64 hi = std::min(a.hi[d], b.hi[d]);
        if (hi < lo) return false;
        if (out) {
            out->lo[d] = lo;
            out->hi[d] = hi;
        }
    }
    return true;
}

i64 box_overlap(const Box &a, const Box &b, int M)
{
    i64 v = 1;
    for (int d = 0; d < M; ++d) {
        i64 lo = std::max(a.lo[d], b.lo[d]);
        i64 hi = std::min(a.hi[d], b.hi[d]);
        if (hi < lo) return 0;
        v *= hi - lo + 1;
    }
    return v;
}

Status check_dims(int M, const i64 *dims)
{
    if (M < 2 || M > kMaxHostDims) return Status::err(-2, "M must be in [2, 6]");
    if (!dims) return Status::err(-1, "dims is null");
    __int128 T = 1;
    for (int d = 0; d < M; ++d) {
        if (dims[d] < 1) return Status::err(-2, "every size must be >= 1");
        T *= dims[d];
        if (T > ((__int128)1 << 62)) return Status::err(-2, "too many points");
    }
    return Status::ok();
}

Status check_perm(int M, const int8_t *perm)
{
    if (!perm) return Status::err(-1, "permutation is null");
    bool seen[kMaxHostDims] = {};
    for (int i = 0; i < M; ++i) {
        int a = perm[i];
        if (a < 0 || a >= M || seen[a]) return Status::err(-3, "not a permutation of the axes");
        seen[a] = true;
    }
    return Status::ok();
}

Status check_order(int M, const int8_t *order)
{
    if (!order) return Status::err(-1, "order is null");
    for (int i = 0; i < M; ++i)
        if (order[i] != i) return Status::err(-3, "the first decomposition must be the natural order");
    bool last_used[kMaxHostDims] = {};
    for (int t = 0; t < M; ++t) {
        Status s = check_perm(M, order + t * M);
        if (!s) return s;
        int last = order[t * M + M - 1];
        if (last_used[last]) return Status::err(-3, "two steps transform the same axis");
        last_used[last] = true;
    }
    return Status::ok();
}

Status make_layout(int M, const i64 *dims, i64 P, const int8_t *perm, Layout *out)
{
    Status s = check_dims(M, dims);
    if (!s) return s;
    s = check_perm(M, perm);
    if (!s) return s;
    if (P < 1) return Status::err(-1, "P must be >= 1");
    Layout L;
    L.M = M;
    L.P = P;
    L.T = 1;
    for (int i = 0; i < M; ++i) {
        L.perm[i] = perm[i];
        L.pos[perm[i]] = i;
        L.pd[i] = dims[perm[i]];
        L.T *= L.pd[i];
    }
    if (P > L.T) return Status::err(-4, "P exceeds the number of points");
    i64 acc = 1;
    L.k = 0;
    for (int i = 0; i < M; ++i) {
        acc *= L.pd[i];
        if (P <= acc) {
            L.k = i + 1;
            L.R = acc;
            break;
        }
    }
    L.W = L.T / L.R;
    i64 st = 1;
    for (int i = M - 1; i >= 0; --i) {
        L.stride[L.perm[i]] = st;
        st *= L.pd[i];
    }
    *out = L;
    return Status::ok();
}

void range_of(const Layout &L, i64 p, i64 *xs, i64 *xe, i64 *start, i64 *end)
{
    i64 s = L.boundary(p);
    i64 e = L.boundary(p + 1) - 1;
    if (xs) *xs = s;
    if (xe) *xe = e;
    // Eqs. (16)-(19): successive floor divisions in the permuted order
    auto split = [&](i64 x, i64 *c) {
        if (!c) return;
        i64 w = L.T;
        for (int r = 0; r < L.M; ++r) {
            w /= L.pd[r];
            c[r] = x / w;
            x -= c[r] * w;
        }
    };
    split(s, start);
    split(e, end);
}

namespace {

// Emit boxes covering rows [a, b] (lexicographic over positions d..k-1 of the
// permuted order; positions < d already fixed in `cur`).
void row_boxes(const Layout &L, int d, i64 a, i64 b, Box cur, std::vector<Box> &out)
{
    if (a > b) return;
    const int k = L.k;
    const int ax = L.perm[d];
    if (d == k - 1) {
        cur.lo[ax] = a;
        cur.hi[ax] = b;
        out.push_back(cur);
        return;
    }
    i64 stride = 1;
    for (int i = d + 1; i < k; ++i) stride *= L.pd[i];
    i64 a0 = a / stride, ar = a % stride;
    i64 b0 = b / stride, br = b % stride;
    if (a0 == b0) {
        cur.lo[ax] = cur.hi[ax] = a0;
        row_boxes(L, d + 1, ar, br, cur, out);
        return;
    }
    if (ar != 0) {
        Box h = cur;
        h.lo[ax] = h.hi[ax] = a0;
        row_boxes(L, d + 1, ar, stride - 1, h, out);
        ++a0;
    }
    bool tail = br != stride - 1;
    i64 mid_hi = tail ? b0 - 1 : b0;
    if (a0 <= mid_hi) {
        Box m = cur;
        m.lo[ax] = a0;
        m.hi[ax] = mid_hi;
        for (int i = d + 1; i < k; ++i) {
            m.lo[L.perm[i]] = 0;
            m.hi[L.perm[i]] = L.pd[i] - 1;
        }
        out.push_back(m);
    }
    if (tail) {
        Box t = cur;
        t.lo[ax] = t.hi[ax] = b0;
        row_boxes(L, d + 1, 0, br, t, out);
    }
}

}  // namespace

std::vector<Box> range_boxes(const Layout &L, i64 p)
{
    std::vector<Box> out;
    Box cur;
    for (int i = 0; i < L.M; ++i) {
        cur.lo[L.perm[i]] = 0;
        cur.hi[L.perm[i]] = L.pd[i] - 1;
    }
    i64 r0 = L.row_lo(p), r1 = L.row_lo(p + 1) - 1;
    row_boxes(L, 0, r0, r1, cur, out);
    return out;
}

i64 kept_literal(const Layout &a, const Layout &b)
{
    i64 kept = 0;
    for (i64 p = 0; p < a.P; ++p) {
        std::vector<Box> ba = range_boxes(a, p);
        std::vector<Box> bb = range_boxes(b, p);
        for (const Box &x : ba)
            for (const Box &y : bb) kept += box_overlap(x, y, a.M);
    }
    return kept;
}

bool product_set_successor(int k, const i64 *l, const i64 *h, const i64 *n, i64 v, i64 *out)
{
    i64 w[kMaxHostDims];
    w[k - 1] = 1;
    for (int i = k - 2; i >= 0; --i) w[i] = w[i + 1] * n[i + 1];
    if (v >= w[0] * n[0]) return false;
    i64 d[kMaxHostDims];
    i64 rem = v;
    for (int i = 0; i < k; ++i) {
        d[i] = rem / w[i];
        rem -= d[i] * w[i];
    }
    for (int i = 0; i < k; ++i) {
        if (d[i] < l[i]) {
            for (int j = i; j < k; ++j) d[j] = l[j];
            break;
        }
        if (d[i] > h[i]) {
            int j = i - 1;
            while (j >= 0 && d[j] >= h[j]) --j;
            if (j < 0) return false;
            d[j] += 1;
            for (int m = j + 1; m < k; ++m) d[m] = l[m];
            break;
        }
    }
    i64 s = 0;
    for (int i = 0; i < k; ++i) s += d[i] * w[i];
    *out = s;
    return true;
}

std::vector<PairCount> pair_counts(const Layout &a, const Layout &b)
{
    std::vector<PairCount> out;
    std::vector<std::pair<i64, i64>> acc;
    // every destination's boxes, computed once
    std::vector<Box> qbox;
    std::vector<i64> qfirst(b.P + 1, 0);
    for (i64 q = 0; q < b.P; ++q) {
        qfirst[q] = (i64)qbox.size();
        for (const Box &C : range_boxes(b, q)) qbox.push_back(C);
    }
    qfirst[b.P] = (i64)qbox.size();
    for (i64 p = 0; p < a.P; ++p) {
        acc.clear();
        for (const Box &B : range_boxes(a, p)) {
            for_each_owner(b, B, [&](i64 q) {
                i64 n = 0;
                for (i64 j = qfirst[q]; j < qfirst[q + 1]; ++j) n += box_overlap(B, qbox[j], a.M);
                if (n) acc.emplace_back(q, n);
            });
        }
        std::sort(acc.begin(), acc.end());
        for (size_t i = 0; i < acc.size();) {
            i64 q = acc[i].first, n = 0;
            while (i < acc.size() && acc[i].first == q) n += acc[i++].second;
            out.push_back({p, q, n});
        }
    }
    return out;
}

namespace {

// Maximum-weight bipartite matching on a sparse graph, exactly: rows
// 0..nr-1, columns 0..nc-1, adj[i] = (column, weight > 0).  Written as a
// rectangular assignment of every row, either to a real column at cost
// W - w or to a private "unmatched" column at cost W (W = the largest
// weight), so all costs are non-negative and the minimum cost is
// nr W - (the maximum matched weight).  Rows are assigned one at a time by a
// shortest augmenting path: Dijkstra over reduced costs c + phi(row) -
// phi(col) (never negative), through matched edges back to their rows, until
// a free column is reached; the potentials of the scanned nodes then move by
// their distance less the path's, which keeps every reduced cost
// non-negative and the matched edges tight.  A row reduction first makes
// each row's cheapest edge tight and matches the rows whose cheapest column
// is free, so only the contested rows search.  Integer costs throughout, and
// the search stays near the row, so a banded overlap graph of any size
// costs about its number of edges per row.  Returns col_of_row (-1 if the
// row stays unmatched).
std::vector<i64> sparse_max_matching(i64 nr, i64 nc, const std::vector<std::vector<std::pair<i64, i64>>> &adj)
{
    i64 W = 1;
    for (const auto &a : adj)
        for (const auto &e : a) W = std::max(W, e.second);
    const i64 INF = std::numeric_limits<i64>::max() / 4;
    const i64 ncol = nc + nr;  // real columns, then row i's private column nc + i
    std::vector<i64> phi_r(nr, 0), phi_c(ncol, 0);
    std::vector<i64> row_of(ncol, -1), col_of(nr, -1);
    std::vector<i64> dist(ncol, INF), pred(ncol, -1);
    std::vector<char> done(ncol, 0);
    std::vector<i64> touched;
    using QE = std::pair<i64, i64>;
    std::priority_queue<QE, std::vector<QE>, std::greater<QE>> pq;
    auto relax = [&](i64 i, i64 di) {
        // edges of row i leaving to columns other than its own matched one
        auto edge = [&](i64 k, i64 c) {
            if (done[k] || k == col_of[i]) return;
            const i64 nd = di + c + phi_r[i] - phi_c[k];
            if (nd < dist[k]) {
                if (dist[k] == INF) touched.push_back(k);
                dist[k] = nd;
                pred[k] = i;
                pq.push({nd, k});
            }
        };
        for (const auto &e : adj[(size_t)i]) edge(e.first, W - e.second);
        edge(nc + i, W);
    };
    // row reduction: phi(row) = -(its cheapest cost) makes that edge tight;
    // rows whose cheapest column is still free take it at once
    for (i64 i = 0; i < nr; ++i) {
        i64 best = W, bk = nc + i;
        for (const auto &e : adj[(size_t)i])
            if (W - e.second < best || (W - e.second == best && e.first < bk)) {
                best = W - e.second;
                bk = e.first;
            }
        phi_r[i] = -best;
        if (row_of[bk] < 0) {
            row_of[bk] = i;
            col_of[i] = bk;
        }
    }
    std::vector<i64> rows_seen;
    for (i64 s = 0; s < nr; ++s) {
        if (col_of[s] >= 0) continue;
        touched.clear();
        rows_seen.assign(1, s);
        std::vector<i64> drow(1, 0);
        relax(s, 0);
        i64 sink = -1, D = 0;
        std::vector<i64> scanned;
        while (!pq.empty()) {
            const auto [d, k] = pq.top();
            pq.pop();
            if (done[k] || d != dist[k]) continue;
            done[k] = 1;
            scanned.push_back(k);
            if (row_of[k] < 0) {
                sink = k;
                D = d;
                break;
            }
            const i64 i = row_of[k];  // the matched edge back is tight: distance d
            rows_seen.push_back(i);
            drow.push_back(d);
            relax(i, d);
        }
        while (!pq.empty()) pq.pop();
        // potentials: scanned nodes move by (distance - D), the rest by 0
        // (a common shift of every node leaves reduced costs unchanged)
        for (i64 k : scanned) phi_c[k] += dist[k] - D;
        for (size_t t = 0; t < rows_seen.size(); ++t) phi_r[rows_seen[t]] += drow[t] - D;
        // augment along the predecessors from the sink back to s
        for (i64 k = sink; k >= 0;) {
            const i64 i = pred[k];
            const i64 prev = col_of[i];
            col_of[i] = k;
            row_of[k] = i;
            k = (i == s) ? -1 : prev;
        }
        for (i64 k : touched) {
            dist[k] = INF;
            done[k] = 0;
            pred[k] = -1;
        }
    }
    std::vector<i64> out(nr, -1);
    for (i64 i = 0; i < nr; ++i) out[i] = col_of[i] < nc ? col_of[i] : -1;
    return out;
}

struct DSU {
    std::vector<i64> par;
    explicit DSU(i64 n) : par(n) { std::iota(par.begin(), par.end(), 0); }
    i64 find(i64 x)
    {
        while (par[x] != x) x = par[x] = par[par[x]];
        return x;
    }
    void unite(i64 a, i64 b) { par[find(a)] = find(b); }
};

}  // namespace

Status max_matching(i64 P, const std::vector<PairCount> &pc, i64 *weight, std::vector<i64> *mu)
{
    // Components of the bipartite overlap graph (rows 0..P-1, columns P..2P-1)
    // are matched independently; nodes left over are paired by zero-weight
    // entries, which does not change the optimum.
    DSU dsu(2 * P);
    for (const PairCount &e : pc) dsu.unite(e.p, P + e.q);
    std::vector<std::vector<i64>> rows_of(2 * P), cols_of(2 * P);
    for (i64 p = 0; p < P; ++p) rows_of[dsu.find(p)].push_back(p);
    for (i64 q = 0; q < P; ++q) cols_of[dsu.find(P + q)].push_back(q);
    std::vector<std::vector<PairCount>> edges_of(2 * P);
    for (const PairCount &e : pc) edges_of[dsu.find(e.p)].push_back(e);

    std::vector<i64> m(P, -1);
    std::vector<char> col_taken(P, 0);
    std::vector<i64> ridx(P, -1), cidx(P, -1);
    i64 total = 0;
    for (i64 c = 0; c < 2 * P; ++c) {
        if (edges_of[c].empty()) continue;
        const auto &R = rows_of[c];
        const auto &C = cols_of[c];
        for (size_t i = 0; i < R.size(); ++i) ridx[R[i]] = (i64)i;
        for (size_t j = 0; j < C.size(); ++j) cidx[C[j]] = (i64)j;
        std::vector<std::vector<std::pair<i64, i64>>> adj(R.size());
        for (const PairCount &e : edges_of[c]) adj[(size_t)ridx[e.p]].push_back({cidx[e.q], e.n});
        const std::vector<i64> col = sparse_max_matching((i64)R.size(), (i64)C.size(), adj);
        for (size_t i = 0; i < R.size(); ++i) {
            const i64 j = col[i];
            if (j < 0) continue;
            for (const auto &e : adj[i])
                if (e.first == j) {
                    m[R[i]] = C[(size_t)j];
                    col_taken[(size_t)C[(size_t)j]] = 1;
                    total += e.second;
                }
        }
    }
    // complete the permutation with the remaining (zero-overlap) pairs
    i64 next_free = 0;
    for (i64 p = 0; p < P; ++p) {
        if (m[p] >= 0) continue;
        // prefer keeping the same label when it is free
        if (!col_taken[p]) {
            m[p] = p;
            col_taken[p] = 1;
        }
    }
    for (i64 p = 0; p < P; ++p) {
        if (m[p] >= 0) continue;
        while (col_taken[next_free]) ++next_free;
        m[p] = next_free;
        col_taken[next_free] = 1;
    }
    if (weight) *weight = total;
    if (mu) *mu = std::move(m);
    return Status::ok();
}

Status transpose_amount(const Layout &a, const Layout &b, int ownership, i64 *moved,
                        std::vector<i64> *mu)
{
    if (ownership == 0) {
        *moved = a.T - kept_literal(a, b);
        if (mu) {
            mu->resize(a.P);
            std::iota(mu->begin(), mu->end(), 0);
        }
        return Status::ok();
    }
    if (ownership != 1) return Status::err(-1, "unknown ownership reading");
    i64 w = 0;
    Status s = max_matching(a.P, pair_counts(a, b), &w, mu);
    if (!s) return s;
    *moved = a.T - w;
    return Status::ok();
}

// ---- orders -------------------------------------------------------------------

std::vector<std::vector<int8_t>> all_perms(int M)
{
    std::vector<int8_t> p(M);
    for (int i = 0; i < M; ++i) p[i] = (int8_t)i;
    std::vector<std::vector<int8_t>> out;
    do {
        out.push_back(p);
    } while (std::next_permutation(p.begin(), p.end()));
    return out;
}

i64 order_count(int M)
{
    if (M < 2 || M > 6) return -1;
    i64 f = 1;
    for (int i = 2; i < M; ++i) f *= i;  // (M-1)!
    i64 c = 1;
    for (int i = 0; i < M; ++i) c *= f;
    return c;
}

namespace {

// number of valid choices at stage s (0-based; stage 0 is the identity)
i64 stage_choices(int M, int s)
{
    if (s == 0) return 1;
    i64 f = 1;
    for (int i = 2; i < M; ++i) f *= i;
    return (i64)(M - s) * f;
}

}  // namespace

Status order_at(int M, i64 index, int8_t *order)
{
    if (M < 2 || M > kMaxHostDims) return Status::err(-2, "M must be in [2, 6]");
    if (!order) return Status::err(-1, "order is null");
    i64 n = order_count(M);
    if (index < 0 || index >= n) return Status::err(-1, "order index out of range");
    auto perms = all_perms(M);
    bool used[kMaxHostDims] = {};
    for (int i = 0; i < M; ++i) order[i] = (int8_t)i;
    used[M - 1] = true;
    i64 rest = index;
    for (int s = 1; s < M; ++s) {
        i64 after = 1;
        for (int s2 = s + 1; s2 < M; ++s2) after *= stage_choices(M, s2);
        i64 digit = rest / after;
        rest -= digit * after;
        i64 seen = 0;
        for (const auto &p : perms) {
            if (used[p[M - 1]]) continue;
            if (seen++ == digit) {
                std::memcpy(order + s * M, p.data(), (size_t)M);
                used[p[M - 1]] = true;
                break;
            }
        }
    }
    return Status::ok();
}

Status order_index(int M, const int8_t *order, i64 *index)
{
    Status s = check_order(M, order);
    if (!s) return s;
    auto perms = all_perms(M);
    bool used[kMaxHostDims] = {};
    used[M - 1] = true;
    i64 idx = 0;
    for (int st = 1; st < M; ++st) {
        i64 after = 1;
        for (int s2 = st + 1; s2 < M; ++s2) after *= stage_choices(M, s2);
        i64 digit = 0;
        for (const auto &p : perms) {
            if (used[p[M - 1]]) continue;
            if (std::memcmp(p.data(), order + st * M, (size_t)M) == 0) break;
            ++digit;
        }
        idx += digit * after;
        used[order[st * M + M - 1]] = true;
    }
    *index = idx;
    return Status::ok();
}

}  // namespace fftrw
