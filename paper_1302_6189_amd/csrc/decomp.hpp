// decomp.hpp -- host-side integer model of the row-wise adaptive decomposition
// (Duy & Ozaki, Section 3: Eqs. (12)-(19)), transpose orders (Eq. (20)) and
// communication amounts.  Pure C++17, no HIP dependency.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace fftrw {

using i64 = int64_t;
constexpr int kMaxDims = 5;      // plans and kernels: M = 2..5
constexpr int kMaxHostDims = 6;  // host model (ranges, amounts, orders): M = 2..6

struct Status {
    int code = 0;
    std::string msg;
    static Status ok() { return {}; }
    static Status err(int c, std::string m) { return Status{c, std::move(m)}; }
    explicit operator bool() const { return code == 0; }
};

// One decomposition pi: the array viewed in axis order perm (slowest first),
// split over P processes on the first k axes (Eq. (13)).
struct Layout {
    int M = 0;
    int perm[kMaxHostDims] = {};  // natural axis at each position
    int pos[kMaxHostDims] = {};   // position of each natural axis
    i64 pd[kMaxHostDims] = {};    // permuted sizes N'_i
    i64 stride[kMaxHostDims] = {};// element stride of each *natural* axis in this layout
    int k = 0;                // level, 1-based
    i64 R = 0;                // rows over the first k axes
    i64 W = 0;                // points per row (product of the other axes)
    i64 P = 0;
    i64 T = 0;

    // first row of process p: floor(R p / P)  (Eq. (13) before the * W)
    i64 row_lo(i64 p) const { return (i64)(((__int128)R * p) / P); }
    // x^s of Eq. (14)
    i64 boundary(i64 p) const { return row_lo(p) * W; }
    // the process whose rows contain row r
    i64 owner_of_row(i64 r) const { return (i64)((((__int128)r + 1) * P - 1) / R); }
    bool row_split() const { return k >= M; }
};

// Axis-aligned box in natural coordinates, inclusive bounds.
struct Box {
    i64 lo[kMaxHostDims];
    i64 hi[kMaxHostDims];
};

i64 box_volume(const Box &b, int M);
i64 box_overlap(const Box &a, const Box &b, int M);
bool box_intersect(const Box &a, const Box &b, int M, Box *out);

Status check_dims(int M, const i64 *dims);
Status check_perm(int M, const int8_t *perm);
Status check_order(int M, const int8_t *order);
Status make_layout(int M, const i64 *dims, i64 P, const int8_t *perm, Layout *out);

// Eqs. (14)-(19) for one process.
void range_of(const Layout &L, i64 p, i64 *xs, i64 *xe, i64 *start, i64 *end);

// The points of process p in L as <= 2k-1 disjoint boxes, in increasing order
// of their 1-D index in L.
std::vector<Box> range_boxes(const Layout &L, i64 p);

// Points kept by the same process id across a -> b (literal reading).
i64 kept_literal(const Layout &a, const Layout &b);

// Visit every process q of layout b whose range meets box B; f(q) is called
// once per q in increasing q.
template <class F>
void for_each_owner(const Layout &b, const Box &B, F &&f);

// Sparse overlap list: for every process p of a, the processes q of b it
// shares points with and how many (sorted by p, then q).
struct PairCount {
    i64 p, q, n;
};
std::vector<PairCount> pair_counts(const Layout &a, const Layout &b);

// Maximum-weight perfect matching on a P x P overlap given sparsely; returns
// the matched weight and mu[p] = q.  Exact (shortest augmenting paths over
// the sparse overlap graph, one connected component at a time).
Status max_matching(i64 P, const std::vector<PairCount> &pc, i64 *weight, std::vector<i64> *mu);

// Transpose a -> b amount under ownership 0 (literal) / 1 (matched);
// mu (nullable) receives the relabelling (identity for literal).
Status transpose_amount(const Layout &a, const Layout &b, int ownership, i64 *moved,
                        std::vector<i64> *mu);

// ---- orders -----------------------------------------------------------------
i64 order_count(int M);
Status order_at(int M, i64 index, int8_t *order);
Status order_index(int M, const int8_t *order, i64 *index);

// All M! permutations in lexicographic order.
std::vector<std::vector<int8_t>> all_perms(int M);

}  // namespace fftrw

// ---- template implementation ---------------------------------------------
namespace fftrw {

// Smallest element >= v of the product set {sum_i y_i w_i : l_i <= y_i <= h_i}
// (mixed radix n[], most significant first).  Returns false if none.
bool product_set_successor(int k, const i64 *l, const i64 *h, const i64 *n, i64 v, i64 *out);

template <class F>
void for_each_owner(const Layout &b, const Box &B, F &&f)
{
    const int k = b.k;
    i64 l[kMaxHostDims], h[kMaxHostDims], n[kMaxHostDims];
    for (int i = 0; i < k; ++i) {
        int ax = b.perm[i];
        l[i] = B.lo[ax];
        h[i] = B.hi[ax];
        n[i] = b.pd[i];
    }
    i64 s;
    if (!product_set_successor(k, l, h, n, 0, &s)) return;
    while (true) {
        i64 q = b.owner_of_row(s);
        f(q);
        i64 next = b.row_lo(q + 1);
        if (next >= b.R) break;
        if (!product_set_successor(k, l, h, n, next, &s)) break;
    }
}

}  // namespace fftrw
