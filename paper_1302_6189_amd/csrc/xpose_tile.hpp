// xpose_tile.hpp -- one tile of the transpose between two decompositions
// (device code shared by the stand-alone kernel and the persistent batched
// kernel).
//
// The array moves from layout A (decomposition pi_t) to layout B (pi_{t+1}).
// Consecutive decompositions always have different last axes, so the
// permutation is a tiled 2-D transpose between u (fastest axis of A) and v
// (fastest axis of B), batched over the other M-2 axes.  A work-group reads a
// TU x TV tile (times G batch slices) along u, transposes it through LDS and
// writes it along v, so both sides are coalesced; with an even u (v) size a
// thread moves two neighbouring values per 16-byte access.
//
// Owner counting: virtual process p owns a contiguous range of rows over the
// first k axes of its decomposition (Eqs. (13)-(15)).  Below level M the
// first k axes of A never include u and those of B never include v, so along
// a (slice, v) row A's owner is fixed and B's row index grows linearly with u:
// the points that keep their owner are the u whose B row falls in that
// owner's range, an interval.  At level M (more processes than rows, the last
// case of Eq. (13)) the row index is the point's whole linear index, so A's
// owner also grows with u (and B's row index also depends on v); the row then
// splits into pieces of constant A owner, each counted the same way (row_keep).
// The rest of the row moves.  Summed over tiles this is the paper's
// communication amount for the transpose.
#pragma once

#include <hip/hip_runtime.h>

#include "cplx.hpp"
#include "kernels.hpp"

namespace fftrw {

constexpr int kMaxG = 256;
constexpr int kTileBatch = 8;  // rows a thread loads (or stores) before it waits

typedef float xf4 __attribute__((ext_vector_type(4)));
typedef float xf2 __attribute__((ext_vector_type(2)));
typedef double xd2 __attribute__((ext_vector_type(2)));

template <typename C> __device__ __forceinline__ C xld(const C *p)
{
    if constexpr (sizeof(C) == 8) {
        xf2 w = gld_nt(reinterpret_cast<const xf2 *>(p));
        return mk<C>(w.x, w.y);
    } else {
        xd2 w = gld_nt(reinterpret_cast<const xd2 *>(p));
        return mk<C>(w.x, w.y);
    }
}
template <typename C> __device__ __forceinline__ void xst(C *p, C v)
{
    if constexpr (sizeof(C) == 8) {
        xf2 w = {v.x, v.y};
        gst_nt(w, reinterpret_cast<xf2 *>(p));
    } else {
        xd2 w = {v.x, v.y};
        gst_nt(w, reinterpret_cast<xd2 *>(p));
    }
}

__device__ __forceinline__ int64_t owner_of_row(int64_t r, int64_t P, int64_t R, bool narrow)
{
    if (narrow) return (int64_t)(((uint32_t)(r + 1) * (uint32_t)P - 1u) / (uint32_t)R);
    return ((r + 1) * P - 1) / R;
}

// coordinates of batch slice s (innermost batch axis first) and its bases;
// plans keep the slice count below 2^31 (sizes are at most 4096), so 32-bit
// divisions suffice
__device__ __forceinline__ void slice_coords(const XposeDesc &d, int64_t s, int *c, int64_t *ab, int64_t *bb)
{
    int64_t a = 0, b = 0;
    uint32_t su = (uint32_t)s;
    for (int i = 0; i < d.nbat; ++i) {
        const uint32_t n = (uint32_t)d.bsize[i];
        const uint32_t q = su / n;
        const uint32_t ci = su - q * n;
        su = q;
        c[i] = (int)ci;
        a += (int64_t)ci * d.ba[i];
        b += (int64_t)ci * d.bb[i];
    }
    *ab = a;
    *bb = b;
}

// Points of the row (batch coordinates c, v) with u in [u0, u0 + nu) that keep
// their owner.  Both row indices are affine in u: B's grows with u when u is
// one of B's leading axes, A's only at level M.  Owners are monotone in the
// row index, so the row is a sequence of pieces of constant A owner o, and
// inside a piece the u whose B row lies in o's range form an interval.
__device__ __forceinline__ int64_t row_keep(const XposeDesc &d, const int *c, int64_t v, int64_t u0, int64_t nu)
{
    const bool narrow = d.owner32 != 0;
    int64_t ra0 = 0, wau = 0, rb0 = 0, wbu = 0;
    for (int j = 0; j < d.ka; ++j) {
        const int src = d.srca[j];
        if (src == 4)
            wau = d.wa[j];
        else
            ra0 += (src == 3 ? v : (int64_t)c[src]) * d.wa[j];
    }
    for (int j = 0; j < d.kb; ++j) {
        const int src = d.srcb[j];
        if (src == 4)
            wbu = d.wb[j];
        else
            rb0 += (src == 3 ? v : (int64_t)c[src]) * d.wb[j];
    }
    // floor(x / y) for x >= 0, y > 0, and ceil(x / w) for w > 0.  When
    // R P < 2^32 for both layouts (narrow) every operand below is under 2^32,
    // so 32-bit divisions suffice.
    auto fdiv = [narrow](int64_t x, int64_t y) -> int64_t {
        return narrow ? (int64_t)((uint32_t)x / (uint32_t)y) : x / y;
    };
    auto cdiv = [&](int64_t x, int64_t w) -> int64_t {
        if (x < 0) return -fdiv(-x, w);
        const int64_t q = fdiv(x, w);
        return q + (q * w != x ? 1 : 0);
    };
    // u in [a, b) whose B row lies in the range of process o
    auto keep_b = [&](int64_t o, int64_t a, int64_t b) -> int64_t {
        if (wbu == 0) return owner_of_row(rb0, d.P, d.Rb, narrow) == o ? b - a : 0;
        const int64_t lo = fdiv(d.Rb * o, d.P) - rb0, hi = fdiv(d.Rb * (o + 1), d.P) - rb0;
        const int64_t k0 = max<int64_t>(a, cdiv(lo, wbu)), k1 = min<int64_t>(b, cdiv(hi, wbu));
        return max<int64_t>(0, k1 - k0);
    };
    if (wau == 0) {
        int64_t o = owner_of_row(ra0, d.P, d.Ra, narrow);
        if (d.mu) o = d.mu[o];
        return keep_b(o, u0, u0 + nu);
    }
    int64_t keep = 0;
    for (int64_t u = u0, end = u0 + nu; u < end;) {
        const int64_t oa = owner_of_row(ra0 + u * wau, d.P, d.Ra, narrow);
        // first u past this piece: A row reaches the start of range oa + 1
        const int64_t next = min<int64_t>(end, cdiv(fdiv(d.Ra * (oa + 1), d.P) - ra0, wau));
        keep += keep_b(d.mu ? (int64_t)d.mu[oa] : oa, u, next);
        u = next;
    }
    return keep;
}

// Points of one tile whose owner changes, this thread's share (one (slice, v)
// row at a time).
__device__ __forceinline__ int tile_moved(const XposeDesc &d, int64_t g0, int ng, int64_t u0, int nu, int64_t v0,
                                          int nv)
{
    int moved = 0;
    for (int i = threadIdx.x; i < ng * nv; i += kThreads) {
        const int g = i / nv, iv = i - g * nv;
        int c[3];
        int64_t ab, bb;
        slice_coords(d, g0 + g, c, &ab, &bb);
        moved += nu - (int)row_keep(d, c, v0 + iv, u0, nu);
    }
    return moved;
}

// LDS bytes of a tile, 16-byte aligned; launchers reserve 16 more bytes
// after it (xpose_tile writes the loads of items past the tile there)
__host__ __device__ inline size_t xpose_tile_bytes(const XposeDesc &d, size_t esz)
{
    size_t b = (size_t)d.G * d.TV * (d.TU + 1) * esz;
    return (b + 15) & ~(size_t)15;
}

// One tile of the transpose: tile index t (u fastest, then v, then slices);
// smem holds the tile.
template <typename C, int VU, int VV>
__device__ __forceinline__ void xpose_tile(const C *__restrict__ in, C *__restrict__ out, const XposeDesc &d,
                                           uint32_t tile_index, unsigned char *smem)
{
    C *tile = reinterpret_cast<C *>(smem);

    const int TU = d.TU, TV = d.TV;
    const int ldt = TU + 1;
    uint32_t t = tile_index;
    const uint32_t tu = t % (uint32_t)d.tiles_u;
    t /= (uint32_t)d.tiles_u;
    const uint32_t tv = t % (uint32_t)d.tiles_v;
    const uint32_t tg = t / (uint32_t)d.tiles_v;
    const int64_t u0 = (int64_t)tu * TU, v0 = (int64_t)tv * TV, g0 = (int64_t)tg * d.G;
    const int nu = (int)min<int64_t>(TU, d.Nu - u0);
    const int nv = (int)min<int64_t>(TV, d.Nv - v0);
    const int ng = (int)min<int64_t>(d.G, d.nslices - g0);

    if (d.count) {
        // each wave publishes its sum at once: work left for the end of the
        // tile would delay the group's exit
        int moved = tile_moved(d, g0, ng, u0, nu, v0, nv);
        for (int off = 32; off > 0; off >>= 1) moved += __shfl_xor(moved, off);
        if ((threadIdx.x & 63) == 0 && moved)
            atomicAdd(d.counter + (tile_index % kCountSlots) * kCountStride, (unsigned long long)moved);
    }

    // load: rows (g, v) of contiguous u-values.  A thread's rows are taken
    // kTileBatch at a time, every load of a batch issued before any value
    // goes to LDS (a loop that writes each value as it arrives runs the
    // thread's loads one HBM round trip at a time).
    {
        const int per_row = TU / VU;
        const int tx = threadIdx.x % per_row;
        const int ty = threadIdx.x / per_row;
        const int ystep = kThreads / per_row;
        const int nrow = ng * nv;
        const int iu = tx * VU;
        const int spare = d.G * TV * ldt;  // first element after the tile
        int gcur = -1;
        int64_t abase = 0;
        for (int rb = ty; rb < nrow; rb += kTileBatch * ystep) {
            C val[kTileBatch][VU];
            int at[kTileBatch];
            // every item loads and writes, so that no load is left pending
            // from one trip to the next: an item past the tile loads an
            // element of the tile again (clamped) and writes it to the spare
            // 16 bytes after the tile, which the launchers reserve
#pragma unroll
            for (int j = 0; j < kTileBatch; ++j) {
                const int r = rb + j * ystep;
                const bool ok = r < nrow && iu < nu;
                const int rc = r < nrow ? r : nrow - 1;
                const int iuc = iu < nu ? iu : 0;
                const int g = rc / nv;
                const int iv = rc - g * nv;
                if (g != gcur) {
                    int c[3];
                    int64_t bb;
                    slice_coords(d, g0 + g, c, &abase, &bb);
                    gcur = g;
                }
                const C *p = in + abase + (v0 + iv) * d.a_sv + u0 + iuc;
                at[j] = ok ? (g * TV + iv) * ldt + iu : spare;
                if constexpr (VU == 2) {
                    const xf4 w = gld_nt(reinterpret_cast<const xf4 *>(p));
                    val[j][0] = mk<C>(w.x, w.y);
                    val[j][1] = mk<C>(w.z, w.w);
                } else {
                    val[j][0] = xld(p);
                }
            }
#pragma unroll
            for (int j = 0; j < kTileBatch; ++j) {
#pragma unroll
                for (int w = 0; w < VU; ++w) tile[at[j] + w] = val[j][w];
            }
        }
    }
    __syncthreads();

    // store: rows (g, u) of contiguous v-values, kTileBatch rows at a time,
    // every LDS read of a batch issued before its first store
    {
        const int per_row = TV / VV;
        const int tx = threadIdx.x % per_row;
        const int ty = threadIdx.x / per_row;
        const int ystep = kThreads / per_row;
        const int nrow = ng * nu;
        const int iv = tx * VV;
        int gcur = -1;
        int64_t bbase = 0;
        for (int rb = ty; rb < nrow; rb += kTileBatch * ystep) {
            C val[kTileBatch][VV];
            C *dst[kTileBatch];
#pragma unroll
            for (int j = 0; j < kTileBatch; ++j) {
                const int r = rb + j * ystep;
                dst[j] = nullptr;
                if (r < nrow && iv < nv) {
                    const int g = r / nu;
                    const int iu = r - g * nu;
                    if (g != gcur) {
                        int c[3];
                        int64_t ab;
                        slice_coords(d, g0 + g, c, &ab, &bbase);
                        gcur = g;
                    }
                    dst[j] = out + bbase + (u0 + iu) * d.b_su + v0 + iv;
                    const C *tcol = tile + (g * TV + iv) * ldt + iu;
                    val[j][0] = tcol[0];
                    if constexpr (VV == 2) val[j][1] = tcol[ldt];
                }
            }
#pragma unroll
            for (int j = 0; j < kTileBatch; ++j)
                if (dst[j]) {
                    if constexpr (VV == 2) {
                        const xf4 w = {val[j][0].x, val[j][0].y, val[j][1].x, val[j][1].y};
                        gst_nt(w, reinterpret_cast<xf4 *>(dst[j]));
                    } else {
                        xst(dst[j], val[j][0]);
                    }
                }
        }
    }
    __syncthreads();  // the LDS block may be reused by the caller's next unit
}

}  // namespace fftrw
