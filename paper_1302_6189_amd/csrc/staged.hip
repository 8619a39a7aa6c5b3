// staged.hip -- the transpose as pack -> exchange -> unpack (Fig. 4, Section 3).
//
// This is the all-to-all the paper's processes perform, with every virtual
// process's buffers held explicitly on the device:
//   pack:     process p copies the points of its range in decomposition A into
//             its send region (the same positions as its range), one segment
//             per destination q in ascending q;
//   exchange: every segment with q != p is copied into q's receive region
//             (segments in ascending p) -- exactly the points that change
//             owner, i.e. the paper's communication amount, counted on the
//             device;
//   unpack:   process q places its received segments, and the segment it kept
//             for itself (read straight from the send array), into its range
//             of decomposition B.
// Inside a segment the points keep A's order, so a segment is a contiguous
// message and sender and receiver agree on it without exchanging indices.
//
// Positions come from closed forms rather than per-point searches.  Let S_p
// be p's range in A, Q_q be q's range in B (each at most 2k-1 boxes) and
// rank_q(z) the number of points of Q_q that precede z in A's order (a box
// count, O(M) per box).  For a point z owned by p in A and by q in B:
//   send position    = D(p, q) + rank_q(z)
//   receive position = start_q + rank_q(z) - (p > q ? kept_q : 0)      (p != q)
//   kept position    = D(q, q) + rank_q(z)                              (p == q)
// with D(p, q) = xs_p + segoff(p, q) - rank_q(first point of p), where
// segoff(p, q), the points of S_p in segments for destinations below q, is the
// number of points of S_p that precede q's first point in B's order -- again
// a box count.  rank_q grows by one along u (A's fastest axis) inside a run of
// constant q, and for a fixed (slice, u) it is affine in v (B's fastest axis):
// v never selects B's owner, so stepping v skips exactly the points of Q_q
// that share the slice.
//
// Both pack and unpack are LDS-tiled over a 3-D block of (u, v, slices along
// one batch axis).  Reads and writes each run along whichever of the three
// axes is contiguous on their side: A is contiguous along u, B along v, and a
// segment along the innermost axis (in A's order) that a typical (p, q) box
// spans -- u when q owns long runs of u, otherwise v or a batch axis (for
// example one value of u and of v but 64 slices per segment).  The plan picks
// that axis and the tile's extents per transpose.
//
// The plan evaluates both closed forms once, so the tiles only look them up:
// rank_q at v = 0 and its step per v for every (slice, u) line (a table of
// T / N_v entries, filled by a kernel when the plan is made), and D(p, q) for
// every pair that shares points (an open-addressing hash table keyed by
// (p, q), filled on the host while the pairs are enumerated: per source p,
// these are the send displacements an all-to-all would take).  A tile computes
// its owners, numbers its distinct sources and destinations, and fetches the
// D of its pairs into LDS once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/fftrw.h"
#include "errors.hpp"
#include "kernels.hpp"
#include "plan.hpp"
#include "xpose_tile.hpp"

namespace fftrw {

constexpr int kRangeBoxes = 2 * (kMaxDims - 1) - 1;  // ranges split at most M - 1 axes

// One box of a range in some axis order, with the number of box points per
// unit step of each axis in that order.  Unused boxes have lo = INT_MAX and
// count nothing.
struct RankBox {
    int lo[kMaxDims];
    int hi[kMaxDims];
    int64_t suf[kMaxDims];
};

struct RecvInfo {              // destination q: its range in B
    int64_t start;             // first point of the range = start of q's receive region
    int64_t kept;              // points of q's range that stay with their process (never exchanged)
    int64_t selfbase;          // D(ksrc, q)
    int first_b[kMaxDims];     // q's first point, coordinates in B's order
    int ksrc;                  // the source range whose points q keeps: q under the literal
                               // reading, the range matched to q under the matched one
    RankBox box[kRangeBoxes];  // in A's order
};

// One slot of the pair table: key p * P + q (-1 = empty), value D(p, q).
struct PairSlot {
    int64_t key;
    int d;
    int pad;
};

__host__ __device__ inline uint64_t pair_hash(int64_t key, int lg)
{
    return ((uint64_t)key * 0x9E3779B97F4A7C15ull) >> (64 - lg);
}

struct SegCopy {
    int64_t xoff;      // position in the concatenation of exchanged segments
    int64_t src, dst;  // send / receive array offsets
    int64_t len;
};

// Tiling of the pack and unpack kernels.  A tile spans TU values of u, TV of
// v and G consecutive slices along the first batch axis of d.  Elements are
// visited with one axis fastest across lanes when read (lane_r) and another
// when written (lane_w): 0 = u, 1 = v, 2 = slices.
struct StagedTile {
    XposeDesc d;
    int lu, lv, lg;         // log2 of TU, TV, G
    int lane_r, lane_w;
    int M;
    int nbq;                // boxes per range in B
    int srcpos[kMaxDims];   // per A position: batch index 0..2, 3 = v, 4 = u
    int vpos;               // A position of v
    int pair_lg;            // log2 of the pair table's slots
    int64_t T, P;
    const RecvInfo *recv;
    const int2 *lrank;      // per (slice, u) line: rank_q at v = 0, step per v
    const PairSlot *pairs;  // D(p, q) of every pair that shares points
};

struct ExchangeArgs {
    const SegCopy *segs;
    const int64_t *chunk_seg;  // per chunk: first and last segment it touches
    int64_t nseg, total;
    unsigned long long *counter;
};

// points of box B that precede coordinates c in the box's axis order
__device__ __forceinline__ int64_t box_rank(const RankBox &B, const int *c, int M)
{
    int64_t r = 0;
#pragma unroll
    for (int i = 0; i < kMaxDims; ++i) {
        if (i >= M) break;
        const int x = c[i];
        if (x < B.lo[i]) break;
        if (x > B.hi[i]) {
            r += (int64_t)(B.hi[i] - B.lo[i] + 1) * B.suf[i];
            break;
        }
        r += (int64_t)(x - B.lo[i]) * B.suf[i];
    }
    return r;
}

// D(p, q) from the pair table (every pair that owns a point of the array is
// present; the table is at most half full, so the probe ends at a free slot)
__device__ __forceinline__ int pair_offset(const StagedTile &a, int p, int q)
{
    const int64_t key = (int64_t)p * a.P + q;
    const uint64_t mask = ((uint64_t)1 << a.pair_lg) - 1;
    uint64_t h = pair_hash(key, a.pair_lg);
    for (uint64_t n = 0; n <= mask; ++n, h = (h + 1) & mask) {
        const int64_t k = a.pairs[h].key;
        if (k == key) return a.pairs[h].d;
        if (k < 0) break;
    }
    return INT_MIN / 2;  // no such pair: the offset falls outside the array and is not written
}

constexpr int kPairTab = 1024;  // dense (p, q) constants per pack tile
constexpr int kTileItems = 16;  // tile elements per thread (tiles hold at most 4096)
constexpr int kOwnHash = 512;   // distinct owners per side a pack tile numbers densely
constexpr size_t kTileLdsMax = 64 * 1024;  // LDS of one pack or unpack tile

// Number owner `key` densely: an open-addressing table (keys, -1 = free)
// whose slots also hold the dense number, given by the thread that claims
// the slot; `list` maps numbers back to owners.  Probing is bounded: past
// kOwnHash steps the table is full and *overflow is set (the tile then looks
// every point's pair up in the plan's pair table).
__device__ __forceinline__ void own_insert(int *keys, int *num, int *list, int *count, int *overflow, int key)
{
    int h = (int)(((uint32_t)key * 2654435761u) >> 23) & (kOwnHash - 1);
    for (int n = 0; n < kOwnHash; ++n, h = (h + 1) & (kOwnHash - 1)) {
        int k = keys[h];
        if (k == -1) {
            k = atomicCAS(&keys[h], -1, key);
            if (k == -1) {
                const int i = atomicAdd(count, 1);
                num[h] = i;
                list[i] = key;
                return;
            }
        }
        if (k == key) return;
    }
    *overflow = 1;
}

// the dense number of an owner already inserted (table not overflowed)
__device__ __forceinline__ int own_lookup(const int *keys, const int *num, int key)
{
    int h = (int)(((uint32_t)key * 2654435761u) >> 23) & (kOwnHash - 1);
    for (int n = 0; n < kOwnHash; ++n, h = (h + 1) & (kOwnHash - 1))
        if (keys[h] == key) return num[h];
    return 0;
}

struct TileLds {
    size_t tile, gbase, gc, r0, wv, rb, sb, kp, ks, pt, own_a, own_b, hash, misc, total;
};

__host__ __device__ inline TileLds tile_lds(int lu, int lv, int lg, size_t esz, bool pack)
{
    const size_t TU = (size_t)1 << lu, TV = (size_t)1 << lv, G = (size_t)1 << lg;
    const size_t SG = TV * (TU + 1) + 1;
    TileLds L;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = (o + bytes + 15) & ~(size_t)15;
        return at;
    };
    // a pack tile's owner hash (keys, numbers, lists for p and q) lives only
    // until the owners are renumbered, before any value reaches the tile, so
    // the two share their LDS
    const size_t hash_bytes = 6 * kOwnHash * 4;
    const size_t tile_bytes = G * SG * esz;
    L.tile = take(pack && hash_bytes > tile_bytes ? hash_bytes : tile_bytes);
    L.gbase = take(G * 4);
    L.gc = take(G * 3 * 4);
    L.r0 = take(G * (TU + 1) * 4);
    L.wv = take(G * (TU + 1) * 4);
    L.rb = pack ? 0 : take(G * (TU + 1) * 4);
    L.sb = pack ? 0 : take(G * (TU + 1) * 4);
    L.kp = pack ? 0 : take(G * (TU + 1) * 4);
    L.ks = pack ? 0 : take(G * (TU + 1) * 4);
    L.pt = pack ? take(kPairTab * 4) : 0;
    L.own_a = take(G * (TV + 1) * 4);
    L.own_b = take(G * (TU + 1) * 4);
    L.hash = L.tile;
    L.misc = take(16);
    L.total = o;
    return L;
}

// One pass over a tile with axis LANE fastest across lanes: thread t owns lane
// position t mod E (E = the axis's extent) and lines t / E, t / E + 256 / E, ...
// of the other two axes.  f(j, g, iv, iu) is called for every element inside
// the tile's valid extents, j numbering the thread's items.
template <int LANE, class F>
__device__ __forceinline__ void tile_pass(int lu, int lv, int lg, int nu, int nv, int ng, F &&f)
{
    const int le = LANE == 0 ? lu : (LANE == 1 ? lv : lg);
    const int x = threadIdx.x & ((1 << le) - 1);
    const int r0 = threadIdx.x >> le;
    const int rstep = kThreads >> le;
    const int nlines = 1 << (lu + lv + lg - le);
#pragma unroll
    for (int j = 0; j < kTileItems; ++j) {
        const int r = r0 + j * rstep;
        if (r >= nlines) break;
        int g, iv, iu;
        if (LANE == 0) {
            iu = x;
            iv = r & ((1 << lv) - 1);
            g = r >> lv;
        } else if (LANE == 1) {
            iv = x;
            iu = r & ((1 << lu) - 1);
            g = r >> lu;
        } else {
            g = x;
            iu = r & ((1 << lu) - 1);
            iv = r >> lu;
        }
        if (g < ng && iv < nv && iu < nu) f(j, g, iv, iu);
    }
}

// PACK:   src = layout A, dst = send array.
// UNPACK: src = receive array, self_src = send array (kept segments), dst = layout B.
template <typename C, bool PACK, int LR, int LW>
__global__ void __launch_bounds__(kThreads)
    staged_tile_kernel(const C *__restrict__ src, const C *__restrict__ self_src, C *__restrict__ dst, StagedTile a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const XposeDesc &d = a.d;
    const int lu = a.lu, lv = a.lv, lg = a.lg;
    const int TU = 1 << lu, TV = 1 << lv, G = 1 << lg;
    const int SV = TU + 1, SG = TV * SV + 1;
    // per-line tables (owners, ranks, q's constants) are padded by one entry
    // per slice: a pass with lanes along the slices then reads them from
    // different banks (a stride of TU = 16 put every fourth slice on one)
    const int KU = TU + 1, KV = TV + 1;
    const int M = a.M;
    uint32_t t = blockIdx.x;
    const uint32_t tu = t % (uint32_t)d.tiles_u;
    t /= (uint32_t)d.tiles_u;
    const uint32_t tv = t % (uint32_t)d.tiles_v;
    const uint32_t tg = t / (uint32_t)d.tiles_v;
    const int64_t u0 = (int64_t)tu * TU, v0 = (int64_t)tv * TV, g0 = (int64_t)tg * G;
    const int nu = (int)min<int64_t>(TU, d.Nu - u0);
    const int nv = (int)min<int64_t>(TV, d.Nv - v0);
    const int ng = (int)min<int64_t>(G, d.nslices - g0);

    const TileLds L = tile_lds(lu, lv, lg, sizeof(C), PACK);
    C *tile = reinterpret_cast<C *>(smem + L.tile);
    int *gbase = reinterpret_cast<int *>(smem + L.gbase);
    int *gc = reinterpret_cast<int *>(smem + L.gc);  // batch coordinates of each slice
    int *r0 = reinterpret_cast<int *>(smem + L.r0);
    int *wv = reinterpret_cast<int *>(smem + L.wv);
    int *rb = reinterpret_cast<int *>(smem + L.rb);
    int *sb = reinterpret_cast<int *>(smem + L.sb);
    int *kp = reinterpret_cast<int *>(smem + L.kp);
    int *ks = reinterpret_cast<int *>(smem + L.ks);
    int *pt = reinterpret_cast<int *>(smem + L.pt);
    int *own_a = reinterpret_cast<int *>(smem + L.own_a);
    int *own_b = reinterpret_cast<int *>(smem + L.own_b);
    int *mm = reinterpret_cast<int *>(smem + L.misc);  // distinct p, distinct q, overflow
    int *hk = reinterpret_cast<int *>(smem + L.hash);  // [side][kOwnHash] keys, numbers, lists
    int *hn = hk + 2 * kOwnHash;
    int *hl = hn + 2 * kOwnHash;

    // owners, slice bases, cleared accumulators
    if (PACK && threadIdx.x == 0) {
        mm[0] = 0;
        mm[1] = 0;
        mm[2] = 0;
    }
    if (PACK)
        for (int i = threadIdx.x; i < 2 * kOwnHash; i += kThreads) hk[i] = -1;
    // each slice's coordinates once, then owners from them
    for (int g = threadIdx.x; g < ng; g += kThreads) {
        int c[3] = {0, 0, 0};
        int64_t ab, bb;
        slice_coords(d, g0 + g, c, &ab, &bb);
        gbase[g] = (int)(PACK ? ab : bb);
        gc[3 * g] = c[0];
        gc[3 * g + 1] = c[1];
        gc[3 * g + 2] = c[2];
    }
    __syncthreads();
    // a pack tile issues the loads that need no owner now and consumes them
    // after the owner arithmetic: its line-table entries (a tile has at most
    // 512 (slice, u) lines) and its values (A's addresses depend only on the
    // slice bases).  (Unpack tiles load their line entries with q's constants:
    // issued early as well, the return transpose's unpack at 512^3 went from
    // 0.42 to 0.63 ms.)
    const int nlines = ng * nu;
    int2 lr[2];
    C val[kTileItems];
    int at[kTileItems];
#pragma unroll
    for (int j = 0; j < kTileItems; ++j) at[j] = -1;
    if constexpr (PACK) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int i = threadIdx.x + j * kThreads;
            if (i < nlines) {
                const int g = i / nu, iu = i - g * nu;
                lr[j] = a.lrank[(g0 + g) * d.Nu + u0 + iu];
            }
        }
        const int a_sv = (int)d.a_sv;
        tile_pass<LR>(lu, lv, lg, nu, nv, ng, [&](int j, int g, int iv, int iu) {
            at[j] = g * SG + iv * SV + iu;
            val[j] = xld(src + (gbase[g] + (int)(v0 + iv) * a_sv + (int)u0 + iu));
        });
    }
    {
        // below level M, A's leading axes are batch axes and v, B's are batch
        // axes and u (the staged path refuses level M)
        const bool narrow = d.owner32 != 0;
        for (int i = threadIdx.x; i < ng * nv; i += kThreads) {
            const int g = i / nv, iv = i - g * nv;
            int64_t r = 0;
            for (int j = 0; j < d.ka; ++j) {
                const int src = d.srca[j];
                r += (src == 3 ? v0 + iv : (int64_t)gc[3 * g + src]) * d.wa[j];
            }
            own_a[g * KV + iv] = (int)owner_of_row(r, d.P, d.Ra, narrow);
        }
        for (int i = threadIdx.x; i < ng * nu; i += kThreads) {
            const int g = i / nu, iu = i - g * nu;
            int64_t r = 0;
            for (int j = 0; j < d.kb; ++j) {
                const int src = d.srcb[j];
                r += (src == 4 ? u0 + iu : (int64_t)gc[3 * g + src]) * d.wb[j];
            }
            own_b[g * KU + iu] = (int)owner_of_row(r, d.P, d.Rb, narrow);
        }
    }
    __syncthreads();

    // per (slice, u) line: rank_q at the tile's first v and its step per v;
    // unpack also picks up q's constants
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int i = threadIdx.x + j * kThreads;
        if (i >= nlines) break;
        const int g = i / nu, iu = i - g * nu;
        const int k = g * KU + iu;
        if (!PACK) lr[j] = a.lrank[(g0 + g) * d.Nu + u0 + iu];
        r0[k] = lr[j].x + (int)v0 * lr[j].y;
        wv[k] = lr[j].y;
        if (!PACK) {
            const RecvInfo &R = a.recv[own_b[k]];
            rb[k] = (int)R.start;
            sb[k] = (int)R.selfbase;
            kp[k] = (int)R.kept;
            ks[k] = R.ksrc;
        }
    }
    if (PACK) {
        // number the tile's distinct owners densely, p (A) and q (B) apart
        for (int i = threadIdx.x; i < ng * nv; i += kThreads)
            own_insert(hk, hn, hl, &mm[0], &mm[2], own_a[(i / nv) * KV + i % nv]);
        for (int i = threadIdx.x; i < ng * nu; i += kThreads)
            own_insert(hk + kOwnHash, hn + kOwnHash, hl + kOwnHash, &mm[1], &mm[2], own_b[(i / nu) * KU + i % nu]);
    }
    __syncthreads();

    // pack: D(p, q) of every pair of the tile's distinct owners (pairs that
    // share no point look up nothing usable and are never read); the owner
    // tables then hold dense numbers
    const int np = PACK ? mm[0] : 0, nq = PACK ? mm[1] : 0;
    const bool dense = PACK && mm[2] == 0 && np * nq <= kPairTab;
    if (PACK && dense) {
        for (int e = threadIdx.x; e < np * nq; e += kThreads) pt[e] = pair_offset(a, hl[e / nq], hl[kOwnHash + e % nq]);
        for (int i = threadIdx.x; i < ng * nv; i += kThreads) {
            int &o = own_a[(i / nv) * KV + i % nv];
            o = own_lookup(hk, hn, o);
        }
        for (int i = threadIdx.x; i < ng * nu; i += kThreads) {
            int &o = own_b[(i / nu) * KU + i % nu];
            o = own_lookup(hk + kOwnHash, hn + kOwnHash, o);
        }
        __syncthreads();
    }

    // unpack reads (every item's load is issued before any LDS store), then
    // the values into the tile
    if constexpr (!PACK) {
        tile_pass<LR>(lu, lv, lg, nu, nv, ng, [&](int j, int g, int iv, int iu) {
            at[j] = g * SG + iv * SV + iu;
            const int k = g * KU + iu;
            const int p = own_a[g * KV + iv];
            const int rk = r0[k] + iv * wv[k];
            const C *from = src;
            int off;
            const int keep_src = ks[k];
            if (p == keep_src) {
                from = self_src;
                off = sb[k] + rk;
            } else {
                off = rb[k] + rk - (p > keep_src ? kp[k] : 0);
            }
            val[j] = (uint32_t)off < (uint32_t)a.T ? xld(from + off) : mk<C>(0, 0);
        });
    }
#pragma unroll
    for (int j = 0; j < kTileItems; ++j)
        if (at[j] >= 0) tile[at[j]] = val[j];
    __syncthreads();
    // write
    if (PACK) {
        if (dense) {
            tile_pass<LW>(lu, lv, lg, nu, nv, ng, [&](int, int g, int iv, int iu) {
                const int k = g * KU + iu;
                const int off = pt[own_a[g * KV + iv] * nq + own_b[k]] + r0[k] + iv * wv[k];
                if ((uint32_t)off < (uint32_t)a.T) xst(dst + off, tile[g * SG + iv * SV + iu]);
            });
        } else {
            tile_pass<LW>(lu, lv, lg, nu, nv, ng, [&](int, int g, int iv, int iu) {
                const int k = g * KU + iu;
                const int off = pair_offset(a, own_a[g * KV + iv], own_b[k]) + r0[k] + iv * wv[k];
                if ((uint32_t)off < (uint32_t)a.T) xst(dst + off, tile[g * SG + iv * SV + iu]);
            });
        }
    } else {
        const int b_su = (int)d.b_su;
        tile_pass<LW>(lu, lv, lg, nu, nv, ng, [&](int, int g, int iv, int iu) {
            xst(dst + (gbase[g] + (int)(u0 + iu) * b_su + (int)v0 + iv), tile[g * SG + iv * SV + iu]);
        });
    }
}

// Plan time: for every (slice, u) line, in the slice numbering of the tiles,
// rank_q of its point at v = 0 and the step of rank_q per unit of v (q = the
// line's owner in B).  q's boxes span all of v, so rank_q is affine in v.
__global__ void __launch_bounds__(kThreads) staged_rank_kernel(StagedTile a, int2 *__restrict__ out)
{
    const XposeDesc &d = a.d;
    const int64_t n = d.nslices * d.Nu;
    for (int64_t x = (int64_t)blockIdx.x * kThreads + threadIdx.x; x < n; x += (int64_t)gridDim.x * kThreads) {
        const int64_t sl = x / d.Nu;
        const int u = (int)(x - sl * d.Nu);
        int bc[3] = {0, 0, 0};
        int64_t ab, bb;
        slice_coords(d, sl, bc, &ab, &bb);
        int64_t r = 0;
        for (int j = 0; j < d.kb; ++j) {
            const int src = d.srcb[j];
            r += (src == 4 ? (int64_t)u : (int64_t)bc[src]) * d.wb[j];
        }
        const RecvInfo &R = a.recv[owner_of_row(r, d.P, d.Rb, d.owner32 != 0)];
        int c[kMaxDims];
#pragma unroll
        for (int m = 0; m < kMaxDims; ++m) {
            const int sp = a.srcpos[m];
            c[m] = sp == 3 ? 0 : sp == 4 ? u : bc[sp < 3 ? sp : 0];
        }
        int64_t ra = 0, rn = 0;
        for (int j = 0; j < a.nbq; ++j) ra += box_rank(R.box[j], c, a.M);
        c[a.vpos] += 1;
        for (int j = 0; j < a.nbq; ++j) rn += box_rank(R.box[j], c, a.M);
        out[x] = make_int2((int)ra, (int)(rn - ra));
    }
}

template <class Key>
__device__ __forceinline__ int64_t upper_index(Key key, int64_t lo, int64_t hi, int64_t x)
{
    // largest i in [lo, hi] with key(i) <= x
    while (lo < hi) {
        int64_t mid = (lo + hi + 1) >> 1;
        if (key(mid) <= x)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

constexpr int kChunk = 4096;  // exchanged points per work-group
constexpr int kChunkItems = kChunk / kThreads;
constexpr int kChunkSegsLds = 512;  // segment starts of a chunk staged in LDS

template <typename C>
__global__ void __launch_bounds__(kThreads)
    exchange_kernel(const C *__restrict__ send, C *__restrict__ recv, ExchangeArgs a)
{
    __shared__ int64_t s_xoff[kChunkSegsLds];
    __shared__ int64_t s_src[kChunkSegsLds], s_dst[kChunkSegsLds];  // segment offsets minus xoff
    __shared__ int copied_wg;
    const int64_t x0 = (int64_t)blockIdx.x * kChunk;
    const int64_t x1 = min<int64_t>(x0 + kChunk, a.total) - 1;
    const int64_t fs = a.chunk_seg[2 * blockIdx.x], ls = a.chunk_seg[2 * blockIdx.x + 1];
    const int n = (int)(x1 - x0 + 1);
    if (threadIdx.x == 0) copied_wg = 0;
    int copied = 0;
    C v[kChunkItems];
    if (fs == ls) {
        // the whole chunk lies in one segment: a straight copy
        const SegCopy S = a.segs[fs];
        const C *from = send + S.src + (x0 - S.xoff);
        C *to = recv + S.dst + (x0 - S.xoff);
#pragma unroll
        for (int j = 0; j < kChunkItems; ++j) {
            const int i = threadIdx.x + j * kThreads;
            if (i < n) v[j] = xld(from + i);
        }
#pragma unroll
        for (int j = 0; j < kChunkItems; ++j) {
            const int i = threadIdx.x + j * kThreads;
            if (i < n) {
                xst(to + i, v[j]);
                ++copied;
            }
        }
    } else {
        // several segments: their descriptors in LDS when few enough, so a
        // point's copy needs one global load (its value), not two
        const int nseg = (int)(ls - fs + 1);
        const bool in_lds = nseg <= kChunkSegsLds;
        if (in_lds)
            for (int i = threadIdx.x; i < nseg; i += kThreads) {
                const SegCopy S = a.segs[fs + i];
                s_xoff[i] = S.xoff;
                s_src[i] = S.src - S.xoff;
                s_dst[i] = S.dst - S.xoff;
            }
        __syncthreads();
        int64_t to[kChunkItems];
#pragma unroll
        for (int j = 0; j < kChunkItems; ++j) {
            const int i = threadIdx.x + j * kThreads;
            to[j] = -1;
            if (i < n) {
                const int64_t x = x0 + i;
                if (in_lds) {
                    const int64_t m = upper_index([&](int64_t q) { return s_xoff[q]; }, 0, nseg - 1, x);
                    to[j] = s_dst[m] + x;
                    v[j] = xld(send + s_src[m] + x);
                } else {
                    const int64_t si = upper_index([&](int64_t q) { return a.segs[q].xoff; }, fs, ls, x);
                    const SegCopy &S = a.segs[si];
                    const int64_t o = x - S.xoff;
                    to[j] = S.dst + o;
                    v[j] = xld(send + S.src + o);
                }
            }
        }
#pragma unroll
        for (int j = 0; j < kChunkItems; ++j) {
            if (to[j] >= 0) {
                xst(recv + to[j], v[j]);
                ++copied;
            }
        }
    }
    __syncthreads();
    for (int off = 32; off > 0; off >>= 1) copied += __shfl_xor(copied, off);
    if ((threadIdx.x & 63) == 0 && copied) atomicAdd(&copied_wg, copied);
    __syncthreads();
    if (threadIdx.x == 0 && copied_wg)
        atomicAdd(a.counter + (blockIdx.x % kCountSlots) * kCountStride, (unsigned long long)copied_wg);
}

namespace {

int copy_to_device(fft_plan_impl *pl, const void *h, size_t bytes, void **d)
{
    if (bytes == 0) bytes = 16;
    if (hipMalloc(d, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(FFTRW_E_NOMEM, "hipMalloc for staged tables failed");
    }
    pl->dev_bytes += bytes;
    if (h && hipMemcpy(*d, h, bytes, hipMemcpyHostToDevice) != hipSuccess)
        return fail(FFTRW_E_DEVICE, "copy of staged tables failed");
    return FFTRW_OK;
}

int ilog2ceil(i64 n)
{
    int l = 0;
    while (((i64)1 << l) < n) ++l;
    return l;
}

// Boxes of a range in the axis order `perm`, padded to kRangeBoxes.
void fill_boxes(const std::vector<Box> &boxes, const int *perm, int M, RankBox *out)
{
    for (int j = 0; j < kRangeBoxes; ++j) {
        RankBox &rb = out[j];
        for (int i = 0; i < kMaxDims; ++i) {
            rb.lo[i] = INT_MAX;
            rb.hi[i] = -1;
            rb.suf[i] = 0;
        }
        if (j >= (int)boxes.size()) continue;
        i64 suf = 1;
        for (int i = M - 1; i >= 0; --i) {
            const int ax = perm[i];
            rb.lo[i] = (int)boxes[j].lo[ax];
            rb.hi[i] = (int)boxes[j].hi[ax];
            rb.suf[i] = suf;
            suf *= boxes[j].hi[ax] - boxes[j].lo[ax] + 1;
        }
    }
}

// The natural axis along which (p, q) segments run: the innermost axis, in A's
// order, that spans more than one value in a representative pair box (the
// largest piece of a middle process's largest range box).
int segment_axis(const Layout &a, const Layout &b, int M)
{
    const std::vector<Box> bx = range_boxes(a, a.P / 2);
    size_t big = 0;
    for (size_t i = 1; i < bx.size(); ++i)
        if (box_volume(bx[i], M) > box_volume(bx[big], M)) big = i;
    Box best = bx[big];
    i64 bestn = -1;
    for_each_owner(b, bx[big], [&](i64 q) {
        for (const Box &C : range_boxes(b, q)) {
            Box X;
            if (box_intersect(bx[big], C, M, &X) && box_volume(X, M) > bestn) {
                bestn = box_volume(X, M);
                best = X;
            }
        }
    });
    for (int i = M - 1; i >= 0; --i) {
        const int ax = a.perm[i];
        if (best.hi[ax] > best.lo[ax]) return ax;
    }
    return a.perm[M - 1];
}

// A tiling for one staged kernel: the transpose's geometry with the segment
// axis moved to the front of the batch axes (it becomes the tile's slice axis
// when it is neither u nor v), and extents favouring the read and write axes.
StagedTileCfg make_tile(const fft_plan_impl *pl, int t, int seg_axis, bool pack)
{
    const Layout &a = pl->lay[t];
    const Layout &b = pl->lay[t + 1];
    const int M = pl->M;
    const int u = a.perm[M - 1], v = b.perm[M - 1];
    StagedTileCfg c;
    c.d = pl->xp[t];
    XposeDesc &d = c.d;
    // batch axes as the transpose orders them (innermost = smallest stride in A)
    int bat[3], nb = 0;
    for (int ax = 0; ax < M; ++ax)
        if (ax != u && ax != v) bat[nb++] = ax;
    std::sort(bat, bat + nb, [&](int x, int y) { return a.stride[x] < a.stride[y]; });
    int order[3] = {0, 1, 2};  // new batch index -> old
    const int sa = (seg_axis != u && seg_axis != v) ? seg_axis : -1;
    if (sa >= 0) {
        int j = 0;
        while (bat[j] != sa) ++j;
        for (int i = j; i > 0; --i) order[i] = order[i - 1];
        order[0] = j;
    }
    int newidx[3] = {0, 1, 2};
    const XposeDesc o = d;
    for (int i = 0; i < nb; ++i) {
        d.bsize[i] = o.bsize[order[i]];
        d.ba[i] = o.ba[order[i]];
        d.bb[i] = o.bb[order[i]];
        newidx[order[i]] = i;
    }
    for (int j = 0; j < d.ka; ++j)
        if (d.srca[j] < 3) d.srca[j] = newidx[o.srca[j]];
    for (int j = 0; j < d.kb; ++j)
        if (d.srcb[j] < 3) d.srcb[j] = newidx[o.srcb[j]];
    for (int i = 0; i < M; ++i) {
        const int ax = a.perm[i];
        if (ax == u)
            c.srcpos[i] = 4;
        else if (ax == v) {
            c.srcpos[i] = 3;
            c.vpos = i;
        } else {
            int j = 0;
            while (bat[j] != ax) ++j;
            c.srcpos[i] = newidx[j];
        }
    }
    // extents: the read and write axes first, then fill up to the budget;
    // each axis at most 256 (one lane pass), slices x u at most 512 (tables).
    // 4096 values per tile (2048 in FP64) spread the per-tile rank and pair
    // set-up over more points; tiles that run along the slices keep 2048
    // (1024): their gathers need the extra resident groups more (measured).
    const int f = seg_axis == u ? 0 : (seg_axis == v ? 1 : 2);
    c.lane_r = pack ? 0 : f;
    c.lane_w = pack ? f : 1;
    const int ra = c.lane_r, wa = c.lane_w;
    const int budget = (pl->esz == 8 ? 12 : 11) - (ra == 2 || wa == 2 ? 1 : 0);
    const int cap[3] = {std::min(8, ilog2ceil(d.Nu)), std::min(8, ilog2ceil(d.Nv)),
                        nb ? std::min(8, ilog2ceil(d.bsize[0])) : 0};
    int l[3] = {0, 0, 0};
    auto room = [&](int ax) {
        int r = std::max(0, budget - l[0] - l[1] - l[2]);
        if (ax != 1) r = std::min(r, std::max(0, 9 - l[0] - l[2]));
        return r;
    };
    auto want = [&](int ax, int lg2) { l[ax] = std::min(cap[ax], std::max(l[ax], std::min(lg2, l[ax] + room(ax)))); };
    auto fill = [&](int ax) { l[ax] = std::min(cap[ax], l[ax] + room(ax)); };
    if (ra == wa) {
        want(ra, 6);
    } else if (ra != 2 && wa != 2) {
        want(ra, (budget + 1) / 2);
        want(wa, budget / 2);
    } else {
        want(ra == 2 ? wa : ra, 4);
        want(2, 4);  // 16 slices: 128-byte runs (measured best; 32 were 10% slower)
    }
    if (ra == 2 && !pack) {
        // unpack tiles reading along the slices widen u before v: A's owner is
        // computed per (slice, v), B's per (slice, u)
        fill(0);
        fill(1);
    } else {
        fill(1);
        fill(0);
    }
    fill(2);
    // a tile that is narrow along u pads every u-line: keep its LDS within 64 KB
    // by shrinking the largest axis that is not a lane axis (else the largest)
    while (tile_lds(l[0], l[1], l[2], pl->esz, pack).total > kTileLdsMax) {
        int ax = -1;
        for (int x = 0; x < 3; ++x)
            if (x != ra && x != wa && l[x] > 0 && (ax < 0 || l[x] > l[ax])) ax = x;
        if (ax < 0)
            for (int x = 0; x < 3; ++x)
                if (l[x] > 0 && (ax < 0 || l[x] > l[ax])) ax = x;
        --l[ax];
    }
    c.lu = l[0];
    c.lv = l[1];
    c.lg = l[2];
    d.TU = 1 << c.lu;
    d.TV = 1 << c.lv;
    d.G = 1 << c.lg;
    d.tiles_u = (d.Nu + d.TU - 1) / d.TU;
    d.tiles_v = (d.Nv + d.TV - 1) / d.TV;
    d.tiles_g = (d.nslices + d.G - 1) / d.G;
    d.count = 1;
    d.counter = nullptr;
    d.mu = nullptr;
    return c;
}

}  // namespace

int staged_build(fft_plan_impl *pl, int t)
{
    const Layout &a = pl->lay[t];
    const Layout &b = pl->lay[t + 1];
    const int M = pl->M;
    const i64 P = pl->P;
    if (a.row_split() || b.row_split())
        return fail(FFTRW_E_ROWSPLIT, "staged transposes need whole rows in both decompositions");
    if (pl->T >= ((i64)1 << 31) || P >= ((i64)1 << 31))
        return fail(FFTRW_E_SIZE, "staged transposes support fewer than 2^31 points");
    if (!pl->send) {
        for (void **buf : {&pl->send, &pl->recv}) {
            if (hipMalloc(buf, (size_t)pl->T * pl->esz) != hipSuccess) {
                (void)hipGetLastError();
                return fail(FFTRW_E_NOMEM, "hipMalloc of staging buffers failed");
            }
            pl->dev_bytes += (size_t)pl->T * pl->esz;
        }
    }
    // every (p, q) pair that shares points, by p then q.  Range p of A is held
    // by the process that keeps range mu[p] of B (mu = identity under the
    // literal reading, the plan's maximum matching under the matched one), so
    // the pair (p, mu[p]) stays put and every other pair is a message.
    const std::vector<PairCount> pc = pair_counts(a, b);
    const std::vector<i64> &mu = pl->mu[t];
    if ((i64)mu.size() != P) return fail(FFTRW_E_DEVICE, "internal: relabelling table size");
    std::vector<RecvInfo> ri(P);
    for (i64 p = 0; p < P; ++p) {
        ri[mu[p]].ksrc = (int)p;
        ri[mu[p]].kept = 0;
        ri[mu[p]].selfbase = 0;
    }
    std::vector<PairSlot> pd;          // (p * P + q, D(p, q)) of every pair
    pd.reserve(pc.size());
    std::vector<i64> before_q(P, 0);   // points of Q_q in the ranges of sources < p
    std::vector<i64> recv_fill(P, 0);  // received points of q so far (sources other than ksrc)
    std::vector<SegCopy> segs;
    i64 moved = 0;
    {
        size_t i = 0;
        for (i64 p = 0; p < P; ++p) {
            const i64 xs = a.boundary(p);
            i64 segoff = 0;
            for (; i < pc.size() && pc[i].p == p; ++i) {
                const i64 q = pc[i].q, n = pc[i].n;
                const i64 D = xs + segoff - before_q[q];
                pd.push_back({p * P + q, (int)D, 0});
                if (q == mu[p]) {
                    ri[q].kept = n;
                    ri[q].selfbase = D;
                } else {
                    segs.push_back({moved, xs + segoff, b.boundary(q) + recv_fill[q], n});
                    moved += n;
                    recv_fill[q] += n;
                }
                before_q[q] += n;
                segoff += n;
            }
            if (segoff != a.boundary(p + 1) - xs)
                return fail(FFTRW_E_DEVICE, "internal: staged pairs do not cover a range");
        }
    }
    // destination ranges as boxes in A's order
    int nbq = 0;
    for (i64 q = 0; q < P; ++q) {
        RecvInfo &r = ri[q];
        r.start = b.boundary(q);
        i64 st[kMaxDims];
        range_of(b, q, nullptr, nullptr, st, nullptr);
        for (int i = 0; i < kMaxDims; ++i) r.first_b[i] = i < M ? (int)st[i] : 0;
        const std::vector<Box> boxes = range_boxes(b, q);
        if ((int)boxes.size() > kRangeBoxes) return fail(FFTRW_E_DEVICE, "internal: too many range boxes");
        nbq = std::max(nbq, (int)boxes.size());
        fill_boxes(boxes, a.perm, M, r.box);
    }
    // the pair table, at most half full
    int lg = 4;
    while (((size_t)1 << lg) < 2 * pd.size()) ++lg;
    std::vector<PairSlot> tab((size_t)1 << lg, PairSlot{-1, 0, 0});
    {
        const uint64_t mask = ((uint64_t)1 << lg) - 1;
        for (const PairSlot &e : pd) {
            uint64_t h = pair_hash(e.key, lg);
            while (tab[h].key >= 0) h = (h + 1) & mask;
            tab[h] = e;
        }
    }

    StagedStep &st = pl->staged[t];
    st.npair = (int64_t)pc.size();
    st.nseg = (int64_t)segs.size();
    st.seg_elems = moved;
    st.nbq = nbq;
    st.pair_lg = lg;
    st.seg_axis = segment_axis(a, b, M);
    st.pack = make_tile(pl, t, st.seg_axis, true);
    st.unpack = make_tile(pl, t, st.seg_axis, false);
    for (const StagedTileCfg *c : {&st.pack, &st.unpack}) {
        if (c->d.tiles_u * c->d.tiles_v * c->d.tiles_g >= (i64)0x7fffffff)
            return fail(FFTRW_E_SIZE, "array too large for one staged launch");
        if (c->lu + c->lv + c->lg > 12 || c->lu + c->lg > 9 || c->lu > 8 || c->lv > 8 || c->lg > 8)
            return fail(FFTRW_E_DEVICE, "internal: staged tile exceeds its LDS tables");
    }
    // pack and unpack index the line table by the same slice numbering
    {
        const XposeDesc &x = st.pack.d, &y = st.unpack.d;
        bool same = x.nbat == y.nbat && x.nslices == y.nslices && x.Nu == y.Nu;
        for (int i = 0; i < x.nbat; ++i) same = same && x.bsize[i] == y.bsize[i];
        for (int i = 0; i < kMaxDims; ++i) same = same && st.pack.srcpos[i] == st.unpack.srcpos[i];
        if (!same) return fail(FFTRW_E_DEVICE, "internal: staged tilings number slices differently");
    }
    // first and last segment of every exchange chunk
    std::vector<int64_t> chunk_seg;
    {
        const i64 nch = (moved + kChunk - 1) / kChunk;
        chunk_seg.resize(2 * (size_t)nch);
        size_t j = 0;
        for (i64 c = 0; c < nch; ++c) {
            const i64 x0 = c * kChunk, x1 = std::min<i64>(x0 + kChunk, moved) - 1;
            while (j + 1 < segs.size() && segs[j + 1].xoff <= x0) ++j;
            size_t k = j;
            while (k + 1 < segs.size() && segs[k + 1].xoff <= x1) ++k;
            chunk_seg[2 * c] = (int64_t)j;
            chunk_seg[2 * c + 1] = (int64_t)k;
        }
    }
    int rc = copy_to_device(pl, ri.data(), sizeof(RecvInfo) * ri.size(), &st.recv_info);
    if (!rc) rc = copy_to_device(pl, tab.data(), sizeof(PairSlot) * tab.size(), &st.pairs);
    if (!rc) rc = copy_to_device(pl, segs.data(), sizeof(SegCopy) * segs.size(), &st.segs);
    if (!rc) rc = copy_to_device(pl, chunk_seg.data(), sizeof(int64_t) * chunk_seg.size(), &st.chunk_seg);
    if (!rc) rc = copy_to_device(pl, nullptr, sizeof(int2) * (size_t)(st.pack.d.nslices * st.pack.d.Nu), &st.lrank);
    if (rc) return rc;
    // the line table, once per plan
    StagedTile g;
    std::memset(&g, 0, sizeof(g));
    g.d = st.pack.d;
    g.M = M;
    g.nbq = nbq;
    for (int i = 0; i < kMaxDims; ++i) g.srcpos[i] = st.pack.srcpos[i];
    g.vpos = st.pack.vpos;
    g.T = pl->T;
    g.P = P;
    g.recv = (const RecvInfo *)st.recv_info;
    const int64_t lines = g.d.nslices * g.d.Nu;
    const int64_t blocks = std::min<int64_t>((lines + kThreads - 1) / kThreads, 65536);
    hipLaunchKernelGGL(staged_rank_kernel, dim3((unsigned)blocks), dim3(kThreads), 0, nullptr, g, (int2 *)st.lrank);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) return fail(FFTRW_E_DEVICE, std::string("staged line table: ") + hipGetErrorString(e));
    return FFTRW_OK;
}

namespace {

StagedTile tile_args(const fft_plan_impl *pl, const StagedStep &st, const StagedTileCfg &c)
{
    StagedTile g;
    std::memset(&g, 0, sizeof(g));
    g.d = c.d;
    g.lu = c.lu;
    g.lv = c.lv;
    g.lg = c.lg;
    g.lane_r = c.lane_r;
    g.lane_w = c.lane_w;
    g.M = pl->M;
    g.nbq = st.nbq;
    for (int i = 0; i < kMaxDims; ++i) g.srcpos[i] = c.srcpos[i];
    g.vpos = c.vpos;
    g.pair_lg = st.pair_lg;
    g.T = pl->T;
    g.P = pl->P;
    g.recv = (const RecvInfo *)st.recv_info;
    g.lrank = (const int2 *)st.lrank;
    g.pairs = (const PairSlot *)st.pairs;
    return g;
}

// part 0: pack (layout A -> send array), 1: exchange (only segments between
// different processes), 2: unpack (receive array and kept segments -> layout B)
template <typename C>
hipError_t launch_staged(const fft_plan_impl *pl, const StagedStep &st, int part, const void *in, void *out,
                         hipStream_t s, int t)
{
    if (part == 0) {
        const StagedTile g = tile_args(pl, st, st.pack);
        const size_t lds = tile_lds(g.lu, g.lv, g.lg, sizeof(C), true).total;
        const unsigned n = (unsigned)(g.d.tiles_u * g.d.tiles_v * g.d.tiles_g);
        const C *i = (const C *)in;
        C *o = (C *)pl->send;
        if (g.lane_w == 0)
            hipLaunchKernelGGL((staged_tile_kernel<C, true, 0, 0>), dim3(n), dim3(kThreads), lds, s, i, i, o, g);
        else if (g.lane_w == 1)
            hipLaunchKernelGGL((staged_tile_kernel<C, true, 0, 1>), dim3(n), dim3(kThreads), lds, s, i, i, o, g);
        else
            hipLaunchKernelGGL((staged_tile_kernel<C, true, 0, 2>), dim3(n), dim3(kThreads), lds, s, i, i, o, g);
        return hipGetLastError();
    }
    if (part == 1) {
        if (st.seg_elems == 0) return hipSuccess;
        ExchangeArgs x;
        x.segs = (const SegCopy *)st.segs;
        x.chunk_seg = (const int64_t *)st.chunk_seg;
        x.nseg = st.nseg;
        x.total = st.seg_elems;
        x.counter = pl->counters + (size_t)t * kCountBlock;
        const unsigned xb = (unsigned)((st.seg_elems + kChunk - 1) / kChunk);
        hipLaunchKernelGGL(exchange_kernel<C>, dim3(xb), dim3(kThreads), 0, s, (const C *)pl->send, (C *)pl->recv,
                           x);
        return hipGetLastError();
    }
    const StagedTile g = tile_args(pl, st, st.unpack);
    const size_t lds = tile_lds(g.lu, g.lv, g.lg, sizeof(C), false).total;
    const unsigned n = (unsigned)(g.d.tiles_u * g.d.tiles_v * g.d.tiles_g);
    const C *r = (const C *)pl->recv, *sd = (const C *)pl->send;
    C *o = (C *)out;
    if (g.lane_r == 0)
        hipLaunchKernelGGL((staged_tile_kernel<C, false, 0, 1>), dim3(n), dim3(kThreads), lds, s, r, sd, o, g);
    else if (g.lane_r == 1)
        hipLaunchKernelGGL((staged_tile_kernel<C, false, 1, 1>), dim3(n), dim3(kThreads), lds, s, r, sd, o, g);
    else
        hipLaunchKernelGGL((staged_tile_kernel<C, false, 2, 1>), dim3(n), dim3(kThreads), lds, s, r, sd, o, g);
    return hipGetLastError();
}

}  // namespace

int staged_part(fft_plan_impl *pl, int t, int part, const void *in, void *out, hipStream_t s)
{
    const StagedStep &st = pl->staged[t];
    const hipError_t e = pl->esz == 16 ? launch_staged<double2>(pl, st, part, in, out, s, t)
                                       : launch_staged<float2>(pl, st, part, in, out, s, t);
    if (e != hipSuccess) return fail(FFTRW_E_DEVICE, std::string("staged transpose launch: ") + hipGetErrorString(e));
    return FFTRW_OK;
}

int staged_run(fft_plan_impl *pl, int t, const void *in, void *out, hipStream_t s)
{
    for (int part = 0; part < 3; ++part)
        if (int rc = staged_part(pl, t, part, in, out, s)) return rc;
    return FFTRW_OK;
}

void staged_free(fft_plan_impl *pl)
{
    for (StagedStep &st : pl->staged) {
        for (void *p : {st.recv_info, st.lrank, st.pairs, st.segs, st.chunk_seg})
            if (p) (void)hipFree(p);
        st = StagedStep{};
    }
    if (pl->send) (void)hipFree(pl->send);
    if (pl->recv) (void)hipFree(pl->recv);
    pl->send = pl->recv = nullptr;
}

}  // namespace fftrw
