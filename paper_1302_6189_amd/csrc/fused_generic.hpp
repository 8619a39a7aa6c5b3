// fused_generic.hpp -- one FFT step fused with the transpose that follows it,
// for rows of any 2,3,5-smooth length (device code shared by single plans and
// the persistent batched kernel).
//
// A unit takes RW rows of layout A that are consecutive in v (the last axis of
// the next layout B) in each of G consecutive batch slices (G > 1 when the
// rows are short): each row is contiguous along u
// (the FFT axis), rows sit a_sv apart.  The rows are staged in LDS (row pitch
// N + 1, or N + 2 for even complex64 rows, see unit_pitch), with the twiddle
// table when it is small, transformed by the same Stockham passes as
// fft_rows_block, and written in layout B: for every
// frequency k the RW results form one run of consecutive v.  One HBM round trip
// replaces two (the FFT step's and the transpose's).  Owner changes are counted
// per row as in the transpose tile (tile_moved).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>

#include "cplx.hpp"
#include "fft_generic.hpp"
#include "kernels.hpp"
#include "xpose_tile.hpp"

namespace fftrw {

constexpr int kUnitItems = 16;  // loads in flight per thread while a unit is staged

// LDS pitch of a unit's rows: one value of padding, two for even complex64
// rows so that every row starts 16 bytes aligned and a 16-byte pair of
// values goes to LDS in one store (two 8-byte stores of the pairs conflict
// on the LDS banks)
__host__ __device__ inline int unit_pitch(int N, size_t esz) { return esz == 8 && N % 2 == 0 ? N + 2 : N + 1; }

// Shape of a fused unit for rows of length N: RW rows consecutive in v per
// slice and G slices (RW G rows, at most kThreads of them, holding at most
// `budget` values with their padding: 4096 complex64, 2048 complex128; each
// row gets a power of two of lanes, unit_lanes, with at most 16 values per
// lane).  RW is the whole v extent when it fits (a slice's outputs are then
// one contiguous block), else a multiple of 16 (runs of whole 128-byte
// lines for complex64), else the largest power of two that fits; among
// those the shape with the fewest units, ceil(N_v / RW) ceil(slices / G),
// is taken (ties: longer runs).  Each unit is one chain of loads, barriers,
// passes and stores, so fuller units mean fewer chains; shorter runs would
// write partial lines.
inline int unit_lanes(int rows)
{
    int lanes = 1;
    while (lanes * 2 * rows <= kThreads) lanes *= 2;
    return lanes;
}

inline void fused_unit_shape(int N, size_t esz, int64_t Nv, int64_t nslices, int budget, int *rw, int *G)
{
    budget = budget < kUnitItems * kThreads ? budget : kUnitItems * kThreads;  // one load pass per unit
    const int P = unit_pitch(N, esz);
    int maxrows = budget / P < kThreads ? budget / P : kThreads;
    // rows such that every row keeps at least ceil(N / 16) lanes
    while (maxrows > 1 && N > 16 * unit_lanes(maxrows)) --maxrows;
    if (maxrows < 1) maxrows = 1;
    int64_t best = -1;
    int br = 1, bg = 1;
    auto consider = [&](int r) {
        const int64_t g = std::min<int64_t>(maxrows / r, nslices);
        const int64_t units = ((Nv + r - 1) / r) * ((nslices + g - 1) / g);
        if (best < 0 || units < best || (units == best && r > br)) {
            best = units;
            br = r;
            bg = (int)g;
        }
    };
    if (Nv <= maxrows) {
        consider((int)Nv);
    } else if (maxrows >= 16) {
        for (int r = 16; r <= maxrows; r += 16) consider(r);
    } else {
        int r = 1;
        while (r * 2 <= maxrows) r *= 2;
        consider(r);
    }
    *rw = br;
    *G = bg;
}

// Units may stage the row length's twiddle table in LDS when its N entries
// take at most 16 KB (the passes then read it there instead of through the
// caches); longer rows keep the unit within 64 KB of LDS.
constexpr size_t kUnitTwLds = 16384;
__host__ __device__ inline bool unit_tw_fits(int N, size_t esz) { return (size_t)N * esz <= kUnitTwLds; }

// LDS bytes of a fused unit: G * RW padded rows, the twiddle table when
// staged, the slices' bases, one int
__host__ __device__ inline size_t fused_unit_bytes(int N, int rw, int G, size_t esz, bool tw_lds)
{
    return (((size_t)G * rw * unit_pitch(N, esz) * esz + 15) & ~(size_t)15) +
           (tw_lds ? (((size_t)N * esz + 15) & ~(size_t)15) : 0) + (size_t)G * 16 + 16;
}

// Element `off` of an array of fewer than 2^32 bytes: the byte offset is
// formed in 32 bits and added to the (uniform) base, so the access takes the
// scalar-base, 32-bit-offset form instead of 64-bit address arithmetic.
template <typename C> __device__ __forceinline__ C *at_off32(C *base, uint32_t off)
{
    return reinterpret_cast<C *>(reinterpret_cast<char *>(base) + off * (uint32_t)sizeof(C));
}
template <typename C> __device__ __forceinline__ const C *at_off32(const C *base, uint32_t off)
{
    return reinterpret_cast<const C *>(reinterpret_cast<const char *>(base) + off * (uint32_t)sizeof(C));
}

// Rows (slice g0 + gi, v0 + r) of a unit into LDS (row rho = gi rw + r at
// rho S), W consecutive values per access (W = 2: 16-byte loads and LDS
// stores of complex64, N and S even, so every row starts on an even element
// in HBM and 16 bytes aligned in LDS).  Group e = rho N / W + c is stepped by
// kThreads without divisions.  A unit holds at most kUnitItems values per
// thread (fused_unit_shape keeps it within kUnitItems * kThreads values), so
// every load of the thread is issued before any is stored to LDS, in one
// pass with no loop around it: a loop would make the compiler wait for the
// loads of one trip before it reuses their registers on the next.  The owner
// changes of the unit's rows are counted while the loads are in flight:
// every thread with rows to count (threadIdx.x < ng nv) has loads too.
template <int W, bool OFF32, typename C>
__device__ __forceinline__ void load_unit_rows(const C *__restrict__ in, C *lds, const FftDesc &f,
                                               const XposeDesc &d, const int64_t *abase, int S, int rw, int nv,
                                               int ng, int64_t g0, int64_t v0, int &moved)
{
    constexpr int ITEMS = kUnitItems / W;
    const int N = f.N;
    const int NW = N / W;
    const int drho = kThreads / NW, dc = kThreads - drho * NW;
    int rho = threadIdx.x / NW, c = threadIdx.x - rho * NW;
    int gi = rho / nv, r = rho - gi * nv;
    const int drg = drho / nv, drr = drho - drg * nv;
    C val[ITEMS][W];
    int at[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        at[j] = -1;
        if (gi < ng) {
            at[j] = (gi * rw + r) * S + c * W;
            const C *p = OFF32 ? at_off32(in, (uint32_t)abase[gi] + (uint32_t)(v0 + r) * (uint32_t)d.a_sv + c * W)
                               : in + abase[gi] + (v0 + r) * d.a_sv + c * W;
            if constexpr (W == 2) {
                const xf4 w = gld_nt(reinterpret_cast<const xf4 *>(p));
                val[j][0] = mk<C>(w.x, w.y);
                val[j][1] = mk<C>(w.z, w.w);
            } else {
                val[j][0] = xld(p);
            }
            // c < NW and r < nv before the step, dc < NW and drr < nv: each
            // wraps at most once
            c += dc;
            gi += drg;
            r += drr;
            if (c >= NW) {
                c -= NW;
                ++r;
            }
            if (r >= nv) {
                r -= nv;
                ++gi;
            }
        }
    }
    if (d.count) moved = tile_moved(d, g0, ng, 0, N, v0, nv);
#pragma unroll
    for (int j = 0; j < ITEMS; ++j)
        if (at[j] >= 0) {
            if constexpr (W == 2) {
                const xf4 w4 = {val[j][0].x, val[j][0].y, val[j][1].x, val[j][1].y};
                *reinterpret_cast<xf4 *>(lds + at[j]) = w4;
            } else {
                lds[at[j]] = val[j][0];
            }
        }
}

// The transformed rows to B: frequency k of row (gi, r) at (slice g0 + gi,
// u = k, v = v0 + r).  Group e = (gi N + k) nv / W + r / W, W consecutive v
// per access (W = 2: 16-byte stores of complex64, nv and every run start
// even).
template <int W, bool OFF32, typename C>
__device__ __forceinline__ void store_unit_runs(C *__restrict__ out, const C *lds, const XposeDesc &d,
                                                const int64_t *bbase, int N, int S, int rw, int nv, int ng,
                                                int64_t v0, typename RealOf<C>::type scale, bool do_scale)
{
    const int nvw = nv / W;
    const int dkk = kThreads / nvw, dr = kThreads - dkk * nvw;
    int kk = threadIdx.x / nvw, r = threadIdx.x - kk * nvw;
    int gi = kk / N, k = kk - gi * N;
    const int dg = dkk / N, dk = dkk - dg * N;
    while (gi < ng) {
        C q[W];
#pragma unroll
        for (int w = 0; w < W; ++w) {
            q[w] = lds[(gi * rw + r * W + w) * S + k];
            if (do_scale) q[w] = cscale(q[w], scale);
        }
        C *p = OFF32 ? at_off32(out, (uint32_t)bbase[gi] + (uint32_t)k * (uint32_t)d.b_su + (uint32_t)v0 + r * W)
                     : out + bbase[gi] + (int64_t)k * d.b_su + v0 + r * W;
        if constexpr (W == 2) {
            const xf4 w = {q[0].x, q[0].y, q[1].x, q[1].y};
            gst_nt(w, reinterpret_cast<xf4 *>(p));
        } else {
            xst(p, q[0]);
        }
        r += dr;
        gi += dg;
        k += dk;
        if (r >= nvw) {
            r -= nvw;
            ++k;
        }
        if (k >= N) {
            k -= N;
            ++gi;
        }
    }
}

struct NoHook {
    __device__ void operator()() const {}
};

// Unit `unit` of a fused step: v-block unit % tiles_v of G consecutive slices.
// TW_LDS: the twiddle table is staged in LDS (the caller checked unit_tw_fits
// and sized the LDS block with it).  LEAN: the step's radices are 2, 3, 4 and
// 5 only (the caller made sure), so the larger passes are not compiled in.
// OFF32: `in` and `out` each hold fewer than 2^32 bytes (the caller made
// sure), and HBM addresses are formed from 32-bit offsets.  hook() runs once the unit's rows are in LDS, after a barrier that every
// thread passed after entering the unit; no HBM access of the unit's is in
// flight then except the owner-count atomics.
template <typename C, int DIR, bool TW_LDS, bool LEAN = false, bool OFF32 = false, typename Hook = NoHook>
__device__ __forceinline__ void fft_xpose_unit(const C *__restrict__ in, C *__restrict__ out, const FftDesc &f,
                                               const XposeDesc &d, int rw, int G, int64_t unit,
                                               typename RealOf<C>::type scale, bool do_scale, unsigned char *smem,
                                               Hook hook = Hook())
{
    const int N = f.N;
    const int S = unit_pitch(N, sizeof(C));
    C *lds = reinterpret_cast<C *>(smem);
    const size_t rows_bytes = ((size_t)G * rw * S * sizeof(C) + 15) & ~(size_t)15;
    C *ltw = reinterpret_cast<C *>(smem + rows_bytes);
    const size_t tw_bytes = TW_LDS ? (((size_t)N * sizeof(C) + 15) & ~(size_t)15) : 0;
    int64_t *abase = reinterpret_cast<int64_t *>(smem + rows_bytes + tw_bytes);
    int64_t *bbase = abase + G;
    // in 32 bits: the plans keep every size at most 4096, the slice count and
    // a step's unit count below 2^31
    const uint32_t tiles_v = ((uint32_t)d.Nv + (uint32_t)rw - 1) / (uint32_t)rw;
    const uint32_t tv = (uint32_t)unit % tiles_v;
    const int64_t g0 = (int64_t)((uint32_t)unit / tiles_v) * G;
    const int64_t v0 = (int64_t)tv * rw;
    const int nv = (int)min<int64_t>(rw, d.Nv - v0);
    const int ng = (int)min<int64_t>(G, d.nslices - g0);
    for (int gi = threadIdx.x; gi < ng; gi += kThreads) {
        int bc[3];
        slice_coords(d, g0 + gi, bc, &abase[gi], &bbase[gi]);
    }
    __syncthreads();

    // a staged twiddle table's first kThreads entries are loaded before the
    // rows, so that both arrive in one memory round trip
    const C *gtw = reinterpret_cast<const C *>(f.tw);
    C tw0 = mk<C>(0, 0);
    if constexpr (TW_LDS)
        if (threadIdx.x < N) tw0 = gld(gtw + threadIdx.x);
    // rows (slice g0 + gi, v0 + r), rho = gi nv + r: N contiguous values each,
    // read in 16-byte pairs when N is even (complex64)
    int moved = 0;
    if constexpr (sizeof(C) == 8) {
        if (N % 2 == 0) {
            load_unit_rows<2, OFF32>(in, lds, f, d, abase, S, rw, nv, ng, g0, v0, moved);
        } else {
            load_unit_rows<1, OFF32>(in, lds, f, d, abase, S, rw, nv, ng, g0, v0, moved);
        }
    } else {
        load_unit_rows<1, OFF32>(in, lds, f, d, abase, S, rw, nv, ng, g0, v0, moved);
    }
    hook();
    if constexpr (TW_LDS) {
        if (threadIdx.x < N) ltw[threadIdx.x] = tw0;
        for (int i = threadIdx.x + kThreads; i < N; i += kThreads) ltw[i] = gld(gtw + i);
    }
    if (d.count) {
        // each wave publishes its sum at once: work left for the end of the
        // unit would delay the group's next unit or its exit
        for (int off = 32; off > 0; off >>= 1) moved += __shfl_xor(moved, off);
        if ((threadIdx.x & 63) == 0 && moved)
            atomicAdd(d.counter + (unit % kCountSlots) * kCountStride, (unsigned long long)moved);
    }
    __syncthreads();
    // each of the G rw rows gets a power of two of lanes; threads past the
    // last row take part in the barriers only (lane N: no butterfly)
    const int lanes = 1 << (31 - __clz(kThreads / (G * rw)));
    const int row = threadIdx.x / lanes;
    const bool in_row = row < G * rw;
    const int lane = in_row ? threadIdx.x - row * lanes : N;
    C *lrow = lds + (in_row ? row : 0) * S;
    const C *tw = TW_LDS ? static_cast<const C *>(ltw) : reinterpret_cast<const C *>(f.tw);
    // a row's lanes are consecutive threads, a power of two of them: at most
    // 64 sit in one wave, and the passes then synchronise that wave only (the
    // stores read across rows and wait for the whole group)
    const bool wave = lanes <= 64;
    int Ns = 1;
    for (int p = 0; p < f.npass; ++p) {
        switch (f.radix[p]) {
        case 2: stockham_pass<2, DIR>(lrow, N, Ns, lanes, lane, tw, wave); break;
        case 3: stockham_pass<3, DIR>(lrow, N, Ns, lanes, lane, tw, wave); break;
        case 4: stockham_pass<4, DIR>(lrow, N, Ns, lanes, lane, tw, wave); break;
        case 5: stockham_pass<5, DIR>(lrow, N, Ns, lanes, lane, tw, wave); break;
        case 8:
            if constexpr (!LEAN) stockham_pass<8, DIR>(lrow, N, Ns, lanes, lane, tw, wave);
            break;
        case 16:
            if constexpr (!LEAN) stockham_pass<16, DIR>(lrow, N, Ns, lanes, lane, tw, wave);
            break;
        default: break;
        }
        Ns *= f.radix[p];
    }
    if (wave) __syncthreads();
    // frequency k of row (gi, r) goes to B at (slice g0 + gi, u = k, v = v0 + r),
    // runs of nv consecutive v; 16-byte pairs of v when N_v and rw are even
    // (complex64: every run then starts on an even element)
    if constexpr (sizeof(C) == 8) {
        if (d.Nv % 2 == 0 && rw % 2 == 0) {
            store_unit_runs<2, OFF32>(out, lds, d, bbase, N, S, rw, nv, ng, v0, scale, do_scale);
        } else {
            store_unit_runs<1, OFF32>(out, lds, d, bbase, N, S, rw, nv, ng, v0, scale, do_scale);
        }
    } else {
        store_unit_runs<1, OFF32>(out, lds, d, bbase, N, S, rw, nv, ng, v0, scale, do_scale);
    }
    __syncthreads();  // the LDS block may be reused by the caller's next unit
}

}  // namespace fftrw
