// fused_generic.hpp -- one FFT step fused with the transpose that follows it,
// for rows of any 2,3,5-smooth length (device code of the persistent batched
// kernel).
//
// A unit takes RW rows of layout A that are consecutive in v (the last axis of
// the next layout B) in each of G consecutive batch slices (G > 1 when the
// rows are short): each row is contiguous along u
// (the FFT axis), rows sit a_sv apart.  The rows are staged in LDS (row stride
// N + 1, so reading a column touches distinct banks), transformed by the same
// Stockham passes as fft_rows_block, and written in layout B: for every
// frequency k the RW results form one run of consecutive v.  One HBM round trip
// replaces two (the FFT step's and the transpose's).  Owner changes are counted
// per row as in the transpose tile (tile_moved).
#pragma once

#include <hip/hip_runtime.h>

#include "cplx.hpp"
#include "fft_generic.hpp"
#include "kernels.hpp"
#include "xpose_tile.hpp"

namespace fftrw {

constexpr int kUnitItems = 16;  // loads in flight per thread while a unit is staged

// Shape of a fused unit for rows of length N: RW rows per slice (a power of
// two covering the v extent when it can) and G slices, so that a unit holds at
// most `budget` values (4096 complex64, 2048 complex128) and every row keeps at
// least one lane of the 256-thread group.
inline void fused_unit_shape(int N, int64_t Nv, int64_t nslices, int budget, int *rw, int *G)
{
    int r = 1;
    while (r * 2 <= 256 && (int64_t)r * 2 * (N + 1) <= budget && r * 2 <= 2 * Nv - 1) r *= 2;
    int g = 1;
    while (g * 2 * r <= 256 && (int64_t)g * 2 * r * (N + 1) <= budget && g * 2 <= 2 * nslices - 1) g *= 2;
    *rw = r;
    *G = g;
}

// LDS bytes of a fused unit: G * RW padded rows, the slices' bases, one int
__host__ __device__ inline size_t fused_unit_bytes(int N, int rw, int G, size_t esz)
{
    return (((size_t)G * rw * (N + 1) * esz + 15) & ~(size_t)15) + (size_t)G * 16 + 16;
}

// Unit `unit` of a fused step: v-block unit % tiles_v of G consecutive slices.
template <typename C, int DIR>
__device__ __forceinline__ void fft_xpose_unit(const C *__restrict__ in, C *__restrict__ out, const FftDesc &f,
                                               const XposeDesc &d, int rw, int G, int64_t unit,
                                               typename RealOf<C>::type scale, bool do_scale, unsigned char *smem)
{
    const int N = f.N;
    const int S = N + 1;
    C *lds = reinterpret_cast<C *>(smem);
    const size_t rows_bytes = ((size_t)G * rw * S * sizeof(C) + 15) & ~(size_t)15;
    int64_t *abase = reinterpret_cast<int64_t *>(smem + rows_bytes);
    int64_t *bbase = abase + G;
    const int64_t tiles_v = (d.Nv + rw - 1) / rw;
    const int64_t tv = unit % tiles_v;
    const int64_t g0 = (unit / tiles_v) * G;
    const int64_t v0 = tv * rw;
    const int nv = (int)min<int64_t>(rw, d.Nv - v0);
    const int ng = (int)min<int64_t>(G, d.nslices - g0);
    for (int gi = threadIdx.x; gi < ng; gi += kThreads) {
        int bc[3];
        slice_coords(d, g0 + gi, bc, &abase[gi], &bbase[gi]);
    }
    __syncthreads();

    // rows (slice g0 + gi, v0 + r), rho = gi nv + r: N contiguous values each;
    // element e = rho N + c, stepped by kThreads without divisions.  Up to
    // kUnitItems loads are issued before any of them is stored to LDS, so a
    // thread keeps its whole share in flight (a unit holds at most 16 values
    // per thread).
    // Every thread with rows to count (threadIdx.x < ng nv) has loads too.
    int moved = 0;
    bool counted = false;
    {
        const int drho = kThreads / N, dc = kThreads - drho * N;
        int rho = threadIdx.x / N, c = threadIdx.x - rho * N;
        int gi = rho / nv, r = rho - gi * nv;
        const int drg = drho / nv, drr = drho - drg * nv;
        while (gi < ng) {
            C val[kUnitItems];
            int at[kUnitItems];
#pragma unroll
            for (int j = 0; j < kUnitItems; ++j) {
                at[j] = -1;
                if (gi < ng) {
                    at[j] = (gi * rw + r) * S + c;
                    val[j] = xld(in + abase[gi] + (v0 + r) * d.a_sv + c);
                    c += dc;
                    gi += drg;
                    r += drr;
                    if (c >= N) {
                        c -= N;
                        ++r;
                    }
                    while (r >= nv) {
                        r -= nv;
                        ++gi;
                    }
                }
            }
            if (d.count && !counted) {  // owner changes, while the first loads are in flight
                moved = tile_moved(d, g0, ng, 0, N, v0, nv);
                counted = true;
            }
#pragma unroll
            for (int j = 0; j < kUnitItems; ++j)
                if (at[j] >= 0) lds[at[j]] = val[j];
        }
    }
    if (d.count) {
        // each wave publishes its sum at once: work left for the end of the
        // unit would delay the group's next unit or its exit
        for (int off = 32; off > 0; off >>= 1) moved += __shfl_xor(moved, off);
        if ((threadIdx.x & 63) == 0 && moved)
            atomicAdd(d.counter + (unit % kCountSlots) * kCountStride, (unsigned long long)moved);
    }
    __syncthreads();
    const int lanes = kThreads / (G * rw);
    const int row = threadIdx.x / lanes;
    const int lane = threadIdx.x - row * lanes;
    C *lrow = lds + row * S;
    const C *tw = reinterpret_cast<const C *>(f.tw);
    int Ns = 1;
    for (int p = 0; p < f.npass; ++p) {
        switch (f.radix[p]) {
        case 2: stockham_pass<2, DIR>(lrow, N, Ns, lanes, lane, tw); break;
        case 3: stockham_pass<3, DIR>(lrow, N, Ns, lanes, lane, tw); break;
        case 4: stockham_pass<4, DIR>(lrow, N, Ns, lanes, lane, tw); break;
        case 5: stockham_pass<5, DIR>(lrow, N, Ns, lanes, lane, tw); break;
        case 8: stockham_pass<8, DIR>(lrow, N, Ns, lanes, lane, tw); break;
        case 16: stockham_pass<16, DIR>(lrow, N, Ns, lanes, lane, tw); break;
        default: break;
        }
        Ns *= f.radix[p];
    }
    // frequency k of row (gi, r) goes to B at (slice g0 + gi, u = k, v = v0 + r):
    // element e = (gi N + k) nv + r, runs of nv consecutive v
    {
        const int dkk = kThreads / nv, dr = kThreads - dkk * nv;
        int kk = threadIdx.x / nv, r = threadIdx.x - kk * nv;
        int gi = kk / N, k = kk - gi * N;
        const int dg = dkk / N, dk = dkk - dg * N;
        while (gi < ng) {
            C q = lds[(gi * rw + r) * S + k];
            if (do_scale) q = cscale(q, scale);
            xst(out + bbase[gi] + (int64_t)k * d.b_su + v0 + r, q);
            r += dr;
            gi += dg;
            k += dk;
            if (r >= nv) {
                r -= nv;
                ++k;
            }
            if (k >= N) {
                k -= N;
                ++gi;
            }
        }
    }
    __syncthreads();  // the LDS block may be reused by the caller's next unit
}

}  // namespace fftrw
