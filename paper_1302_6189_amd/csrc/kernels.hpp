// kernels.hpp -- argument blocks shared by the host driver and the HIP kernels.
#pragma once

#include <cstdint>

namespace fftrw {

constexpr int kMaxPasses = 12;
constexpr int kThreads = 256;  // work-group size of every kernel here (4 waves of 64)

// A device owner-change counter is kCountSlots partial sums on separate
// 128-byte lines; work-group i adds to slot i % kCountSlots and readers sum
// the slots.  One address shared by every work-group would serialise their
// atomics across the chip's L2 slices.
constexpr int kCountSlots = 32;
constexpr int kCountStride = 16;  // 64-bit words between slots
constexpr int kCountBlock = kCountSlots * kCountStride;

// One batched 1-D FFT pass set: nrows contiguous rows of length N, transformed
// by Stockham autosort passes with the given radices (product = N).
struct FftDesc {
    int N;
    int npass;
    int radix[kMaxPasses];
    int rows_per_wg;   // RW: rows held in LDS by one work-group (power of two)
    int lanes_per_row; // 256 / RW threads cooperate on one row
    int64_t nrows;
    const void *tw;    // forward twiddles w_N^e, e = 0..N-1 (float2 or double2),
                       // or the per-pass table of the power-of-two kernel
    int pow2;          // 1: compile-time power-of-two kernel (fft_pow2.hip)
    int mfma;          // > 0: 256/512-point split-precision MFMA kernel (fft_mfma.hip)
    int tw_count;      // entries in the twiddle table
};

// Fused permutation of the whole array from layout A to layout B with a
// per-tile count of points whose owner changes (see transpose kernels).
struct XposeDesc {
    // fast axes: u = fastest axis of A (read contiguously), v = fastest of B
    int64_t Nu, Nv;
    int64_t a_sv;   // stride of v in A
    int64_t b_su;   // stride of u in B
    // batch axes (the other M-2 axes), innermost first
    int nbat;
    int64_t bsize[3], ba[3], bb[3];
    int64_t nslices;  // product of bsize
    // tiling
    int TU, TV, G;    // tile extents along u, v and number of batch slices per tile
    int64_t tiles_u, tiles_v, tiles_g;
    // owner counting (0 = off)
    int count;
    int ka, kb;              // levels of A and B
    int srca[5], srcb[5];    // for each leading axis: 0..2 batch index, 3 = v, 4 = u
                             // (u leads in A and v in B only at level M)
    int64_t wa[5], wb[5];    // row-index weights of the leading axes
    int64_t Ra, Rb, P;
    int owner32;             // (r+1) P - 1 fits in 32 bits for both layouts
    const int *mu;           // relabelling of A's ranges (nullable = identity)
    unsigned long long *counter;  // kCountBlock words (slots, see kCountSlots)
};

}  // namespace fftrw
