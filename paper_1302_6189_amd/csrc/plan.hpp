// plan.hpp -- the execution plan behind fft_plan_t.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "decomp.hpp"
#include "kernels.hpp"

namespace fftrw {

// Tiling of a staged pack or unpack kernel (see staged.hip).
struct StagedTileCfg {
    XposeDesc d;                  // geometry; batch axis 0 is the tile's slice axis
    int lu = 0, lv = 0, lg = 0;   // log2 of the tile's extents along u, v, slices
    int lane_r = 0, lane_w = 0;   // axis fastest across lanes when reading / writing
    int srcpos[kMaxDims] = {};    // per A position: batch index 0..2, 3 = v, 4 = u
    int vpos = 0;                 // A position of v
};

// Staged transpose tables (pack -> exchange -> unpack), see staged.hip.
struct StagedStep {
    int64_t npair = 0;            // (p, q) pairs that share points
    void *recv_info = nullptr;    // device RecvInfo[P]: destination ranges
    void *lrank = nullptr;        // device int2 per (slice, u) line: rank at v = 0, step per v
    void *pairs = nullptr;        // device pair table: D(p, q) of every pair, by hash of (p, q)
    int pair_lg = 0;              // log2 of the pair table's slots
    int nbq = 0;                  // boxes per destination range
    int64_t nseg = 0;
    void *segs = nullptr;         // device SegCopy[nseg] (p != q only)
    void *chunk_seg = nullptr;    // device int64[2 * chunks]: first/last segment of each exchange chunk
    int64_t seg_elems = 0;        // = the transpose's amount (points exchanged)
    int seg_axis = -1;            // natural axis along which segments run
    StagedTileCfg pack, unpack;   // tilings of the two kernels
};

// Device memory handed to a plan in place of hipMalloc: bump allocation from
// a fixed region (nothing is freed), twiddle tables generated on `stream`.
struct DevArena {
    unsigned char *base = nullptr;
    size_t cap = 0, used = 0;
    hipStream_t stream = nullptr;
};

// An FFT step at level M run as a binary exchange among the processes that
// share each row (staged plans; see rowsplit.hip): every range holds b points,
// a row is c = 2^s ranges.
struct SplitStep {
    int b = 0, c = 0, s = 0;      // c = 0: the step's rows are whole
    void *tw = nullptr;           // w_N^e, e < N (the butterflies' twiddles)
    FftDesc local = {};           // the b-point DFTs of the blocks (b > 1)
};

struct fft_plan_impl {
    int M = 0;
    i64 dims[kMaxDims] = {};
    i64 P = 0;
    int8_t order[kMaxDims * kMaxDims] = {};
    int dtype = 1;
    int precision = 0;
    unsigned flags = 0;
    int ownership = 0;
    i64 T = 0;
    size_t esz = 8;
    int device = 0;

    Layout lay[kMaxDims + 1];           // pi_1..pi_M, then natural
    std::vector<FftDesc> fft;           // per step
    std::vector<XposeDesc> xp;          // per transpose (M of them)
    std::vector<i64> analytic;          // M: steps then return transpose
    std::vector<std::vector<i64>> mu;   // per transpose relabelling (matched)
    std::vector<StagedStep> staged;     // per transpose (STAGED flag)
    bool xp_staged[kMaxDims] = {};      // transpose t runs through staged tables
    std::vector<SplitStep> split;       // per step (staged plans at level M)
    std::vector<i64> split_analytic;    // per step: points the split rows' exchange moves

    // device memory
    void *work = nullptr;
    void *send = nullptr, *recv = nullptr;
    unsigned long long *counters = nullptr;  // M blocks (transposes), + M (split-row exchanges) when staged
    int n_counters = 0;                      // 64-bit words in counters
    std::vector<void *> allocs;
    DevArena *arena = nullptr;          // set: device memory comes from the arena, never hipMalloc
    std::map<int, void *> twiddles;
    size_t dev_bytes = 0;
    bool executed = false;
    bool fused = false;                 // FFT steps fused with the following transpose
    int fuse_kind[kMaxDims] = {};       // per step: 1 power-of-two kernel, 2 generic smooth-length unit

    // per-stage timing events (fft_plan_set_timing)
    bool timing = false;
    std::vector<hipEvent_t> events;  // stage boundaries of the last exec
    int n_recorded = 0;
};

}  // namespace fftrw

struct fft_plan_s : fftrw::fft_plan_impl {};
