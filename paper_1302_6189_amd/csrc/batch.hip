// batch.hip -- many uneven transforms in one persistent launch.
//
// Each item is a whole Fig. 4 pipeline (M FFT steps and M transposes) with its
// own sizes, process count and order.  The work of all items is cut into
// units -- a block of rows of one FFT step, or a tile of one transpose --
// grouped into stage levels: level s holds stage s of every item that has
// one.  One grid of work-groups, sized to stay resident, sweeps the levels:
// inside a level units are taken from the level's atomic counter, a few
// consecutive units per claim.  A work-group leaving a level adds the number
// of units it completed there to the level's done counter (after a release
// at device scope, issued by one wave for the group) and waits until the
// counter holds every unit of the level (then acquires, so data written on
// one XCD is seen on the others), which keeps every item's FFT -> transpose
// -> FFT order.  Counting units rather than arrivals means no
// work-group waits for one that has not started: a unit is only ever claimed
// by a running work-group, and a level is left only once all its units are
// claimed, so the wait ends whether or not the whole grid is resident
// (another kernel may hold part of the device).  Waiting polls a
// device-coherent counter without invalidating caches, and every wait is
// bounded by the real-time clock: past the bound the work-group adds one to
// a sticky time-out count and goes on, so the grid always drains and the
// host can refuse the result.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/fftrw.h"
#include "decomp.hpp"
#include "errors.hpp"
#include "fft_generic.hpp"
#include "fused_generic.hpp"
#include "kernels.hpp"
#include "plan.hpp"
#include "tune.hpp"
#include "xpose_tile.hpp"

namespace fftrw {

constexpr int kMaxStages = 2 * kMaxDims;

struct BatchItemDev {
    float2 *buf[3];                 // 0 in (read only), 1 out, 2 work
    int M;
    int nstage;                     // 2M (2M - 1 with LEAVE_PERMUTED); fused: M
    int fused;                      // stage t = FFT step t fused with transpose t
    int nx;                         // transposes executed (M, or M - 1 with LEAVE_PERMUTED)
    int frw[kMaxDims];              // rows (consecutive v) per slice of a fused unit of stage t
    int fg[kMaxDims];               // slices per fused unit of stage t
    int src[kMaxStages];            // 0 in, 1 out, 2 work
    int dst[kMaxStages];
    int64_t prefix[kMaxStages + 1]; // units of this item before stage s
    float inv_scale;                // 1/T for the inverse's last FFT step
    int xv[kMaxDims];               // 16-byte access flags of transpose t: bit0 u, bit1 v
    FftDesc fft[kMaxDims];
    XposeDesc xp[kMaxDims];
};

struct BatchTask {
    int item, stage;
    int64_t unit0, nunits;  // unit0 counts from the start of the task's level
};

// zeroed before every launch: one claim counter and one done counter per level
struct BatchCounters {
    unsigned long long next[kMaxStages];
    unsigned long long done[kMaxStages];
};

// task starts of one level held in LDS for the per-unit search
constexpr int kLevelTasksLds = 256;

// s_waitcnt operand: vector memory count 0 (bits 3:0 and 15:14), the export
// and LDS/scalar counts at their maxima (bits 6:4 and 11:8)
constexpr int kWaitVmcnt0 = 0x0F70;

// units per claim of the level counter, and the level's last units claimed
// one at a time (this many per work-group of the grid)
constexpr int kClaimUnits = 3;
constexpr int kClaimTail = 4;

// real-time clock ticks (100 MHz) a work-group may wait at one barrier
constexpr unsigned long long kWaitTicks = 200000000ull;

// Takes the next unit index from a level's claim counter (a 64-bit word
// whose low half counts; levels hold fewer than 2^32 units).  A wrapping
// increment rather than an add: the compiler rewrites a single lane's atomic
// add into a wave-wide scan that needs the result at once, which would wait
// for every load and store the wave has in flight; the increment's result is
// waited for only where it is used.
__device__ __forceinline__ unsigned claim(unsigned long long *ctr)
{
    return __builtin_amdgcn_atomic_inc32(reinterpret_cast<unsigned *>(ctr), 0xffffffffu, __ATOMIC_RELAXED, "agent");
}

// The buffer of a stage.  One uniform address, read through the scalar
// cache: a vector load would count on the wait counter that the unit's HBM
// stores also count on, and waiting for it would wait for the previous
// unit's stores as well.
__device__ __forceinline__ float2 *batch_buf(const BatchItemDev &it, int kind)
{
    return it.buf[__builtin_amdgcn_readfirstlane(kind)];
}

// The inverse (whose last stage also scales) is held to three waves per SIMD
// (at most 168 VGPRs; it needs one more otherwise, which would leave two).
// The forward fits without the hint and runs 1% faster without it.
// LEAN: every stage of every item is a fused unit with radices 2, 3, 4 and 5
// only, and every item's buffers hold fewer than 2^32 bytes (32-bit offsets);
// without the other stage kernels and the larger passes the kernel fits four
// waves per SIMD.
template <int DIR, bool TW_LDS, bool LEAN>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(LEAN ? 4 : (DIR > 0 ? 3 : 1))))
    batch_kernel(const BatchItemDev *__restrict__ items, const BatchTask *__restrict__ tasks,
                 const int *__restrict__ level_task0, const int64_t *__restrict__ level_units, int nlevels,
                 BatchCounters *ctr, unsigned long long *timeouts, unsigned long long wait_ticks)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int64_t s_unit0[kLevelTasksLds];
    __shared__ int64_t s_unit;
    __shared__ int s_task, s_end;
    for (int lv = 0; lv < nlevels; ++lv) {
        const int64_t nunits = level_units[lv];
        const int t0 = level_task0[lv], t1 = level_task0[lv + 1];
        // the level's task starts, searched in LDS when they fit
        const bool in_lds = t1 - t0 <= kLevelTasksLds;
        if (in_lds)
            for (int i = threadIdx.x; i < t1 - t0; i += kThreads) s_unit0[i] = tasks[t0 + i].unit0;
        __syncthreads();
        // Thread 0 claims units from the level's counter and finds each one's
        // task (a binary search over the level's task starts, skipped while
        // the units stay in one task).  A claim takes a chunk of kClaimUnits
        // consecutive units, and single units for the level's last
        // kClaimTail x grid, so that few atomics reach the one counter and
        // the level still ends evenly.  A unit's successor is handed to the
        // work-group (s_unit, s_task) in the middle of the unit, once the
        // unit's own row loads have arrived, and a new chunk is claimed when
        // the last unit of the current one starts: loads, stores and atomics
        // count on one wait counter in issue order, so reading a claim at
        // the next unit's start would also wait for this unit's stores.
        // (a level has fewer than 2^31 units, and claims stop one chunk past
        // its end per work-group, so unit numbers fit in 32 bits)
        const int nu32 = (int)nunits;
        const int tail = min(nu32, (int)gridDim.x * kClaimTail);
        const int nchunk = (nu32 - tail) / kClaimUnits;  // chunks of kClaimUnits
        const int head = nchunk * kClaimUnits;
        // Thread 0 keeps the unit being run and its task in s_unit and s_task
        // (which the work-group reads), the end of its chunk in s_end, and
        // the claim in flight in a register.
        unsigned pending = 0, ndone = 0;
        // thread 0: publish unit `cur` of chunk end `end`, its task searched
        // from task index `task` (counted from t0) on
        auto publish_unit = [&](int cur, int end, int task) {
            const int last = t1 - t0 - 1;
            if (cur < nu32 && task < last &&
                cur >= (in_lds ? s_unit0[task + 1] : tasks[t0 + task + 1].unit0)) {
                int lo = task + 1, hi = last;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if ((in_lds ? s_unit0[mid] : tasks[t0 + mid].unit0) <= cur)
                        lo = mid;
                    else
                        hi = mid - 1;
                }
                task = lo;
            }
            s_unit = cur;
            s_end = end;
            s_task = t0 + task;
        };
        // thread 0: the first unit of claimed chunk c
        auto publish_chunk = [&](unsigned c, int task) {
            const int ci = (int)min(c, (unsigned)nu32);  // past the end: a unit >= nunits
            const int cur = ci < nchunk ? ci * kClaimUnits : min(head + (ci - nchunk), nu32);
            publish_unit(cur, ci < nchunk ? cur + kClaimUnits : cur + 1, task);
        };
        auto publish = [&]() {
            if (threadIdx.x == 0) {
                const int cur = (int)s_unit, end = s_end, task = s_task - t0;
                if (cur + 1 < end)
                    publish_unit(cur + 1, end, task);
                else
                    publish_chunk(pending, task);
            }
        };
        if (threadIdx.x == 0) publish_chunk(claim(&ctr->next[lv]), 0);
        __syncthreads();
        for (;;) {
            // every unit function synchronises the work-group before it calls
            // publish (and non-fused units are preceded by a barrier), so these
            // reads are done before thread 0 overwrites the values
            const int64_t u = s_unit;
            const int lo = s_task;
            if (u >= nunits) break;
            if (threadIdx.x == 0) {
                ++ndone;
                if (u + 1 >= s_end) pending = claim(&ctr->next[lv]);
            }
            const BatchTask tk = tasks[lo];
            const BatchItemDev &it = items[tk.item];
            const int64_t local = u - tk.unit0;
            const int st = tk.stage;
            const float2 *src = batch_buf(it, it.src[st]);
            float2 *dst = batch_buf(it, it.dst[st]);
            if constexpr (LEAN) {
                const bool last = st == it.M - 1;
                fft_xpose_unit<float2, DIR, TW_LDS, true, true>(src, dst, it.fft[st], it.xp[st], it.frw[st], it.fg[st],
                                                                local,
                                                                DIR > 0 && last ? it.inv_scale : 1.f, DIR > 0 && last,
                                                                smem, publish);
                continue;
            }
            if (it.fused && st < it.nx) {
                const bool last = st == it.M - 1;
                fft_xpose_unit<float2, DIR, TW_LDS>(src, dst, it.fft[st], it.xp[st], it.frw[st], it.fg[st], local,
                                                    DIR > 0 && last ? it.inv_scale : 1.f, DIR > 0 && last, smem,
                                                    publish);
                continue;
            }
            // the other unit kinds take the next unit before they start
            __syncthreads();
            publish();
            if (it.fused) {
                const bool last = st == it.M - 1;
                fft_rows_block<float2, DIR>(src, dst, it.fft[st], local, DIR > 0 && last ? it.inv_scale : 1.f,
                                            DIR > 0 && last, reinterpret_cast<float2 *>(smem));
                continue;
            }
            const int t = st >> 1;
            if ((st & 1) == 0) {
                const bool last = t == it.M - 1;
                fft_rows_block<float2, DIR>(src, dst, it.fft[t], local, DIR > 0 && last ? it.inv_scale : 1.f,
                                            DIR > 0 && last, reinterpret_cast<float2 *>(smem));
            } else {
                switch (it.xv[t]) {
                case 3: xpose_tile<float2, 2, 2>(src, dst, it.xp[t], (uint32_t)local, smem); break;
                case 1: xpose_tile<float2, 2, 1>(src, dst, it.xp[t], (uint32_t)local, smem); break;
                case 2: xpose_tile<float2, 1, 2>(src, dst, it.xp[t], (uint32_t)local, smem); break;
                default: xpose_tile<float2, 1, 1>(src, dst, it.xp[t], (uint32_t)local, smem); break;
                }
            }
        }
        if (lv + 1 == nlevels) break;
        // Level barrier: publish the units this group completed, wait for
        // all.  Every wave first waits until its own stores have completed
        // (they are then in the L2; a workgroup-scope release does not wait
        // for them); the agent-scope fences are issued by thread 0's wave
        // alone: its release writes back the L2 (whatever wave wrote the
        // lines) before the count is published, and its acquire invalidates
        // the L2 and this CU's L1, which the group's other waves read
        // through after the second barrier.
        __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
        __syncthreads();
        if (threadIdx.x == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            const unsigned long long target = (unsigned long long)nunits;
            if (ndone) atomicAdd(&ctr->done[lv], (unsigned long long)ndone);
            const unsigned long long w0 = wall_clock64();
            while (__hip_atomic_load(&ctr->done[lv], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                if (wall_clock64() - w0 > wait_ticks) {
                    atomicAdd(timeouts, 1ull);
                    break;
                }
                __builtin_amdgcn_s_sleep(10);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
    }
}

__global__ void batch_reset_kernel(unsigned long long *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

}  // namespace fftrw

// ---- host side ----------------------------------------------------------------
namespace fftrw {

int plan_create(fft_plan_t *plan, int M, const int64_t *dims, int64_t P, const int8_t *order, int dtype,
                int precision, unsigned flags, bool generic_rows, const TuneTable *tune, DevArena *arena);
void plan_free(fft_plan_t plan);

struct fft_batch_impl {
    int n = 0;
    unsigned flags = 0;
    std::vector<fft_plan_t> plans;
    std::vector<BatchItemDev> h_items;
    std::vector<BatchTask> h_tasks;
    BatchItemDev *d_items = nullptr;
    BatchTask *d_tasks = nullptr;
    unsigned long long *d_ctr = nullptr;  // BatchCounters, then moved[sum of M_i]
    unsigned long long *d_timeouts = nullptr;  // sticky count of timed-out waits (never reset)
    bool timed_out = false;               // a stats call has seen d_timeouts != 0
    unsigned long long wait_ticks = kWaitTicks;  // bound of one level wait (real-time clock ticks)
    int64_t nctr = 0;
    std::vector<int> level_task0;         // first task of each level (+ end)
    std::vector<int64_t> level_units;     // units of each level
    int *d_level_task0 = nullptr;
    int64_t *d_level_units = nullptr;
    std::vector<int64_t> moved_off;       // first moved counter of each item
    int64_t total = 0;
    int grid = 0;
    size_t lds = 0;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    bool pointers_set = false;
    bool tuned = false;  // a matching autotuner cache was applied
    bool any_fused = false;
    bool tw_lds = false;  // fused units stage their twiddle tables in LDS
    bool lean = false;    // every stage a fused unit of radices 2..5 (batch_kernel's LEAN form)
};

namespace {

int batch_fail_hip(hipError_t e, const char *what)
{
    return fail(FFTRW_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

void batch_free(fft_batch_impl *b)
{
    if (!b) return;
    for (int d = 0; d < 2; ++d) {
        if (b->gexec[d]) (void)hipGraphExecDestroy(b->gexec[d]);
        if (b->graph[d]) (void)hipGraphDestroy(b->graph[d]);
    }
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    for (void *p : {(void *)b->d_items, (void *)b->d_tasks, (void *)b->d_ctr, (void *)b->d_level_task0,
                    (void *)b->d_level_units, (void *)b->d_timeouts})
        if (p) (void)hipFree(p);
    for (fft_plan_t p : b->plans) plan_free(p);
    delete b;
}

// enqueue reset + persistent kernel on stream s
int batch_enqueue(fft_batch_impl *b, int dir, hipStream_t s)
{
    const int64_t nctr = b->nctr;
    hipLaunchKernelGGL(batch_reset_kernel, dim3((unsigned)((nctr + 255) / 256)), dim3(256), 0, s, b->d_ctr, nctr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return batch_fail_hip(e, "batch reset launch");
    BatchCounters *ctr = reinterpret_cast<BatchCounters *>(b->d_ctr);
    const int nl = (int)b->level_units.size();
#define FFTRW_LAUNCH(D, T, L)                                                                                   \
    hipLaunchKernelGGL((batch_kernel<D, T, L>), dim3(b->grid), dim3(kThreads), b->lds, s, b->d_items, b->d_tasks, \
                       b->d_level_task0, b->d_level_units, nl, ctr, b->d_timeouts, b->wait_ticks)
    if (b->lean) {
        if (dir < 0) {
            if (b->tw_lds) FFTRW_LAUNCH(-1, true, true); else FFTRW_LAUNCH(-1, false, true);
        } else {
            if (b->tw_lds) FFTRW_LAUNCH(1, true, true); else FFTRW_LAUNCH(1, false, true);
        }
    } else {
        if (dir < 0) {
            if (b->tw_lds) FFTRW_LAUNCH(-1, true, false); else FFTRW_LAUNCH(-1, false, false);
        } else {
            if (b->tw_lds) FFTRW_LAUNCH(1, true, false); else FFTRW_LAUNCH(1, false, false);
        }
    }
#undef FFTRW_LAUNCH
    e = hipGetLastError();
    if (e != hipSuccess) return batch_fail_hip(e, "batch kernel launch");
    return FFTRW_OK;
}

}  // namespace
}  // namespace fftrw

struct fft_batch_s : fftrw::fft_batch_impl {};

using namespace fftrw;

extern "C" {

int fft_batch_plan(fft_batch_t *out, int n, const fft_item_desc *items, int precision, const char *tune_cache,
                   unsigned flags)
{
    g_last_error.clear();
    if (!out || !items || n < 1) return fail(FFTRW_E_ARG, "null output, null items or n < 1");
    TuneTable tune;
    const bool tuned = tune_cache && tune_load(tune_cache, tune_device_name(), fft_version(), &tune);
    *out = nullptr;
    if (precision != FFTRW_PREC_NATIVE)
        return fail(FFTRW_E_UNSUPPORTED, "the batched form runs the FP32 Stockham kernels");
    if (flags & ~(unsigned)(FFTRW_FLAG_COUNT_MOVED | FFTRW_FLAG_LEAVE_PERMUTED | FFTRW_FLAG_BATCH_NO_GRAPH |
                            FFTRW_FLAG_BATCH_NO_FUSE))
        return fail(FFTRW_E_UNSUPPORTED,
                    "the batched form supports COUNT_MOVED, LEAVE_PERMUTED, BATCH_NO_GRAPH and BATCH_NO_FUSE only");
    fft_batch_s *b = new (std::nothrow) fft_batch_s();
    if (!b) return fail(FFTRW_E_NOMEM, "out of host memory");
    b->n = n;
    b->flags = flags;
    // test hook: FFTRW_BATCH_WAIT_TICKS bounds each level wait (100 MHz
    // ticks) instead of 2 s, so tests can force the time-out path
    if (const char *w = std::getenv("FFTRW_BATCH_WAIT_TICKS")) b->wait_ticks = std::strtoull(w, nullptr, 10);
    const unsigned pflags = flags & (FFTRW_FLAG_COUNT_MOVED | FFTRW_FLAG_LEAVE_PERMUTED);
    const bool leave = (flags & FFTRW_FLAG_LEAVE_PERMUTED) != 0;
    b->h_items.resize(n);
    size_t lds = 16, lds_tw = 16;  // LDS per group without and with staged twiddles
    bool tw_fits = true;          // every fused step's table fits (unit_tw_fits)
    int max_stage = 0;
    for (int i = 0; i < n; ++i) {
        const fft_item_desc &it = items[i];
        fft_plan_t p = nullptr;
        int rc = plan_create(&p, it.M, it.dims, it.P, it.has_order ? it.order : nullptr, FFTRW_C64,
                             FFTRW_PREC_NATIVE, pflags, true, tuned ? &tune : nullptr, nullptr);
        if (rc) {
            std::string m = "item " + std::to_string(i) + ": " + g_last_error;
            batch_free(b);
            return fail(rc, m);
        }
        b->plans.push_back(p);
        BatchItemDev &d = b->h_items[i];
        std::memset(&d, 0, sizeof(d));
        d.M = it.M;
        const int nx = leave ? it.M - 1 : it.M;
        d.nx = nx;
        d.buf[2] = (float2 *)p->work;
        d.inv_scale = (float)(1.0 / (double)p->T);
        int64_t units = 0;
        // fused schedule: one unit = RW rows consecutive in v of one slice, the
        // largest power of two with RW (N + padding) <= 4096 that the v axis can fill
        d.fused = !(flags & FFTRW_FLAG_BATCH_NO_FUSE);
        if (d.fused) {
            d.nstage = it.M;
            int cur = 0;
            for (int t = 0; t < it.M; ++t) {
                d.prefix[t] = units;
                d.fft[t] = p->fft[t];
                if (t < nx) {
                    d.xp[t] = p->xp[t];
                    const int N = d.fft[t].N;
                    if (tuned) {
                        // the radix order the autotuner timed in the fused unit
                        // (it differs from the separate row kernel's), checked
                        // as the plan checks the row kernel's
                        auto ft = tune.fused.find({N, (int)d.xp[t].Nv});
                        if (ft != tune.fused.end()) {
                            const std::vector<int> &rad = ft->second;
                            int64_t prod = 1;
                            bool ok = !rad.empty() && (int)rad.size() <= kMaxPasses;
                            for (int r : rad) {
                                ok = ok && (r == 2 || r == 3 || r == 4 || r == 5 || r == 8 || r == 16);
                                prod *= r;
                            }
                            if (ok && prod == N) {
                                d.fft[t].npass = (int)rad.size();
                                for (int q = 0; q < d.fft[t].npass; ++q) d.fft[t].radix[q] = rad[q];
                            }
                        }
                    }
                    int rw = 1, G = 1;
                    fused_unit_shape(N, 8, d.xp[t].Nv, d.xp[t].nslices, 4096, &rw, &G);
                    d.frw[t] = rw;
                    d.fg[t] = G;
                    d.src[t] = t == 0 ? 0 : cur;
                    d.dst[t] = ((nx - 1 - t) % 2 == 0) ? 1 : 2;
                    cur = d.dst[t];
                    units += ((d.xp[t].Nv + rw - 1) / rw) * ((d.xp[t].nslices + G - 1) / G);
                    lds = std::max(lds, fused_unit_bytes(N, rw, G, 8, false));
                    lds_tw = std::max(lds_tw, fused_unit_bytes(N, rw, G, 8, true));
                    tw_fits = tw_fits && unit_tw_fits(N, 8);
                } else {
                    // LEAVE_PERMUTED: the last FFT step runs in place on the output
                    d.src[t] = 1;
                    d.dst[t] = 1;
                    units += (d.fft[t].nrows + d.fft[t].rows_per_wg - 1) / d.fft[t].rows_per_wg;
                    lds = std::max(lds, (size_t)d.fft[t].rows_per_wg * d.fft[t].N * 8);
                }
            }
            d.prefix[d.nstage] = units;
            max_stage = std::max(max_stage, d.nstage);
            b->any_fused = true;
            continue;
        }
        d.nstage = it.M + nx;
        // buffer sequence of the pipeline: FFT 0 reads the input; transposes alternate
        const int b0 = (nx % 2 == 0) ? 1 : 2, b1 = b0 == 1 ? 2 : 1;
        int cur = b0, other = b1;
        for (int st = 0; st < d.nstage; ++st) {
            d.prefix[st] = units;
            const int t = st >> 1;
            if ((st & 1) == 0) {
                d.src[st] = t == 0 ? 0 : cur;
                d.dst[st] = cur;
                d.fft[t] = p->fft[t];
                units += (d.fft[t].nrows + d.fft[t].rows_per_wg - 1) / d.fft[t].rows_per_wg;
                lds = std::max(lds, (size_t)d.fft[t].rows_per_wg * d.fft[t].N * 8);
            } else {
                d.src[st] = cur;
                d.dst[st] = other;
                std::swap(cur, other);
                d.xp[t] = p->xp[t];
                d.xv[t] = ((d.xp[t].Nu % 2 == 0 && d.xp[t].TU >= 2) ? 1 : 0) |
                          ((d.xp[t].Nv % 2 == 0 && d.xp[t].TV >= 2) ? 2 : 0);
                units += d.xp[t].tiles_u * d.xp[t].tiles_v * d.xp[t].tiles_g;
                lds = std::max(lds, xpose_tile_bytes(d.xp[t], 8) + 16);
            }
        }
        d.prefix[d.nstage] = units;
        max_stage = std::max(max_stage, d.nstage);
    }
    // stage level by stage level, items in order; units numbered within a level
    for (int s = 0; s < max_stage; ++s) {
        b->level_task0.push_back((int)b->h_tasks.size());
        int64_t lvl = 0;
        for (int i = 0; i < n; ++i) {
            const BatchItemDev &d = b->h_items[i];
            if (s >= d.nstage) continue;
            const int64_t cnt = d.prefix[s + 1] - d.prefix[s];
            if (cnt <= 0) continue;
            b->h_tasks.push_back({i, s, lvl, cnt});
            lvl += cnt;
        }
        // claims count in 32 bits (see claim); every group claims at most
        // once past the end of a level
        if (lvl >= (int64_t{1} << 31)) {
            batch_free(b);
            return fail(FFTRW_E_SIZE, "a stage level of the batch has 2^31 or more units");
        }
        b->level_units.push_back(lvl);
        b->total += lvl;
    }
    b->level_task0.push_back((int)b->h_tasks.size());
    // twiddles in LDS when every fused step's table fits; the groups of the
    // separate stages need no more LDS either way
    b->tw_lds = b->any_fused && tw_fits;
    b->lds = (std::max(lds, b->tw_lds ? lds_tw : (size_t)0) + 15) & ~(size_t)15;
    // Every FFT step of a batch runs radices 2, 3, 4 and 5 only (8 and 16
    // become 4 x 2 and 4 x 4, in place), in the fused and the separate
    // schedules alike so that the two stay bit-identical.  When every stage is
    // a fused unit (no LEAVE_PERMUTED, no BATCH_NO_FUSE) the batch then runs
    // batch_kernel's LEAN form: without the separate stage kernels and the
    // larger passes it holds four waves per SIMD instead of three (config 5:
    // 5.95 -> 5.33 ms).
    b->lean = !(flags & (FFTRW_FLAG_LEAVE_PERMUTED | FFTRW_FLAG_BATCH_NO_FUSE));
    for (fft_plan_t p : b->plans)
        if (p->T * (int64_t)sizeof(float2) >= (int64_t{1} << 32)) b->lean = false;  // 32-bit offsets
    for (int i = 0; i < n; ++i) {
        BatchItemDev &d = b->h_items[i];
        for (int t = 0; t < d.M; ++t) {
            FftDesc &f = d.fft[t];
            int rad[kMaxPasses], np = 0;
            bool fits = true;
            for (int q = 0; q < f.npass && fits; ++q) {
                const int r = f.radix[q];
                const int nparts = (r == 8 || r == 16) ? 2 : 1;
                const int parts[2] = {nparts == 2 ? 4 : r, r == 16 ? 4 : 2};
                if (np + nparts > kMaxPasses) {
                    fits = false;
                    break;
                }
                for (int k = 0; k < nparts; ++k) rad[np++] = parts[k];
            }
            if (!fits) {
                b->lean = false;  // keeps the step's own radices
                continue;
            }
            f.npass = np;
            for (int q = 0; q < np; ++q) f.radix[q] = rad[q];
        }
    }
    b->moved_off.resize(n);
    b->nctr = (int64_t)(sizeof(BatchCounters) / sizeof(unsigned long long));
    for (int i = 0; i < n; ++i) {
        b->moved_off[i] = b->nctr;
        b->nctr += (int64_t)b->h_items[i].M * kCountBlock;
    }
    int dev = 0, ncu = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu,
            b->lean ? (b->tw_lds ? batch_kernel<-1, true, true> : batch_kernel<-1, false, true>)
                    : (b->tw_lds ? batch_kernel<-1, true, false> : batch_kernel<-1, false, false>),
            kThreads, b->lds);
    if (e != hipSuccess || per_cu < 1 || ncu < 1) {
        batch_free(b);
        return e != hipSuccess ? batch_fail_hip(e, "occupancy query") : fail(FFTRW_E_DEVICE, "kernel does not fit");
    }
    b->grid = per_cu * ncu;
    e = hipMalloc(&b->d_items, sizeof(BatchItemDev) * (size_t)n);
    if (e == hipSuccess) e = hipMalloc(&b->d_tasks, sizeof(BatchTask) * b->h_tasks.size());
    if (e == hipSuccess) e = hipMalloc(&b->d_ctr, sizeof(unsigned long long) * (size_t)b->nctr);
    if (e == hipSuccess) e = hipMalloc(&b->d_timeouts, sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMemset(b->d_timeouts, 0, sizeof(unsigned long long));
    if (e == hipSuccess && (flags & FFTRW_FLAG_COUNT_MOVED)) {
        // owner-change counters of every transpose live in the batch's counter
        // block, which the graph's reset kernel clears before each launch
        for (int i = 0; i < n; ++i)
            for (int t = 0; t < b->h_items[i].M; ++t)
                if (b->h_items[i].xp[t].count)
                    b->h_items[i].xp[t].counter = b->d_ctr + b->moved_off[i] + (int64_t)t * kCountBlock;
    }
    if (e == hipSuccess)
        e = hipMemcpy(b->d_tasks, b->h_tasks.data(), sizeof(BatchTask) * b->h_tasks.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&b->d_level_task0, sizeof(int) * b->level_task0.size());
    if (e == hipSuccess) e = hipMalloc(&b->d_level_units, sizeof(int64_t) * b->level_units.size());
    if (e == hipSuccess)
        e = hipMemcpy(b->d_level_task0, b->level_task0.data(), sizeof(int) * b->level_task0.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->d_level_units, b->level_units.data(), sizeof(int64_t) * b->level_units.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        batch_free(b);
        return fail(FFTRW_E_NOMEM, "device allocation for the batch failed");
    }
    b->tuned = tuned;
    int64_t units = 0;
    for (int64_t u : b->level_units) units += u;
    log_line(1, "batch of %d items: %lld units in %zu stage levels, %d resident groups, %s stages%s%s", n,
             (long long)units, b->level_units.size(), b->grid, b->any_fused ? "fused" : "separate",
             b->lean ? " (lean kernel: fused units of radices 2..5)" : "", tuned ? ", tuned" : "");
    *out = b;
    return FFTRW_OK;
}

static int batch_exec(fft_batch_t b, void *const *in, void *const *out, void *stream, int dir)
{
    g_last_error.clear();
    if (!b || !in || !out) return fail(FFTRW_E_ARG, "null batch or pointer arrays");
    if (b->timed_out)
        return fail(FFTRW_E_DEVICE, "an earlier launch of this batch timed out at a level barrier");
    bool changed = !b->pointers_set;
    for (int i = 0; i < b->n; ++i) {
        if (!in[i] || !out[i]) return fail(FFTRW_E_ARG, "null buffer for item " + std::to_string(i));
        if (b->h_items[i].fused && in[i] == out[i])
            return fail(FFTRW_E_ARG, "item " + std::to_string(i) +
                                         ": fused stages need in != out (plan with FFTRW_FLAG_BATCH_NO_FUSE for in place)");
        BatchItemDev &d = b->h_items[i];
        if (d.buf[0] != in[i] || d.buf[1] != out[i]) changed = true;
        d.buf[0] = (float2 *)in[i];
        d.buf[1] = (float2 *)out[i];
    }
    hipStream_t s = (hipStream_t)stream;
    if (changed) {
        // the item table is read by the kernel; update it in stream order
        hipError_t e = hipStreamSynchronize(s);
        if (e == hipSuccess)
            e = hipMemcpy(b->d_items, b->h_items.data(), sizeof(BatchItemDev) * (size_t)b->n, hipMemcpyHostToDevice);
        if (e != hipSuccess) return batch_fail_hip(e, "item table update");
        b->pointers_set = true;
    }
    if (b->flags & FFTRW_FLAG_BATCH_NO_GRAPH) return batch_enqueue(b, dir, s);
    const int di = dir < 0 ? 0 : 1;
    if (!b->gexec[di]) {
        hipError_t e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return batch_fail_hip(e, "graph capture begin");
        int rc = batch_enqueue(b, dir, b->cap_stream);
        e = hipStreamEndCapture(b->cap_stream, &b->graph[di]);
        if (rc) return rc;
        if (e != hipSuccess) return batch_fail_hip(e, "graph capture end");
        e = hipGraphInstantiate(&b->gexec[di], b->graph[di], nullptr, nullptr, 0);
        if (e != hipSuccess) return batch_fail_hip(e, "graph instantiate");
    }
    hipError_t e = hipGraphLaunch(b->gexec[di], s);
    if (e != hipSuccess) return batch_fail_hip(e, "graph launch");
    return FFTRW_OK;
}

int fft_batch_exec_fwd(fft_batch_t b, void *const *in, void *const *out, void *stream)
{
    return batch_exec(b, in, out, stream, -1);
}

int fft_batch_exec_inv(fft_batch_t b, void *const *in, void *const *out, void *stream)
{
    return batch_exec(b, in, out, stream, 1);
}

int fft_batch_stats(fft_batch_t b, int64_t *moved, int64_t *analytic, int64_t *units, int *error)
{
    g_last_error.clear();
    if (!b) return fail(FFTRW_E_ARG, "null batch");
    if (units) *units = b->total;
    std::vector<unsigned long long> h((size_t)b->nctr, 0ull);
    unsigned long long timeouts = 0;
    {
        hipError_t e = hipDeviceSynchronize();
        if (e == hipSuccess && moved)
            e = hipMemcpy(h.data(), b->d_ctr, sizeof(unsigned long long) * h.size(), hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(&timeouts, b->d_timeouts, sizeof(timeouts), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return batch_fail_hip(e, "reading batch counters");
    }
    const bool leave = (b->flags & FFTRW_FLAG_LEAVE_PERMUTED) != 0;
    const bool counted = (b->flags & FFTRW_FLAG_COUNT_MOVED) != 0;
    int off = 0;
    for (int i = 0; i < b->n; ++i) {
        const int M = b->h_items[i].M;
        for (int t = 0; t < M; ++t) {
            if (analytic) analytic[off + t] = b->plans[i]->analytic[t];
            if (moved) {
                int64_t sum = -1;
                if (counted && !(leave && t == M - 1)) {
                    sum = 0;
                    for (int k = 0; k < kCountSlots; ++k)
                        sum += (int64_t)h[b->moved_off[i] + (int64_t)t * kCountBlock + (int64_t)k * kCountStride];
                }
                moved[off + t] = sum;
            }
        }
        off += M;
    }
    if (error) *error = (int)std::min<unsigned long long>(timeouts, 0x7fffffffull);
    if (timeouts) {
        b->timed_out = true;
        return fail(FFTRW_E_DEVICE, std::to_string(timeouts) +
                                        " level-barrier wait(s) timed out; results of this batch are unreliable");
    }
    return FFTRW_OK;
}

int fft_batch_destroy(fft_batch_t b)
{
    g_last_error.clear();
    batch_free(b);
    return FFTRW_OK;
}

}  // extern "C"
