/*
 * fftrw.h -- row-wise decomposed multi-dimensional complex FFTs on one MI355X.
 *
 * Implements the parallel M-D FFT of Duy & Ozaki, "A decomposition method with
 * minimum communication amount for parallelization of multi-dimensional FFTs":
 * N_p processes each own a contiguous 1-D range of the array in the current
 * axis order (the row-wise adaptive decomposition, Eqs. (12)-(19)); step t
 * runs 1-D FFTs (Eq. (1)) along the last axis of decomposition pi_t and then
 * transposes to pi_{t+1}, re-decomposing (Fig. 4).  Here all N_p processes
 * are *virtual*: their ranges are consecutive slices of one device buffer, so
 * every transpose is an on-device permutation through HBM whose count of
 * points that change owner is the paper's communication amount.
 *
 * Conventions used by every entry point
 * -------------------------------------
 * - M in [2, 5] for plans, batches and the autotuner; the host functions on
 *   ranges, amounts and orders (fft_decomp, fft_comm_volume,
 *   fft_rowsplit_volume, fft_pair_counts, fft_transpose_volumes,
 *   fft_order_*) also take M = 6.  dims[0..M) = (N_1, ..., N_M), N_1 slowest
 *   (row-major, C order).
 * - An axis permutation `perm` (M int8) lists natural axis indices from the
 *   slowest to the fastest position: {2,0,1} is the paper's "cab".
 * - A transpose order `order` (M*M int8) is M permutations, row t = pi_{t+1}:
 *   order[t*M + i] = natural axis at position i of decomposition t.  Row 0 must
 *   be the identity and the last entries of the M rows must all differ (the
 *   FFT axis of each step; Section 3.2, Eq. (20)).
 * - Complex data are interleaved (re, im).  FFTRW_C64 = 2 x float, FFTRW_C128 =
 *   2 x double.  Forward uses w_N = exp(-2 pi i / N) with no scaling (Eq. (1));
 *   inverse uses exp(+2 pi i / N) and scales by 1/T, T = prod(dims).
 * - Every function returns an int status (0 = FFTRW_OK, < 0 = error) unless
 *   stated otherwise; no C++ exception crosses this interface.  The text of the
 *   last error on the calling thread is returned by fft_last_error().
 * - Pointers named `in`/`out` and the `stream` argument are HIP device
 *   pointers and a hipStream_t (NULL = the default stream).  Host pointers are
 *   named otherwise and are only read/written during the call.
 * - Diagnostics: the environment variable FFTRW_LOG (read once per process)
 *   selects lines on stderr, each starting "fftrw: ": 1 = every error and
 *   every plan or batch created (order, kernels, workspace), 2 = also each
 *   order search, 3 = also each execution.  Unset or 0: silent.
 */
#ifndef FFTRW_H
#define FFTRW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
enum {
    FFTRW_OK = 0,
    FFTRW_E_ARG = -1,         /* null pointer, bad enum, bad index            */
    FFTRW_E_SIZE = -2,        /* M out of range (see conventions), a size < 1,
                                 or a row length the FFT kernels do not support
                                 (see fft_plan)                                */
    FFTRW_E_ORDER = -3,       /* malformed permutation or transpose order      */
    FFTRW_E_ROWSPLIT = -4,    /* N_p > T (no level of Eq. (13) applies); or a
                                 step at level M (N_p > T / N_last: rows along
                                 its FFT axis split over processes) that a
                                 staged plan cannot run as a binary exchange
                                 (see fft_plan_rowsplit_stats), or as a flag
                                 from fft_comm_volume (see there)               */
    FFTRW_E_NOMEM = -5,       /* host or device allocation failed             */
    FFTRW_E_DEVICE = -6,      /* a HIP call failed; see fft_last_error()       */
    FFTRW_E_UNSUPPORTED = -7  /* combination not implemented                   */
};

/* ---- enums ----------------------------------------------------------------- */
enum { FFTRW_C64 = 1, FFTRW_C128 = 2 };

enum {
    FFTRW_PREC_NATIVE = 0,        /* FP32 math for C64, FP64 math for C128        */
    FFTRW_PREC_SPLIT_F16 = 1,     /* radix-16 stages on FP16 MFMA, hi/lo split    */
    FFTRW_PREC_SPLIT_BF16 = 2,    /* radix-16 stages on BF16 MFMA, hi/lo split    */
    FFTRW_PREC_SPLIT_BF16X3 = 3   /* radix-16 stages on BF16 MFMA, 3-term split   */
};

enum { FFTRW_OWN_LITERAL = 0, FFTRW_OWN_MATCHED = 1 };

enum {
    FFTRW_FLAG_LEAVE_PERMUTED = 1u,  /* skip the final transpose back to natural
                                        order: output stays in layout pi_M       */
    FFTRW_FLAG_STAGED = 2u,          /* transposes as pack -> exchange -> unpack
                                        with explicit per-process send/receive
                                        segments (default: one fused permutation) */
    FFTRW_FLAG_COUNT_MOVED = 4u,     /* count, on the device, the points whose
                                        owner changes in every transpose          */
    FFTRW_FLAG_OWN_MATCHED = 8u,     /* ownership reading R2 (see fft_comm_volume):
                                        device counts, and with STAGED the
                                        exchange itself, follow the matching     */
    FFTRW_FLAG_FUSED_FFT = 16u,      /* fuse each FFT step with the transpose that
                                        follows it (one HBM pass per step).  The
                                        default: a plan fuses whenever every step
                                        qualifies (see fft_plan); the flag only
                                        states it                                 */
    FFTRW_FLAG_BATCH_NO_GRAPH = 32u, /* batched form: launch the persistent kernel
                                        directly instead of replaying a graph     */
    FFTRW_FLAG_BATCH_NO_FUSE = 64u,  /* batched form: separate FFT and transpose
                                        stages (allows in == out)                 */
    FFTRW_FLAG_SEPARATE = 128u       /* plans: run every FFT step and every
                                        transpose as kernels of their own (two HBM
                                        passes per step); excludes FUSED_FFT      */
};

typedef struct fft_plan_s *fft_plan_t;

/* ---- host-only integer functions (no device needed) ----------------------- */

/*
 * fft_decomp -- Eqs. (13)-(19): the range of process `myid` in decomposition
 * `perm` of an array of sizes `dims` over P processes.
 *   level : k of Eq. (13) (1-based): the smallest k with P <= N'_1 ... N'_k,
 *           where N'_i = dims[perm[i]].
 *   xs,xe : first and last 1-D index (Eq. (12) in the order perm), inclusive.
 *   start,end (M int64 each, nullable): Eqs. (16)-(19), coordinates in the
 *           permuted order (start[i] runs along natural axis perm[i]).
 * Errors: FFTRW_E_ARG (myid out of [0,P), null level/xs/xe), FFTRW_E_SIZE,
 * FFTRW_E_ORDER (perm not a permutation), FFTRW_E_ROWSPLIT if P > T.
 */
int fft_decomp(int M, const int64_t *dims, int64_t P, const int8_t *perm,
               int64_t myid, int *level, int64_t *xs, int64_t *xe,
               int64_t *start, int64_t *end);

/*
 * fft_comm_volume -- the communication amount of a transpose order
 * (Sections 3.1 and 3.3; the quantity compared in Section 4).
 *   per_step[M-1] (nullable): points that change owner in transpose
 *       pi_t -> pi_{t+1}, t = 1..M-1.
 *   total: sum of per_step.
 *   return_volume (nullable): the same count for the final transpose
 *       pi_M -> natural order of Fig. 4, which is NOT part of `total`.
 * ownership FFTRW_OWN_LITERAL (R1): process p owns range p of Eqs. (14)-(15)
 *   in every decomposition.  FFTRW_OWN_MATCHED (R2): the ranges of each new
 *   decomposition are assigned to processes one-to-one so that the most
 *   points stay put (maximum-weight matching on the overlap counts).
 * Counts are exact int64.  Row-split orders (a step at level M) are counted
 * like any other, and the call returns FFTRW_E_ROWSPLIT after filling the
 * outputs: the amounts then leave out whatever the split rows' own 1-D FFTs
 * would exchange, which the paper does not define.
 */
int fft_comm_volume(int M, const int64_t *dims, int64_t P, const int8_t *order,
                    int ownership, int64_t *per_step, int64_t *total,
                    int64_t *return_volume);

/*
 * fft_rowsplit_volume -- what the 1-D FFTs of split rows would exchange, for
 * the steps at level M of Eq. (13) (N_p > T / N_last), which the transposes'
 * amount leaves out.  The paper does not say how a split row is transformed;
 * the reading here is a binary exchange: a row of length N held by c > 1
 * processes runs ceil(log2 c) butterfly stages whose partners sit on other
 * processes, each sending every point of the row once, so the row adds
 * N * ceil(log2 c) points.  With it the 64^3 comparison of Section 4 against
 * the 3-D method (Eq. (23)) peaks at 8,192 processes at 11.6 times.  This
 * reading was chosen because it reproduces that printed 11.6 (the paper's
 * own algorithm for a split row is unknown); given the reading, the count is
 * the number of points an executed binary-exchange FFT sends.
 *   per_step[M] (nullable): one count per FFT step t = 1..M (0 below level M).
 *   total: their sum.
 * Errors: FFTRW_E_ARG, FFTRW_E_SIZE, FFTRW_E_ORDER, FFTRW_E_ROWSPLIT if P > T.
 * Cost O(M * P) on the host.
 */
int fft_rowsplit_volume(int M, const int64_t *dims, int64_t P, const int8_t *order,
                        int64_t *per_step, int64_t *total);

/*
 * fft_pair_counts -- overlap counts C[p][q] = points owned by p in
 * decomposition perm_a and by q in perm_b (literal ownership), written densely
 * into C[P*P] (host, caller-owned).  For checking; P <= 4096.
 */
int fft_pair_counts(int M, const int64_t *dims, int64_t P, const int8_t *perm_a,
                    const int8_t *perm_b, int64_t *C);

/* (M-1)!^M, the number of transpose orders (Eq. (20), Table 1); -1 if M is
 * outside [2, 6]. */
int64_t fft_order_count(int M);

/* Order number `index` (0-based) in canonical enumeration: (pi_2, ..., pi_M)
 * in lexicographic order, each permutation compared as a string over
 * "abcde".  order: M*M int8 output (host). */
int fft_order_at(int M, int64_t index, int8_t *order);

/* Inverse of fft_order_at; FFTRW_E_ORDER if the order is not valid. */
int fft_order_index(int M, const int8_t *order, int64_t *index);

/*
 * fft_transpose_volumes -- the amount of every single transpose
 * pi_a -> pi_b that an order can contain (Sections 3.1, 3.3), as a table over
 * the M! permutations in lexicographic order: table[a * M! + b] (host array of
 * (M!)^2 int64, caller-owned).  Pairs no order contains are -1: two
 * permutations with the same last axis, and pairs that involve a permutation
 * other than the identity ending with the identity's last axis.  The amount of
 * an order is the sum of its M-1 entries.  Computed on several host threads.
 */
int fft_transpose_volumes(int M, const int64_t *dims, int64_t P, int ownership,
                          int64_t *table);

/*
 * fft_order_search -- the smallest and largest total communication amount
 * over all (M-1)!^M orders (Sections 3.1, 3.3; for 6-D, 2,985,984,000,000
 * orders, which Section 3.3 leaves unsearched).  Exact, without listing the
 * orders: the amount of an order is a sum over consecutive decompositions, so
 * a dynamic program over (current decomposition, axes already transformed)
 * gives the optimum and the number of orders attaining it.
 * Ties go to the lowest canonical index; n_best / n_worst count the tied
 * orders.  best_order / worst_order (M*M int8, nullable) receive the orders.
 * The best order is the one fft_plan uses when given order == NULL.
 */
int fft_order_search(int M, const int64_t *dims, int64_t P, int ownership,
                     int64_t *best_index, int64_t *best_volume, int64_t *n_best,
                     int64_t *worst_index, int64_t *worst_volume, int64_t *n_worst,
                     int8_t *best_order, int8_t *worst_order);

/*
 * fft_order_volumes -- total amount of every order (host array of
 * fft_order_count(M) int64, in canonical order).  M <= 5
 * (FFTRW_E_UNSUPPORTED for 6-D: use fft_order_search).
 */
int fft_order_volumes(int M, const int64_t *dims, int64_t P, int ownership,
                      int64_t *volumes);

/*
 * fft_compare_models -- the amounts of the fixed-degree methods compared in
 * Section 4 for an N^M array: Eq. (21) 1-D (slab), Eq. (22) 2-D (pencil),
 * Eq. (23) 3-D, Eq. (24) 4-D, Eq. (25) 5-D, evaluated as printed in double
 * precision.  out[5] receives A_1D, A_2D, A_3D, A_4D, A_5D (the 1-D, 2-D and
 * 3-D forms are stated for M = 3, the 4-D form for M = 4 and the 5-D form for
 * M = 5; each is returned as printed regardless of M).
 */
int fft_compare_models(double N, double P, double *out);

/* ---- plans and device execution ------------------------------------------ */

/*
 * fft_plan -- build an execution plan on the current HIP device.
 *   order: M*M int8 as above, or NULL for the best order of fft_order_search
 *          (literal ownership, lowest canonical index on ties).
 *   dtype: FFTRW_C64 or FFTRW_C128.   precision: FFTRW_PREC_*; the split MFMA
 *          forms need dtype C64; axes of 256 and 512 points run on MFMA,
 *          other axes keep the FP32 Stockham kernels.
 *   flags: FFTRW_FLAG_*.
 * Row lengths: every dims[i] must factor into 2, 3, 5 and be <= 4096.
 * 1 <= P <= T.  Steps at level M of Eq. (13) (P > T / N_last, rows split
 * along the FFT axis) run: the processes sharing a row share device memory,
 * so the row is transformed whole, and the transposes are counted exactly as
 * at other levels.  Staged plans run such a step's split rows as a binary
 * exchange (see fft_plan_rowsplit_stats), and its transposes as the counted
 * fused permutation.
 * Fusion: unless flags hold FFTRW_FLAG_SEPARATE or FFTRW_FLAG_STAGED, each
 * FFT step runs fused with the transpose that follows it when every step
 * qualifies (power-of-two rows of 16..512 points for C64, 16..256 for C128,
 * whose work-group's run along the next layout's last axis fits that axis;
 * other 2,3,5-smooth rows up to 4095 points for C64, 2047 for C128; 256- and
 * 512-point rows of the split MFMA forms); otherwise, and for execs with in == out, the
 * steps and transposes run as separate kernels.  Results are bit-identical
 * either way; fft_plan_describe's text starts with "fused|" when it fuses.
 * The plan owns its device workspace (fft_workspace_bytes) and twiddle
 * tables; it must outlive every exec enqueued with it.  One exec per plan may
 * be in flight at a time.
 * Errors: FFTRW_E_ARG, FFTRW_E_SIZE, FFTRW_E_ORDER, FFTRW_E_ROWSPLIT,
 * FFTRW_E_UNSUPPORTED, FFTRW_E_NOMEM, FFTRW_E_DEVICE.
 */
int fft_plan(fft_plan_t *plan, int M, const int64_t *dims, int64_t P,
             const int8_t *order, int dtype, int precision, unsigned flags);

/*
 * fft_exec_fwd / fft_exec_inv -- enqueue the whole Fig. 4 pipeline on
 * `stream`: for t = 1..M, 1-D FFTs along the last axis of pi_t, then the
 * transpose to pi_{t+1} (to natural order after step M unless
 * LEAVE_PERMUTED).  in: T elements in natural layout; out: T elements in
 * natural layout (or pi_M layout with LEAVE_PERMUTED).  in == out is allowed;
 * otherwise `in` is not modified.  Asynchronous: returns after enqueueing.
 */
int fft_exec_fwd(fft_plan_t plan, const void *in, void *out, void *stream);
int fft_exec_inv(fft_plan_t plan, const void *in, void *out, void *stream);

/*
 * fft_exec_fft_step -- enqueue only step t (0-based) of the pipeline: 1-D FFTs
 * along the last axis of pi_{t+1}.  in/out hold T elements in that layout
 * (in == out allowed).  direction: -1 forward, +1 inverse (unscaled).
 */
int fft_exec_fft_step(fft_plan_t plan, int t, int direction, const void *in,
                      void *out, void *stream);

/*
 * fft_exec_transpose -- enqueue only transpose t (0-based): layout pi_{t+1}
 * -> pi_{t+2}, or pi_M -> natural for t = M-1, with the plan's mode (fused or
 * staged) and counter.  in and out must not overlap.
 */
int fft_exec_transpose(fft_plan_t plan, int t, const void *in, void *out,
                       void *stream);

/*
 * fft_plan_stats -- host copies of the plan's analytic amounts and the
 * device counters of the last exec.
 *   per_step[M] (nullable): analytic counts for transposes 1..M-1, then the
 *       return transpose (the same numbers as fft_comm_volume).
 *   moved[M] (nullable): points counted on the device as changing owner in
 *       each transpose of the last exec (COUNT_MOVED), or the points copied by
 *       the exchange kernel (STAGED); -1 where nothing was counted.  This call
 *       synchronises the device.
 */
int fft_plan_stats(fft_plan_t plan, int64_t *per_step, int64_t *moved);

/*
 * fft_plan_messages -- for a plan built with FFTRW_FLAG_STAGED, the number of
 * messages of each transpose's all-to-all: the (p, q) pairs with p != q that
 * exchange at least one point (Fig. 4's transposes, as a distributed run
 * would send them); with FFTRW_FLAG_OWN_MATCHED, the pairs that share points
 * other than each range and its matched range.  -1 for a transpose that
 * touches a decomposition at level M: staged plans run it as the fused
 * permutation, its owner changes counted (see fft_plan_stats).  per_step[M] receives transposes 1..M-1 then the return
 * transpose.  FFTRW_E_UNSUPPORTED for plans without staged tables.
 */
int fft_plan_messages(fft_plan_t plan, int64_t *per_step);

/*
 * fft_plan_rowsplit_stats -- for a plan built with FFTRW_FLAG_STAGED, the
 * exchange of the FFT steps whose rows are split over processes (level M of
 * Eq. (13), N_p > T / N_last).  A staged plan runs such a step as a binary
 * exchange among the processes that share each row (the reading of
 * fft_rowsplit_volume): it needs every range to hold b = T / N_p points and
 * each row to be c = N / b ranges with c a power of two (otherwise fft_plan
 * returns FFTRW_E_ROWSPLIT), and sends every point once in each of the
 * log2 c stages.
 *   per_step[M] (nullable): fft_rowsplit_volume's count for each FFT step
 *       (0 below level M), or -1 for a plan that is not staged.
 *   moved[M] (nullable): points copied between processes by the last exec's
 *       split-row exchanges, counted on the device; -1 where not executed.
 * Synchronises the device.
 */
int fft_plan_rowsplit_stats(fft_plan_t plan, int64_t *per_step, int64_t *moved);

/*
 * fft_plan_set_timing -- when enable != 0, every later exec records a HIP
 * event on its stream after each stage (FFT step or transpose), so
 * fft_plan_timings can report per-stage durations.  Creates the events on the
 * current device; FFTRW_E_DEVICE if that fails.
 */
int fft_plan_set_timing(fft_plan_t plan, int enable);

/*
 * fft_plan_timings -- durations in milliseconds of the stages of the last
 * exec with timing enabled, in launch order: FFT step 1, transpose 1, FFT
 * step 2, ..., FFT step M, return transpose (absent with LEAVE_PERMUTED).
 * With FFTRW_FLAG_STAGED each transpose is three stages: pack, exchange,
 * unpack.  When the plan fuses (see fft_plan) each stage is one FFT step
 * together with the transpose that follows it.
 * ms: host array of capacity `cap`; *n receives the number of stages.
 * Synchronises on the last event.
 */
int fft_plan_timings(fft_plan_t plan, float *ms, int cap, int *n);

/* Device bytes the plan holds (workspace, staging, tables). */
int fft_workspace_bytes(fft_plan_t plan, size_t *bytes);

/* Information about the plan: its order (M*M int8), and per step the radix
 * factorisation of the FFT axis as a string "8x8x8" (buffer of `cap` bytes). */
int fft_plan_describe(fft_plan_t plan, int8_t *order, char *text, size_t cap);

int fft_destroy(fft_plan_t plan);

/*
 * fft_exec_noalloc -- for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): plan and run the whole pipeline of fft_exec_fwd (direction -1)
 * or fft_exec_inv (+1) in one call, allocating nothing on the device.  The
 * arguments mean what they mean for fft_plan and fft_exec_*; in and out are
 * caller-owned device buffers of T elements (in == out allowed; otherwise in
 * is not modified).  The workspace and twiddle tables live in one fixed
 * device array of the library (64 MiB of workspace plus 1 MiB for tables;
 * each GPU the library runs on holds its own copy until the process ends), so
 * T * element size must be at most 64 MiB (8,388,608 complex64 points,
 * 4,194,304 complex128): larger arrays return FFTRW_E_SIZE.  flags: only
 * LEAVE_PERMUTED, FUSED_FFT, SEPARATE (FFTRW_E_UNSUPPORTED otherwise: staged
 * tables, device counters and relabelling tables would need memory of their
 * own).  Results equal fft_plan + fft_exec_* with the same arguments bit for
 * bit.  Asynchronous on `stream`.  Every call on a GPU shares that GPU's
 * array: calls that overlap on one GPU (other streams or threads) race; calls
 * on one stream are ordered.  The host side allocates only host memory.
 * Errors: as fft_plan, plus FFTRW_E_ARG for a direction other than -1 / +1.
 */
int fft_exec_noalloc(int M, const int64_t *dims, int64_t P, const int8_t *order,
                     int dtype, int precision, unsigned flags, int direction,
                     const void *in, void *out, void *stream);

/* ---- batched form: many uneven transforms in one persistent launch ------- */

/* One item of a batch: an M-D complex64 transform of sizes dims[0..M) over P
 * virtual processes, with the transpose order `order` (M*M int8 as for
 * fft_plan) when has_order != 0, else the best order of fft_order_search. */
typedef struct {
    int M;
    int64_t dims[5];
    int64_t P;
    int8_t order[25];
    int has_order;
} fft_item_desc;

typedef struct fft_batch_s *fft_batch_t;

/*
 * fft_batch_plan -- plan n independent transforms (each the Fig. 4 pipeline)
 * to run together in ONE persistent kernel launch, replayed from a HIP graph.
 * The work of every item is cut into units, numbered stage level by stage
 * level (level s holds stage s of every item).  By default stage t of an item
 * is its FFT step t fused with the transpose that follows (a unit: a block of
 * rows consecutive in the next layout's last axis); with BATCH_NO_FUSE the
 * FFT steps (row blocks) and transposes (tiles) are stages of their own.
 * Work-groups claim units from a per-level atomic counter; between levels
 * each waits until every unit of the level is done (a count of completed
 * units, so the wait ends even when other kernels keep part of the grid from
 * being resident).  A wait past its time limit (2 s) adds one to a sticky
 * time-out count that fft_batch_stats reports.  precision must be FFTRW_PREC_NATIVE; flags:
 * COUNT_MOVED, LEAVE_PERMUTED, BATCH_NO_GRAPH, BATCH_NO_FUSE.  tune_cache:
 * path of the autotuner's cache (fft_autotune) or NULL for the built-in plan.
 * Each item's row lengths follow fft_plan's rules; the batch owns one
 * T_i-element workspace per item.
 */
int fft_batch_plan(fft_batch_t *batch, int n, const fft_item_desc *items,
                   int precision, const char *tune_cache, unsigned flags);

/* Forward / inverse of every item: in[i], out[i] are device pointers to T_i
 * complex64 values in natural layout (host arrays of n pointers); in[i] must
 * differ from out[i] unless the batch was planned with BATCH_NO_FUSE
 * (FFTRW_E_ARG otherwise).  One graph
 * launch on `stream` (the first call per direction captures it). */
int fft_batch_exec_fwd(fft_batch_t batch, void *const *in, void *const *out,
                       void *stream);
int fft_batch_exec_inv(fft_batch_t batch, void *const *in, void *const *out,
                       void *stream);

/*
 * fft_batch_stats -- moved (sum of M_i, nullable): device-counted owner
 * changes per transpose of every item (COUNT_MOVED) in the last exec, items
 * in order; analytic (same shape, nullable): the plan's amounts; units:
 * number of work units of one exec; error (nullable): the number of level
 * waits that exceeded their limit, summed over every exec of this batch so far
 * (no launch resets it).  Synchronises the device.  When that count is not
 * zero the call fills the outputs and returns FFTRW_E_DEVICE, and later execs
 * of the batch return FFTRW_E_DEVICE: a timed-out exec's results are not
 * reliable.
 */
int fft_batch_stats(fft_batch_t batch, int64_t *moved, int64_t *analytic,
                    int64_t *units, int *error);

int fft_batch_destroy(fft_batch_t batch);

/*
 * fft_autotune -- time candidate kernel parameters for the row lengths and
 * transposes of the given items on the current device and write the winners
 * to the JSON file cache_path: per row length, the radix order and rows per
 * work-group of the generic row kernel; per (u size, v size) transpose, the
 * tile shape, and the radix order of the FFT step fused with it (the built-in
 * order unless another is at least 3% faster); fused batch stages use the
 * latter, separate stages the former.  The cache records the device architecture and library
 * version; fft_batch_plan ignores a cache whose tags do not match.  Uses
 * about 260 MB of device memory while it runs; synchronous.  flags: 0.
 */
int fft_autotune(int n, const fft_item_desc *items, const char *cache_path,
                 unsigned flags);

/*
 * fft_fused_unit_shape -- the work-group unit of a step whose 1-D FFTs along
 * u (rows of N points, Eq. (1)) are fused with the transpose that follows
 * (Fig. 4): rw rows consecutive in v, the next layout's fastest axis, in each
 * of G slices.  The plans and the batched form use this rule; the call is
 * for tests and tools, host only (no device needed).  esz: bytes per complex
 * value, 8 (complex64: units of at most 4096 values with padding) or 16
 * (complex128: 2048).  Nv: extent of v; nslices: number of batch slices.
 * The unit count of the step is ceil(Nv / rw) * ceil(nslices / G).  Returns
 * FFTRW_OK, or FFTRW_E_ARG for N < 2, Nv < 1, nslices < 1, another esz or
 * a null output.
 */
int fft_fused_unit_shape(int N, int esz, int64_t Nv, int64_t nslices, int *rw, int *G);

/* Text of the last error on the calling thread ("" if none). */
const char *fft_last_error(void);

/* Library version string. */
const char *fft_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FFTRW_H */
