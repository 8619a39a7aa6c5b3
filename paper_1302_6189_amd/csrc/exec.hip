// exec.hip -- plans and the Fig. 4 pipeline on one device (device half of the C ABI).
//
// Step t (t = 1..M) runs 1-D FFTs along the last axis of decomposition pi_t,
// then transposes to pi_{t+1} (and after step M back to natural order).  The
// N_p virtual processes own consecutive slices of the one buffer that holds
// the array in the current layout, so the transpose is an on-device
// permutation; the plan knows each transpose's analytic amount, and the
// kernels can count it on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "../../include/fftrw.h"
#include "decomp.hpp"
#include "errors.hpp"
#include "kernels.hpp"
#include "plan.hpp"
#include "tune.hpp"

namespace fftrw {

hipError_t launch_twiddles(void *out, int64_t n, bool fp64, hipStream_t s);
bool pow2_supported(int N, bool fp64);
void pow2_describe(int N, bool fp64, int *tw_count, int *radices, int *npass);
hipError_t pow2_make_twiddles(int N, bool fp64, void *tw, hipStream_t s);
hipError_t launch_fft_pow2(int N, bool fp64, const void *tw, int64_t nrows, int dir, const void *in, void *out,
                           double scale, hipStream_t s);
int pow2_rows_per_wg(int N, bool fp64);
hipError_t launch_fft_xpose_generic(const FftDesc &f, const XposeDesc &d, bool fp64, int dir, const void *in,
                                    void *out, double scale, hipStream_t s);
hipError_t launch_fft_xpose_pow2(int N, bool fp64, const void *tw, const XposeDesc &fx, int dir, const void *in,
                                 void *out, double scale, hipStream_t s);
hipError_t launch_fft_mfma_xpose(int precision, int dir, int N, const void *twN, const XposeDesc &d, const void *in,
                                 void *out, double scale, hipStream_t s);
hipError_t launch_fft_mfma(int precision, int dir, int N, const void *twN, int64_t nrows, const void *in, void *out,
                           double scale, hipStream_t s);
hipError_t launch_fft_rows(const FftDesc &d, bool fp64, int dir, const void *in, void *out, double scale,
                           hipStream_t s);
hipError_t launch_xpose(const XposeDesc &d, size_t esz, const void *in, void *out, hipStream_t s);
size_t xpose_lds_bytes(const XposeDesc &d, size_t esz);
hipError_t launch_zero_u64(unsigned long long *p, int n, hipStream_t s);
hipError_t launch_bx_exchange(bool fp64, const void *data, void *recv, int64_t T, int N, int b, int hb,
                              unsigned long long *counter, hipStream_t s);
hipError_t launch_bx_butterfly(bool fp64, int dir, void *data, const void *recv, int64_t T, int N, int h,
                               const void *tw, hipStream_t s);
hipError_t launch_bx_unscramble(bool fp64, const void *in, void *out, int64_t T, int N, int b, int sbits,
                                double scale, hipStream_t s);
int staged_build(fft_plan_impl *pl, int t);
int staged_run(fft_plan_impl *pl, int t, const void *in, void *out, hipStream_t s);
int staged_part(fft_plan_impl *pl, int t, int part, const void *in, void *out, hipStream_t s);
void staged_free(fft_plan_impl *pl);

// Radix factorisation of a row length: powers of two as 8s with a 16, 4 or 2
// to finish, then 3s and 5s.  Returns the number of passes.  The autotuner
// times this built-in order too.
int factor_radices(i64 n, int *rad)
{
    int np = 0;
    int e2 = 0;
    while (n % 2 == 0) {
        n /= 2;
        ++e2;
    }
    int e3 = 0, e5 = 0;
    while (n % 3 == 0) {
        n /= 3;
        ++e3;
    }
    while (n % 5 == 0) {
        n /= 5;
        ++e5;
    }
    // power-of-two part
    int n8 = e2 / 3, rem = e2 % 3;
    if (rem == 1 && n8 >= 1) {  // 2^(3m+1) = 16 * 8^(m-1)
        rad[np++] = 16;
        --n8;
        rem = 0;
    }
    for (int i = 0; i < n8; ++i) rad[np++] = 8;
    if (rem == 2) rad[np++] = 4;
    if (rem == 1) rad[np++] = 2;
    for (int i = 0; i < e3; ++i) rad[np++] = 3;
    for (int i = 0; i < e5; ++i) rad[np++] = 5;
    return np;
}

namespace {

int hip_fail(hipError_t e, const char *what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(FFTRW_E_DEVICE, m);
}

#define HIP_TRY(expr, what)                     \
    do {                                        \
        hipError_t _e = (expr);                 \
        if (_e != hipSuccess) return hip_fail(_e, what); \
    } while (0)

bool smooth235(i64 n)
{
    if (n < 1) return false;
    for (int p : {2, 3, 5})
        while (n % p == 0) n /= p;
    return n == 1;
}


i64 pow2ceil(i64 x)
{
    i64 p = 1;
    while (p < x) p <<= 1;
    return p;
}

int make_len_desc(fft_plan_impl *pl, i64 N, FftDesc *d, bool generic_rows, const TuneTable *tune)
{
    if (!smooth235(N) || N > 4096)
        return fail(FFTRW_E_SIZE, "row length " + std::to_string(N) + " must be 2^a 3^b 5^c and <= 4096");
    std::memset(d, 0, sizeof(*d));
    d->N = (int)N;
    d->nrows = pl->T / N;
    if (pl->precision != FFTRW_PREC_NATIVE && (N == 256 || N == 512)) {
        // two radix-16 DFT contractions on MFMA (per half row for 512, then a
        // radix-2 combination), generic N-entry twiddle table
        d->mfma = pl->precision;
        d->npass = N == 256 ? 2 : 3;
        d->radix[0] = d->radix[1] = 16;
        d->radix[2] = 2;
        d->tw_count = (int)N;
        return FFTRW_OK;
    }
    if (!generic_rows && pow2_supported((int)N, pl->esz == 16)) {
        d->pow2 = 1;
        pow2_describe((int)N, pl->esz == 16, &d->tw_count, d->radix, &d->npass);
        return FFTRW_OK;
    }
    d->npass = factor_radices(N, d->radix);
    d->tw_count = (int)N;
    const i64 elems = pl->esz == 8 ? 4096 : 2048;
    i64 rw = 1;
    while (rw * 2 <= 256 && rw * 2 * N <= elems) rw *= 2;
    if (tune) {
        // autotuned radix order and rows per work-group, checked against the
        // kernel's limits (radix set, product, LDS size, 16 values per lane)
        auto it = tune->rows.find((int)N);
        if (it != tune->rows.end()) {
            const RowTune &rt = it->second;
            i64 prod = 1;
            bool ok = !rt.radix.empty() && (int)rt.radix.size() <= kMaxPasses;
            for (int r : rt.radix) {
                ok = ok && (r == 2 || r == 3 || r == 4 || r == 5 || r == 8 || r == 16);
                prod *= r;
            }
            if (ok && prod == N) {
                d->npass = (int)rt.radix.size();
                for (int q = 0; q < d->npass; ++q) d->radix[q] = rt.radix[q];
            }
            const i64 trw = rt.rows_per_wg;
            if (trw >= 1 && trw <= rw && (trw & (trw - 1)) == 0) rw = trw;
        }
    }
    d->rows_per_wg = (int)rw;
    d->lanes_per_row = (int)(256 / rw);
    d->nrows = pl->T / N;
    return FFTRW_OK;
}

int make_fft_desc(fft_plan_impl *pl, int t, FftDesc *d, bool generic_rows, const TuneTable *tune)
{
    const int ax = pl->order[t * pl->M + pl->M - 1];
    return make_len_desc(pl, pl->dims[ax], d, generic_rows, tune);
}

int dev_alloc(fft_plan_impl *pl, void **p, size_t bytes);

// The twiddle table a descriptor's kernel reads: the per-pass table of the
// compile-time power-of-two kernel, else w_N^e for e < N, generated on the
// device in FP64 and rounded.
int make_desc_twiddles(fft_plan_impl *pl, const FftDesc &d, void **tw)
{
    if (int rc = dev_alloc(pl, tw, (size_t)std::max(1, d.tw_count) * pl->esz)) return rc;
    hipStream_t ts = pl->arena ? pl->arena->stream : nullptr;
    hipError_t e = (d.pow2 && !d.mfma) ? pow2_make_twiddles(d.N, pl->esz == 16, *tw, ts)
                                       : launch_twiddles(*tw, d.N, pl->esz == 16, ts);
    if (e != hipSuccess) return hip_fail(e, "twiddle generation");
    return FFTRW_OK;
}

int make_xpose_desc(fft_plan_impl *pl, const Layout &a, const Layout &b, const std::vector<i64> *mu,
                    unsigned long long *counter, XposeDesc *d, const TuneTable *tune)
{
    const int M = pl->M;
    std::memset(d, 0, sizeof(*d));
    const int u = a.perm[M - 1], v = b.perm[M - 1];
    if (u == v) return fail(FFTRW_E_ORDER, "consecutive decompositions share their last axis");
    d->Nu = pl->dims[u];
    d->Nv = pl->dims[v];
    d->a_sv = a.stride[v];
    d->b_su = b.stride[u];
    // batch axes, innermost = smallest stride in A
    int bat[3], nb = 0;
    for (int ax = 0; ax < M; ++ax)
        if (ax != u && ax != v) bat[nb++] = ax;
    std::sort(bat, bat + nb, [&](int x, int y) { return a.stride[x] < a.stride[y]; });
    d->nbat = nb;
    d->nslices = 1;
    int batpos[kMaxDims];
    for (int i = 0; i < kMaxDims; ++i) batpos[i] = -1;
    for (int i = 0; i < nb; ++i) {
        d->bsize[i] = pl->dims[bat[i]];
        d->ba[i] = a.stride[bat[i]];
        d->bb[i] = b.stride[bat[i]];
        d->nslices *= d->bsize[i];
        batpos[bat[i]] = i;
    }
    d->TU = (int)std::min<i64>(64, pow2ceil(d->Nu));
    d->TV = (int)std::min<i64>(64, pow2ceil(d->Nv));
    const i64 elems = pl->esz == 8 ? 4096 : 2048;
    i64 G = std::max<i64>(1, elems / ((i64)d->TU * d->TV));
    if (tune) {
        auto it = tune->tiles.find({(int)d->Nu, (int)d->Nv});
        if (it != tune->tiles.end()) {
            const TileTune &tt = it->second;
            auto pow2ok = [](int x) { return x >= 1 && x <= 64 && (x & (x - 1)) == 0; };
            if (pow2ok(tt.TU) && pow2ok(tt.TV) && tt.G >= 1 && (i64)tt.G * tt.TU * tt.TV <= elems) {
                d->TU = tt.TU;
                d->TV = tt.TV;
                G = tt.G;
            }
        }
    }
    G = std::min<i64>(G, 256);
    G = std::min<i64>(G, d->nslices);
    d->G = (int)G;
    d->tiles_u = (d->Nu + d->TU - 1) / d->TU;
    d->tiles_v = (d->Nv + d->TV - 1) / d->TV;
    d->tiles_g = (d->nslices + G - 1) / G;
    if (d->tiles_u * d->tiles_v * d->tiles_g >= (i64)0x7fffffff || d->nslices >= (i64)0x7fffffff)
        return fail(FFTRW_E_SIZE, "array too large for one transpose launch");
    d->count = counter != nullptr;
    d->counter = counter;
    d->P = pl->P;
    d->ka = a.k;
    d->kb = b.k;
    d->Ra = a.R;
    d->Rb = b.R;
    d->owner32 = (__int128)a.R * pl->P < ((__int128)1 << 32) && (__int128)b.R * pl->P < ((__int128)1 << 32);
    for (int j = 0; j < a.k; ++j) {
        const int ax = a.perm[j];
        d->srca[j] = ax == v ? 3 : ax == u ? 4 : batpos[ax];
        i64 w = 1;
        for (int i = j + 1; i < a.k; ++i) w *= a.pd[i];
        d->wa[j] = w;
    }
    for (int j = 0; j < b.k; ++j) {
        const int ax = b.perm[j];
        d->srcb[j] = ax == u ? 4 : ax == v ? 3 : batpos[ax];
        i64 w = 1;
        for (int i = j + 1; i < b.k; ++i) w *= b.pd[i];
        d->wb[j] = w;
    }
    (void)mu;
    return FFTRW_OK;
}

void free_plan(fft_plan_impl *pl)
{
    if (!pl) return;
    for (hipEvent_t e : pl->events) (void)hipEventDestroy(e);
    pl->events.clear();
    staged_free(pl);
    for (void *p : pl->allocs) (void)hipFree(p);
    pl->allocs.clear();
    delete static_cast<fft_plan_s *>(pl);
}

int dev_alloc(fft_plan_impl *pl, void **p, size_t bytes)
{
    if (bytes == 0) bytes = 16;
    if (pl->arena) {
        DevArena &a = *pl->arena;
        const size_t off = (a.used + 255) & ~(size_t)255;
        if (off > a.cap || bytes > a.cap - off)
            return fail(FFTRW_E_SIZE, "the fixed device region holds " + std::to_string(a.cap) + " bytes, " +
                                          std::to_string(off + bytes) + " needed");
        *p = a.base + off;
        a.used = off + bytes;
        pl->dev_bytes += bytes;
        return FFTRW_OK;
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(FFTRW_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    pl->allocs.push_back(*p);
    pl->dev_bytes += bytes;
    return FFTRW_OK;
}

int run_fft_desc(fft_plan_impl *pl, const FftDesc &d, int dir, const void *in, void *out, double scale,
                 hipStream_t s)
{
    if (d.mfma) {
        HIP_TRY(launch_fft_mfma(d.mfma, dir, d.N, d.tw, d.nrows, in, out, scale, s), "mfma fft pass launch");
        return FFTRW_OK;
    }
    if (d.pow2) {
        HIP_TRY(launch_fft_pow2(d.N, pl->esz == 16, d.tw, d.nrows, dir, in, out, scale, s), "fft pass launch");
        return FFTRW_OK;
    }
    HIP_TRY(launch_fft_rows(d, pl->esz == 16, dir, in, out, scale, s), "fft pass launch");
    return FFTRW_OK;
}

// Step t at level M in a staged plan: the split rows' binary exchange (see
// rowsplit.hip), then b-point DFTs of the blocks and the permutation to
// natural order within each row.  Works in place on `out` (copied from `in`
// first when they differ); the staging receive array carries the messages.
int run_split_step(fft_plan_impl *pl, int t, int dir, const void *in, void *out, double scale, hipStream_t s)
{
    const SplitStep &sp = pl->split[t];
    const bool fp64 = pl->esz == 16;
    const int N = pl->fft[t].N;
    if (in != out)
        HIP_TRY(hipMemcpyAsync(out, in, (size_t)pl->T * pl->esz, hipMemcpyDeviceToDevice, s), "split-row copy");
    unsigned long long *ctr = pl->counters + (size_t)(pl->M + t) * kCountBlock;
    for (int st = 0; st < sp.s; ++st) {
        const int h = N >> (st + 1);
        HIP_TRY(launch_bx_exchange(fp64, out, pl->recv, pl->T, N, sp.b, h / sp.b, ctr, s), "split-row exchange");
        HIP_TRY(launch_bx_butterfly(fp64, dir, out, pl->recv, pl->T, N, h, sp.tw, s), "split-row butterflies");
    }
    if (sp.b > 1)
        if (int rc = run_fft_desc(pl, sp.local, dir, out, out, 1.0, s)) return rc;
    HIP_TRY(launch_bx_unscramble(fp64, out, pl->recv, pl->T, N, sp.b, sp.s, scale, s), "split-row order");
    HIP_TRY(hipMemcpyAsync(out, pl->recv, (size_t)pl->T * pl->esz, hipMemcpyDeviceToDevice, s), "split-row copy");
    return FFTRW_OK;
}

int run_fft_step(fft_plan_impl *pl, int t, int dir, const void *in, void *out, double scale, hipStream_t s)
{
    if (!pl->split.empty() && pl->split[t].c > 0) return run_split_step(pl, t, dir, in, out, scale, s);
    return run_fft_desc(pl, pl->fft[t], dir, in, out, scale, s);
}

int run_transpose(fft_plan_impl *pl, int t, const void *in, void *out, hipStream_t s)
{
    if ((pl->flags & FFTRW_FLAG_STAGED) && pl->xp_staged[t]) return staged_run(pl, t, in, out, s);
    HIP_TRY(launch_xpose(pl->xp[t], pl->esz, in, out, s), "transpose launch");
    return FFTRW_OK;
}

int run_pipeline(fft_plan_impl *pl, const void *in, void *out, hipStream_t s, int dir)
{
    const int M = pl->M;
    const bool leave = (pl->flags & FFTRW_FLAG_LEAVE_PERMUTED) != 0;
    const int nx = leave ? M - 1 : M;
    if (pl->counters) HIP_TRY(launch_zero_u64(pl->counters, pl->n_counters, s), "counter reset");
    int nev = 0;
    auto mark = [&]() -> int {
        if (!pl->timing) return FFTRW_OK;
        HIP_TRY(hipEventRecord(pl->events[nev++], s), "timing event");
        return FFTRW_OK;
    };
    if (int rc = mark()) return rc;
    if (pl->fused && in != out) {
        // every step is one out-of-place kernel: FFT along u, written in the
        // next layout; the buffers alternate so the last one lands in out
        const void *src = in;
        for (int t = 0; t < nx; ++t) {
            void *dst = ((nx - 1 - t) % 2 == 0) ? out : pl->work;
            const double scale = (dir > 0 && t == M - 1) ? 1.0 / (double)pl->T : 1.0;
            const FftDesc &d = pl->fft[t];
            if (pl->fuse_kind[t] == 1)
                HIP_TRY(launch_fft_xpose_pow2(d.N, pl->esz == 16, d.tw, pl->xp[t], dir, src, dst, scale, s),
                        "fused fft+transpose launch");
            else if (pl->fuse_kind[t] == 3)
                HIP_TRY(launch_fft_mfma_xpose(d.mfma, dir, d.N, d.tw, pl->xp[t], src, dst, scale, s),
                        "fused mfma fft+transpose launch");
            else
                HIP_TRY(launch_fft_xpose_generic(d, pl->xp[t], pl->esz == 16, dir, src, dst, scale, s),
                        "fused fft+transpose launch");
            if (int rc = mark()) return rc;
            src = dst;
        }
        if (leave) {
            const double scale = dir > 0 ? 1.0 / (double)pl->T : 1.0;
            if (int rc = run_fft_step(pl, M - 1, dir, out, out, scale, s)) return rc;
            if (int rc = mark()) return rc;
        }
        pl->n_recorded = nev;
        pl->executed = true;
        return FFTRW_OK;
    }
    void *b0 = (nx % 2 == 0) ? out : pl->work;
    void *b1 = (b0 == out) ? pl->work : out;
    void *cur = b0, *other = b1;
    for (int t = 0; t < M; ++t) {
        const double scale = (dir > 0 && t == M - 1) ? 1.0 / (double)pl->T : 1.0;
        int rc = run_fft_step(pl, t, dir, t == 0 ? in : cur, cur, scale, s);
        if (rc || (rc = mark())) return rc;
        if (t < nx) {
            if (pl->timing && (pl->flags & FFTRW_FLAG_STAGED) && pl->xp_staged[t]) {
                // pack, exchange and unpack as stages of their own
                for (int part = 0; part < 3 && !rc; ++part) {
                    rc = staged_part(pl, t, part, cur, other, s);
                    if (!rc) rc = mark();
                }
                if (rc) return rc;
            } else {
                rc = run_transpose(pl, t, cur, other, s);
                if (rc || (rc = mark())) return rc;
            }
            std::swap(cur, other);
        }
    }
    pl->n_recorded = nev;
    pl->executed = true;
    return FFTRW_OK;
}

}  // namespace

// Build a plan; generic_rows forces the runtime-radix row kernel for every
// step (the persistent batched kernel runs only that one).
int plan_create(fft_plan_t *plan, int M, const int64_t *dims, int64_t P, const int8_t *order, int dtype,
                int precision, unsigned flags, bool generic_rows, const TuneTable *tune, DevArena *arena)
{
    g_last_error.clear();
    if (!plan) return fail(FFTRW_E_ARG, "plan must not be null");
    *plan = nullptr;
    if (M < 2 || M > kMaxDims) return fail(FFTRW_E_SIZE, "plans run M = 2..5");
    Status st = check_dims(M, dims);
    if (!st) return fail(st);
    if (P < 1) return fail(FFTRW_E_ARG, "P must be >= 1");
    if (dtype != FFTRW_C64 && dtype != FFTRW_C128) return fail(FFTRW_E_ARG, "unknown dtype");
    if (precision < FFTRW_PREC_NATIVE || precision > FFTRW_PREC_SPLIT_BF16X3)
        return fail(FFTRW_E_ARG, "unknown precision");
    if (precision != FFTRW_PREC_NATIVE && dtype != FFTRW_C64)
        return fail(FFTRW_E_UNSUPPORTED, "the split-precision MFMA form computes complex64 data");
    if (flags & ~(unsigned)(FFTRW_FLAG_LEAVE_PERMUTED | FFTRW_FLAG_STAGED | FFTRW_FLAG_COUNT_MOVED |
                            FFTRW_FLAG_OWN_MATCHED | FFTRW_FLAG_FUSED_FFT | FFTRW_FLAG_BATCH_NO_GRAPH |
                            FFTRW_FLAG_SEPARATE))
        return fail(FFTRW_E_ARG, "unknown flag bits");
    if ((flags & FFTRW_FLAG_SEPARATE) && (flags & FFTRW_FLAG_FUSED_FFT))
        return fail(FFTRW_E_ARG, "FFTRW_FLAG_SEPARATE and FFTRW_FLAG_FUSED_FFT exclude each other");

    fft_plan_s *pl = new (std::nothrow) fft_plan_s();
    if (!pl) return fail(FFTRW_E_NOMEM, "out of host memory");
    pl->M = M;
    pl->P = P;
    pl->dtype = dtype;
    pl->precision = precision;
    pl->flags = flags;
    pl->arena = arena;
    pl->ownership = (flags & FFTRW_FLAG_OWN_MATCHED) ? FFTRW_OWN_MATCHED : FFTRW_OWN_LITERAL;
    pl->esz = dtype == FFTRW_C64 ? 8 : 16;
    pl->T = 1;
    for (int i = 0; i < M; ++i) {
        pl->dims[i] = dims[i];
        pl->T *= dims[i];
    }
    if (order) {
        st = check_order(M, order);
        if (!st) {
            free_plan(pl);
            return fail(st);
        }
        std::memcpy(pl->order, order, (size_t)(M * M));
    } else {
        int64_t bi = 0;
        int rc = fft_order_search(M, dims, P, FFTRW_OWN_LITERAL, &bi, nullptr, nullptr, nullptr, nullptr,
                                  nullptr, pl->order, nullptr);
        if (rc) {
            free_plan(pl);
            return rc;
        }
    }
    // layouts
    int8_t ident[kMaxDims];
    for (int i = 0; i < M; ++i) ident[i] = (int8_t)i;
    for (int t = 0; t <= M; ++t) {
        st = make_layout(M, dims, P, t < M ? pl->order + t * M : ident, &pl->lay[t]);
        if (!st) {
            free_plan(pl);
            return fail(st);
        }
    }
    // analytic amounts (and relabellings for the matched reading)
    pl->analytic.assign(M, 0);
    pl->mu.assign(M, {});
    for (int t = 0; t < M; ++t) {
        st = transpose_amount(pl->lay[t], pl->lay[t + 1], pl->ownership, &pl->analytic[t], &pl->mu[t]);
        if (!st) {
            free_plan(pl);
            return fail(st);
        }
    }
    int rc = hipGetDevice(&pl->device) == hipSuccess ? 0 : -1;
    if (rc) {
        free_plan(pl);
        return fail(FFTRW_E_DEVICE, "no HIP device");
    }
    // FFT descriptors and twiddles
    pl->fft.resize(M);
    for (int t = 0; t < M; ++t) {
        rc = make_fft_desc(pl, t, &pl->fft[t], generic_rows, tune);
        if (rc) {
            free_plan(pl);
            return rc;
        }
        const int N = pl->fft[t].N;
        if (!pl->twiddles.count(N)) {
            void *tw = nullptr;
            rc = dev_alloc(pl, &tw, (size_t)std::max(1, pl->fft[t].tw_count) * pl->esz);
            if (rc) {
                free_plan(pl);
                return rc;
            }
            hipStream_t ts = arena ? arena->stream : nullptr;
            hipError_t e = (pl->fft[t].pow2 && !pl->fft[t].mfma) ? pow2_make_twiddles(N, pl->esz == 16, tw, ts)
                                                                 : launch_twiddles(tw, N, pl->esz == 16, ts);
            if (e != hipSuccess) {
                free_plan(pl);
                return hip_fail(e, "twiddle generation");
            }
            pl->twiddles[N] = tw;
        }
        pl->fft[t].tw = pl->twiddles[N];
    }
    // staged plans at level M: each split step must be c = 2^s whole ranges of
    // b = T / N_p points per row, run as a binary exchange (rowsplit.hip)
    bool any_split = false;
    if (flags & FFTRW_FLAG_STAGED) {
        pl->split.assign(M, SplitStep{});
        pl->split_analytic.assign(M, 0);
        int64_t tot = 0;
        if ((rc = fft_rowsplit_volume(M, dims, P, pl->order, pl->split_analytic.data(), &tot))) {
            free_plan(pl);
            return rc;
        }
        for (int t = 0; t < M; ++t) {
            if (!pl->lay[t].row_split()) continue;
            const i64 N = pl->fft[t].N;
            const i64 b = pl->T / P;
            const i64 c = b > 0 && pl->T % P == 0 && N % b == 0 ? N / b : 0;
            if (c < 2 || (c & (c - 1)) != 0) {
                free_plan(pl);
                return fail(FFTRW_E_ROWSPLIT,
                            "staged plans run a step at level M (rows split over processes) as a binary exchange "
                            "only when every range holds T / N_p points and each row is a power-of-two number of "
                            "ranges; here T = " + std::to_string(pl->T) + ", N_p = " + std::to_string(P) +
                                ", row length " + std::to_string(N));
            }
            SplitStep &sp = pl->split[t];
            sp.b = (int)b;
            sp.c = (int)c;
            while ((1 << sp.s) < sp.c) ++sp.s;
            FftDesc full = {};
            full.N = (int)N;
            full.tw_count = (int)N;  // w_N^e, e < N
            if ((rc = make_desc_twiddles(pl, full, &sp.tw))) {
                free_plan(pl);
                return rc;
            }
            if (b > 1) {
                if ((rc = make_len_desc(pl, b, &sp.local, false, tune)) ||
                    (rc = make_desc_twiddles(pl, sp.local, const_cast<void **>(&sp.local.tw)))) {
                    free_plan(pl);
                    return rc;
                }
            }
            any_split = true;
        }
    }
    // workspace and counters (staged plans also count each split step's exchange)
    rc = dev_alloc(pl, &pl->work, (size_t)pl->T * pl->esz);
    if (!rc && (flags & (FFTRW_FLAG_COUNT_MOVED | FFTRW_FLAG_STAGED))) {
        pl->n_counters = ((flags & FFTRW_FLAG_STAGED) ? 2 : 1) * M * kCountBlock;
        rc = dev_alloc(pl, (void **)&pl->counters, sizeof(unsigned long long) * (size_t)pl->n_counters);
    }
    if (!rc && any_split && !pl->send) {
        // the staging arrays (freed with the staged tables); the split steps'
        // messages go through the receive array
        for (void **buf : {&pl->send, &pl->recv}) {
            if (hipMalloc(buf, (size_t)pl->T * pl->esz) != hipSuccess) {
                (void)hipGetLastError();
                rc = fail(FFTRW_E_NOMEM, "hipMalloc of staging buffers failed");
                break;
            }
            pl->dev_bytes += (size_t)pl->T * pl->esz;
        }
    }
    if (rc) {
        free_plan(pl);
        return rc;
    }
    // relabelling tables on the device (matched reading)
    std::vector<int *> mu_dev(M, nullptr);
    if (pl->ownership == FFTRW_OWN_MATCHED) {
        for (int t = 0; t < M; ++t) {
            std::vector<int> m32(pl->mu[t].begin(), pl->mu[t].end());
            void *p = nullptr;
            rc = dev_alloc(pl, &p, sizeof(int) * m32.size());
            if (!rc && hipMemcpy(p, m32.data(), sizeof(int) * m32.size(), hipMemcpyHostToDevice) != hipSuccess)
                rc = fail(FFTRW_E_DEVICE, "copy of relabelling table failed");
            if (rc) {
                free_plan(pl);
                return rc;
            }
            mu_dev[t] = (int *)p;
        }
    }
    // transposes
    pl->xp.resize(M);
    pl->staged.resize(M);
    for (int t = 0; t < M; ++t) {
        // staged plans: transposes between whole-row layouts run pack ->
        // exchange -> unpack; one that touches a level-M layout (rows split)
        // runs the fused permutation with its owner changes counted
        const bool staged = (flags & FFTRW_FLAG_STAGED) && !pl->lay[t].row_split() && !pl->lay[t + 1].row_split();
        pl->xp_staged[t] = staged;
        unsigned long long *ctr = (flags & (FFTRW_FLAG_COUNT_MOVED | FFTRW_FLAG_STAGED))
                                      ? pl->counters + (size_t)t * kCountBlock
                                      : nullptr;
        rc = make_xpose_desc(pl, pl->lay[t], pl->lay[t + 1], &pl->mu[t], ctr, &pl->xp[t], tune);
        if (rc) {
            free_plan(pl);
            return rc;
        }
        pl->xp[t].mu = mu_dev[t];
        if (staged) {
            rc = staged_build(pl, t);
            if (rc) {
                free_plan(pl);
                return rc;
            }
        }
    }
    // fusion of every FFT step with its transpose (the default): power-of-two
    // rows of 16..512 (256 in FP64) whose work-group's run of consecutive
    // v-values fits the v axis use the compile-time kernel; 2,3,5-smooth rows
    // use the generic unit; steps of the split-precision form (256 and 512
    // points) use the MFMA kernel
    if (!(flags & (FFTRW_FLAG_SEPARATE | FFTRW_FLAG_STAGED)) && !generic_rows) {
        const bool fp64 = pl->esz == 16;
        const int nx = (flags & FFTRW_FLAG_LEAVE_PERMUTED) ? M - 1 : M;
        bool ok = true;
        for (int t = 0; t < nx && ok; ++t) {
            const FftDesc &d = pl->fft[t];
            const bool pow2_ok = d.pow2 && !d.mfma && d.N >= 16 && d.N <= (fp64 ? 256 : 512) &&
                                 pow2_rows_per_wg(d.N, fp64) <= pl->xp[t].Nv;
            const bool generic_ok = !d.pow2 && !d.mfma && d.N + 1 <= (fp64 ? 2048 : 4096);
            pl->fuse_kind[t] = d.mfma ? 3 : (pow2_ok ? 1 : (generic_ok ? 2 : 0));
            ok = pl->fuse_kind[t] != 0;
        }
        pl->fused = ok;
    }
    // (an arena plan only enqueues: its caller's stream orders the twiddle
    // kernels before the transform)
    if (!arena && hipDeviceSynchronize() != hipSuccess) {
        free_plan(pl);
        return fail(FFTRW_E_DEVICE, "device error during plan creation");
    }
    if (log_level() >= 1) {
        char text[256];
        (void)fft_plan_describe(pl, nullptr, text, sizeof(text));
        std::string dd, oo;
        for (int i = 0; i < M; ++i) dd += (i ? "x" : "") + std::to_string(dims[i]);
        for (int t = 0; t < M; ++t) {
            if (t) oo += "->";
            for (int i = 0; i < M; ++i) oo += (char)('a' + pl->order[t * M + i]);
        }
        log_line(1, "plan %s P=%lld order %s kernels %s flags 0x%x workspace %zu bytes", dd.c_str(), (long long)P,
                 oo.c_str(), text, flags, pl->dev_bytes);
    }
    *plan = pl;
    return FFTRW_OK;
}

void plan_free(fft_plan_t plan) { free_plan(plan); }

int plan_run(fft_plan_impl *pl, const void *in, void *out, hipStream_t s, int dir)
{
    return run_pipeline(pl, in, out, s, dir);
}

}  // namespace fftrw

using namespace fftrw;

extern "C" {

int fft_plan(fft_plan_t *plan, int M, const int64_t *dims, int64_t P, const int8_t *order, int dtype,
             int precision, unsigned flags)
{
    return fftrw::plan_create(plan, M, dims, P, order, dtype, precision, flags, false, nullptr, nullptr);
}

int fft_exec_fwd(fft_plan_t plan, const void *in, void *out, void *stream)
{
    g_last_error.clear();
    if (!plan || !in || !out) return fail(FFTRW_E_ARG, "null plan or buffer");
    log_line(3, "exec forward plan %p in %p out %p stream %p", (void *)plan, in, out, stream);
    return run_pipeline(plan, in, out, (hipStream_t)stream, -1);
}

int fft_exec_inv(fft_plan_t plan, const void *in, void *out, void *stream)
{
    g_last_error.clear();
    if (!plan || !in || !out) return fail(FFTRW_E_ARG, "null plan or buffer");
    log_line(3, "exec inverse plan %p in %p out %p stream %p", (void *)plan, in, out, stream);
    return run_pipeline(plan, in, out, (hipStream_t)stream, +1);
}

int fft_exec_fft_step(fft_plan_t plan, int t, int direction, const void *in, void *out, void *stream)
{
    g_last_error.clear();
    if (!plan || !in || !out) return fail(FFTRW_E_ARG, "null plan or buffer");
    if (t < 0 || t >= plan->M) return fail(FFTRW_E_ARG, "step out of range");
    if (direction != -1 && direction != 1) return fail(FFTRW_E_ARG, "direction must be -1 or +1");
    return run_fft_step(plan, t, direction, in, out, 1.0, (hipStream_t)stream);
}

int fft_exec_transpose(fft_plan_t plan, int t, const void *in, void *out, void *stream)
{
    g_last_error.clear();
    if (!plan || !in || !out) return fail(FFTRW_E_ARG, "null plan or buffer");
    if (t < 0 || t >= plan->M) return fail(FFTRW_E_ARG, "transpose index out of range");
    if (in == out) return fail(FFTRW_E_ARG, "a transpose cannot run in place");
    hipStream_t s = (hipStream_t)stream;
    if (plan->counters) {
        hipError_t e = launch_zero_u64(plan->counters + (size_t)t * kCountBlock, kCountBlock, s);
        if (e != hipSuccess) return fail(FFTRW_E_DEVICE, hipGetErrorString(e));
    }
    int rc = run_transpose(plan, t, in, out, s);
    if (!rc) plan->executed = true;
    return rc;
}

int fft_plan_stats(fft_plan_t plan, int64_t *per_step, int64_t *moved)
{
    g_last_error.clear();
    if (!plan) return fail(FFTRW_E_ARG, "null plan");
    const int M = plan->M;
    if (per_step)
        for (int t = 0; t < M; ++t) per_step[t] = plan->analytic[t];
    if (moved) {
        for (int t = 0; t < M; ++t) moved[t] = -1;
        if (plan->counters && plan->executed) {
            std::vector<unsigned long long> h((size_t)M * kCountBlock);
            if (hipDeviceSynchronize() != hipSuccess)
                return fail(FFTRW_E_DEVICE, "device error before reading counters");
            if (hipMemcpy(h.data(), plan->counters, sizeof(unsigned long long) * h.size(), hipMemcpyDeviceToHost) !=
                hipSuccess)
                return fail(FFTRW_E_DEVICE, "reading counters failed");
            const bool leave = (plan->flags & FFTRW_FLAG_LEAVE_PERMUTED) != 0;
            for (int t = 0; t < M; ++t) {
                if (leave && t == M - 1) continue;
                unsigned long long sum = 0;
                for (int k = 0; k < kCountSlots; ++k) sum += h[(size_t)t * kCountBlock + (size_t)k * kCountStride];
                moved[t] = (int64_t)sum;
            }
        }
    }
    return FFTRW_OK;
}

int fft_plan_messages(fft_plan_t plan, int64_t *per_step)
{
    g_last_error.clear();
    if (!plan || !per_step) return fail(FFTRW_E_ARG, "null plan or output");
    if (!(plan->flags & FFTRW_FLAG_STAGED)) return fail(FFTRW_E_UNSUPPORTED, "the plan has no staged tables");
    for (int t = 0; t < plan->M; ++t) per_step[t] = plan->xp_staged[t] ? plan->staged[t].nseg : -1;
    return FFTRW_OK;
}

int fft_plan_rowsplit_stats(fft_plan_t plan, int64_t *per_step, int64_t *moved)
{
    g_last_error.clear();
    if (!plan) return fail(FFTRW_E_ARG, "null plan");
    const int M = plan->M;
    const bool staged = (plan->flags & FFTRW_FLAG_STAGED) != 0;
    if (per_step)
        for (int t = 0; t < M; ++t) per_step[t] = staged ? plan->split_analytic[t] : -1;
    if (moved) {
        for (int t = 0; t < M; ++t) moved[t] = -1;
        if (staged && plan->executed) {
            std::vector<unsigned long long> h((size_t)M * kCountBlock);
            if (hipDeviceSynchronize() != hipSuccess)
                return fail(FFTRW_E_DEVICE, "device error before reading counters");
            if (hipMemcpy(h.data(), plan->counters + (size_t)M * kCountBlock, sizeof(unsigned long long) * h.size(),
                          hipMemcpyDeviceToHost) != hipSuccess)
                return fail(FFTRW_E_DEVICE, "reading counters failed");
            for (int t = 0; t < M; ++t) {
                unsigned long long sum = 0;
                for (int k = 0; k < kCountSlots; ++k) sum += h[(size_t)t * kCountBlock + (size_t)k * kCountStride];
                moved[t] = (int64_t)sum;
            }
        }
    }
    return FFTRW_OK;
}

int fft_plan_set_timing(fft_plan_t plan, int enable)
{
    g_last_error.clear();
    if (!plan) return fail(FFTRW_E_ARG, "null plan");
    if (enable && plan->events.empty()) {
        plan->events.resize(4 * plan->M + 1);
        for (hipEvent_t &e : plan->events)
            if (hipEventCreate(&e) != hipSuccess) return fail(FFTRW_E_DEVICE, "hipEventCreate failed");
    }
    plan->timing = enable != 0;
    plan->n_recorded = 0;
    return FFTRW_OK;
}

int fft_plan_timings(fft_plan_t plan, float *ms, int cap, int *n)
{
    g_last_error.clear();
    if (!plan || !n) return fail(FFTRW_E_ARG, "null argument");
    const int stages = plan->n_recorded > 0 ? plan->n_recorded - 1 : 0;
    *n = stages;
    if (stages == 0) return FFTRW_OK;
    if (hipEventSynchronize(plan->events[stages]) != hipSuccess)
        return fail(FFTRW_E_DEVICE, "waiting for timing events failed");
    for (int i = 0; i < stages && i < cap; ++i) {
        float v = 0.f;
        if (hipEventElapsedTime(&v, plan->events[i], plan->events[i + 1]) != hipSuccess)
            return fail(FFTRW_E_DEVICE, "hipEventElapsedTime failed");
        if (ms) ms[i] = v;
    }
    return FFTRW_OK;
}

int fft_workspace_bytes(fft_plan_t plan, size_t *bytes)
{
    g_last_error.clear();
    if (!plan || !bytes) return fail(FFTRW_E_ARG, "null argument");
    *bytes = plan->dev_bytes;
    return FFTRW_OK;
}

int fft_plan_describe(fft_plan_t plan, int8_t *order, char *text, size_t cap)
{
    g_last_error.clear();
    if (!plan) return fail(FFTRW_E_ARG, "null plan");
    if (order) std::memcpy(order, plan->order, (size_t)(plan->M * plan->M));
    if (text && cap) {
        std::string s = plan->fused ? "fused|" : "";
        for (int t = 0; t < plan->M; ++t) {
            if (t) s += ";";
            if (plan->fft[t].mfma) s += "mfma:";
            for (int p = 0; p < plan->fft[t].npass; ++p) {
                if (p) s += "x";
                s += std::to_string(plan->fft[t].radix[p]);
            }
        }
        std::snprintf(text, cap, "%s", s.c_str());
    }
    return FFTRW_OK;
}

int fft_destroy(fft_plan_t plan)
{
    g_last_error.clear();
    if (!plan) return FFTRW_OK;
    free_plan(plan);
    return FFTRW_OK;
}

}  // extern "C"
