// fft_mfma.hip -- 256- and 512-point row FFTs as radix-16 DFT contractions on
// MFMA.
//
// The precision form of a step of Fig. 4: with N = 256 = 16 x 16 and the row
// x viewed as the 16 x 16 matrix X[n1][n2] = x[16 n1 + n2], Eq. (1) factors as
//     Y  = F16 X                        (16-point DFTs of the 16 columns)
//     Y'[k1][n2] = Y[k1][n2] w_256^{n2 k1}
//     Z  = F16 Y'^T,   xbar[16 k2 + k1] = Z[k2][k1],
// F16[k][n] = w_16^{kn}.  Both products are 16 x 16 complex matrices times
// 16 x 16 complex matrices, run in real form on one wave as
//     Re = [Fr | -Fi] [Br; Bi],   Im = [Fi | Fr] [Br; Bi]
// (16x32 by 32x16, one v_mfma_f32_16x16x32 each).  Operands are split into a
// high and a low half-precision part (FP16, or BF16 with two or three parts)
// after a power-of-two scaling per column (one 16-point input vector), and
// the partial products are accumulated in FP32:
//     two parts:   A_h B_h + A_h B_l + A_l B_h
//     three parts: the six products whose parts' orders sum to at most 2.
// The twiddles between the stages are applied in FP32 from a table computed
// in FP64; F16 itself is generated in FP64 on the device.  A 512-point row is
// split into its even and odd points: two such 256-point transforms, then one
// radix-2 combination in FP32.  The table is w_N^e for e < N (w_256 = w_512^2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>

#include "cplx.hpp"
#include "kernels.hpp"
#include "xpose_tile.hpp"

namespace fftrw {

typedef _Float16 mh8 __attribute__((ext_vector_type(8)));
typedef __bf16 mb8 __attribute__((ext_vector_type(8)));
typedef float mf4 __attribute__((ext_vector_type(4)));
typedef float mf2v __attribute__((ext_vector_type(2)));

enum { kPrecF16 = 1, kPrecBF16 = 2, kPrecBF16x3 = 3 };

template <int PREC> struct Parts;
template <> struct Parts<kPrecF16> {
    using V = mh8;
    static constexpr int n = 2;
    static __device__ __forceinline__ float round(float x) { return (float)(_Float16)x; }
    static __device__ __forceinline__ mf4 mma(V a, V b, mf4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ void set(V &v, int i, float x) { v[i] = (_Float16)x; }
};
template <int PREC> struct PartsBF16 {
    using V = mb8;
    static constexpr int n = PREC == kPrecBF16 ? 2 : 3;
    static __device__ __forceinline__ float round(float x) { return (float)(__bf16)x; }
    static __device__ __forceinline__ mf4 mma(V a, V b, mf4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ void set(V &v, int i, float x) { v[i] = (__bf16)x; }
};
template <> struct Parts<kPrecBF16> : PartsBF16<kPrecBF16> {};
template <> struct Parts<kPrecBF16x3> : PartsBF16<kPrecBF16x3> {};

// split 8 values into PT::n parts (x = p0 + p1 [+ p2] up to rounding of the last)
template <class PT>
__device__ __forceinline__ void split8(const float *x, typename PT::V *p)
{
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        float r = x[i];
#pragma unroll
        for (int q = 0; q < PT::n; ++q) {
            const float h = PT::round(r);
            PT::set(p[q], i, h);
            r -= h;
        }
    }
}

// C += A B over the split parts, smallest terms first
template <class PT>
__device__ __forceinline__ mf4 split_product(const typename PT::V *a, const typename PT::V *b)
{
    mf4 acc = {0.f, 0.f, 0.f, 0.f};
    if constexpr (PT::n == 3) {
        acc = PT::mma(a[1], b[1], acc);
        acc = PT::mma(a[2], b[0], acc);
        acc = PT::mma(a[0], b[2], acc);
    }
    acc = PT::mma(a[1], b[0], acc);
    acc = PT::mma(a[0], b[1], acc);
    acc = PT::mma(a[0], b[0], acc);
    return acc;
}

// power-of-two exponent s such that max|x| * 2^s lies in [2^14, 2^15)
__device__ __forceinline__ int column_exponent(const float *b, int lane)
{
    float m = 0.f;
#pragma unroll
    for (int v = 0; v < 8; ++v) m = fmaxf(m, fabsf(b[v]));
    // the 32 reals of a column sit in lanes c, c+16, c+32, c+48
    m = fmaxf(m, __shfl_xor(m, 16));
    m = fmaxf(m, __shfl_xor(m, 32));
    if (!(m > 0.f)) return 0;
    int e;
    (void)frexpf(m, &e);
    return 15 - e;
}

__device__ __forceinline__ void wave_sync()
{
    // LDS blocks here are private to one wave: order writes before other
    // lanes' reads with a wave-level barrier (no work-group barrier)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

typedef float mf4v __attribute__((ext_vector_type(4)));

// One 256-point DFT on MFMA over the subsequence s[m] = x[R m + h] (m < 256)
// of the row held in LDS with x[j] at xb[j XS] (R = 1: the row itself; R = 2:
// its even or odd points).
// Lane (g, c) returns Z[16 k2 + c] for k2 = 4 g + v in z[v].  tw holds
// w_256^{c k1} for k1 = 4 g + v.  yb is the wave's stage-1 block; the call
// begins and ends with a wave barrier, so consecutive calls may reuse it.
template <class PT, int DIR, int R, int XS>
__device__ __forceinline__ void dft256_mfma(const float2 *xb, float2 *yb, int h, const typename PT::V *a1,
                                            const typename PT::V *a2, const float2 *tw, int lane, float2 *z)
{
    using V = typename PT::V;
    const int g = lane >> 4;
    const int c = lane & 15;
    const bool im = g >= 2;
    const int n1base = 8 * (g & 1);
    wave_sync();

    // ---- stage 1: B[k][c] = s[16 n1 + c], k = 8g + v ------------------------
    float b[8];
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        const float2 e = xb[(R * (16 * (n1base + v) + c) + h) * XS];
        b[v] = im ? e.y : e.x;
    }
    const int s1 = column_exponent(b, lane);
#pragma unroll
    for (int v = 0; v < 8; ++v) b[v] = ldexpf(b[v], s1);
    V bp[PT::n];
    split8<PT>(b, bp);
    mf4 cr = split_product<PT>(a1, bp);
    mf4 ci = split_product<PT>(a2, bp);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const float re = ldexpf(cr[v], -s1), imv = ldexpf(ci[v], -s1);
        yb[(4 * g + v) * 17 + c] = DIR < 0 ? cmul(mk<float2>(re, imv), tw[v]) : cmulc(mk<float2>(re, imv), tw[v]);
    }
    wave_sync();

    // ---- stage 2: B2[n2][k1] = Y'[k1][n2], column k1 = c ----------------------
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        const float2 e = yb[c * 17 + n1base + v];
        b[v] = im ? e.y : e.x;
    }
    const int s2 = column_exponent(b, lane);
#pragma unroll
    for (int v = 0; v < 8; ++v) b[v] = ldexpf(b[v], s2);
    split8<PT>(b, bp);
    cr = split_product<PT>(a1, bp);
    ci = split_product<PT>(a2, bp);
#pragma unroll
    for (int v = 0; v < 4; ++v) z[v] = mk<float2>(ldexpf(cr[v], -s2), ldexpf(ci[v], -s2));
    wave_sync();
}

// The F16 operands [Fr | -Fi] and [Fi | Fr] of lane (g, c): row c, k = 8 g + v,
// computed in FP64 and split once per wave.
template <class PT, int DIR>
__device__ __forceinline__ void dft16_operands(int lane, typename PT::V *a1, typename PT::V *a2)
{
    const int g = lane >> 4;
    const int c = lane & 15;
    float f1[8], f2[8];
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        const int k = 8 * g + v;
        const int kk = k & 15;
        double sn, co;
        sincospi(2.0 * (double)((c * kk) & 15) / 16.0, &sn, &co);
        const float fr = (float)co, fi = (float)(DIR * sn);
        f1[v] = k < 16 ? fr : -fi;
        f2[v] = k < 16 ? fi : fr;
    }
    split8<PT>(f1, a1);
    split8<PT>(f2, a2);
}

// The whole N = 256 R point transform of the row in xb: for every lane's four
// frequencies k = 16 (4 g + v) + c, out[v] = X[k] and, for R = 2, out[4 + v] =
// X[k + 256].  R = 2 splits the row into its even and odd points (Eq. (1) with
// N = 2 x 256): X[k] = E[k] + w_512^k O[k], X[k + 256] = E[k] - w_512^k O[k],
// the combination in FP32 with w_512^k from the table (twc).
template <class PT, int DIR, int R, int XS>
__device__ __forceinline__ void dft_row_mfma(const float2 *xb, float2 *yb, const typename PT::V *a1,
                                             const typename PT::V *a2, const float2 *tw, const float2 *twc,
                                             int lane, float2 *out)
{
    dft256_mfma<PT, DIR, R, XS>(xb, yb, 0, a1, a2, tw, lane, out);
    if constexpr (R == 2) {
        float2 o[4];
        dft256_mfma<PT, DIR, R, XS>(xb, yb, 1, a1, a2, tw, lane, o);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const float2 t = DIR < 0 ? cmul(o[v], twc[v]) : cmulc(o[v], twc[v]);
            const float2 e = out[v];
            out[v] = mk<float2>(e.x + t.x, e.y + t.y);
            out[4 + v] = mk<float2>(e.x - t.x, e.y - t.y);
        }
    }
}

// Per-lane twiddles from the w_N^e table (N = 256 R): w_256^{c k1} = w_N^{R c k1}
// for the stage between the contractions, w_512^k for the combination.
template <int R>
__device__ __forceinline__ void mfma_twiddles(const float2 *__restrict__ twN, int lane, float2 *tw, float2 *twc)
{
    const int g = lane >> 4;
    const int c = lane & 15;
#pragma unroll
    for (int v = 0; v < 4; ++v) tw[v] = twN[R * c * (4 * g + v)];
#pragma unroll
    for (int v = 0; v < 4; ++v) twc[v] = R == 2 ? twN[16 * (4 * g + v) + c] : mk<float2>(1.f, 0.f);
}

template <int PREC, int DIR, int R>
__global__ void __launch_bounds__(kThreads)
    fft_mfma_kernel(const float2 *in, float2 *out, int64_t nrows, const float2 *__restrict__ twN, float scale,
                    int do_scale)
{
    using PT = Parts<PREC>;
    using V = typename PT::V;
    constexpr int N = 256 * R;
    constexpr int NQ = N / 128;  // 16-byte pieces of a row per lane
    __shared__ __align__(16) float2 xbuf[kThreads / 64][N];     // row in / row out
    __shared__ float2 ybuf[kThreads / 64][16 * 17];              // stage-1 result, padded

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4;
    const int c = lane & 15;
    float2 *xb = xbuf[wave];
    float2 *yb = ybuf[wave];

    V a1[PT::n], a2[PT::n];
    dft16_operands<PT, DIR>(lane, a1, a2);
    float2 tw[4], twc[4];
    mfma_twiddles<R>(twN, lane, tw, twc);

    const int64_t wstride = (int64_t)gridDim.x * (kThreads / 64);
    int64_t row = (int64_t)blockIdx.x * (kThreads / 64) + wave;
    mf4v p[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) p[q] = mf4v{0.f, 0.f, 0.f, 0.f};
    if (row < nrows) {
        const mf4v *src = reinterpret_cast<const mf4v *>(in + row * N);
#pragma unroll
        for (int q = 0; q < NQ; ++q) p[q] = __builtin_nontemporal_load(src + 64 * q + lane);
    }
    for (; row < nrows; row += wstride) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) reinterpret_cast<mf4v *>(xb)[64 * q + lane] = p[q];
        const int64_t nxt = row + wstride;
        if (nxt < nrows) {  // prefetch the next row while this one is transformed
            const mf4v *src = reinterpret_cast<const mf4v *>(in + nxt * N);
#pragma unroll
            for (int q = 0; q < NQ; ++q) p[q] = __builtin_nontemporal_load(src + 64 * q + lane);
        }
        float2 z[4 * R];
        dft_row_mfma<PT, DIR, R, 1>(xb, yb, a1, a2, tw, twc, lane, z);
        // X[k] (k = 16 (4g + v) + c [+ 256]) staged in xb for 16-byte stores
#pragma unroll
        for (int v = 0; v < 4 * R; ++v) {
            float2 e = z[v];
            if (do_scale) {
                e.x *= scale;
                e.y *= scale;
            }
            xb[256 * (v >> 2) + 16 * (4 * g + (v & 3)) + c] = e;
        }
        wave_sync();
        mf4v *dst = reinterpret_cast<mf4v *>(out + row * N);
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            __builtin_nontemporal_store(reinterpret_cast<mf4v *>(xb)[64 * q + lane], dst + 64 * q + lane);
        wave_sync();  // xb is rewritten by the next row
    }
}

// The same transform fused with the transpose that follows: a unit is 16
// rows consecutive in v (the next layout's last axis) of one batch slice;
// each wave transforms every fourth of them, the results meet in an LDS block
// S[k][row] and every frequency k leaves as one run of 16 consecutive v
// (128 bytes) in the next layout.  A 512-point row's input is staged in its
// own column of that block (x[j] at S[j][row]) and overwritten by its output
// once both contractions have read it, so the 70 KB block is the only row
// buffer and two work-groups fit a CU (8-row units, 64-byte runs, fit three
// and ran 40% slower); a 256-point row goes through a per-wave buffer.  A resident grid walks the units, so the
// split F16 operands (FP64 sin/cos) are built once per work-group.  Owner
// changes are counted per row (tile_moved).
constexpr int kMaxDevices = 64;  // devices whose resident grid size is cached

constexpr int kMfmaRows = 16;

template <int PREC, int DIR, int R>
__global__ void __launch_bounds__(kThreads)
    fft_mfma_xpose_kernel(const float2 *in, float2 *out, XposeDesc d, const float2 *__restrict__ twN, float scale,
                          int do_scale)
{
    using PT = Parts<PREC>;
    using V = typename PT::V;
    constexpr int N = 256 * R;
    constexpr int NQ = N / 128;
    constexpr int RW = kMfmaRows;
    constexpr int SR = RW + 1;
    constexpr bool kCol = R == 2;  // rows staged in their columns of stg
    __shared__ __align__(16) float2 xbuf[kCol ? 1 : kThreads / 64][kCol ? 1 : N];
    __shared__ float2 ybuf[kThreads / 64][16 * 17];
    __shared__ float2 stg[N * SR];
    __shared__ int moved_wg;

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4;
    const int c = lane & 15;
    float2 *yb = ybuf[wave];

    // the F16 operands and twiddles are set up once; the resident grid then
    // walks the units u = blockIdx.x, + gridDim.x, ...
    V a1[PT::n], a2[PT::n];
    dft16_operands<PT, DIR>(lane, a1, a2);
    float2 tw[4], twc[4];
    mfma_twiddles<R>(twN, lane, tw, twc);
    if (threadIdx.x == 0) moved_wg = 0;
    int moved = 0;

    const int64_t tiles_v = (d.Nv + RW - 1) / RW;
    const int64_t nunits = tiles_v * d.nslices;
    for (int64_t unit = blockIdx.x; unit < nunits; unit += gridDim.x) {
        const int64_t tv = unit % tiles_v;
        const int64_t slice = unit / tiles_v;
        const int64_t v0 = tv * RW;
        const int nv = (int)min<int64_t>(RW, d.Nv - v0);
        int bc[3];
        int64_t abase, bbase;
        slice_coords(d, slice, bc, &abase, &bbase);

        // rows of this wave: r = wave, wave + 4, ... (< nv); load the first
        int r = wave;
        mf4v p[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) p[q] = mf4v{0.f, 0.f, 0.f, 0.f};
        if (r < nv) {
            const mf4v *src = reinterpret_cast<const mf4v *>(in + abase + (v0 + r) * d.a_sv);
#pragma unroll
            for (int q = 0; q < NQ; ++q) p[q] = __builtin_nontemporal_load(src + 64 * q + lane);
        }
        if (d.count) moved += tile_moved(d, slice, 1, 0, N, v0, nv);
        for (; r < nv; r += kThreads / 64) {
            float2 *xb = kCol ? stg + r : xbuf[kCol ? 0 : wave];  // x[j] at xb[j XS]
            if constexpr (kCol) {
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    const int j = 2 * (64 * q + lane);
                    xb[j * SR] = mk<float2>(p[q][0], p[q][1]);
                    xb[(j + 1) * SR] = mk<float2>(p[q][2], p[q][3]);
                }
            } else {
#pragma unroll
                for (int q = 0; q < NQ; ++q) reinterpret_cast<mf4v *>(xb)[64 * q + lane] = p[q];
            }
            const int rn = r + kThreads / 64;
            if (rn < nv) {  // the wave's next row loads while this one is transformed
                const mf4v *src = reinterpret_cast<const mf4v *>(in + abase + (v0 + rn) * d.a_sv);
#pragma unroll
                for (int q = 0; q < NQ; ++q) p[q] = __builtin_nontemporal_load(src + 64 * q + lane);
            }
            float2 z[4 * R];
            dft_row_mfma<PT, DIR, R, kCol ? SR : 1>(xb, yb, a1, a2, tw, twc, lane, z);
            // X[k] (k = 16 (4g + v) + c [+ 256]) into row r of the staging block
            // (both contractions have read the row: dft_row_mfma ends with a
            // wave barrier)
#pragma unroll
            for (int v = 0; v < 4 * R; ++v) {
                float2 e = z[v];
                if (do_scale) {
                    e.x *= scale;
                    e.y *= scale;
                }
                stg[(256 * (v >> 2) + 16 * (4 * g + (v & 3)) + c) * SR + r] = e;
            }
        }
        __syncthreads();
        // runs of consecutive v for every k, two values per 16-byte store when
        // N_v is even (every other stride of layout B is then a multiple of
        // N_v, so pairs start 16 bytes aligned); 8-byte stores otherwise
        constexpr int HP = RW / 2;
        const int npair = (nv + 1) / 2;
        const bool wide = (d.Nv & 1) == 0;
        float2 *dstb = out + bbase + v0;
        for (int idx = threadIdx.x; idx < N * HP; idx += kThreads) {
            const int rp = idx % HP;
            const int k = idx / HP;
            if (rp >= npair) continue;
            const int r0 = 2 * rp;
            float2 *q = dstb + (int64_t)k * d.b_su + r0;
            const float2 a0 = stg[k * SR + r0];
            if (r0 + 1 < nv && wide) {
                const float2 a1v = stg[k * SR + r0 + 1];
                mf4v w = {a0.x, a0.y, a1v.x, a1v.y};
                __builtin_nontemporal_store(w, reinterpret_cast<mf4v *>(q));
            } else {
                xst(q, a0);
                if (r0 + 1 < nv) xst(q + 1, stg[k * SR + r0 + 1]);
            }
        }
        __syncthreads();  // the staging block is refilled by the next unit
    }
    if (d.count) {
        for (int off = 32; off > 0; off >>= 1) moved += __shfl_xor(moved, off);
        if ((threadIdx.x & 63) == 0 && moved) atomicAdd(&moved_wg, moved);
        __syncthreads();
        if (threadIdx.x == 0 && moved_wg)
            atomicAdd(d.counter + (blockIdx.x % kCountSlots) * kCountStride, (unsigned long long)moved_wg);
    }
}

// Work-groups of the fused kernel resident on the device, queried once per
// device and row factor.
template <int R>
hipError_t mfma_resident_grid(int *resident)
{
    static std::atomic<int> resident_of[kMaxDevices];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return hipErrorInvalidDevice;
    int n = dev < kMaxDevices ? resident_of[dev].load(std::memory_order_relaxed) : 0;
    if (n == 0) {
        int ncu = 0, per_cu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fft_mfma_xpose_kernel<kPrecF16, -1, R>, kThreads,
                                                         0) != hipSuccess ||
            ncu < 1 || per_cu < 1)
            return hipErrorInvalidDeviceFunction;
        n = ncu * per_cu;
        if (dev < kMaxDevices) resident_of[dev].store(n, std::memory_order_relaxed);
    }
    *resident = n;
    return hipSuccess;
}

template <int R>
hipError_t launch_mfma_xpose_r(int precision, int dir, const void *twN, const XposeDesc &d, const void *in,
                               void *out, double scale, hipStream_t s)
{
    constexpr int RW = kMfmaRows;
    const int64_t nunits = ((d.Nv + RW - 1) / RW) * d.nslices;
    if (nunits <= 0) return hipSuccess;
    int resident = 0;
    if (hipError_t e = mfma_resident_grid<R>(&resident)) return e;
    const int ds = scale != 1.0;
    dim3 grid((unsigned)std::min<int64_t>(nunits, resident)), block(kThreads);
    const float2 *i = (const float2 *)in;
    float2 *o = (float2 *)out;
    const float2 *t = (const float2 *)twN;
    const float sc = (float)scale;
#define FFTRW_LAUNCH(P, D) \
    hipLaunchKernelGGL((fft_mfma_xpose_kernel<P, D, R>), grid, block, 0, s, i, o, d, t, sc, ds)
    if (precision == kPrecF16) {
        if (dir < 0) FFTRW_LAUNCH(kPrecF16, -1); else FFTRW_LAUNCH(kPrecF16, 1);
    } else if (precision == kPrecBF16) {
        if (dir < 0) FFTRW_LAUNCH(kPrecBF16, -1); else FFTRW_LAUNCH(kPrecBF16, 1);
    } else if (precision == kPrecBF16x3) {
        if (dir < 0) FFTRW_LAUNCH(kPrecBF16x3, -1); else FFTRW_LAUNCH(kPrecBF16x3, 1);
    } else {
        return hipErrorInvalidValue;
    }
#undef FFTRW_LAUNCH
    return hipGetLastError();
}

hipError_t launch_fft_mfma_xpose(int precision, int dir, int N, const void *twN, const XposeDesc &d, const void *in,
                                 void *out, double scale, hipStream_t s)
{
    if (N == 256) return launch_mfma_xpose_r<1>(precision, dir, twN, d, in, out, scale, s);
    if (N == 512) return launch_mfma_xpose_r<2>(precision, dir, twN, d, in, out, scale, s);
    return hipErrorInvalidValue;
}

template <int R>
hipError_t launch_mfma_r(int precision, int dir, const void *twN, int64_t nrows, const void *in, void *out,
                         double scale, hipStream_t s)
{
    // waves loop over rows; about 8 work-groups per CU of 256
    const int64_t nblk = std::min<int64_t>((nrows + 3) / 4, 2048);
    if (nblk <= 0) return hipSuccess;
    const int ds = scale != 1.0;
    dim3 grid((unsigned)nblk), block(kThreads);
    const float2 *i = (const float2 *)in;
    float2 *o = (float2 *)out;
    const float2 *t = (const float2 *)twN;
    const float sc = (float)scale;
#define FFTRW_LAUNCH(P, D) \
    hipLaunchKernelGGL((fft_mfma_kernel<P, D, R>), grid, block, 0, s, i, o, nrows, t, sc, ds)
    if (precision == kPrecF16) {
        if (dir < 0) FFTRW_LAUNCH(kPrecF16, -1); else FFTRW_LAUNCH(kPrecF16, 1);
    } else if (precision == kPrecBF16) {
        if (dir < 0) FFTRW_LAUNCH(kPrecBF16, -1); else FFTRW_LAUNCH(kPrecBF16, 1);
    } else if (precision == kPrecBF16x3) {
        if (dir < 0) FFTRW_LAUNCH(kPrecBF16x3, -1); else FFTRW_LAUNCH(kPrecBF16x3, 1);
    } else {
        return hipErrorInvalidValue;
    }
#undef FFTRW_LAUNCH
    return hipGetLastError();
}

hipError_t launch_fft_mfma(int precision, int dir, int N, const void *twN, int64_t nrows, const void *in, void *out,
                           double scale, hipStream_t s)
{
    if (N == 256) return launch_mfma_r<1>(precision, dir, twN, nrows, in, out, scale, s);
    if (N == 512) return launch_mfma_r<2>(precision, dir, twN, nrows, in, out, scale, s);
    return hipErrorInvalidValue;
}

}  // namespace fftrw
