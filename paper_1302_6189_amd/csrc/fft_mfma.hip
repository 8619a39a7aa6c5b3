// fft_mfma.hip -- 256-point row FFTs as radix-16 DFT contractions on MFMA.
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
// in FP64; F16 itself is generated in FP64 on the device.
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

template <int PREC, int DIR>
__global__ void __launch_bounds__(kThreads)
    fft256_mfma_kernel(const float2 *in, float2 *out, int64_t nrows, const float2 *__restrict__ tw256, float scale,
                       int do_scale)
{
    using PT = Parts<PREC>;
    using V = typename PT::V;
    __shared__ __align__(16) float2 xbuf[kThreads / 64][256];     // row in / row out
    __shared__ float2 ybuf[kThreads / 64][16 * 17];                // stage-1 result, padded

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4;   // lane group 0..3
    const int c = lane & 15;   // column (A: row) index
    float2 *xb = xbuf[wave];
    float2 *yb = ybuf[wave];
    const bool im = g >= 2;
    const int n1base = 8 * (g & 1);

    // A operands [Fr | -Fi] and [Fi | Fr], lane holds row c, k = 8g + v (FP64 once per wave)
    V a1[PT::n], a2[PT::n];
    {
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
    // twiddles w_256^{n2 k1} of this lane (n2 = c, k1 = 4g + v)
    float2 tw[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) tw[v] = tw256[c * (4 * g + v)];

    const int64_t wstride = (int64_t)gridDim.x * (kThreads / 64);
    int64_t row = (int64_t)blockIdx.x * (kThreads / 64) + wave;
    mf4v p0 = {0.f, 0.f, 0.f, 0.f}, p1 = p0;
    if (row < nrows) {
        const mf4v *src = reinterpret_cast<const mf4v *>(in + row * 256);
        p0 = __builtin_nontemporal_load(src + lane);
        p1 = __builtin_nontemporal_load(src + 64 + lane);
    }
    for (; row < nrows; row += wstride) {
        reinterpret_cast<mf4v *>(xb)[lane] = p0;
        reinterpret_cast<mf4v *>(xb)[64 + lane] = p1;
        const int64_t nxt = row + wstride;
        if (nxt < nrows) {  // prefetch the next row while this one is transformed
            const mf4v *src = reinterpret_cast<const mf4v *>(in + nxt * 256);
            p0 = __builtin_nontemporal_load(src + lane);
            p1 = __builtin_nontemporal_load(src + 64 + lane);
        }
        wave_sync();

        // ---- stage 1: B[k][c] = x[16 n1 + c], k = 8g + v ------------------------
        float b[8];
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const float2 e = xb[16 * (n1base + v) + c];
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
        // Z[k2][k1] (k2 = 4g + v, k1 = c) lands at y[16 k2 + k1]: stage in xb
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            float re = ldexpf(cr[v], -s2), imv = ldexpf(ci[v], -s2);
            if (do_scale) {
                re *= scale;
                imv *= scale;
            }
            xb[16 * (4 * g + v) + c] = mk<float2>(re, imv);
        }
        wave_sync();
        mf4v* dst = reinterpret_cast<mf4v *>(out + row * 256);
        __builtin_nontemporal_store(reinterpret_cast<mf4v *>(xb)[lane], dst + lane);
        __builtin_nontemporal_store(reinterpret_cast<mf4v *>(xb)[64 + lane], dst + 64 + lane);
        wave_sync();  // xb is rewritten by the next row
    }
}

// The same 256-point transform fused with the transpose that follows: a unit
// is 16 rows consecutive in v (the next layout's last axis) of one batch slice;
// each wave transforms 4 of them, the results meet in an LDS block S[k][row]
// and every frequency k leaves as one run of 16 consecutive v (128 bytes) in
// the next layout.  A resident grid walks the units, so the split F16
// operands (FP64 sin/cos) are built once per work-group.  Owner changes are
// counted per row (tile_moved).
constexpr int kMfmaRows = 16;
constexpr int kMaxDevices = 64;  // devices whose resident grid size is cached

template <int PREC, int DIR>
__global__ void __launch_bounds__(kThreads)
    fft256_mfma_xpose_kernel(const float2 *in, float2 *out, XposeDesc d, const float2 *__restrict__ tw256,
                             float scale, int do_scale)
{
    using PT = Parts<PREC>;
    using V = typename PT::V;
    constexpr int SR = kMfmaRows + 1;
    __shared__ __align__(16) float2 xbuf[kThreads / 64][256];
    __shared__ float2 ybuf[kThreads / 64][16 * 17];
    __shared__ float2 stg[256 * SR];
    __shared__ int moved_wg;

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4;
    const int c = lane & 15;
    float2 *xb = xbuf[wave];
    float2 *yb = ybuf[wave];
    const bool im = g >= 2;
    const int n1base = 8 * (g & 1);

    // the F16 operands and twiddles are set up once; the resident grid then
    // walks the units (groups of 16 rows) u = blockIdx.x, + gridDim.x, ...
    V a1[PT::n], a2[PT::n];
    {
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
    float2 tw[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) tw[v] = tw256[c * (4 * g + v)];
    if (threadIdx.x == 0) moved_wg = 0;
    int moved = 0;

    const int64_t tiles_v = (d.Nv + kMfmaRows - 1) / kMfmaRows;
    const int64_t nunits = tiles_v * d.nslices;
    for (int64_t unit = blockIdx.x; unit < nunits; unit += gridDim.x) {
        const int64_t tv = unit % tiles_v;
        const int64_t slice = unit / tiles_v;
        const int64_t v0 = tv * kMfmaRows;
        const int nv = (int)min<int64_t>(kMfmaRows, d.Nv - v0);
        int bc[3];
        int64_t abase, bbase;
        slice_coords(d, slice, bc, &abase, &bbase);

        // rows of this wave: r = wave, wave + 4, ... (< nv); load the first
        int r = wave;
        mf4v p0 = {0.f, 0.f, 0.f, 0.f}, p1 = p0;
        if (r < nv) {
            const mf4v *src = reinterpret_cast<const mf4v *>(in + abase + (v0 + r) * d.a_sv);
            p0 = __builtin_nontemporal_load(src + lane);
            p1 = __builtin_nontemporal_load(src + 64 + lane);
        }
        if (d.count) moved += tile_moved(d, slice, 1, 0, 256, v0, nv);
        for (; r < nv; r += kThreads / 64) {
            reinterpret_cast<mf4v *>(xb)[lane] = p0;
            reinterpret_cast<mf4v *>(xb)[64 + lane] = p1;
            const int rn = r + kThreads / 64;
            if (rn < nv) {  // the wave's next row loads while this one is transformed
                const mf4v *src = reinterpret_cast<const mf4v *>(in + abase + (v0 + rn) * d.a_sv);
                p0 = __builtin_nontemporal_load(src + lane);
                p1 = __builtin_nontemporal_load(src + 64 + lane);
            }
            wave_sync();
            float b[8];
#pragma unroll
            for (int v = 0; v < 8; ++v) {
                const float2 e = xb[16 * (n1base + v) + c];
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
                yb[(4 * g + v) * 17 + c] =
                    DIR < 0 ? cmul(mk<float2>(re, imv), tw[v]) : cmulc(mk<float2>(re, imv), tw[v]);
            }
            wave_sync();
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
            // xbar[16 k2 + k1] = Z[k2][k1] (k2 = 4g + v, k1 = c) into row r of the staging block
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                float re = ldexpf(cr[v], -s2), imv = ldexpf(ci[v], -s2);
                if (do_scale) {
                    re *= scale;
                    imv *= scale;
                }
                stg[(16 * (4 * g + v) + c) * SR + r] = mk<float2>(re, imv);
            }
            wave_sync();  // xb and yb are rewritten by the wave's next row
        }
        __syncthreads();
        // runs of consecutive v for every k, two values per 16-byte store when
        // N_v is even (every other stride of layout B is then a multiple of
        // N_v, so pairs start 16 bytes aligned); 8-byte stores otherwise
        constexpr int HP = kMfmaRows / 2;
        const int npair = (nv + 1) / 2;
        const bool wide = (d.Nv & 1) == 0;
        float2 *dstb = out + bbase + v0;
        for (int idx = threadIdx.x; idx < 256 * HP; idx += kThreads) {
            const int rp = idx % HP;
            const int k = idx / HP;
            if (rp >= npair) continue;
            const int r0 = 2 * rp;
            float2 *p = dstb + (int64_t)k * d.b_su + r0;
            const float2 a0 = stg[k * SR + r0];
            if (r0 + 1 < nv && wide) {
                const float2 a1v = stg[k * SR + r0 + 1];
                mf4v w = {a0.x, a0.y, a1v.x, a1v.y};
                __builtin_nontemporal_store(w, reinterpret_cast<mf4v *>(p));
            } else {
                xst(p, a0);
                if (r0 + 1 < nv) xst(p + 1, stg[k * SR + r0 + 1]);
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

hipError_t launch_fft256_mfma_xpose(int precision, int dir, const void *tw256, const XposeDesc &d, const void *in,
                                    void *out, double scale, hipStream_t s)
{
    const int64_t nunits = ((d.Nv + kMfmaRows - 1) / kMfmaRows) * d.nslices;
    if (nunits <= 0) return hipSuccess;
    // a resident grid (work-groups walk the units), sized once per device
    static std::atomic<int> resident_of[kMaxDevices];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return hipErrorInvalidDevice;
    int resident = dev < kMaxDevices ? resident_of[dev].load(std::memory_order_relaxed) : 0;
    if (resident == 0) {
        int ncu = 0, per_cu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fft256_mfma_xpose_kernel<kPrecF16, -1>, kThreads,
                                                         0) != hipSuccess ||
            ncu < 1 || per_cu < 1)
            return hipErrorInvalidDeviceFunction;
        resident = ncu * per_cu;
        if (dev < kMaxDevices) resident_of[dev].store(resident, std::memory_order_relaxed);
    }
    const int ds = scale != 1.0;
    dim3 grid((unsigned)std::min<int64_t>(nunits, resident)), block(kThreads);
    const float2 *i = (const float2 *)in;
    float2 *o = (float2 *)out;
    const float2 *t = (const float2 *)tw256;
    const float sc = (float)scale;
#define FFTRW_LAUNCH(P, D) \
    hipLaunchKernelGGL((fft256_mfma_xpose_kernel<P, D>), grid, block, 0, s, i, o, d, t, sc, ds)
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

hipError_t launch_fft256_mfma(int precision, int dir, const void *tw256, int64_t nrows, const void *in, void *out,
                              double scale, hipStream_t s)
{
    // waves loop over rows; about 8 work-groups per CU of 256
    const int64_t nblk = std::min<int64_t>((nrows + 3) / 4, 2048);
    if (nblk <= 0) return hipSuccess;
    const int ds = scale != 1.0;
    dim3 grid((unsigned)nblk), block(kThreads);
    const float2 *i = (const float2 *)in;
    float2 *o = (float2 *)out;
    const float2 *t = (const float2 *)tw256;
    const float sc = (float)scale;
#define FFTRW_LAUNCH(P, D) \
    hipLaunchKernelGGL((fft256_mfma_kernel<P, D>), grid, block, 0, s, i, o, nrows, t, sc, ds)
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

}  // namespace fftrw
