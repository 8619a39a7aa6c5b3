// fft_rows.hip -- stand-alone launch of the generic row FFT (fft_generic.hpp)
// for 2,3,5-smooth lengths, the FP64 twiddle table w_N^e it reads, and the
// fused unit's shape rule exported for tests (fft_fused_unit_shape).
#include <hip/hip_runtime.h>

#include "../../include/fftrw.h"
#include "errors.hpp"
#include "fft_generic.hpp"
#include "fused_generic.hpp"

namespace fftrw {

// ---- twiddle table: w_N^e = exp(-2 pi i e / N), computed in FP64 -------------
template <typename C>
__global__ void __launch_bounds__(kThreads) twiddle_kernel(C *out, int64_t n)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    double s, c;
    // sin/cos of pi * (-2 e / n); the argument is reduced exactly first
    sincospi(-2.0 * (double)e / (double)n, &s, &c);
    out[e] = mk<C>((typename RealOf<C>::type)c, (typename RealOf<C>::type)s);
}

hipError_t launch_twiddles(void *out, int64_t n, bool fp64, hipStream_t s)
{
    dim3 grid((unsigned)((n + kThreads - 1) / kThreads));
    if (fp64)
        hipLaunchKernelGGL(twiddle_kernel<double2>, grid, dim3(kThreads), 0, s, (double2 *)out, n);
    else
        hipLaunchKernelGGL(twiddle_kernel<float2>, grid, dim3(kThreads), 0, s, (float2 *)out, n);
    return hipGetLastError();
}

template <typename C, int DIR, bool TW_LDS, bool LEAN>
__global__ void __launch_bounds__(kThreads)
    fft_rows_kernel(const C *in, C *out, FftDesc d, typename RealOf<C>::type scale, int do_scale)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    fft_rows_block<C, DIR, TW_LDS, LEAN>(in, out, d, blockIdx.x, scale, do_scale != 0, reinterpret_cast<C *>(smem_raw));
}

// Radix lists without 8 and 16 (lengths with at most two factors 2, or the
// lists the autotuner picks that way) run the kernels compiled for radices 2
// to 5 only: the same passes with fewer registers (complex64 118-119 VGPRs
// instead of 131-135, four waves per SIMD instead of three).
bool lean_radices(const FftDesc &d)
{
    for (int q = 0; q < d.npass; ++q)
        if (d.radix[q] == 8 || d.radix[q] == 16) return false;
    return true;
}

hipError_t launch_fft_rows(const FftDesc &d, bool fp64, int dir, const void *in, void *out, double scale,
                           hipStream_t s)
{
    const int64_t nblk = (d.nrows + d.rows_per_wg - 1) / d.rows_per_wg;
    if (nblk <= 0) return hipSuccess;
    const size_t esz = fp64 ? 16 : 8;
    // the twiddle table goes to LDS after the rows when it takes at most 16 KB
    const bool tw = unit_tw_fits(d.N, esz);
    const size_t lds = ((size_t)d.rows_per_wg * d.N + (tw ? d.N : 0)) * esz;
    const int do_scale = scale != 1.0;
    dim3 grid((unsigned)nblk), block(kThreads);
    const bool lean = lean_radices(d);
#define FFTRW_LAUNCH(C, D, T, SC)                                                                                  \
    do {                                                                                                         \
        if (lean)                                                                                                \
            hipLaunchKernelGGL((fft_rows_kernel<C, D, T, true>), grid, block, lds, s, (const C *)in, (C *)out, d, SC, \
                               do_scale);                                                                        \
        else                                                                                                     \
            hipLaunchKernelGGL((fft_rows_kernel<C, D, T, false>), grid, block, lds, s, (const C *)in, (C *)out, d, SC, \
                               do_scale);                                                                        \
    } while (0)
    if (fp64) {
        if (dir < 0) {
            if (tw) FFTRW_LAUNCH(double2, -1, true, scale); else FFTRW_LAUNCH(double2, -1, false, scale);
        } else {
            if (tw) FFTRW_LAUNCH(double2, 1, true, scale); else FFTRW_LAUNCH(double2, 1, false, scale);
        }
    } else {
        if (dir < 0) {
            if (tw) FFTRW_LAUNCH(float2, -1, true, (float)scale); else FFTRW_LAUNCH(float2, -1, false, (float)scale);
        } else {
            if (tw) FFTRW_LAUNCH(float2, 1, true, (float)scale); else FFTRW_LAUNCH(float2, 1, false, (float)scale);
        }
    }
#undef FFTRW_LAUNCH
    return hipGetLastError();
}

template <typename C, int DIR, bool TW_LDS, bool LEAN>
__global__ void __launch_bounds__(kThreads)
    fft_xpose_generic_kernel(const C *in, C *out, FftDesc f, XposeDesc d, int rw, int G,
                             typename RealOf<C>::type scale, int do_scale)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    fft_xpose_unit<C, DIR, TW_LDS, LEAN>(in, out, f, d, rw, G, blockIdx.x, scale, do_scale != 0, smem_raw);
}

// one FFT step of 2,3,5-smooth rows fused with the transpose that follows
hipError_t launch_fft_xpose_generic(const FftDesc &f, const XposeDesc &d, bool fp64, int dir, const void *in,
                                    void *out, double scale, hipStream_t s)
{
    const size_t esz = fp64 ? 16 : 8;
    int rw = 1, G = 1;
    fused_unit_shape(f.N, esz, d.Nv, d.nslices, fp64 ? 2048 : 4096, &rw, &G);
    const int64_t nblk = ((d.Nv + rw - 1) / rw) * ((d.nslices + G - 1) / G);
    if (nblk <= 0) return hipSuccess;
    if (nblk >= (int64_t)0x7fffffff) return hipErrorInvalidValue;
    const bool tw = unit_tw_fits(f.N, esz);
    const size_t lds = fused_unit_bytes(f.N, rw, G, esz, tw);
    const int do_scale = scale != 1.0;
    dim3 grid((unsigned)nblk), block(kThreads);
    const bool lean = lean_radices(f);
#define FFTRW_LAUNCH(C, D, T, SC)                                                                             \
    do {                                                                                                    \
        if (lean)                                                                                           \
            hipLaunchKernelGGL((fft_xpose_generic_kernel<C, D, T, true>), grid, block, lds, s, (const C *)in, \
                               (C *)out, f, d, rw, G, SC, do_scale);                                        \
        else                                                                                                \
            hipLaunchKernelGGL((fft_xpose_generic_kernel<C, D, T, false>), grid, block, lds, s, (const C *)in, \
                               (C *)out, f, d, rw, G, SC, do_scale);                                        \
    } while (0)
    if (fp64) {
        if (dir < 0) {
            if (tw) FFTRW_LAUNCH(double2, -1, true, scale); else FFTRW_LAUNCH(double2, -1, false, scale);
        } else {
            if (tw) FFTRW_LAUNCH(double2, 1, true, scale); else FFTRW_LAUNCH(double2, 1, false, scale);
        }
    } else {
        if (dir < 0) {
            if (tw) FFTRW_LAUNCH(float2, -1, true, (float)scale); else FFTRW_LAUNCH(float2, -1, false, (float)scale);
        } else {
            if (tw) FFTRW_LAUNCH(float2, 1, true, (float)scale); else FFTRW_LAUNCH(float2, 1, false, (float)scale);
        }
    }
#undef FFTRW_LAUNCH
    return hipGetLastError();
}

}  // namespace fftrw

extern "C" int fft_fused_unit_shape(int N, int esz, int64_t Nv, int64_t nslices, int *rw, int *G)
{
    fftrw::g_last_error.clear();
    if (N < 2 || Nv < 1 || nslices < 1 || (esz != 8 && esz != 16) || !rw || !G)
        return fftrw::fail(FFTRW_E_ARG, "fft_fused_unit_shape: N >= 2, Nv >= 1, nslices >= 1, esz 8 or 16, "
                                        "non-null outputs");
    fftrw::fused_unit_shape(N, (size_t)esz, Nv, nslices, esz == 16 ? 2048 : 4096, rw, G);
    return FFTRW_OK;
}
