// fft_generic.hpp -- batched 1-D FFTs along contiguous rows of any 2,3,5-smooth
// length (device code shared by the stand-alone kernel and the persistent
// batched kernel).
//
// Every step of the paper's parallel M-D FFT runs independent 1-D FFTs (Eq. (1))
// along the last axis of the current decomposition; after the preceding
// transpose those rows are contiguous.  A work-group stages RW whole rows
// (RW * N <= 4096 complex values for FP32, 2048 for FP64) in LDS with 16-byte
// coalesced loads, runs the Stockham autosort passes there (one radix-R
// butterfly per thread per R outputs, values staged in registers between two
// barriers so one LDS buffer suffices), and stores the rows back coalesced.
#pragma once

#include <hip/hip_runtime.h>

#include "cplx.hpp"
#include "kernels.hpp"

namespace fftrw {

// ---- one Stockham pass in LDS ----------------------------------------------------
// Pass with radix R after sub-transforms of size Ns: butterfly j (< N/R) reads
// x[j + i N/R], multiplies by w_{Ns R}^{i k} (k = j mod Ns), runs DFT_R and
// writes y[(j - k) R + k + i Ns].
// Synchronisation between a pass's reads and writes: the row's own lanes only
// when they all sit in one wave (wave = true), else the whole work-group.
__device__ __forceinline__ void row_sync(bool wave)
{
    if (wave) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

template <int R, int DIR, typename C>
__device__ __forceinline__ void stockham_pass(C *row, int N, int Ns, int lanes, int lane, const C *tw, bool wave)
{
    constexpr int MAXB = (16 + R - 1) / R;  // N / lanes <= 16 by construction
    const int nbf = N / R;
    const int twstep = N / (Ns * R);
    // j mod Ns by a multiply: with mg = ceil(2^32 / Ns), floor(j mg / 2^32) =
    // floor(j / Ns) exactly for j, Ns <= 4096 (the rounding error of mg adds
    // less than j / 2^32 < 1 / Ns to j / Ns)
    const uint32_t mg = (uint32_t)(0xffffffffu / (uint32_t)Ns) + 1u;
    C v[MAXB][R];
    int kk[MAXB];
#pragma unroll
    for (int m = 0; m < MAXB; ++m) {
        const int j = lane + m * lanes;
        if (j < nbf) {
            const int k = Ns == 1 ? 0 : j - (int)__umulhi((uint32_t)j, mg) * Ns;
            kk[m] = k;
#pragma unroll
            for (int i = 0; i < R; ++i) v[m][i] = row[j + i * nbf];
            if (Ns > 1) {
#pragma unroll
                for (int i = 1; i < R; ++i) v[m][i] = twmul<DIR>(v[m][i], tw[i * k * twstep]);
            }
            Dft<R, DIR, C>::run(v[m]);
        }
    }
    row_sync(wave);
#pragma unroll
    for (int m = 0; m < MAXB; ++m) {
        const int j = lane + m * lanes;
        if (j < nbf) {
            const int k = kk[m];
            const int base = (j - k) * R + k;
#pragma unroll
            for (int i = 0; i < R; ++i) row[base + i * Ns] = v[m][i];
        }
    }
    row_sync(wave);
}

// Copies cnt values into LDS; each thread issues up to kLoadBatch loads before
// storing any of them, so its share of the block is in flight at once.
constexpr int kLoadBatch = 8;

template <typename T>
__device__ __forceinline__ void load_batched(T *lds, const T *__restrict__ src, int n)
{
    for (int e0 = threadIdx.x; e0 < n; e0 += kThreads * kLoadBatch) {
        T t[kLoadBatch];
#pragma unroll
        for (int j = 0; j < kLoadBatch; ++j) {
            const int e = e0 + j * kThreads;
            if (e < n) t[j] = src[e];
        }
#pragma unroll
        for (int j = 0; j < kLoadBatch; ++j) {
            const int e = e0 + j * kThreads;
            if (e < n) lds[e] = t[j];
        }
    }
}

template <typename C>
__device__ __forceinline__ void load_block(C *lds, const C *__restrict__ src, int cnt)
{
    // native vector types keep the batch in registers
    typedef float f2v __attribute__((ext_vector_type(2)));
    typedef float f4v __attribute__((ext_vector_type(4)));
    typedef double d2v __attribute__((ext_vector_type(2)));
    if constexpr (sizeof(C) == 8) {
        // two complex floats per 16-byte access when the block is even-sized
        if ((cnt & 1) == 0 && (((uintptr_t)src) & 15) == 0) {
            load_batched(reinterpret_cast<f4v *>(lds), reinterpret_cast<const f4v *>(src), cnt >> 1);
            return;
        }
        load_batched(reinterpret_cast<f2v *>(lds), reinterpret_cast<const f2v *>(src), cnt);
    } else {
        load_batched(reinterpret_cast<d2v *>(lds), reinterpret_cast<const d2v *>(src), cnt);
    }
}

template <typename C>
__device__ __forceinline__ void store_block(C *__restrict__ dst, const C *lds, int cnt,
                                            typename RealOf<C>::type scale, bool do_scale)
{
    if constexpr (sizeof(C) == 8) {
        if ((cnt & 1) == 0 && (((uintptr_t)dst) & 15) == 0) {
            float4 *d4 = reinterpret_cast<float4 *>(dst);
            const float4 *l4 = reinterpret_cast<const float4 *>(lds);
            for (int e = threadIdx.x; e < (cnt >> 1); e += kThreads) {
                float4 q = l4[e];
                if (do_scale) {
                    q.x *= scale;
                    q.y *= scale;
                    q.z *= scale;
                    q.w *= scale;
                }
                d4[e] = q;
            }
            return;
        }
    }
    for (int e = threadIdx.x; e < cnt; e += kThreads) {
        C q = lds[e];
        if (do_scale) q = cscale(q, scale);
        dst[e] = q;
    }
}

// One work-group's share of a batched row FFT: rows [blk * RW, blk * RW + RW).
// TW_LDS: the N-entry twiddle table is staged in LDS after the rows (the
// caller sized the block for it), so the passes read it there.  LEAN: the
// radices are 2, 3, 4 and 5 only (the caller checked), so the passes of 8 and
// 16 are not compiled in and the kernel holds fewer registers.
template <typename C, int DIR, bool TW_LDS = false, bool LEAN = false>
__device__ __forceinline__ void fft_rows_block(const C *in, C *out, const FftDesc &d, int64_t blk,
                                               typename RealOf<C>::type scale, bool do_scale, C *lds)
{
    const int N = d.N;
    const int64_t row0 = blk * d.rows_per_wg;
    const int64_t left = d.nrows - row0;
    const int rows_here = left < d.rows_per_wg ? (int)left : d.rows_per_wg;
    const int cnt = rows_here * N;
    load_block(lds, in + row0 * N, cnt);
    C *ltw = lds + (int64_t)d.rows_per_wg * N;
    if constexpr (TW_LDS) {
        const C *gtw = reinterpret_cast<const C *>(d.tw);
        for (int i = threadIdx.x; i < N; i += kThreads) ltw[i] = gtw[i];
    }
    __syncthreads();
    const int lanes = d.lanes_per_row;
    const int row = threadIdx.x / lanes;
    const int lane = threadIdx.x - row * lanes;
    C *lrow = lds + row * N;
    const C *tw = TW_LDS ? static_cast<const C *>(ltw) : reinterpret_cast<const C *>(d.tw);
    // a row's lanes are consecutive threads, a power of two of them: at most
    // 64 sit in one wave, and the passes then synchronise that wave only (the
    // stores read across rows and wait for the whole group)
    const bool wave = lanes <= 64;
    int Ns = 1;
    for (int p = 0; p < d.npass; ++p) {
        switch (d.radix[p]) {
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
        Ns *= d.radix[p];
    }
    if (wave) __syncthreads();
    store_block(out + row0 * N, lds, cnt, scale, do_scale);
    __syncthreads();  // the LDS block may be reused by the caller's next unit
}

}  // namespace fftrw
