// rowsplit.hip -- the 1-D FFT of rows split over processes (level M of
// Eq. (13)), executed as a binary exchange between the processes that share
// each row.
//
// At level M (N_p > T / N, N the row length along the step's FFT axis) the
// processes' ranges of Eqs. (14)-(15) cut the rows.  The paper does not say
// how such a row is transformed.  The reading implemented here: when every
// range holds b = T / N_p points and each row is c = N / b whole ranges with c
// a power of two, the c processes of a row run the first s = log2 c stages of
// a radix-2 decimation-in-frequency FFT across processes.  In stage st the
// half-span is h = N / 2^(st+1) (a multiple of b), block i pairs with block
// i XOR (h / b), and every process sends its whole block to its partner: N
// points per row and stage, N log2 c per row in all, the count
// fft_rowsplit_volume reports.  The block that holds the lower half keeps
// x[j] + x[j + h], the other (x[j] - x[j + h]) w_{2h}^{j mod h}.  After the s
// stages each block is an independent b-point DFT (the plan's ordinary row
// kernels on rows of length b), and block i position m holds frequency
// bitrev_s(i) + c m of the row; a last permutation puts the row in natural
// order.  That permutation is what a distributed code would fold into the
// transpose that follows, so it is not part of the exchanged amount.
//
// Here the blocks' messages go through an explicit receive array, copied and
// counted on the device like the staged transposes' exchange.
#include <hip/hip_runtime.h>

#include "cplx.hpp"
#include "kernels.hpp"
#include "xpose_tile.hpp"

namespace fftrw {

// Stage st, the exchange: every block is copied into its partner's slot of
// the receive array (recv[x + (i' - i) b] = data[x] for x in block i of its
// row, i' = i XOR hb); each thread counts its copies.
template <typename C>
__global__ void __launch_bounds__(kThreads)
    bx_exchange_kernel(const C *__restrict__ data, C *__restrict__ recv, int64_t T, int N, int b, int hb,
                       unsigned long long *counter)
{
    __shared__ int copied_wg;
    if (threadIdx.x == 0) copied_wg = 0;
    __syncthreads();
    int copied = 0;
    for (int64_t x = (int64_t)blockIdx.x * kThreads + threadIdx.x; x < T; x += (int64_t)gridDim.x * kThreads) {
        const int pos = (int)(x % N);
        const int i = pos / b;
        const int ip = i ^ hb;
        xst(recv + x + (int64_t)(ip - i) * b, xld(data + x));
        ++copied;
    }
    for (int off = 32; off > 0; off >>= 1) copied += __shfl_xor(copied, off);
    if ((threadIdx.x & 63) == 0 && copied) atomicAdd(&copied_wg, copied);
    __syncthreads();
    if (threadIdx.x == 0 && copied_wg)
        atomicAdd(counter + (blockIdx.x % kCountSlots) * kCountStride, (unsigned long long)copied_wg);
}

// Stage st, the butterflies: each block combines its own values with the
// partner's (now in recv at the same positions).  tw: w_N^e, e < N.
template <typename C, int DIR>
__global__ void __launch_bounds__(kThreads)
    bx_butterfly_kernel(C *__restrict__ data, const C *__restrict__ recv, int64_t T, int N, int h,
                        const C *__restrict__ tw)
{
    const int step = N / (2 * h);  // w_{2h}^j = w_N^{j N / (2h)}
    for (int64_t x = (int64_t)blockIdx.x * kThreads + threadIdx.x; x < T; x += (int64_t)gridDim.x * kThreads) {
        const int pos = (int)(x % N);
        const C own = data[x], other = recv[x];
        if (((pos / h) & 1) == 0) {
            data[x] = cadd(own, other);
        } else {
            const C w = tw[(pos % h) * step];
            data[x] = twmul<DIR>(csub(other, own), w);
        }
    }
}

// Natural order: block i position m of each row holds frequency
// bitrev_s(i) + c m.  scale: 1/T on the inverse's last step.
template <typename C>
__global__ void __launch_bounds__(kThreads)
    bx_unscramble_kernel(const C *__restrict__ in, C *__restrict__ out, int64_t T, int N, int b, int s,
                         typename RealOf<C>::type scale, int do_scale)
{
    const int c = N / b;
    for (int64_t x = (int64_t)blockIdx.x * kThreads + threadIdx.x; x < T; x += (int64_t)gridDim.x * kThreads) {
        const int64_t row0 = x - x % N;
        const int pos = (int)(x - row0);
        const int i = pos / b, m = pos - i * b;
        const int f = s ? (int)(__brev((unsigned)i) >> (32 - s)) : 0;
        C v = in[x];
        if (do_scale) v = cscale(v, scale);
        out[row0 + f + (int64_t)c * m] = v;
    }
}

namespace {

unsigned grid_for(int64_t T)
{
    const int64_t g = (T + kThreads - 1) / kThreads;
    return (unsigned)(g < 65536 ? (g < 1 ? 1 : g) : 65536);
}

}  // namespace

hipError_t launch_bx_exchange(bool fp64, const void *data, void *recv, int64_t T, int N, int b, int hb,
                              unsigned long long *counter, hipStream_t s)
{
    if (fp64)
        hipLaunchKernelGGL(bx_exchange_kernel<double2>, dim3(grid_for(T)), dim3(kThreads), 0, s,
                           (const double2 *)data, (double2 *)recv, T, N, b, hb, counter);
    else
        hipLaunchKernelGGL(bx_exchange_kernel<float2>, dim3(grid_for(T)), dim3(kThreads), 0, s,
                           (const float2 *)data, (float2 *)recv, T, N, b, hb, counter);
    return hipGetLastError();
}

hipError_t launch_bx_butterfly(bool fp64, int dir, void *data, const void *recv, int64_t T, int N, int h,
                               const void *tw, hipStream_t s)
{
#define FFTRW_BX(C, D)                                                                                        \
    hipLaunchKernelGGL((bx_butterfly_kernel<C, D>), dim3(grid_for(T)), dim3(kThreads), 0, s, (C *)data,     \
                       (const C *)recv, T, N, h, (const C *)tw)
    if (fp64) {
        if (dir < 0) FFTRW_BX(double2, -1); else FFTRW_BX(double2, 1);
    } else {
        if (dir < 0) FFTRW_BX(float2, -1); else FFTRW_BX(float2, 1);
    }
#undef FFTRW_BX
    return hipGetLastError();
}

hipError_t launch_bx_unscramble(bool fp64, const void *in, void *out, int64_t T, int N, int b, int sbits,
                                double scale, hipStream_t s)
{
    const int ds = scale != 1.0;
    if (fp64)
        hipLaunchKernelGGL(bx_unscramble_kernel<double2>, dim3(grid_for(T)), dim3(kThreads), 0, s,
                           (const double2 *)in, (double2 *)out, T, N, b, sbits, scale, ds);
    else
        hipLaunchKernelGGL(bx_unscramble_kernel<float2>, dim3(grid_for(T)), dim3(kThreads), 0, s,
                           (const float2 *)in, (float2 *)out, T, N, b, sbits, (float)scale, ds);
    return hipGetLastError();
}

}  // namespace fftrw
