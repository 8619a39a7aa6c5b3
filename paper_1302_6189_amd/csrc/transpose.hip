// transpose.hip -- the transpose between two decompositions (Fig. 4), fused.
//
// The array moves from layout A (decomposition pi_t) to layout B (pi_{t+1}).
// Consecutive decompositions always have different last axes, so the
// permutation is a tiled 2-D transpose between u (fastest axis of A) and v
// (fastest axis of B), batched over the other M-2 axes.  A work-group reads a
// TU x TV tile (times G batch slices) along u, transposes it through LDS and
// writes it along v, so both sides are coalesced.
//
// Owner counting: virtual process p owns a contiguous range of rows over the
// first k axes of its decomposition (Eqs. (13)-(15)).  The first k axes of A
// never include u and those of B never include v (k < M), so inside a tile
// A's owner depends only on (slice, v) and B's only on (slice, u).  Each tile
// computes the two owner vectors once, then counts the (u, v) pairs whose
// owners differ: the points this tile moves between processes.  Summed over
// tiles this is the paper's communication amount for the transpose.
#include <hip/hip_runtime.h>

#include "cplx.hpp"
#include "kernels.hpp"

namespace fftrw {

constexpr int kMaxG = 256;

__device__ __forceinline__ int64_t owner_of_row(int64_t r, int64_t P, int64_t R)
{
    return ((r + 1) * P - 1) / R;
}

template <typename C>
__global__ void __launch_bounds__(kThreads) xpose_kernel(const C *__restrict__ in, C *__restrict__ out, XposeDesc d)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *tile = reinterpret_cast<C *>(smem_raw);
    __shared__ int64_t abase[kMaxG], bbase[kMaxG];
    __shared__ int bcoord[kMaxG][3];
    __shared__ int moved_wg;

    const int TU = d.TU, TV = d.TV;
    const int ldt = TU + 1;
    int64_t t = blockIdx.x;
    const int64_t tu = t % d.tiles_u;
    t /= d.tiles_u;
    const int64_t tv = t % d.tiles_v;
    const int64_t tg = t / d.tiles_v;
    const int64_t u0 = tu * TU, v0 = tv * TV, g0 = tg * d.G;
    const int nu = (int)min<int64_t>(TU, d.Nu - u0);
    const int nv = (int)min<int64_t>(TV, d.Nv - v0);
    const int ng = (int)min<int64_t>(d.G, d.nslices - g0);

    for (int g = threadIdx.x; g < ng; g += kThreads) {
        int64_t s = g0 + g, ab = 0, bb = 0;
        for (int i = 0; i < d.nbat; ++i) {
            int64_t c = s % d.bsize[i];
            s /= d.bsize[i];
            ab += c * d.ba[i];
            bb += c * d.bb[i];
            bcoord[g][i] = (int)c;
        }
        abase[g] = ab;
        bbase[g] = bb;
    }
    if (threadIdx.x == 0) moved_wg = 0;
    __syncthreads();

    // load: rows (g, v) of TU contiguous u-values
    {
        const int tx = threadIdx.x % TU;
        const int ty = threadIdx.x / TU;
        const int ystep = kThreads / TU;
        const int nrow = ng * nv;
        for (int r = ty; r < nrow; r += ystep) {
            const int g = r / nv;
            const int iv = r - g * nv;
            if (tx < nu) tile[(g * TV + iv) * ldt + tx] = in[abase[g] + (v0 + iv) * d.a_sv + u0 + tx];
        }
    }
    __syncthreads();

    // owner vectors of this tile (counting mode)
    int *own_a = nullptr, *own_b = nullptr;
    if (d.count) {
        own_a = reinterpret_cast<int *>(tile + (size_t)d.G * TV * ldt);
        own_b = own_a + d.G * TV;
        for (int i = threadIdx.x; i < ng * nv; i += kThreads) {
            const int g = i / nv, iv = i - g * nv;
            int64_t r = 0;
            for (int j = 0; j < d.ka; ++j) {
                const int src = d.srca[j];
                const int64_t c = src == 3 ? v0 + iv : (int64_t)bcoord[g][src];
                r += c * d.wa[j];
            }
            int64_t o = owner_of_row(r, d.P, d.Ra);
            if (d.mu) o = d.mu[o];
            own_a[g * TV + iv] = (int)o;
        }
        for (int i = threadIdx.x; i < ng * nu; i += kThreads) {
            const int g = i / nu, iu = i - g * nu;
            int64_t r = 0;
            for (int j = 0; j < d.kb; ++j) {
                const int src = d.srcb[j];
                const int64_t c = src == 4 ? u0 + iu : (int64_t)bcoord[g][src];
                r += c * d.wb[j];
            }
            own_b[g * TU + iu] = (int)owner_of_row(r, d.P, d.Rb);
        }
        __syncthreads();
    }

    // store: rows (g, u) of TV contiguous v-values
    int moved = 0;
    {
        const int tx = threadIdx.x % TV;
        const int ty = threadIdx.x / TV;
        const int ystep = kThreads / TV;
        const int nrow = ng * nu;
        for (int r = ty; r < nrow; r += ystep) {
            const int g = r / nu;
            const int iu = r - g * nu;
            if (tx < nv) {
                out[bbase[g] + (u0 + iu) * d.b_su + v0 + tx] = tile[(g * TV + tx) * ldt + iu];
                if (d.count) moved += own_a[g * TV + tx] != own_b[g * TU + iu];
            }
        }
    }
    if (d.count) {
        for (int off = 32; off > 0; off >>= 1) moved += __shfl_xor(moved, off);
        if ((threadIdx.x & 63) == 0 && moved) atomicAdd(&moved_wg, moved);
        __syncthreads();
        if (threadIdx.x == 0 && moved_wg) atomicAdd(d.counter, (unsigned long long)moved_wg);
    }
}

size_t xpose_lds_bytes(const XposeDesc &d, size_t esz)
{
    size_t b = (size_t)d.G * d.TV * (d.TU + 1) * esz;
    if (d.count) b += (size_t)d.G * (d.TU + d.TV) * sizeof(int);
    return (b + 15) & ~(size_t)15;
}

hipError_t launch_xpose(const XposeDesc &d, size_t esz, const void *in, void *out, hipStream_t s)
{
    const int64_t nblk = d.tiles_u * d.tiles_v * d.tiles_g;
    if (nblk <= 0) return hipSuccess;
    const size_t lds = xpose_lds_bytes(d, esz);
    dim3 grid((unsigned)nblk), block(kThreads);
    if (esz == 8)
        hipLaunchKernelGGL(xpose_kernel<float2>, grid, block, lds, s, (const float2 *)in, (float2 *)out, d);
    else
        hipLaunchKernelGGL(xpose_kernel<double2>, grid, block, lds, s, (const double2 *)in, (double2 *)out, d);
    return hipGetLastError();
}

__global__ void zero_u64_kernel(unsigned long long *p, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

hipError_t launch_zero_u64(unsigned long long *p, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_u64_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace fftrw
