// transpose.hip -- stand-alone launch of the fused transpose (xpose_tile.hpp).
#include <hip/hip_runtime.h>

#include "xpose_tile.hpp"

namespace fftrw {

template <typename C, int VU, int VV>
__global__ void __launch_bounds__(kThreads) xpose_kernel(const C *__restrict__ in, C *__restrict__ out, XposeDesc d)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    xpose_tile<C, VU, VV>(in, out, d, blockIdx.x, smem_raw);
}

size_t xpose_lds_bytes(const XposeDesc &d, size_t esz) { return xpose_tile_bytes(d, esz) + 16; }

hipError_t launch_xpose(const XposeDesc &d, size_t esz, const void *in, void *out, hipStream_t s)
{
    const int64_t nblk = d.tiles_u * d.tiles_v * d.tiles_g;
    if (nblk <= 0) return hipSuccess;
    const size_t lds = xpose_lds_bytes(d, esz);
    dim3 grid((unsigned)nblk), block(kThreads);
    // 16-byte accesses for complex64 along an even fast axis
    const bool vu = esz == 8 && d.Nu % 2 == 0 && d.TU >= 2;
    const bool vv = esz == 8 && d.Nv % 2 == 0 && d.TV >= 2;
    if (esz == 8) {
        const float2 *i = (const float2 *)in;
        float2 *o = (float2 *)out;
        if (vu && vv)
            hipLaunchKernelGGL((xpose_kernel<float2, 2, 2>), grid, block, lds, s, i, o, d);
        else if (vu)
            hipLaunchKernelGGL((xpose_kernel<float2, 2, 1>), grid, block, lds, s, i, o, d);
        else if (vv)
            hipLaunchKernelGGL((xpose_kernel<float2, 1, 2>), grid, block, lds, s, i, o, d);
        else
            hipLaunchKernelGGL((xpose_kernel<float2, 1, 1>), grid, block, lds, s, i, o, d);
    } else {
        hipLaunchKernelGGL((xpose_kernel<double2, 1, 1>), grid, block, lds, s, (const double2 *)in,
                           (double2 *)out, d);
    }
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
