// fft_pow2.hip -- batched 1-D FFTs along contiguous rows of power-of-two length.
//
// Same computation as fft_rows.hip (Eq. (1) on every row of the current
// decomposition), specialised at compile time for N = 2^n <= 4096:
//   * every thread owns E consecutive-butterfly values (E = 16 for FP32,
//     8 for FP64), so a row is handled by N/E threads and a 256-thread
//     work-group holds 256 E / N rows;
//   * the first Stockham pass reads straight from HBM into registers and the
//     last one writes straight back (its outputs land at j + i N/R, so both
//     sides stay coalesced, 16 bytes per access when a thread owns two
//     adjacent butterflies); only the passes in between go through LDS, whose
//     index is padded by one element every 16 to spread the Stockham strides
//     over the banks;
//   * twiddles of pass p are read from a per-pass table w_{Ns R}^{i k}
//     (k < Ns, i = 1..R-1) generated in FP64 on the device.
// Streaming accesses use non-temporal hints: every value is touched once.
#include <hip/hip_runtime.h>

#include "cplx.hpp"
#include "kernels.hpp"
#include "xpose_tile.hpp"

namespace fftrw {

template <int... Rs> struct RadixList {
    static constexpr int n = sizeof...(Rs);
    static constexpr int r[n] = {Rs...};
};

__device__ __forceinline__ int lds_pad(int e) { return e + (e >> 4); }

template <typename C> struct Vec2;
template <> struct Vec2<float2> {
    typedef float type __attribute__((ext_vector_type(4)));
};
typedef float f2v __attribute__((ext_vector_type(2)));
typedef double d2v __attribute__((ext_vector_type(2)));

// one complex value with a non-temporal hint (8 or 16 bytes in one access)
template <typename C>
__device__ __forceinline__ C ld_nt(const C *p)
{
    if constexpr (sizeof(C) == 8) {
        f2v w = __builtin_nontemporal_load(reinterpret_cast<const f2v *>(p));
        return mk<C>(w.x, w.y);
    } else {
        d2v w = __builtin_nontemporal_load(reinterpret_cast<const d2v *>(p));
        return mk<C>(w.x, w.y);
    }
}
template <typename C>
__device__ __forceinline__ void st_nt(C *p, C v)
{
    if constexpr (sizeof(C) == 8) {
        f2v w = {v.x, v.y};
        __builtin_nontemporal_store(w, reinterpret_cast<f2v *>(p));
    } else {
        d2v w = {v.x, v.y};
        __builtin_nontemporal_store(w, reinterpret_cast<d2v *>(p));
    }
}

// load n consecutive complex values (n = 1, 2 or a multiple of 2 for float2)
template <int NV, typename C>
__device__ __forceinline__ void load_run(const C *p, C *dst)
{
    if constexpr (sizeof(C) == 8 && NV % 2 == 0) {
        using V = typename Vec2<float2>::type;
#pragma unroll
        for (int q = 0; q < NV / 2; ++q) {
            V w = __builtin_nontemporal_load(reinterpret_cast<const V *>(p) + q);
            dst[2 * q] = mk<C>(w.x, w.y);
            dst[2 * q + 1] = mk<C>(w.z, w.w);
        }
    } else {
#pragma unroll
        for (int q = 0; q < NV; ++q) dst[q] = ld_nt(p + q);
    }
}

template <int NV, typename C>
__device__ __forceinline__ void store_run(C *p, const C *src)
{
    if constexpr (sizeof(C) == 8 && NV % 2 == 0) {
        using V = typename Vec2<float2>::type;
#pragma unroll
        for (int q = 0; q < NV / 2; ++q) {
            V w = {src[2 * q].x, src[2 * q].y, src[2 * q + 1].x, src[2 * q + 1].y};
            __builtin_nontemporal_store(w, reinterpret_cast<V *>(p) + q);
        }
    } else {
#pragma unroll
        for (int q = 0; q < NV; ++q) st_nt(p + q, src[q]);
    }
}

// compile-time description of pass P of a radix list
template <int N, class RL, int P> struct PassInfo {
    static constexpr int R = RL::r[P];
    static constexpr int Ns = PassInfo<N, RL, P - 1>::Ns * RL::r[P - 1];
    static constexpr int NB = N / R;  // butterflies per row
    static constexpr int tw_off = PassInfo<N, RL, P - 1>::tw_off + PassInfo<N, RL, P - 1>::Ns * (RL::r[P - 1] - 1);
};
template <int N, class RL> struct PassInfo<N, RL, 0> {
    static constexpr int R = RL::r[0];
    static constexpr int Ns = 1;
    static constexpr int NB = N / R;
    static constexpr int tw_off = 0;
};

// The twiddles w^{i k} of the thread's butterflies in pass P (k = j mod Ns
// for butterfly j = lane B + b), read from the pass's table.  They depend on
// the lane only, so run_passes loads each pass's twiddles one pass ahead,
// before the exchange that precedes it; they arrive while the exchange runs.
template <int N, int E, class RL, int P, typename C> struct PassTwiddles {
    static constexpr int R = PassInfo<N, RL, P>::R;
    static constexpr int B = E / R;
    C t[PassInfo<N, RL, P>::Ns > 1 ? B : 1][R - 1];
};

template <int N, int E, class RL, int P, typename C>
__device__ __forceinline__ void load_twiddles(PassTwiddles<N, E, RL, P, C> &w, int lane, const C *tw)
{
    using PI = PassInfo<N, RL, P>;
    constexpr int R = PI::R, B = E / R;
    if constexpr (PI::Ns > 1) {
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int j = lane * B + b;
            const int k = j % PI::Ns;
            const C *t = tw + PI::tw_off + k * (R - 1);
#pragma unroll
            for (int i = 1; i < R; ++i) w.t[b][i - 1] = t[i - 1];
        }
    }
}

// twiddle v[b R + i] *= w^{i k} for the thread's butterflies of pass P
template <int N, int E, int DIR, class RL, int P, typename C>
__device__ __forceinline__ void apply_twiddles(C *v, const PassTwiddles<N, E, RL, P, C> &w)
{
    using PI = PassInfo<N, RL, P>;
    constexpr int R = PI::R, B = E / R;
    if constexpr (PI::Ns > 1) {
#pragma unroll
        for (int b = 0; b < B; ++b)
#pragma unroll
            for (int i = 1; i < R; ++i) v[b * R + i] = twmul<DIR>(v[b * R + i], w.t[b][i - 1]);
    }
}

template <int E, int DIR, class RL, int P, typename C>
__device__ __forceinline__ void butterflies(C *v)
{
    constexpr int R = RL::r[P], B = E / R;
#pragma unroll
    for (int b = 0; b < B; ++b) Dft<R, DIR, C>::run(v + b * R);
}

// write pass P's outputs to LDS (Stockham positions), read pass P+1's inputs
template <int N, int E, class RL, int P, typename C>
__device__ __forceinline__ void exchange(C *v, C *row, int lane)
{
    using A = PassInfo<N, RL, P>;
    using B2 = PassInfo<N, RL, P + 1>;
    constexpr int RA = A::R, BA = E / RA;
#pragma unroll
    for (int b = 0; b < BA; ++b) {
        const int j = lane * BA + b;
        const int k = j % A::Ns;
        const int base = (j - k) * RA + k;
#pragma unroll
        for (int i = 0; i < RA; ++i) row[lds_pad(base + i * A::Ns)] = v[b * RA + i];
    }
    __syncthreads();
    constexpr int RB = B2::R, BB = E / RB;
#pragma unroll
    for (int b = 0; b < BB; ++b) {
        const int j = lane * BB + b;
#pragma unroll
        for (int i = 0; i < RB; ++i) v[b * RB + i] = row[lds_pad(j + i * B2::NB)];
    }
    __syncthreads();
}

// passes P.. of the thread's E values; w holds pass P's twiddles (loaded by
// the caller), pass P + 1's are loaded before the exchange between the two
template <int N, int E, int DIR, class RL, int P, typename C>
__device__ __forceinline__ void run_passes(C *v, C *row, int lane, const C *tw,
                                           const PassTwiddles<N, E, RL, P, C> &w)
{
    apply_twiddles<N, E, DIR, RL, P>(v, w);
    butterflies<E, DIR, RL, P>(v);
    if constexpr (P + 1 < RL::n) {
        PassTwiddles<N, E, RL, P + 1, C> wn;
        load_twiddles<N, E, RL, P + 1>(wn, lane, tw);
        exchange<N, E, RL, P>(v, row, lane);
        run_passes<N, E, DIR, RL, P + 1>(v, row, lane, tw, wn);
    }
}

// all passes, from the first (whose twiddles are all 1: Ns = 1)
template <int N, int E, int DIR, class RL, typename C>
__device__ __forceinline__ void run_passes(C *v, C *row, int lane, const C *tw)
{
    PassTwiddles<N, E, RL, 0, C> w0;
    load_twiddles<N, E, RL, 0>(w0, lane, tw);
    run_passes<N, E, DIR, RL, 0>(v, row, lane, tw, w0);
}

template <typename C, int N, int E, int DIR, class RL>
__global__ void __launch_bounds__(kThreads)
    fft_pow2_kernel(const C *in, C *out, int64_t nrows, const C *__restrict__ tw,
                    typename RealOf<C>::type scale, int do_scale)
{
    constexpr int L = N / E;        // threads per row
    constexpr int RW = kThreads / L;  // rows per work-group
    constexpr int NP = RL::n;
    __shared__ C lds[NP > 1 ? RW * (N + N / 16) : 1];
    const int lane = threadIdx.x % L;
    const int lrow = threadIdx.x / L;
    const int64_t grow = (int64_t)blockIdx.x * RW + lrow;
    const bool active = grow < nrows;
    const C *src = in + grow * N;
    C *dst = out + grow * N;
    C v[E];

    {   // first pass inputs straight from HBM
        using PI = PassInfo<N, RL, 0>;
        constexpr int R = PI::R, B = E / R;
        if (active) {
#pragma unroll
            for (int i = 0; i < R; ++i) {
                C t[B];
                load_run<B>(src + lane * B + i * PI::NB, t);
#pragma unroll
                for (int b = 0; b < B; ++b) v[b * R + i] = t[b];
            }
        } else {
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = mk<C>(0, 0);
        }
    }
    run_passes<N, E, DIR, RL>(v, lds + lrow * (N + N / 16), lane, tw);
    {   // last pass outputs straight to HBM at j + i N/R
        using PI = PassInfo<N, RL, NP - 1>;
        constexpr int R = PI::R, B = E / R;
        if (do_scale) {
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = cscale(v[e], scale);
        }
        if (active) {
#pragma unroll
            for (int i = 0; i < R; ++i) {
                C t[B];
#pragma unroll
                for (int b = 0; b < B; ++b) t[b] = v[b * R + i];
                store_run<B>(dst + lane * B + i * PI::NB, t);
            }
        }
    }
}

// ---- FFT step fused with the transpose that follows it -------------------------
// A work-group transforms RW rows along u (the last axis of layout A) that are
// consecutive in v (the last axis of layout B) within one batch slice, then
// writes the results in layout B: the last pass lands in an LDS staging block
// S[k][r] and each k becomes one run of RW consecutive v-values in HBM.  Owner
// counting as in the transpose (row_keep).

// threads per work-group of the fused kernel: 512 when a 256-thread group
// would hold fewer than 16 rows (runs of 16 values = 128 bytes)
template <int N, int E> struct FusedThreads {
    static constexpr int value = (kThreads / (N / E) < 16 && 512 / (N / E) <= 64) ? 512 : kThreads;
};

template <typename C, int N, int E, int DIR, class RL>
__global__ void __launch_bounds__((FusedThreads<N, E>::value))
    fft_xpose_kernel(const C *in, C *out, XposeDesc d, const C *__restrict__ tw, typename RealOf<C>::type scale,
                     int do_scale)
{
    constexpr int NT = FusedThreads<N, E>::value;
    constexpr int L = N / E;
    constexpr int RW = NT / L;
    constexpr int NP = RL::n;
    constexpr int SROW = RW + 1;
    constexpr int LDS_FFT = NP > 1 ? RW * (N + N / 16) : 1;
    constexpr int LDS_STG = N * SROW;
    __shared__ C lds[LDS_FFT > LDS_STG ? LDS_FFT : LDS_STG];
    __shared__ int moved_wg;

    // block coordinates in 32 bits (sizes are at most 4096, a launch has
    // fewer than 2^31 groups): they come before the first row load
    const uint32_t tiles_v = ((uint32_t)d.Nv + RW - 1) / RW;
    const uint32_t tv = blockIdx.x % tiles_v;
    const uint32_t slice = blockIdx.x / tiles_v;
    const int64_t v0 = (int64_t)tv * RW;
    const int nv = (int)min<int64_t>(RW, d.Nv - v0);
    int bc[3] = {0, 0, 0};
    int64_t abase = 0, bbase = 0;
    slice_coords(d, slice, bc, &abase, &bbase);
    const int lane = threadIdx.x % L;
    const int r = threadIdx.x / L;
    const bool active = r < nv;
    const C *src = in + abase + (v0 + r) * d.a_sv;
    C v[E];
    {
        using PI = PassInfo<N, RL, 0>;
        constexpr int R = PI::R, B = E / R;
        if (active) {
#pragma unroll
            for (int i = 0; i < R; ++i) {
                C t[B];
                load_run<B>(src + lane * B + i * PI::NB, t);
#pragma unroll
                for (int b = 0; b < B; ++b) v[b * R + i] = t[b];
            }
        } else {
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = mk<C>(0, 0);
        }
    }
    // (computed while the row loads are in flight) owner changes of this
    // group's rows: thread r counts row v0 + r.  With rows < nv <= 64 wave 0
    // holds every term and publishes the sum at once: work left for the end
    // of the kernel delays the group's exit and costs more than it does here
    int moved = 0;
    if (d.count) {
        if (threadIdx.x == 0) moved_wg = 0;
        if (threadIdx.x < nv) moved = (int)(N - row_keep(d, bc, v0 + threadIdx.x, 0, N));
        if constexpr (RW <= 64) {
            if (threadIdx.x < 64) {
                for (int off = 32; off > 0; off >>= 1) moved += __shfl_xor(moved, off);
                if (threadIdx.x == 0 && moved)
                    atomicAdd(d.counter + (blockIdx.x % kCountSlots) * kCountStride, (unsigned long long)moved);
            }
        }
    }

    run_passes<N, E, DIR, RL>(v, lds + r * (N + N / 16), lane, tw);
    {   // last pass outputs (row r, k = j + i N/R) into the staging block
        using PI = PassInfo<N, RL, NP - 1>;
        constexpr int R = PI::R, B = E / R;
#pragma unroll
        for (int i = 0; i < R; ++i)
#pragma unroll
            for (int b = 0; b < B; ++b) {
                C q = v[b * R + i];
                if (do_scale) q = cscale(q, scale);
                lds[(lane * B + b + i * PI::NB) * SROW + r] = q;
            }
    }
    __syncthreads();
    // runs of consecutive v for every k, two values per 16-byte store when
    // N_v is even: every stride of layout B other than v's is then a multiple
    // of N_v, so each pair starts 16 bytes aligned (odd N_v: 8-byte stores)
    constexpr int HP = RW / 2;
    const int npair = (nv + 1) / 2;
    const bool wide = (d.Nv & 1) == 0;
    C *dstb = out + bbase + v0;
    if constexpr (sizeof(C) == 8 && N * HP % NT == 0) {
        if (nv == RW && wide) {
            // a full tile in 16-byte pairs, with no branch per run: every LDS
            // read of the thread is issued before the first store waits
            using V4 = typename Vec2<float2>::type;
            constexpr int IT = N * HP / NT;
            V4 w[IT];
#pragma unroll
            for (int it = 0; it < IT; ++it) {
                const int idx = threadIdx.x + it * NT;
                const int r0 = 2 * (idx % HP), k = idx / HP;
                const C a0 = lds[k * SROW + r0], a1 = lds[k * SROW + r0 + 1];
                w[it] = V4{a0.x, a0.y, a1.x, a1.y};
            }
#pragma unroll
            for (int it = 0; it < IT; ++it) {
                const int idx = threadIdx.x + it * NT;
                const int r0 = 2 * (idx % HP), k = idx / HP;
                __builtin_nontemporal_store(w[it], reinterpret_cast<V4 *>(dstb + (int64_t)k * d.b_su + r0));
            }
            goto stored;
        }
    }
    for (int idx = threadIdx.x; idx < N * HP; idx += NT) {
        const int rp = idx % HP;
        const int k = idx / HP;
        if (rp >= npair) continue;
        const int r0 = 2 * rp;
        C *p = dstb + (int64_t)k * d.b_su + r0;
        const C a0 = lds[k * SROW + r0];
        if (r0 + 1 < nv) {
            const C a1 = lds[k * SROW + r0 + 1];
            if constexpr (sizeof(C) == 8) {
                if (wide) {
                    using V4 = typename Vec2<float2>::type;
                    V4 w = {a0.x, a0.y, a1.x, a1.y};
                    __builtin_nontemporal_store(w, reinterpret_cast<V4 *>(p));
                } else {
                    st_nt(p, a0);
                    st_nt(p + 1, a1);
                }
            } else {
                st_nt(p, a0);
                st_nt(p + 1, a1);
            }
        } else {
            st_nt(p, a0);
        }
    }
stored:
    if constexpr (RW > 64) {
        if (d.count) {
            for (int off = 32; off > 0; off >>= 1) moved += __shfl_xor(moved, off);
            if ((threadIdx.x & 63) == 0 && moved) atomicAdd(&moved_wg, moved);
            __syncthreads();
            if (threadIdx.x == 0 && moved_wg)
                atomicAdd(d.counter + (blockIdx.x % kCountSlots) * kCountStride, (unsigned long long)moved_wg);
        }
    }
}

// radix lists per N (every radix divides E so each thread owns whole butterflies)
template <int N> struct Pow2Plan;
template <> struct Pow2Plan<2> { using RL = RadixList<2>; };
template <> struct Pow2Plan<4> { using RL = RadixList<4>; };
template <> struct Pow2Plan<8> { using RL = RadixList<8>; };
template <> struct Pow2Plan<16> { using RL = RadixList<16>; };
template <> struct Pow2Plan<32> { using RL = RadixList<4, 8>; };
template <> struct Pow2Plan<64> { using RL = RadixList<8, 8>; };
template <> struct Pow2Plan<128> { using RL = RadixList<2, 8, 8>; };
template <> struct Pow2Plan<256> { using RL = RadixList<4, 8, 8>; };
template <> struct Pow2Plan<512> { using RL = RadixList<8, 8, 8>; };
template <> struct Pow2Plan<1024> { using RL = RadixList<2, 8, 8, 8>; };
template <> struct Pow2Plan<2048> { using RL = RadixList<4, 8, 8, 8>; };
template <> struct Pow2Plan<4096> { using RL = RadixList<8, 8, 8, 8>; };

// FP64 rows: 8 values per thread, so radices <= 8
template <int N> struct Pow2Plan64 { using RL = typename Pow2Plan<N>::RL; };
template <> struct Pow2Plan64<16> { using RL = RadixList<2, 8>; };

template <int N, class RL> struct TwSize {
    static constexpr int value = PassInfo<N, RL, RL::n - 1>::tw_off + PassInfo<N, RL, RL::n - 1>::Ns * (RL::r[RL::n - 1] - 1);
};

struct RadixArg {
    int r[kMaxPasses];
    int n;
};

// per-pass twiddle table, FP64 arithmetic: entry (pass p, k, i) = w_{Ns R}^{i k}
template <typename C>
__global__ void pow2_twiddle_kernel(C *out, RadixArg ra)
{
    const int *radix = ra.r;
    const int npass = ra.n;
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    int off = 0, Ns = 1;
    for (int p = 0; p < npass; ++p) {
        const int R = radix[p];
        const int cnt = Ns * (R - 1);
        if (idx >= off && idx < off + cnt) {
            const int rel = idx - off;
            const int k = rel / (R - 1), i = rel % (R - 1) + 1;
            const long e = (long)i * k, n = (long)Ns * R;
            double s, c;
            sincospi(-2.0 * (double)(e % n) / (double)n, &s, &c);
            out[idx] = mk<C>((typename RealOf<C>::type)c, (typename RealOf<C>::type)s);
        }
        off += cnt;
        Ns *= R;
    }
}

namespace {

template <typename C, int N, int E, class RL>
hipError_t launch_one(bool make_tw, void *tw, int64_t nrows, int dir, const void *in, void *out, double scale,
                      hipStream_t s, int *tw_count, int *radices, int *npass, const XposeDesc *fx = nullptr)
{
    if (tw_count) *tw_count = TwSize<N, RL>::value;
    if (npass) {
        *npass = RL::n;
        for (int p = 0; p < RL::n; ++p) radices[p] = RL::r[p];
    }
    if (make_tw) {
        const int cnt = TwSize<N, RL>::value;
        if (cnt == 0) return hipSuccess;
        RadixArg ra{};
        for (int p = 0; p < RL::n; ++p) ra.r[p] = RL::r[p];
        ra.n = RL::n;
        hipLaunchKernelGGL(pow2_twiddle_kernel<C>, dim3((cnt + 255) / 256), dim3(256), 0, s, (C *)tw, ra);
        return hipGetLastError();
    }
    if (!in) return hipSuccess;
    constexpr int L = N / E, RW = kThreads / L;
    if (fx) {
        using Real = typename RealOf<C>::type;
        constexpr int NTF = FusedThreads<N, E>::value, RWF = NTF / L;
        const int64_t nblk = ((fx->Nv + RWF - 1) / RWF) * fx->nslices;
        if (nblk <= 0) return hipSuccess;
        const int ds = scale != 1.0;
        if (dir < 0)
            hipLaunchKernelGGL((fft_xpose_kernel<C, N, E, -1, RL>), dim3((unsigned)nblk), dim3(NTF), 0, s,
                               (const C *)in, (C *)out, *fx, (const C *)tw, (Real)scale, ds);
        else
            hipLaunchKernelGGL((fft_xpose_kernel<C, N, E, 1, RL>), dim3((unsigned)nblk), dim3(NTF), 0, s,
                               (const C *)in, (C *)out, *fx, (const C *)tw, (Real)scale, ds);
        return hipGetLastError();
    }
    const int64_t nblk = (nrows + RW - 1) / RW;
    if (nblk <= 0) return hipSuccess;
    using Real = typename RealOf<C>::type;
    const int do_scale = scale != 1.0;
    if (dir < 0)
        hipLaunchKernelGGL((fft_pow2_kernel<C, N, E, -1, RL>), dim3((unsigned)nblk), dim3(kThreads), 0, s,
                           (const C *)in, (C *)out, nrows, (const C *)tw, (Real)scale, do_scale);
    else
        hipLaunchKernelGGL((fft_pow2_kernel<C, N, E, 1, RL>), dim3((unsigned)nblk), dim3(kThreads), 0, s,
                           (const C *)in, (C *)out, nrows, (const C *)tw, (Real)scale, do_scale);
    return hipGetLastError();
}

template <typename C, int N>
hipError_t dispatch_n(bool make_tw, void *tw, int64_t nrows, int dir, const void *in, void *out, double scale,
                      hipStream_t s, int *tw_count, int *radices, int *npass, const XposeDesc *fx)
{
    if constexpr (sizeof(C) == 8) {
        constexpr int E = N < 16 ? N : 16;
        return launch_one<C, N, E, typename Pow2Plan<N>::RL>(make_tw, tw, nrows, dir, in, out, scale, s, tw_count,
                                                             radices, npass, fx);
    } else if constexpr (N <= 2048) {
        constexpr int E = N < 8 ? N : 8;
        return launch_one<C, N, E, typename Pow2Plan64<N>::RL>(make_tw, tw, nrows, dir, in, out, scale, s,
                                                                tw_count, radices, npass, fx);
    } else {
        return hipErrorInvalidValue;
    }
}

template <typename C>
hipError_t dispatch(int N, bool make_tw, void *tw, int64_t nrows, int dir, const void *in, void *out,
                    double scale, hipStream_t s, int *tw_count, int *radices, int *npass,
                    const XposeDesc *fx = nullptr)
{
#define FFTRW_CASE(n) \
    case n: return dispatch_n<C, n>(make_tw, tw, nrows, dir, in, out, scale, s, tw_count, radices, npass, fx);
    switch (N) {
        FFTRW_CASE(2) FFTRW_CASE(4) FFTRW_CASE(8) FFTRW_CASE(16) FFTRW_CASE(32) FFTRW_CASE(64)
        FFTRW_CASE(128) FFTRW_CASE(256) FFTRW_CASE(512) FFTRW_CASE(1024) FFTRW_CASE(2048) FFTRW_CASE(4096)
    default: return hipErrorInvalidValue;
    }
#undef FFTRW_CASE
}

}  // namespace

bool pow2_supported(int N, bool fp64)
{
    return N >= 2 && N <= (fp64 ? 2048 : 4096) && (N & (N - 1)) == 0;
}

// Describe the kernel for N: number of twiddle entries and the radix list.
void pow2_describe(int N, bool fp64, int *tw_count, int *radices, int *npass)
{
    if (fp64)
        (void)dispatch<double2>(N, false, nullptr, 0, -1, nullptr, nullptr, 1.0, nullptr, tw_count, radices, npass);
    else
        (void)dispatch<float2>(N, false, nullptr, 0, -1, nullptr, nullptr, 1.0, nullptr, tw_count, radices, npass);
}

hipError_t pow2_make_twiddles(int N, bool fp64, void *tw, hipStream_t s)
{
    return fp64 ? dispatch<double2>(N, true, tw, 0, -1, nullptr, nullptr, 1.0, s, nullptr, nullptr, nullptr)
                : dispatch<float2>(N, true, tw, 0, -1, nullptr, nullptr, 1.0, s, nullptr, nullptr, nullptr);
}

// rows per work-group of the fused kernel for N (its run length along v)
int pow2_rows_per_wg(int N, bool fp64)
{
    const int E = fp64 ? (N < 8 ? N : 8) : (N < 16 ? N : 16);
    const int L = N / E;
    const int nt = (kThreads / L < 16 && 512 / L <= 64) ? 512 : kThreads;
    return nt / L;
}

hipError_t launch_fft_xpose_pow2(int N, bool fp64, const void *tw, const XposeDesc &fx, int dir, const void *in,
                                 void *out, double scale, hipStream_t s)
{
    return fp64 ? dispatch<double2>(N, false, (void *)tw, 0, dir, in, out, scale, s, nullptr, nullptr, nullptr, &fx)
                : dispatch<float2>(N, false, (void *)tw, 0, dir, in, out, scale, s, nullptr, nullptr, nullptr, &fx);
}

hipError_t launch_fft_pow2(int N, bool fp64, const void *tw, int64_t nrows, int dir, const void *in, void *out,
                           double scale, hipStream_t s)
{
    return fp64 ? dispatch<double2>(N, false, (void *)tw, nrows, dir, in, out, scale, s, nullptr, nullptr, nullptr)
                : dispatch<float2>(N, false, (void *)tw, nrows, dir, in, out, scale, s, nullptr, nullptr, nullptr);
}

}  // namespace fftrw
