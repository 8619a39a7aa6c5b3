// cplx.hpp -- complex arithmetic and small DFT butterflies for the FFT passes.
//
// Every butterfly computes y_k = sum_j w^{jk} x_j for a short length R, the
// 1-D DFT of Eq. (1), with w = exp(DIR * 2 pi i / R): DIR = -1 is the paper's
// forward transform, DIR = +1 the (unscaled) inverse.  The formulas are the
// usual splittings of that sum into even/odd or symmetric parts.
#pragma once

#include <hip/hip_runtime.h>

namespace fftrw {

template <typename Real> struct CplxOf;
template <> struct CplxOf<float> { using type = float2; };
template <> struct CplxOf<double> { using type = double2; };

template <typename C> struct RealOf;
template <> struct RealOf<float2> { using type = float; };
template <> struct RealOf<double2> { using type = double; };

// Pointers that a kernel reads out of a descriptor in memory are generic
// (flat) pointers to the compiler, and flat accesses count on the LDS wait
// counter as well: a wait for one LDS read then also waits for every flat
// load and store still in flight, which serialises a thread's HBM accesses.
// Passing such a pointer through the global address space lets the compiler
// issue global_ loads and stores, whose waits are separate from the LDS's.
template <typename T> __device__ __forceinline__ T *as_global(T *p)
{
    return (T *)(__attribute__((address_space(1))) T *)p;
}

// HBM accesses through the global address space.  A pointer a kernel reads
// out of a descriptor in memory is a generic (flat) pointer to the compiler,
// and flat accesses count on the LDS wait counter too: a wait for one LDS
// read then also waits for every flat load and store still in flight, which
// serialises a thread's HBM accesses.  Global loads and stores have waits of
// their own.  Only for pointers into device memory (never LDS).
template <typename T> __device__ __forceinline__ T gld_nt(const T *p)
{
    return __builtin_nontemporal_load((const __attribute__((address_space(1))) T *)p);
}
template <typename T> __device__ __forceinline__ void gst_nt(T v, T *p)
{
    __builtin_nontemporal_store(v, (__attribute__((address_space(1))) T *)p);
}
// one complex value (float2 or double2), cached
template <typename T> __device__ __forceinline__ T gld(const T *p)
{
    if constexpr (sizeof(T) == 8) {
        typedef float v2 __attribute__((ext_vector_type(2)));
        const v2 w = *(const __attribute__((address_space(1))) v2 *)p;
        T r;
        r.x = w.x;
        r.y = w.y;
        return r;
    } else {
        typedef double v2 __attribute__((ext_vector_type(2)));
        const v2 w = *(const __attribute__((address_space(1))) v2 *)p;
        T r;
        r.x = w.x;
        r.y = w.y;
        return r;
    }
}

template <typename C> __device__ __forceinline__ C mk(typename RealOf<C>::type x, typename RealOf<C>::type y)
{
    C r;
    r.x = x;
    r.y = y;
    return r;
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return mk<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return mk<C>(a.x - b.x, a.y - b.y); }
template <typename C> __device__ __forceinline__ C cmul(C a, C b)
{
    return mk<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename C> __device__ __forceinline__ C cmulc(C a, C b)
{
    return mk<C>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename C> __device__ __forceinline__ C cscale(C a, typename RealOf<C>::type s)
{
    return mk<C>(a.x * s, a.y * s);
}
// a * (DIR * i)
template <int DIR, typename C> __device__ __forceinline__ C rot90(C a)
{
    return DIR < 0 ? mk<C>(a.y, -a.x) : mk<C>(-a.y, a.x);
}
// twiddle product: a * w (forward) or a * conj(w) (inverse); w from a forward table
template <int DIR, typename C> __device__ __forceinline__ C twmul(C a, C w)
{
    return DIR < 0 ? cmul(a, w) : cmulc(a, w);
}

template <int R, int DIR, typename C> struct Dft;

template <int DIR, typename C> struct Dft<2, DIR, C> {
    static __device__ __forceinline__ void run(C *x)
    {
        C a = x[0], b = x[1];
        x[0] = cadd(a, b);
        x[1] = csub(a, b);
    }
};

template <int DIR, typename C> struct Dft<4, DIR, C> {
    static __device__ __forceinline__ void run(C *x)
    {
        C a = cadd(x[0], x[2]), b = csub(x[0], x[2]);
        C c = cadd(x[1], x[3]), d = rot90<DIR>(csub(x[1], x[3]));
        x[0] = cadd(a, c);
        x[2] = csub(a, c);
        x[1] = cadd(b, d);
        x[3] = csub(b, d);
    }
};

template <int DIR, typename C> struct Dft<8, DIR, C> {
    static __device__ __forceinline__ void run(C *x)
    {
        using Real = typename RealOf<C>::type;
        const Real h = (Real)0.70710678118654752440084436210485;
        C e[4] = {x[0], x[2], x[4], x[6]};
        C o[4] = {x[1], x[3], x[5], x[7]};
        Dft<4, DIR, C>::run(e);
        Dft<4, DIR, C>::run(o);
        // w8^k = (cos(pi k/4), DIR sin(pi k/4))
        C o1 = mk<C>(h * (o[1].x - DIR * o[1].y), h * (o[1].y + DIR * o[1].x));
        C o2 = rot90<DIR>(o[2]);
        C o3 = mk<C>(h * (-o[3].x - DIR * o[3].y), h * (-o[3].y + DIR * o[3].x));
        x[0] = cadd(e[0], o[0]);
        x[4] = csub(e[0], o[0]);
        x[1] = cadd(e[1], o1);
        x[5] = csub(e[1], o1);
        x[2] = cadd(e[2], o2);
        x[6] = csub(e[2], o2);
        x[3] = cadd(e[3], o3);
        x[7] = csub(e[3], o3);
    }
};

template <int DIR, typename C> struct Dft<16, DIR, C> {
    static __device__ __forceinline__ void run(C *x)
    {
        using Real = typename RealOf<C>::type;
        // cos(pi k / 8), sin(pi k / 8), k = 0..7
        const Real cs[8] = {(Real)1.0,
                            (Real)0.92387953251128675612818318939679,
                            (Real)0.70710678118654752440084436210485,
                            (Real)0.38268343236508977172845998403040,
                            (Real)0.0,
                            (Real)-0.38268343236508977172845998403040,
                            (Real)-0.70710678118654752440084436210485,
                            (Real)-0.92387953251128675612818318939679};
        const Real sn[8] = {(Real)0.0,
                            (Real)0.38268343236508977172845998403040,
                            (Real)0.70710678118654752440084436210485,
                            (Real)0.92387953251128675612818318939679,
                            (Real)1.0,
                            (Real)0.92387953251128675612818318939679,
                            (Real)0.70710678118654752440084436210485,
                            (Real)0.38268343236508977172845998403040};
        C e[8], o[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            e[j] = x[2 * j];
            o[j] = x[2 * j + 1];
        }
        Dft<8, DIR, C>::run(e);
        Dft<8, DIR, C>::run(o);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            C w = mk<C>(cs[k], DIR * sn[k]);
            C t = cmul(o[k], w);
            x[k] = cadd(e[k], t);
            x[k + 8] = csub(e[k], t);
        }
    }
};

template <int DIR, typename C> struct Dft<3, DIR, C> {
    static __device__ __forceinline__ void run(C *x)
    {
        using Real = typename RealOf<C>::type;
        const Real s3 = (Real)0.86602540378443864676372317075294;
        C t = cadd(x[1], x[2]);
        C m = mk<C>(x[0].x - (Real)0.5 * t.x, x[0].y - (Real)0.5 * t.y);
        C s = rot90<DIR>(cscale(csub(x[1], x[2]), s3));
        x[0] = cadd(x[0], t);
        x[1] = cadd(m, s);
        x[2] = csub(m, s);
    }
};

template <int DIR, typename C> struct Dft<5, DIR, C> {
    static __device__ __forceinline__ void run(C *x)
    {
        using Real = typename RealOf<C>::type;
        const Real c1 = (Real)0.30901699437494742410229341718282;   // cos(2 pi/5)
        const Real c2 = (Real)-0.80901699437494742410229341718282;  // cos(4 pi/5)
        const Real s1 = (Real)0.95105651629515357211643933337938;   // sin(2 pi/5)
        const Real s2 = (Real)0.58778525229247312916870595463907;   // sin(4 pi/5)
        C a1 = cadd(x[1], x[4]), a2 = cadd(x[2], x[3]);
        C b1 = csub(x[1], x[4]), b2 = csub(x[2], x[3]);
        C y0 = cadd(x[0], cadd(a1, a2));
        C m1 = mk<C>(x[0].x + c1 * a1.x + c2 * a2.x, x[0].y + c1 * a1.y + c2 * a2.y);
        C m2 = mk<C>(x[0].x + c2 * a1.x + c1 * a2.x, x[0].y + c2 * a1.y + c1 * a2.y);
        C n1 = rot90<DIR>(mk<C>(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y));
        C n2 = rot90<DIR>(mk<C>(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y));
        x[0] = y0;
        x[1] = cadd(m1, n1);
        x[4] = csub(m1, n1);
        x[2] = cadd(m2, n2);
        x[3] = csub(m2, n2);
    }
};

}  // namespace fftrw
