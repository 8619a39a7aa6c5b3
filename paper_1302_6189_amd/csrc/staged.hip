// staged.hip -- the transpose as pack -> exchange -> unpack (Fig. 4, Section 3).
//
// This is the all-to-all the paper's processes perform, with every virtual
// process's buffers held explicitly on the device:
//   pack:     process p copies the points of its range in decomposition A into
//             its send buffer, one segment per destination q (ascending q);
//   exchange: every segment with q != p is copied into q's receive buffer
//             (segments ordered by source p) -- exactly the points that change
//             owner, i.e. the paper's communication amount, counted on the
//             device;
//   unpack:   process q places its received segments, and the segment it kept
//             for itself (read straight from its send buffer), into its range
//             of decomposition B.
// A (p, q) segment is the intersection of p's range in A with q's range in B:
// a union of axis-aligned boxes (each range is at most 2k-1 boxes).  Inside a
// segment the boxes follow p's range order and the points of a box run in A's
// axis order; sender and receiver both derive that convention from the plan,
// so nothing but point values is exchanged.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/fftrw.h"
#include "errors.hpp"
#include "kernels.hpp"
#include "plan.hpp"

namespace fftrw {

struct BoxCopy {
    int lo[kMaxDims];
    int ext[kMaxDims];
    int64_t send_off;  // first point in the global send array
    int64_t recv_off;  // first point in the global receive array
    int self;          // p == q: unpack reads the send array
    int pad;
};

struct SegCopy {
    int64_t xoff;      // position in the concatenation of exchanged segments
    int64_t src, dst;  // send / receive array offsets
    int64_t len;
};

struct StagedArgs {
    int M;
    int ord_a[kMaxDims];     // natural axes of A from slowest to fastest
    int64_t stride_a[kMaxDims], stride_b[kMaxDims];
    const BoxCopy *boxes;    // sorted by send_off (pack) or by recv_off (unpack)
    int64_t nbox;
    int64_t total;           // points covered (T, or the exchanged count)
    const SegCopy *segs;
    int64_t nseg;
    unsigned long long *counter;
};

constexpr int kChunk = 4096;  // points per work-group

template <class Key>
__device__ __forceinline__ int64_t upper_index(Key key, int64_t lo, int64_t hi, int64_t x)
{
    // largest i in [lo, hi] with key(i) <= x
    while (lo < hi) {
        int64_t mid = (lo + hi + 1) >> 1;
        if (key(mid) <= x)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

template <typename C, bool UNPACK>
__global__ void __launch_bounds__(kThreads)
    box_copy_kernel(const C *__restrict__ src, const C *__restrict__ send, C *__restrict__ dst, StagedArgs a)
{
    __shared__ int64_t first_box, last_box;
    const int64_t s0 = (int64_t)blockIdx.x * kChunk;
    const int64_t s1 = min<int64_t>(s0 + kChunk, a.total) - 1;
    auto key = [&](int64_t i) { return UNPACK ? a.boxes[i].recv_off : a.boxes[i].send_off; };
    if (threadIdx.x == 0) first_box = upper_index(key, 0, a.nbox - 1, s0);
    if (threadIdx.x == 1) last_box = upper_index(key, 0, a.nbox - 1, s1);
    __syncthreads();
    const int64_t b_lo = first_box, b_hi = last_box;
    for (int64_t s = s0 + threadIdx.x; s <= s1; s += kThreads) {
        const int64_t bi = upper_index(key, b_lo, b_hi, s);
        const BoxCopy &B = a.boxes[bi];
        int64_t e = s - key(bi);
        // coordinates inside the box, A's fastest axis first
        int64_t addr_a = 0, addr_b = 0;
        for (int i = a.M - 1; i >= 0; --i) {
            const int ax = a.ord_a[i];
            const int64_t c = e % B.ext[ax];
            e /= B.ext[ax];
            const int64_t g = B.lo[ax] + c;
            addr_a += g * a.stride_a[ax];
            addr_b += g * a.stride_b[ax];
        }
        if (!UNPACK) {
            dst[s] = src[addr_a];  // layout A -> send array
        } else {
            const C v = B.self ? send[B.send_off + (s - B.recv_off)] : src[s];
            dst[addr_b] = v;       // receive (or kept) array -> layout B
        }
    }
}

template <typename C>
__global__ void __launch_bounds__(kThreads)
    exchange_kernel(const C *__restrict__ send, C *__restrict__ recv, StagedArgs a)
{
    __shared__ int64_t first_seg, last_seg;
    const int64_t x0 = (int64_t)blockIdx.x * kChunk;
    const int64_t x1 = min<int64_t>(x0 + kChunk, a.total) - 1;
    auto key = [&](int64_t i) { return a.segs[i].xoff; };
    if (threadIdx.x == 0) first_seg = upper_index(key, 0, a.nseg - 1, x0);
    if (threadIdx.x == 1) last_seg = upper_index(key, 0, a.nseg - 1, x1);
    __syncthreads();
    int copied = 0;
    for (int64_t x = x0 + threadIdx.x; x <= x1; x += kThreads) {
        const int64_t si = upper_index(key, first_seg, last_seg, x);
        const SegCopy &S = a.segs[si];
        const int64_t o = x - S.xoff;
        recv[S.dst + o] = send[S.src + o];
        ++copied;
    }
    for (int off = 32; off > 0; off >>= 1) copied += __shfl_xor(copied, off);
    if ((threadIdx.x & 63) == 0 && copied) atomicAdd(a.counter, (unsigned long long)copied);
}

namespace {

struct HostBox {
    int64_t p, q;
    int64_t seq;  // order of the box inside p's range
    Box box;
    int64_t n;
};

int copy_to_device(fft_plan_impl *pl, const void *h, size_t bytes, void **d)
{
    if (bytes == 0) bytes = 16;
    if (hipMalloc(d, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(FFTRW_E_NOMEM, "hipMalloc for staged tables failed");
    }
    pl->dev_bytes += bytes;
    if (h && hipMemcpy(*d, h, bytes, hipMemcpyHostToDevice) != hipSuccess)
        return fail(FFTRW_E_DEVICE, "copy of staged tables failed");
    return FFTRW_OK;
}

}  // namespace

int staged_build(fft_plan_impl *pl, int t)
{
    if (pl->ownership != FFTRW_OWN_LITERAL)
        return fail(FFTRW_E_UNSUPPORTED, "staged transposes use the literal ownership reading");
    const Layout &a = pl->lay[t];
    const Layout &b = pl->lay[t + 1];
    const int M = pl->M;
    if (!pl->send) {
        for (void **buf : {&pl->send, &pl->recv}) {
            if (hipMalloc(buf, (size_t)pl->T * pl->esz) != hipSuccess) {
                (void)hipGetLastError();
                return fail(FFTRW_E_NOMEM, "hipMalloc of staging buffers failed");
            }
            pl->dev_bytes += (size_t)pl->T * pl->esz;
        }
    }
    // every (p, q) box, in p's range order
    std::vector<HostBox> hb;
    for (int64_t p = 0; p < a.P; ++p) {
        int64_t seq = 0;
        for (const Box &B : range_boxes(a, p)) {
            for_each_owner(b, B, [&](int64_t q) {
                for (const Box &Cq : range_boxes(b, q)) {
                    Box X;
                    if (box_intersect(B, Cq, M, &X)) hb.push_back({p, q, seq++, X, box_volume(X, M)});
                }
            });
        }
    }
    // send order: (p, q, seq); a process's send array starts at its range start
    std::stable_sort(hb.begin(), hb.end(), [](const HostBox &x, const HostBox &y) {
        return x.p != y.p ? x.p < y.p : (x.q != y.q ? x.q < y.q : x.seq < y.seq);
    });
    std::vector<BoxCopy> boxes(hb.size());
    std::vector<int64_t> seg_send;  // per box: offset of its (p,q) segment start
    {
        int64_t pos = 0;
        for (size_t i = 0; i < hb.size(); ++i) {
            BoxCopy &bc = boxes[i];
            for (int d = 0; d < kMaxDims; ++d) {
                bc.lo[d] = d < M ? (int)hb[i].box.lo[d] : 0;
                bc.ext[d] = d < M ? (int)(hb[i].box.hi[d] - hb[i].box.lo[d] + 1) : 1;
            }
            bc.send_off = pos;
            bc.self = hb[i].p == hb[i].q;
            bc.pad = 0;
            pos += hb[i].n;
        }
        if (pos != pl->T) return fail(FFTRW_E_DEVICE, "internal: staged boxes do not cover the array");
    }
    // receive order: (q, p, seq)
    std::vector<size_t> ridx(hb.size());
    for (size_t i = 0; i < ridx.size(); ++i) ridx[i] = i;
    std::stable_sort(ridx.begin(), ridx.end(), [&](size_t x, size_t y) {
        const HostBox &X = hb[x], &Y = hb[y];
        return X.q != Y.q ? X.q < Y.q : (X.p != Y.p ? X.p < Y.p : X.seq < Y.seq);
    });
    {
        int64_t pos = 0;
        for (size_t r : ridx) {
            boxes[r].recv_off = pos;
            pos += hb[r].n;
        }
    }
    // exchanged segments: maximal runs of boxes with the same (p, q), p != q;
    // in both orders the boxes of one segment are consecutive
    std::vector<SegCopy> segs;
    int64_t moved = 0;
    for (size_t i = 0; i < hb.size();) {
        size_t j = i;
        int64_t len = 0;
        while (j < hb.size() && hb[j].p == hb[i].p && hb[j].q == hb[i].q) len += hb[j++].n;
        if (hb[i].p != hb[i].q) {
            segs.push_back({moved, boxes[i].send_off, boxes[i].recv_off, len});
            moved += len;
        }
        i = j;
    }
    std::vector<BoxCopy> boxes_recv(hb.size());
    for (size_t k = 0; k < ridx.size(); ++k) boxes_recv[k] = boxes[ridx[k]];

    StagedStep &st = pl->staged[t];
    st.nbox = (int64_t)boxes.size();
    st.nseg = (int64_t)segs.size();
    st.seg_elems = moved;
    int rc = copy_to_device(pl, boxes.data(), sizeof(BoxCopy) * boxes.size(), &st.boxes);
    if (!rc) rc = copy_to_device(pl, boxes_recv.data(), sizeof(BoxCopy) * boxes_recv.size(), &st.pack_prefix);
    if (!rc) rc = copy_to_device(pl, segs.data(), sizeof(SegCopy) * segs.size(), &st.segs);
    return rc;
}

int staged_run(fft_plan_impl *pl, int t, const void *in, void *out, hipStream_t s)
{
    const StagedStep &st = pl->staged[t];
    const Layout &a = pl->lay[t];
    const Layout &b = pl->lay[t + 1];
    StagedArgs g;
    std::memset(&g, 0, sizeof(g));
    g.M = pl->M;
    for (int i = 0; i < pl->M; ++i) {
        g.ord_a[i] = a.perm[i];
        g.stride_a[i] = a.stride[i];
        g.stride_b[i] = b.stride[i];
    }
    g.nbox = st.nbox;
    g.total = pl->T;
    g.counter = pl->counters + t;
    const unsigned nblk = (unsigned)((pl->T + kChunk - 1) / kChunk);
    const bool fp64 = pl->esz == 16;
    // pack: layout A -> send array
    g.boxes = (const BoxCopy *)st.boxes;
    if (fp64)
        hipLaunchKernelGGL((box_copy_kernel<double2, false>), dim3(nblk), dim3(kThreads), 0, s,
                           (const double2 *)in, (const double2 *)nullptr, (double2 *)pl->send, g);
    else
        hipLaunchKernelGGL((box_copy_kernel<float2, false>), dim3(nblk), dim3(kThreads), 0, s,
                           (const float2 *)in, (const float2 *)nullptr, (float2 *)pl->send, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(FFTRW_E_DEVICE, std::string("pack launch: ") + hipGetErrorString(e));
    // exchange: only segments between different processes
    if (st.seg_elems > 0) {
        StagedArgs x = g;
        x.segs = (const SegCopy *)st.segs;
        x.nseg = st.nseg;
        x.total = st.seg_elems;
        const unsigned xb = (unsigned)((st.seg_elems + kChunk - 1) / kChunk);
        if (fp64)
            hipLaunchKernelGGL(exchange_kernel<double2>, dim3(xb), dim3(kThreads), 0, s,
                               (const double2 *)pl->send, (double2 *)pl->recv, x);
        else
            hipLaunchKernelGGL(exchange_kernel<float2>, dim3(xb), dim3(kThreads), 0, s,
                               (const float2 *)pl->send, (float2 *)pl->recv, x);
        e = hipGetLastError();
        if (e != hipSuccess) return fail(FFTRW_E_DEVICE, std::string("exchange launch: ") + hipGetErrorString(e));
    }
    // unpack: receive array (and kept segments) -> layout B
    g.boxes = (const BoxCopy *)st.pack_prefix;
    if (fp64)
        hipLaunchKernelGGL((box_copy_kernel<double2, true>), dim3(nblk), dim3(kThreads), 0, s,
                           (const double2 *)pl->recv, (const double2 *)pl->send, (double2 *)out, g);
    else
        hipLaunchKernelGGL((box_copy_kernel<float2, true>), dim3(nblk), dim3(kThreads), 0, s,
                           (const float2 *)pl->recv, (const float2 *)pl->send, (float2 *)out, g);
    e = hipGetLastError();
    if (e != hipSuccess) return fail(FFTRW_E_DEVICE, std::string("unpack launch: ") + hipGetErrorString(e));
    return FFTRW_OK;
}

void staged_free(fft_plan_impl *pl)
{
    for (StagedStep &st : pl->staged) {
        for (void *p : {st.boxes, st.pack_prefix, st.unpack_prefix, st.segs, st.seg_prefix})
            if (p) (void)hipFree(p);
        st = StagedStep{};
    }
    if (pl->send) (void)hipFree(pl->send);
    if (pl->recv) (void)hipFree(pl->recv);
    pl->send = pl->recv = nullptr;
}

}  // namespace fftrw
