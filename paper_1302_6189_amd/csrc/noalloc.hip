// noalloc.hip -- the whole Fig. 4 pipeline without any device allocation, for
// callers that cannot allocate (code under HIP graph capture, serving loops,
// harnesses that forbid hipMalloc).
//
// fft_plan + fft_exec_fwd/inv allocate the plan's workspace (the ping-pong
// buffer of the transposes) and twiddle tables with hipMalloc.  This entry
// point builds the same plan on the host for one call and takes that device
// memory from one fixed array, `scratch`, instead: the workspace of at most
// kScratchWork bytes and the twiddle tables, which are regenerated into it on
// the caller's stream every call.  The same kernels then run, so the results
// equal those of a plan with the same arguments bit for bit.
//
// `scratch` is a device-side object of the library's code object: each GPU the
// library runs on holds its own copy (kScratchBytes) until the process ends.
// In host code its name is only a stand-in for the symbol; the device address
// is looked up once per device (hipGetSymbolAddress, with that device
// current) and only that address is ever handed to kernels.  Every call on a
// GPU shares that GPU's copy, so calls that overlap on one GPU (other streams,
// other threads) race; calls on one stream are ordered by the stream.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/fftrw.h"
#include "errors.hpp"
#include "plan.hpp"
#include "tune.hpp"

namespace fftrw {

int plan_create(fft_plan_t *plan, int M, const int64_t *dims, int64_t P, const int8_t *order, int dtype,
                int precision, unsigned flags, bool generic_rows, const TuneTable *tune, DevArena *arena);
void plan_free(fft_plan_t plan);
int plan_run(fft_plan_impl *pl, const void *in, void *out, hipStream_t s, int dir);

constexpr size_t kScratchWork = (size_t)64 << 20;              // the workspace: one array of T elements
constexpr size_t kScratchBytes = kScratchWork + ((size_t)1 << 20);  // + twiddle tables (<= 5 x 64 KB)
constexpr int kScratchDevices = 64;

}  // namespace fftrw

static __device__ __align__(256) unsigned char scratch[fftrw::kScratchBytes];

namespace {

std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[fftrw::kScratchDevices];  // device address of `scratch`, per device

// The device address of this device's `scratch`, looked up on its first use
// with the device current.
int scratch_of(int dev, unsigned char **out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fftrw::fail(FFTRW_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<unsigned char *>(p);
    }
    *out = g_scratch_ptr[dev];
    return FFTRW_OK;
}

}  // namespace

using namespace fftrw;

extern "C" int fft_exec_noalloc(int M, const int64_t *dims, int64_t P, const int8_t *order, int dtype,
                                int precision, unsigned flags, int direction, const void *in, void *out,
                                void *stream)
{
    g_last_error.clear();
    if (!dims || !in || !out) return fail(FFTRW_E_ARG, "null dims or buffer");
    if (direction != -1 && direction != 1) return fail(FFTRW_E_ARG, "direction must be -1 or +1");
    if (flags & ~(unsigned)(FFTRW_FLAG_LEAVE_PERMUTED | FFTRW_FLAG_FUSED_FFT | FFTRW_FLAG_SEPARATE))
        return fail(FFTRW_E_UNSUPPORTED,
                    "fft_exec_noalloc takes LEAVE_PERMUTED, FUSED_FFT and SEPARATE only (staged tables, "
                    "device counters and matched relabelling tables would need memory of their own)");
    if (dtype != FFTRW_C64 && dtype != FFTRW_C128) return fail(FFTRW_E_ARG, "unknown dtype");
    if (M < 2 || M > 5) return fail(FFTRW_E_SIZE, "plans run M = 2..5");
    // the size limit, checked before anything else is built
    const size_t esz = dtype == FFTRW_C64 ? 8 : 16;
    size_t T = 1;
    for (int i = 0; i < M; ++i) {
        if (dims[i] < 1) return fail(FFTRW_E_SIZE, "sizes must be >= 1");
        if ((size_t)dims[i] > kScratchWork / esz / T)
            return fail(FFTRW_E_SIZE, "fft_exec_noalloc handles at most " + std::to_string(kScratchWork / esz) +
                                          " points of this type (" + std::to_string(kScratchWork >> 20) +
                                          " MiB of workspace); use fft_plan for larger arrays");
        T *= (size_t)dims[i];
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(FFTRW_E_DEVICE, "no HIP device");
    if (dev < 0 || dev >= kScratchDevices) return fail(FFTRW_E_DEVICE, "device index beyond the scratch table");
    unsigned char *base = nullptr;
    if (int rc = scratch_of(dev, &base)) return rc;
    DevArena arena;
    arena.base = base;
    arena.cap = kScratchBytes;
    arena.stream = (hipStream_t)stream;
    fft_plan_t pl = nullptr;
    int rc = plan_create(&pl, M, dims, P, order, dtype, precision, flags, false, nullptr, &arena);
    if (rc) return rc;
    log_line(3, "exec (no allocation) %s plan %p in %p out %p stream %p", direction < 0 ? "forward" : "inverse",
             (void *)pl, in, out, stream);
    rc = plan_run(pl, in, out, (hipStream_t)stream, direction);
    plan_free(pl);  // host memory only: the device memory is the scratch array's
    return rc;
}
