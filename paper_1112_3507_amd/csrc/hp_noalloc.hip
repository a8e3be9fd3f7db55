// hp_noalloc.hip -- the entry point that allocates nothing: hp_dot_noalloc.
//
// hp_dot reduces its per-workgroup partial sums in the handle's workspace (allocated by
// hp_setup) and returns the result on the host. hp_dot_noalloc runs the same two kernels (first
// stage: one partial per workgroup in a fixed grid; second stage: one workgroup sums them in index
// order), so its result is bitwise that of hp_dot, but the partials live in a file-scope device
// array and the result goes to a caller-owned device double, stream-ordered, without a host
// synchronisation: callers that cannot allocate (code under stream capture, tight serving loops)
// can use it.
#include "hp.h"
#include "hp_internal.h"

#include <mutex>
#include <string>

using namespace hp;

namespace {

// Partial sums of the first reduction stage: the dot kernel launches at most this many
// workgroups for any length (one per 1024 entries, capped), so every n >= 0 fits.
constexpr int kScratchPartials = 2048;
constexpr int kMaxDevices = 64;

// One copy per GPU, held until the process ends. Host code never uses this name as an address
// (on the host it is a stand-in, not the device address): it takes the address per device from
// hipGetSymbolAddress and passes that.
static __device__ __align__(256) double scratch[kScratchPartials];

std::mutex g_mu;
double* g_scratch_ptr[kMaxDevices] = {};

thread_local std::string g_na_err;

int na_fail(int code, const char* msg, hipError_t e = hipSuccess) {
    g_na_err = msg;
    if (e != hipSuccess) {
        g_na_err += ": ";
        g_na_err += hipGetErrorString(e);
    }
    return code;
}

// Device address of `scratch` on the current device, looked up once per device.
int scratch_ptr(double** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return na_fail(HP_EHIP, "hipGetDevice failed", e);
    if (dev < 0 || dev >= kMaxDevices) return na_fail(HP_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return na_fail(HP_EHIP, "hipGetSymbolAddress(scratch) failed", e);
        g_scratch_ptr[dev] = (double*)p;
    }
    *out = g_scratch_ptr[dev];
    return HP_OK;
}

}  // namespace

extern "C" {

const char* hp_noalloc_last_error(void) { return g_na_err.c_str(); }

int hp_dot_noalloc(const double* x, const double* y, long long n, double* result, void* stream) {
    g_na_err.clear();
    if (!result || (n > 0 && (!x || !y))) return na_fail(HP_EINVAL, "null argument");
    if (n < 0) return na_fail(HP_EINVAL, "negative length");
    if (reduce_blocks_vec(n) > kScratchPartials)
        return na_fail(HP_EINVAL, "length needs more partial sums than the static scratch holds");
    double* part = nullptr;
    int rc = scratch_ptr(&part);
    if (rc != HP_OK) return rc;
    // the second stage stores its total into result[0] (slot 0 of a one-entry scalar array);
    // every partial it reads is written by the first stage of the same call, so nothing in the
    // scratch needs clearing
    RedCtl red;
    red.partials = part;
    red.scal = result;
    red.op = OP_STORE;
    red.slot = 0;
    launch_dot<double>(x, y, (int64_t)n, red, (hipStream_t)stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return na_fail(HP_EHIP, "kernel launch failed", e);
    return HP_OK;
}

}  // extern "C"
