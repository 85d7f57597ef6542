// Error norms without a state or workspace, for callers that cannot
// allocate device memory: the reduction of mpdc_diagnostics (the normalised
// L1/L2/Linf of Eq. 2 and min/max) over plain device arrays, with its
// per-work-group partial sums in a file-scope device array instead of the
// state's workspace.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <sstream>

#include "dycore_kernels.h"
#include "mpdc_internal.h"

namespace mpdc {
namespace {

// One 9-double partial per work-group of the reduction (the layout of
// k_diag's output); the reduction strides over any number of elements with
// at most this many work-groups.
constexpr int kStaticBlocks = 1024;
constexpr int kStaticVals = 9;
constexpr size_t kScratchBytes = (size_t)kStaticBlocks * kStaticVals * sizeof(double);

// Each GPU the library runs on holds its own copy until the process ends.
// In host code the name is only a stand-in: kernels get the device address
// from hipGetSymbolAddress (scratch_ptr below), never the name itself.
static __device__ __align__(256) double scratch[kStaticBlocks * kStaticVals];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {nullptr};

// Device address of this GPU's scratch, looked up once per device (with that
// device current, as it is when this is called).
hipError_t scratch_ptr(double **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace
}  // namespace mpdc

using namespace mpdc;

extern "C" int mpdc_error_norms_noalloc(const double *x, const double *ref, const double *weight, size_t n,
                                        size_t inner, double *out, void *stream) {
    if (!x || !ref || !out) return fail(MPDC_E_INVAL, "null field, reference or output");
    if (n == 0 || inner == 0) return fail(MPDC_E_INVAL, "empty field (n and inner must be positive)");
    if (n > (size_t)LONG_MAX / inner) return fail(MPDC_E_INVAL, "n x inner overflows the element count");
    hipStream_t s = (hipStream_t)stream;
    double *part_dev = nullptr;
    hipError_t e = scratch_ptr(&part_dev);
    if (e != hipSuccess) {
        std::ostringstream o;
        o << "hipGetSymbolAddress of the norms scratch: " << hipGetErrorString(e);
        return fail(MPDC_E_DEVICE, o.str());
    }
    const long total = (long)(n * inner);
    const long want = (total + 255) / 256;
    const int nblocks = (int)(want < kStaticBlocks ? want : kStaticBlocks);
    if ((size_t)nblocks * kStaticVals * sizeof(double) > kScratchBytes)
        return fail(MPDC_E_NOMEM, "the reduction needs more partials than the static scratch holds");
    DiagArgs a{};
    a.area = weight;
    a.x = x;
    a.ref = ref;
    a.n = (long)n;
    a.inner = (long)inner;
    a.xs = 1;
    a.xo = 0;
    a.partial = part_dev;   // every slot the launch uses is written by it: nothing to clear
    e = launch_diag(a, nblocks, s);
    double part[kStaticBlocks * kStaticVals];
    if (e == hipSuccess)
        e = hipMemcpyAsync(part, part_dev, (size_t)nblocks * kStaticVals * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        std::ostringstream o;
        o << "norms reduction: " << hipGetErrorString(e);
        return fail(MPDC_E_DEVICE, o.str());
    }
    double r[kStaticVals] = {0.0, (double)INFINITY, -(double)INFINITY, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = 0; b < nblocks; b++) {   // fixed order
        const double *p = part + (size_t)b * kStaticVals;
        r[1] = p[1] < r[1] ? p[1] : r[1];
        r[2] = p[2] > r[2] ? p[2] : r[2];
        for (int v = 3; v < 7; v++) r[v] += p[v];
        r[7] = p[7] > r[7] ? p[7] : r[7];
        r[8] = p[8] > r[8] ? p[8] : r[8];
    }
    out[0] = r[3] / r[4];
    out[1] = std::sqrt(r[5] / r[6]);
    out[2] = r[7] / r[8];
    out[3] = r[1];
    out[4] = r[2];
    return MPDC_OK;
}
