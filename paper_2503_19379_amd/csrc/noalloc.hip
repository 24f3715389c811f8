// mfd_lambda_re_static: Alg 4.1's recompute (lambda_re of every field of a
// block) with no device allocation, for callers that cannot allocate (code
// under HIP graph capture, tight serving loops).  The per-workgroup partial
// sums and their totals live in a file-scope device array instead of buffers
// allocated per call; the ratios go to a caller-owned device array, so the
// call is stream-ordered from start to end.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "../../include/mfdkc.h"
#include "internal.h"
#include "solver.h"

namespace {

// Partial sums: LAMRE_PARTS workgroups x 2 sums x nb fields, then the 2 nb
// totals.  nb <= LAMRE_MAX_NB.
constexpr int LAMRE_PARTS = 128;
constexpr int LAMRE_MAX_NB = 64;
constexpr size_t SCRATCH_DOUBLES = (size_t)LAMRE_PARTS * 2 * LAMRE_MAX_NB + 2 * LAMRE_MAX_NB;

// One copy per GPU, held until the process ends.  Host code never passes
// this name to a kernel: it is a host-side stand-in for the symbol; the
// device address comes from hipGetSymbolAddress, per device.
__device__ __align__(256) double scratch[SCRATCH_DOUBLES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
double* g_scratch[MAX_DEVICES] = {};

// The device address of `scratch` on the current device (set up on the first
// call on that device); nullptr on failure.
double* scratch_ptr(int dev) {
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        g_scratch[dev] = static_cast<double*>(ptr);
    }
    return g_scratch[dev];
}

__global__ void ratio_kernel(const double* __restrict__ sums, int nb, double* __restrict__ out) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nb) out[b] = sums[2 * b] / sums[2 * b + 1];
}

}  // namespace

namespace mfd {
OpParams ctx_params(const mfd_ctx* ctx, const double k[3]);
int ctx_device(const mfd_ctx* ctx);
const void* ctx_mu64(const mfd_ctx* ctx);
int set_error(int status, const char* msg);
}  // namespace mfd

extern "C" int mfd_lambda_re_static(mfd_ctx* ctx, const double k[3], int nb, const void* X, double* out,
                                    void* stream) {
    using namespace mfd;
    if (!ctx || !k || !X || !out) return set_error(MFD_EINVAL, "NULL argument");
    if (nb <= 0) return set_error(MFD_EINVAL, "nb must be > 0");
    if (nb > LAMRE_MAX_NB) return set_error(MFD_EINVAL, "nb exceeds 64, the size of the static scratch");
    if (!std::isfinite(k[0]) || !std::isfinite(k[1]) || !std::isfinite(k[2]))
        return set_error(MFD_EINVAL, "k must be finite");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return set_error(MFD_EDEVICE, "hipGetDevice failed");
    if (dev != ctx_device(ctx)) return set_error(MFD_EINVAL, "the context was built on another device");
    if (dev < 0 || dev >= MAX_DEVICES) return set_error(MFD_EUNSUPPORTED, "device index beyond 63");
    double* base = scratch_ptr(dev);
    if (!base) return set_error(MFD_EDEVICE, "hipGetSymbolAddress of the static scratch failed");
    double* partial = base;
    double* sums = base + (size_t)LAMRE_PARTS * 2 * LAMRE_MAX_NB;
    const OpParams p = ctx_params(ctx, k);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_lambda_re(p, nb, X, ctx_mu64(ctx), partial, LAMRE_PARTS, sums, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(ratio_kernel, dim3((nb + 63) / 64), dim3(64), 0, s, sums, nb, out);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return set_error(MFD_EDEVICE, hipGetErrorString(e));
    return MFD_OK;
}
