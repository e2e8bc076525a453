// noalloc.hip -- the library-owned scratch of the allocation-free run
// (mcrt_run_into_noalloc) and the kernel that prepares it.
//
// The transport kernel needs, besides its inputs (the scene) and outputs
// (the result), two pieces of scratch memory per launch: the work-queue
// counter (chunks of packet ids handed out so far, must start at zero) and
// the per-wavelength optics staged for the launch (kappa, albedo, g, the
// packet luminosity L0 = L / n_per_lambda, the proposal's wavelength
// feature).  mcrt_run_into takes the counter from the result and rewrites the
// sim's optics buffer from the host.  The allocation-free run takes both from
// one file-scope device array per GPU instead, prepared on the device from the
// sim's device copies, so a call allocates nothing, copies nothing from the
// host and creates no events.  Every call on a GPU shares that GPU's array.

#define MCRT_HD __device__ __forceinline__
#include "internal.h"
#include "transport_core.h"

#include <mutex>

namespace mcrt {

namespace {

constexpr size_t kScratchBytes = kNoAllocHeader + (size_t)kNoAllocMaxLambda * sizeof(Optics<double>);

// Device address: taken once per device with hipGetSymbolAddress at context
// creation; host code uses that address, never this name.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch_ptr[kMaxDevices] = {};

template <typename Real>
__global__ void __launch_bounds__(256) noalloc_setup_kernel(unsigned char *base, const Optics<Real> *optics,
                                                            const double *lum, int n_lambda, double n_per_lambda)
{
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l == 0) *reinterpret_cast<unsigned long long *>(base) = 0ull; // the queue counter starts at zero
    if (l >= n_lambda) return;
    Optics<Real> o = optics[l];
    // the same rounding as the host's (Real)(L / (double)n_per_lambda)
    o.L0 = (Real)(lum[l] / n_per_lambda);
    reinterpret_cast<Optics<Real> *>(base + kNoAllocHeader)[l] = o;
}

} // namespace

size_t noalloc_scratch_bytes() { return kScratchBytes; }

hipError_t noalloc_scratch_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = p;
    return hipSuccess;
}

void *noalloc_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    return g_scratch_ptr[device];
}

template <typename Real>
hipError_t launch_noalloc_setup(void *scratch_dev, const Optics<Real> *optics_base, const double *lum, int n_lambda,
                                uint64_t n_per_lambda, hipStream_t stream)
{
    if (!scratch_dev || n_lambda < 1 || n_lambda > kNoAllocMaxLambda) return hipErrorInvalidValue;
    const int blocks = (n_lambda + 255) / 256;
    hipLaunchKernelGGL(noalloc_setup_kernel<Real>, dim3(blocks), dim3(256), 0, stream,
                       static_cast<unsigned char *>(scratch_dev), optics_base, lum, n_lambda, (double)n_per_lambda);
    return hipGetLastError();
}

template hipError_t launch_noalloc_setup<float>(void *, const Optics<float> *, const double *, int, uint64_t,
                                                hipStream_t);
template hipError_t launch_noalloc_setup<double>(void *, const Optics<double> *, const double *, int, uint64_t,
                                                 hipStream_t);

} // namespace mcrt
