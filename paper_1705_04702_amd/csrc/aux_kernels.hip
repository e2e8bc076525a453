// aux_kernels.hip -- fills and readback conversions around the transport
// kernel: zeroing of tallies (a kernel rather than a memset, so the sequence
// stays valid under stream capture), the (wavelength, cell) -> (cell,
// wavelength) table transpose of the readback, and image scaling to flux.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace mcrt {

__global__ void fill_zero_kernel(uint4 *p, size_t n16, unsigned char *tail, size_t ntail)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n16; i += stride) p[i] = make_uint4(0u, 0u, 0u, 0u);
    if (blockIdx.x == 0 && threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t stream)
{
    if (bytes == 0) return hipSuccess;
    size_t n16 = bytes / 16;
    size_t ntail = bytes - n16 * 16;
    size_t blocks = (n16 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, (uint4 *)p, n16,
                       (unsigned char *)p + n16 * 16, ntail);
    return hipGetLastError();
}

struct Layout {
    int n[3], bs[3], nb[3], sh[3];
    int bricked;
};

__device__ __forceinline__ int64_t layout_store(const Layout &L, int64_t c)
{
    if (!L.bricked) return c;
    int ix = (int)(c % L.n[0]);
    int iy = (int)((c / L.n[0]) % L.n[1]);
    int iz = (int)(c / ((int64_t)L.n[0] * L.n[1]));
    int brick = (ix >> L.bs[0]) + L.nb[0] * ((iy >> L.bs[1]) + L.nb[1] * (iz >> L.bs[2]));
    int in = ((ix & ((1 << L.bs[0]) - 1)) << L.sh[0]) + ((iy & ((1 << L.bs[1]) - 1)) << L.sh[1]) +
             ((iz & ((1 << L.bs[2]) - 1)) << L.sh[2]);
    return (int64_t)brick * 32 + in;
}

// dst[(c - cell0) * n_lambda + l] = src[l * n_store + store(c)]: one thread per
// (cell, wavelength) pair, wavelength fastest so the writes are coalesced.
__global__ void table_readback_kernel(const double *src, double *dst, int64_t n_store, int n_lambda, Layout L,
                                      int64_t cell0, int64_t ncell)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t total = ncell * n_lambda;
    for (; i < total; i += stride) {
        int64_t c = cell0 + i / n_lambda;
        int l = (int)(i % n_lambda);
        dst[i] = src[(int64_t)l * n_store + layout_store(L, c)];
    }
}

hipError_t launch_table_readback(const double *src, double *dst, int64_t n_store, int n_lambda, const int *n,
                                 const int *bs, const int *sh, const int *nb, int64_t cell0, int64_t ncell,
                                 hipStream_t stream)
{
    Layout L{};
    L.bricked = bs != nullptr;
    for (int a = 0; a < 3; ++a) {
        L.n[a] = n ? n[a] : 1;
        L.bs[a] = bs ? bs[a] : 0;
        L.sh[a] = sh ? sh[a] : 0;
        L.nb[a] = nb ? nb[a] : 1;
    }
    int64_t total = ncell * n_lambda;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(table_readback_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, src, dst, n_store,
                       n_lambda, L, cell0, ncell);
    return hipGetLastError();
}

template <typename ImgT>
__global__ void image_scale_kernel(const ImgT *src, double *dst, int64_t n, double scale)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) dst[i] = (double)src[i] * scale;
}

template <typename ImgT>
hipError_t launch_image_scale(const ImgT *src, double *dst, int64_t n, double scale, hipStream_t stream)
{
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(image_scale_kernel<ImgT>, dim3((unsigned)blocks), dim3(256), 0, stream, src, dst, n, scale);
    return hipGetLastError();
}

template hipError_t launch_image_scale<float>(const float *, double *, int64_t, double, hipStream_t);
template hipError_t launch_image_scale<double>(const double *, double *, int64_t, double, hipStream_t);

// SED of an instrument: sed[l] = scale * sum over the pixels of wavelength
// slice l.  One block per slice; each thread sums a fixed stride of pixels in
// FP64, then a fixed-shape tree in LDS, so the result does not depend on
// timing.
template <typename ImgT>
__global__ void __launch_bounds__(256) sed_kernel(const ImgT *img, double *sed, int64_t npix, double scale)
{
    __shared__ double part[256];
    const ImgT *row = img + (int64_t)blockIdx.x * npix;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < npix; i += 256) acc += (double)row[i];
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) sed[blockIdx.x] = part[0] * scale;
}

template <typename ImgT>
hipError_t launch_sed(const ImgT *img, double *sed, int n_lambda, int64_t npix, double scale, hipStream_t stream)
{
    if (n_lambda <= 0) return hipSuccess;
    hipLaunchKernelGGL(sed_kernel<ImgT>, dim3((unsigned)n_lambda), dim3(256), 0, stream, img, sed, npix, scale);
    return hipGetLastError();
}

template hipError_t launch_sed<float>(const float *, double *, int, int64_t, double, hipStream_t);
template hipError_t launch_sed<double>(const double *, double *, int, int64_t, double, hipStream_t);

} // namespace mcrt
