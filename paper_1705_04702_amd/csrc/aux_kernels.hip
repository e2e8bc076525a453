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

// dst[(c - cell0) * n_lambda + l] = src[l * n_cells + c] for c in [cell0, cell0 + ncell);
// 64 x 64 tiles through LDS so both sides are coalesced.
__global__ void table_transpose_kernel(const double *src, double *dst, int64_t n_cells, int n_lambda,
                                       int64_t cell0, int64_t ncell)
{
    __shared__ double tile[64][65];
    int64_t c_base = cell0 + (int64_t)blockIdx.x * 64;
    int l_base = blockIdx.y * 64;
    int tx = threadIdx.x & 63, ty = threadIdx.x >> 6; // 256 threads: 64 x 4
    for (int r = ty; r < 64; r += 4) {
        int l = l_base + r;
        int64_t c = c_base + tx;
        if (l < n_lambda && c < cell0 + ncell) tile[r][tx] = src[(int64_t)l * n_cells + c];
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        int64_t c = c_base + r;
        int l = l_base + tx;
        if (l < n_lambda && c < cell0 + ncell) dst[(c - cell0) * n_lambda + l] = tile[tx][r];
    }
}

hipError_t launch_table_transpose(const double *src, double *dst, int64_t n_cells, int n_lambda,
                                  int64_t cell0, int64_t ncell, hipStream_t stream)
{
    dim3 grid((unsigned)((ncell + 63) / 64), (unsigned)((n_lambda + 63) / 64));
    hipLaunchKernelGGL(table_transpose_kernel, grid, dim3(256), 0, stream, src, dst, n_cells, n_lambda,
                       cell0, ncell);
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

} // namespace mcrt
