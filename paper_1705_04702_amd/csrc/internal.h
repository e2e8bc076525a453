// internal.h -- declarations shared by the library's translation units (not
// part of the public C-ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcrt {

constexpr int kBlock = 256;    // threads per workgroup (4 waves)
constexpr int kNumStats = 9;   // packets, events, prop, locate, peel cells, adds, dropped, capped, guard

template <typename Real, typename ImgT> struct View;
template <typename Real> struct Optics;
template <typename Real> struct InsDesc;

template <typename Real, typename ImgT> struct TransportArgs {
    View<Real, ImgT> view;
    const Optics<Real> *optics;   // global copies, staged into LDS by the kernel
    const InsDesc<Real> *ins;
    uint64_t total;               // packets in this launch: n_lambda * count
    uint64_t count;               // packets per wavelength in this launch
    uint64_t first_id;            // first packet id
    uint32_t chunk;               // packets taken per queue grab
    int threshold;                // lanes that must finish a march before events run
    unsigned long long *counter;  // queue position (chunks handed out)
    double *energy;               // [4] emitted, absorbed, escaped, truncated
    unsigned long long *stats;    // [kNumStats]
};

hipError_t launch_transport_f32(const TransportArgs<float, float> &a, int grid, hipStream_t stream);
hipError_t launch_transport_f64(const TransportArgs<double, double> &a, int grid, hipStream_t stream);

// auxiliary kernels (aux_kernels.hip)
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t stream);
hipError_t launch_table_transpose(const double *src, double *dst, int64_t n_cells, int n_lambda,
                                  int64_t cell0, int64_t ncell, hipStream_t stream);
template <typename ImgT>
hipError_t launch_image_scale(const ImgT *src, double *dst, int64_t n, double scale, hipStream_t stream);

} // namespace mcrt
