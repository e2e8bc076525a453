// internal.h -- declarations shared by the library's translation units (not
// part of the public C-ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcrt {

constexpr int kBlock = 256;    // threads per workgroup (4 waves)
constexpr int kNumStats = 10;  // packets, events, prop, locate, peel cells, adds, dropped, capped, guard, nonfinite

template <typename Real, typename ImgT, int G> struct View;
template <typename Real> struct Optics;
template <typename Real> struct InsDesc;

template <typename Real, typename ImgT, int G> struct TransportArgs {
    View<Real, ImgT, G> view;
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
    const void *mlp_frags;        // learned FP32: forward fragments (bf16, fragment order)
    const float *mlp_bias;        // learned FP32: biases [176]
};

// G = 0 Cartesian, 1 octree
hipError_t launch_transport_f32c(const TransportArgs<float, float, 0> &a, int grid, hipStream_t stream);
hipError_t launch_transport_f32o(const TransportArgs<float, float, 1> &a, int grid, hipStream_t stream);
hipError_t launch_transport_f64c(const TransportArgs<double, double, 0> &a, int grid, hipStream_t stream);
hipError_t launch_transport_f64o(const TransportArgs<double, double, 1> &a, int grid, hipStream_t stream);

// Allocation-free runs (noalloc.hip): a file-scope device array per GPU
// holds the queue counter (first kNoAllocHeader bytes) and the launch's
// per-wavelength optics (at most kNoAllocMaxLambda).  setup takes the
// array's device address for `device` (that device current) once; scratch
// returns it (NULL before setup).  launch_noalloc_setup zeroes the counter and
// writes the optics from the sim's device copies with L0 = lum / n_per_lambda.
constexpr size_t kNoAllocHeader = 256;
constexpr int kNoAllocMaxLambda = 4096;
size_t noalloc_scratch_bytes();
hipError_t noalloc_scratch_setup(int device);
void *noalloc_scratch(int device);
template <typename Real>
hipError_t launch_noalloc_setup(void *scratch_dev, const Optics<Real> *optics_base, const double *lum, int n_lambda,
                                uint64_t n_per_lambda, hipStream_t stream);

// auxiliary kernels (aux_kernels.hip)
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t stream);
// dst[(c - cell0) * n_lambda + l] = src[l * n_store + store(c)] for cells c in
// [cell0, cell0 + ncell); store() is the bricked layout (bs, sh, nb) of a
// Cartesian grid with n cells per axis, or the identity when bs == NULL.
hipError_t launch_table_readback(const double *src, double *dst, int64_t n_store, int n_lambda,
                                 const int *n, const int *bs, const int *sh, const int *nb, int64_t cell0,
                                 int64_t ncell, hipStream_t stream);
template <typename ImgT>
hipError_t launch_image_scale(const ImgT *src, double *dst, int64_t n, double scale, hipStream_t stream);
// Dust emission (dust.hip).  Cartesian cells in natural order
// m = ix + nx (iy + ny iz), tables and density in the bricked storage order;
// octree leaves in leaf order (storage order too).
struct DustGrid {
    long long n_cells, n_store;
    int n_lambda;
    int n[3], bs[3], sh[3], nb[3];
    const int *leaf; // octree: per leaf (origin x, y, z, level); NULL for Cartesian
};
struct DustTables {
    const double *t[4]; // absorption tables [n_lambda][n_store], summed
    int n;
};
int dust_blocks(long long n);          // blocks of the per-cell kernels over n cells (partial sums)
int dust_scan_tiles(long long n);       // tiles per row of the scan
// absorbed[s] = sum over wavelengths of the summed tables, s in storage
// order (n_store entries); part_* per block of dust_blocks(n_store)
hipError_t launch_dust_absorbed(const DustGrid &g, const DustTables &tabs, const float *density, double *absorbed,
                                double *part_abs, double *part_mass, hipStream_t st);
// T[m] and emis[l][m] (see dust.hip)
hipError_t launch_dust_emission(const DustGrid &g, const double *absorbed, const float *density,
                                const double *lambda_um, const double *kw, double u0, double T0, double beta,
                                double *T, double *emis, hipStream_t st);
// x[rows][n] := inclusive running sums of each row; tile_sums[rows][tiles]
hipError_t launch_dust_scan(double *x, long long n, int rows, double *tile_sums, hipStream_t st);
// guide[rows][K]: first index whose running sum exceeds k (row total / K)
hipError_t launch_dust_guide(const double *cdf, long long n, int K, int rows, int *guide, hipStream_t st);

// sed[l] = scale * sum of the npix pixels of slice l (n_lambda slices)
template <typename ImgT>
hipError_t launch_sed(const ImgT *img, double *sed, int n_lambda, int64_t npix, double scale, hipStream_t stream);

} // namespace mcrt

namespace mcrt {

// One model of a batched launch: its scene view (pointers to global optics and
// instrument arrays), its packet range and its own tally accumulators.
template <typename Real, typename ImgT> struct ModelDesc {
    View<Real, ImgT, 0> view;
    const Optics<Real> *optics;
    const InsDesc<Real> *ins;
    uint64_t count;       // packets per wavelength in this launch
    uint64_t first_id;
    uint64_t total;       // count * n_lambda
    uint64_t chunk0;      // index of the model's first chunk in the batch queue
    double *energy;       // [4]
    unsigned long long *stats; // [kNumStats]
};

template <typename Real, typename ImgT> struct BatchArgs {
    const ModelDesc<Real, ImgT> *models;
    int n_models;
    uint64_t total_chunks;
    uint32_t chunk;
    int threshold;
    unsigned long long *counter;
};

// slots: the deposit tile per lane, 8 or 16
hipError_t launch_batch_f32(const BatchArgs<float, float> &a, int grid, hipStream_t stream, int slots);

// learned proposal (proposal.hip)
struct GradArgs {
    const uint16_t *frags;    // all 60 fragments
    const float *bias;        // [176]
    const float *X, *KP, *C;  // samples: features [n][9], direction [n][3], weight [n]
    int64_t n;                // samples available
    int64_t m;                // samples in this pass
    int random;               // 0: samples 0 .. m-1; 1: m uniform draws (with replacement) from [0, n)
    uint32_t key0, key1, step;
    float scale;              // multiplies every weight (1 / sum of the weights of the pass)
    float *partial;           // [waves][kGradStride]
    double *loss_partial;     // [waves]
};
struct AdamArgs {
    float *theta, *m, *v;     // FP32 master parameters and moments [7400]
    float lr, b1, b2, eps;
    int step;                 // Adam time step (>= 1)
    int update;               // 0: only sum the gradient
    float *grad_out;          // optional [7400]: the summed gradient
    double *loss_out;         // optional: the summed loss
};
constexpr int kGradStrideFloats = 7424;
constexpr int kFragAllElems = 60 * 64 * 4; // bf16 values of all fragments
hipError_t launch_sum_f32(const float *x, int64_t n, double *out, hipStream_t stream);
hipError_t launch_proposal_pack(const float *theta, uint16_t *frags, float *bias, double *theta64,
                                hipStream_t stream);
hipError_t launch_proposal_forward(const uint16_t *frags, const float *bias, const float *X, int64_t n, float *out,
                                   hipStream_t stream);
hipError_t launch_proposal_grad(const GradArgs &g, int waves, hipStream_t stream);
hipError_t launch_proposal_adam(const float *partial, int waves, const double *loss_partial, const AdamArgs &a,
                                hipStream_t stream);
hipError_t launch_hist_count(const void *h, const void *tot, bool fp64, int64_t n_slots, int E, uint32_t *count,
                             uint64_t *offset, uint64_t *block_sums, uint64_t *total, hipStream_t st);
hipError_t launch_hist_write(const void *h, const void *tot, bool fp64, int64_t n_slots, int E,
                             const uint64_t *offset, float *X, float *KP, float *C, hipStream_t st);
hipError_t launch_batch_f64(const BatchArgs<double, double> &a, int grid, hipStream_t stream);

} // namespace mcrt
