// dust.hip -- the dust emission of a grid's cells on the device (Section
// 3.2, dust emission and self-absorption phases; a modified blackbody stands
// in for the paper's dust model files):
//   1. per cell, the absorbed luminosity summed over the wavelengths of one or
//      more absorption tables (wavelength-major) and per-block sums of it and
//      of the mass, density x volume (Cartesian cells 1, octree leaves 8^-L;
//      the heating unit u0 = total absorbed / total mass);
//   2. per cell, the temperature T = T0 (u / u0)^(1 / (4 + beta)) and the
//      emission of each wavelength bin, absorbed * kw B_lambda(T) / sum, with
//      kw = kappa (1 - albedo) * bin width (the cell emits what it absorbed);
//   3. per wavelength, running sums of the emission over the cells (a fixed
//      three-pass scan: the same result on every run);
//   4. per wavelength, a guide of K entries for the launch's cell search.
// All in FP64.
#include <hip/hip_runtime.h>

#define MCRT_HD __device__ __forceinline__
#include "det_math.h"
#include "internal.h"

namespace mcrt {

namespace {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 16; // per thread
constexpr int kScanTile = kScanBlock * kScanItems;

__device__ __forceinline__ long long brick_index(const int n[3], const int bs[3], const int sh[3], const int nb[3],
                                                 long long m)
{
    // (octree leaves are stored in leaf order: callers use m itself)
    const int ix = (int)(m % n[0]), iy = (int)((m / n[0]) % n[1]), iz = (int)(m / ((long long)n[0] * n[1]));
    const long long brick = (ix >> bs[0]) + (long long)nb[0] * ((iy >> bs[1]) + (long long)nb[1] * (iz >> bs[2]));
    const int in = ((ix & ((1 << bs[0]) - 1)) << sh[0]) + ((iy & ((1 << bs[1]) - 1)) << sh[1]) +
                   ((iz & ((1 << bs[2]) - 1)) << sh[2]);
    return brick * 32 + in;
}

// fixed-shape block sum of one value per thread (kScanBlock threads)
__device__ __forceinline__ double block_sum(double x, double *part)
{
    part[threadIdx.x] = x;
    __syncthreads();
    for (int w = kScanBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    const double r = part[0];
    __syncthreads();
    return r;
}

// In storage order (consecutive lanes read consecutive table elements); the
// bricks' padding cells hold zeros and add nothing.
__global__ void __launch_bounds__(kScanBlock)
absorbed_kernel(DustGrid g, DustTables tabs, const float *density, double *absorbed, double *part_abs,
                double *part_mass)
{
    __shared__ double part[kScanBlock];
    const long long sidx = (long long)blockIdx.x * kScanBlock + threadIdx.x;
    double La = 0.0, rho = 0.0;
    if (sidx < g.n_store) {
        for (int l = 0; l < g.n_lambda; ++l) {
            double t = tabs.t[0][(long long)l * g.n_store + sidx];
            for (int k = 1; k < tabs.n; ++k) t = t + tabs.t[k][(long long)l * g.n_store + sidx];
            La += t;
        }
        rho = (double)density[sidx] * (g.leaf ? ldexp(1.0, -3 * g.leaf[4 * sidx + 3]) : 1.0); // mass
        absorbed[sidx] = La;
    }
    const double sa = block_sum(La, part);
    const double sm = block_sum(rho, part);
    if (threadIdx.x == 0) {
        part_abs[blockIdx.x] = sa;
        part_mass[blockIdx.x] = sm;
    }
}

__device__ __forceinline__ double planck(double lambda_um, double T)
{
    const double h = 6.62607015e-34, c = 2.99792458e8, k = 1.380649e-23;
    const double lam = lambda_um * 1e-6;
    const double x = h * c / (lam * k * T);
    return 2.0 * h * c * c / (lam * lam * lam * lam * lam) / dm::expm1(x);
}

__global__ void __launch_bounds__(kScanBlock)
emission_kernel(DustGrid g, const double *absorbed, const float *density, const double *lambda_um, const double *kw,
                double u0, double T0, double beta, double *T, double *emis)
{
    const long long m = (long long)blockIdx.x * kScanBlock + threadIdx.x;
    if (m >= g.n_cells) return;
    const long long sidx = g.leaf ? m : brick_index(g.n, g.bs, g.sh, g.nb, m);
    const double La = absorbed[sidx];
    const double rho = (double)density[sidx] * (g.leaf ? ldexp(1.0, -3 * g.leaf[4 * m + 3]) : 1.0); // mass
    double Tm = 0.0;
    double sum = 0.0;
    const bool emits = La > 0.0 && rho > 0.0 && u0 > 0.0;
    if (emits) {
        Tm = T0 * dm::exp(dm::log((La / rho) / u0) / (4.0 + beta));
        // each bin's shape kw B(T) goes to the output first, scaled below
        for (int l = 0; l < g.n_lambda; ++l) {
            const double w = kw[l] * planck(lambda_um[l], Tm);
            emis[(long long)l * g.n_cells + m] = w;
            sum += w;
        }
    }
    T[m] = Tm;
    const bool ok = emits && sum > 0.0;
    for (int l = 0; l < g.n_lambda; ++l) {
        double *e = emis + (long long)l * g.n_cells + m;
        *e = ok ? La * (*e / sum) : 0.0;
    }
}

// a tile of a row into LDS with coalesced loads (zeros past the end); each
// thread then owns kScanItems consecutive elements (padded rows: no bank
// conflicts on the per-thread reads)
constexpr int kPad = kScanItems + 1;
__device__ __forceinline__ void load_tile(const double *row, long long n, double *tile)
{
    const long long t0 = (long long)blockIdx.x * kScanTile;
    for (int i = 0; i < kScanItems; ++i) {
        const int e = i * kScanBlock + threadIdx.x; // element within the tile
        const long long g = t0 + e;
        tile[(e / kScanItems) * kPad + e % kScanItems] = g < n ? row[g] : 0.0;
    }
    __syncthreads();
}

// scan pass 1: per tile of one row, its sum (thread sums of consecutive
// elements, then the same fixed-shape scan as pass 3: its last element)
__device__ __forceinline__ double thread_scan(double acc, double *part)
{
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int d = 1; d < kScanBlock; d <<= 1) {
        const double add = (int)threadIdx.x >= d ? part[threadIdx.x - d] : 0.0;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    return part[threadIdx.x]; // inclusive
}

__global__ void __launch_bounds__(kScanBlock) scan_tiles_kernel(const double *x, long long n, double *tile_sums)
{
    __shared__ double tile[kScanBlock * kPad];
    __shared__ double part[kScanBlock];
    load_tile(x + (long long)blockIdx.y * n, n, tile);
    double acc = 0.0;
    for (int i = 0; i < kScanItems; ++i) acc += tile[threadIdx.x * kPad + i];
    const double incl = thread_scan(acc, part);
    if (threadIdx.x == kScanBlock - 1) tile_sums[(long long)blockIdx.y * gridDim.x + blockIdx.x] = incl;
}

// scan pass 2: per row, exclusive running sums of its tiles (one thread a row)
__global__ void scan_offsets_kernel(double *tile_sums, int tiles, int rows)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    double acc = 0.0;
    for (int t = 0; t < tiles; ++t) {
        const double v = tile_sums[(long long)r * tiles + t];
        tile_sums[(long long)r * tiles + t] = acc;
        acc += v;
    }
}

// scan pass 3: inclusive running sums inside each tile, plus the tile offset
// (the tile is staged through LDS both ways, so global accesses coalesce)
__global__ void __launch_bounds__(kScanBlock) scan_apply_kernel(double *x, long long n, const double *offsets)
{
    __shared__ double tile[kScanBlock * kPad];
    __shared__ double part[kScanBlock];
    double *row = x + (long long)blockIdx.y * n;
    load_tile(row, n, tile);
    double acc = 0.0;
    for (int i = 0; i < kScanItems; ++i) acc += tile[threadIdx.x * kPad + i];
    // exclusive scan of the thread sums (Hillis-Steele over a fixed shape)
    const double incl = thread_scan(acc, part);
    double run = offsets[(long long)blockIdx.y * gridDim.x + blockIdx.x] + (incl - acc);
    for (int i = 0; i < kScanItems; ++i) {
        run += tile[threadIdx.x * kPad + i];
        tile[threadIdx.x * kPad + i] = run;
    }
    __syncthreads();
    const long long t0 = (long long)blockIdx.x * kScanTile;
    for (int i = 0; i < kScanItems; ++i) {
        const int e = i * kScanBlock + threadIdx.x;
        const long long g = t0 + e;
        if (g < n) row[g] = tile[(e / kScanItems) * kPad + e % kScanItems];
    }
}

// guide[k] = first cell whose running sum exceeds k (total / K)
__global__ void guide_kernel(const double *cdf, long long n, int K, int rows, int *guide)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)K * rows) return;
    const int r = (int)(t / K), k = (int)(t % K);
    const double *row = cdf + (long long)r * n;
    const double total = row[n - 1];
    const double x = (double)k * (total / (double)K);
    long long lo = 0, hi = n - 1;
    while (lo < hi) {
        const long long mid = lo + (hi - lo) / 2;
        if (row[mid] > x) hi = mid;
        else lo = mid + 1;
    }
    guide[t] = (int)lo;
}

} // namespace

int dust_blocks(long long n) { return (int)((n + kScanBlock - 1) / kScanBlock); }

hipError_t launch_dust_absorbed(const DustGrid &g, const DustTables &tabs, const float *density, double *absorbed,
                                double *part_abs, double *part_mass, hipStream_t st)
{
    hipLaunchKernelGGL(absorbed_kernel, dim3(dust_blocks(g.n_store)), dim3(kScanBlock), 0, st, g, tabs, density,
                       absorbed, part_abs, part_mass);
    return hipGetLastError();
}

hipError_t launch_dust_emission(const DustGrid &g, const double *absorbed, const float *density,
                                const double *lambda_um, const double *kw, double u0, double T0, double beta,
                                double *T, double *emis, hipStream_t st)
{
    hipLaunchKernelGGL(emission_kernel, dim3(dust_blocks(g.n_cells)), dim3(kScanBlock), 0, st, g, absorbed, density,
                       lambda_um, kw, u0, T0, beta, T, emis);
    return hipGetLastError();
}

int dust_scan_tiles(long long n) { return (int)((n + kScanTile - 1) / kScanTile); }

hipError_t launch_dust_scan(double *x, long long n, int rows, double *tile_sums, hipStream_t st)
{
    const int tiles = dust_scan_tiles(n);
    hipLaunchKernelGGL(scan_tiles_kernel, dim3(tiles, rows), dim3(kScanBlock), 0, st, x, n, tile_sums);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(scan_offsets_kernel, dim3((rows + 63) / 64), dim3(64), 0, st, tile_sums, tiles, rows);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(scan_apply_kernel, dim3(tiles, rows), dim3(kScanBlock), 0, st, x, n, tile_sums);
    return hipGetLastError();
}

hipError_t launch_dust_guide(const double *cdf, long long n, int K, int rows, int *guide, hipStream_t st)
{
    const long long total = (long long)K * rows;
    hipLaunchKernelGGL(guide_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, cdf, n, K, rows, guide);
    return hipGetLastError();
}

} // namespace mcrt
