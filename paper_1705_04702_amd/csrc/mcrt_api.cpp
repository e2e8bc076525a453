// mcrt_api.cpp -- implementation of the C-ABI declared in include/mcrt.h:
// handle management, argument validation, scene upload, run orchestration
// and result readback.  All arithmetic of the photon life cycle runs in the
// HIP kernels; this file only prepares constants and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mcrt.h"

#define MCRT_HD inline
#include "transport_core.h"
#include "internal.h"
#include "scene_setup.h"

using namespace mcrt;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                                 \
    do {                                                                                              \
        hipError_t e_ = (expr);                                                                       \
        if (e_ != hipSuccess) return fail(MCRT_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

bool debug_fail_alloc()
{
    const char *s = std::getenv("MCRT_DEBUG_FAIL_ALLOC");
    return s && s[0] == '1';
}

int dev_alloc(void **p, size_t bytes)
{
    *p = nullptr;
    if (debug_fail_alloc()) return fail(MCRT_ENOMEM, "device allocation refused (MCRT_DEBUG_FAIL_ALLOC=1)");
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(MCRT_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
    }
    return MCRT_OK;
}

void dev_free(void *p)
{
    if (p) (void)hipFree(p);
}

// Owners released on every return path (HIP_TRY returns early).
struct DevPtr {
    void *p = nullptr;
    DevPtr() = default;
    DevPtr(const DevPtr &) = delete;
    DevPtr &operator=(const DevPtr &) = delete;
    ~DevPtr() { dev_free(p); }
};

struct EventPair {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    EventPair() = default;
    EventPair(const EventPair &) = delete;
    EventPair &operator=(const EventPair &) = delete;
    ~EventPair()
    {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

bool finite_box(const double b[6])
{
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(b[a]) || !std::isfinite(b[3 + a]) || !(b[3 + a] > b[a])) return false;
    return true;
}

} // namespace

namespace mcrt {
// Error reporting for the other host sources of the library (output.cpp).
int report_error(int code, const std::string &msg) { return fail(code, msg); }
} // namespace mcrt

struct mcrt_context {
    int device = 0;
    hipStream_t stream = nullptr;
    int n_cu = 0;
};

struct mcrt_grid {
    mcrt_context *ctx = nullptr;
    int type = kCartesian;
    double box[6] = {};
    int n[3] = {0, 0, 0};
    int depth = 0;
    int64_t n_cells = 0;
    std::vector<int32_t> first_child;
};

struct mcrt_medium {
    mcrt_grid *grid = nullptr;
    std::vector<float> density;
    int n_lambda = 0;
    std::vector<double> kappa, albedo, g;
    std::vector<double> lambda_um; // empty when not given
};

struct mcrt_source {
    mcrt_context *ctx = nullptr;
    int type = kPointIso;
    double pos[3] = {0, 0, 0};
    double hR = 0, zs = 0;
    std::vector<double> L;
};

struct mcrt_instrument {
    mcrt_context *ctx = nullptr;
    HostInstrument h{};
};

struct mcrt_sim {
    mcrt_context *ctx = nullptr;
    mcrt_medium *medium = nullptr;
    mcrt_source *source = nullptr;
    int n_ins = 0;
    HostInstrument ins[kMaxIns];
    double inv4pid2[kMaxIns];
    long long ins_offset[kMaxIns];
    long long image_elems = 0;
    mcrt_options opt{};
    int depth = 0, top_level = 0;
    int bs[3] = {0, 0, 0}, nb[3] = {1, 1, 1}, sh[3] = {0, 0, 0}; // Cartesian brick layout
    long long n_store = 0;                     // stored cells per wavelength slice
    // device copies of the scene
    float *d_density = nullptr;
    unsigned long long *d_node = nullptr; // octree walk blocks (64-bit entries)
    unsigned long long *d_top = nullptr;  // octree walk top table
    void *d_optics = nullptr; // Optics<Real>[n_lambda], rewritten per run
    void *d_optics_base = nullptr; // Optics<Real>[n_lambda] with L0 = 0 (allocation-free runs)
    double *d_lum = nullptr;       // source luminosity per wavelength, FP64 (allocation-free runs)
    void *d_ins = nullptr;    // InsDesc<Real>[n_ins]
    void *d_col[kMaxIns] = {}; // column maps of axis-aligned instruments (Cartesian), Real[n_store]
    std::atomic<int> busy{0};
    // learned proposal
    mcrt_proposal *prop = nullptr;
    double alpha = 0.2;
    double r_out = 0.0, rho_mean = 0.0; // feature scales
    std::vector<double> lamf;            // wavelength feature per bin
};

struct mcrt_proposal {
    mcrt_context *ctx = nullptr;
    float *d_theta = nullptr, *d_m = nullptr, *d_v = nullptr; // FP32 master, Adam moments [7400]
    uint16_t *d_frags = nullptr;  // bf16 fragments [60][64][4]
    float *d_bias = nullptr;      // [176]
    double *d_theta64 = nullptr;  // FP64 copy for the scalar network [7400]
    int step = 0;                 // Adam time step
    std::atomic<int> busy{0};
};

struct mcrt_histories {
    mcrt_context *ctx = nullptr;
    int fp64 = 0;
    int64_t n_packets = 0;
    int events = 0;
    void *d_hist = nullptr;   // Real [n_packets][events][14]
    void *d_total = nullptr;  // Real [n_packets]
    int64_t n_samples = 0;
    float *d_X = nullptr, *d_KP = nullptr, *d_C = nullptr;
    double c_sum = 0.0;
};

struct mcrt_dust {
    mcrt_sim *sim = nullptr;
    mcrt_dust_params params{};
    int K = 0;                   // guide entries per wavelength
    double *d_cdf = nullptr;     // [n_lambda][n_cells] running sums of the emission
    int *d_guide = nullptr;      // [n_lambda][K]
    double *d_T = nullptr;       // [n_cells] temperatures
    int *d_leaf = nullptr;       // octree: [n_cells][4] leaf origin and level
    std::vector<double> L;       // emitted luminosity per wavelength
};

struct mcrt_result {
    mcrt_sim *sim = nullptr;
    double *d_table = nullptr;    // [n_lambda][n_cells]
    void *d_images = nullptr;     // float or double, [ins][lambda][y][x]
    double *d_energy = nullptr;   // [4]
    unsigned long long *d_stats = nullptr;   // [kNumStats]
    unsigned long long *d_counter = nullptr; // queue position
    double kernel_ms = 0.0;
    // the cumulative counters after the last launch into this result, so
    // that a launch reports (return code, run log) only what it added itself
    unsigned long long seen[kNumStats] = {};
};

// The automatic chunk times 2^shift (at least 1, at most 2^24 packets).
static uint64_t shifted_chunk(uint64_t c, int shift)
{
    c = shift >= 0 ? c << shift : c >> (-shift);
    return c < 1 ? 1 : (c > (uint64_t(1) << 24) ? (uint64_t(1) << 24) : c);
}

// Codes after which a launch's results are still there to use.
static inline bool soft_code(int rc) { return rc == MCRT_ELIMIT || rc == MCRT_ENONFINITE; }

// The return code of a launch into r from the cumulative stats it left
// (stats[7] capped, stats[9] non-finite): MCRT_ENONFINITE or MCRT_ELIMIT when
// this launch raised the count, else MCRT_OK.  delta (optional) receives what
// the launch added to every counter.
static int launch_outcome(mcrt_result *r, const unsigned long long *stats, unsigned long long *delta = nullptr)
{
    const bool capped = stats[7] > r->seen[7], nonfinite = stats[9] > r->seen[9];
    for (int k = 0; k < kNumStats; ++k) {
        if (delta) delta[k] = stats[k] - r->seen[k];
        r->seen[k] = stats[k];
    }
    if (nonfinite)
        return fail(MCRT_ENONFINITE, "packets whose luminosity became NaN or infinite were ended (see "
                                     "stats.nonfinite); the other packets' results are valid");
    if (capped) return fail(MCRT_ELIMIT, "packets hit the event cap (results valid; see stats.capped)");
    return MCRT_OK;
}

// ---------------------------------------------------------------------------
// Run log.  With the environment variable MCRT_LOG set to a positive integer,
// every timed transport launch appends one JSON line to the file that
// MCRT_LOG_FILE names (else to stderr): what ran, the counters the launch
// added, its kernel time, and the rates derived from them -- packets/s,
// deposits/s (propagation cells plus pixel additions) and the algorithmic
// HBM bytes (per propagation cell a 4-byte density read and a table deposit
// of 8 bytes, per interaction-search or peel-off cell a 4-byte density read,
// per pixel addition the image element) over the kernel time, also as a
// fraction of 8 TB/s.  The variables are read at every launch.  Autotuner
// trials and allocation-free launches (untimed) are not logged.
// ---------------------------------------------------------------------------
namespace {

std::mutex g_log_mu;
thread_local int g_log_muted = 0;
constexpr double kHbmPeakGBs = 8000.0;

struct Counters {
    unsigned long long v[kNumStats];
};

int log_level()
{
    const char *s = std::getenv("MCRT_LOG");
    return s ? std::atoi(s) : 0;
}

struct LogMute {
    LogMute() { ++g_log_muted; }
    ~LogMute() { --g_log_muted; }
};

// One launch's line.  sims/deltas: the launch's models (one, except for a
// batch) and the counters each added; fields that differ between a batch's
// models are summed (cells, wavelengths, instruments, counters).
void log_launch(const char *entry, mcrt_sim *const *sims, int n, const Counters *deltas,
                uint64_t n_per_lambda, uint64_t first_id, uint64_t count, uint64_t seed, double kernel_ms, int rc)
{
    if (g_log_muted || log_level() <= 0) return;
    const mcrt_sim *s0 = sims[0];
    const bool fp32 = s0->opt.precision == MCRT_FP32;
    unsigned long long d[kNumStats] = {};
    long long cells = 0;
    int n_lambda = 0, n_ins = 0;
    for (int i = 0; i < n; ++i) {
        for (int k = 0; k < kNumStats; ++k) d[k] += deltas[i].v[k];
        cells += (long long)sims[i]->medium->grid->n_cells;
        n_lambda += sims[i]->medium->n_lambda;
        n_ins += sims[i]->n_ins;
    }
    const double bytes = 12.0 * (double)d[2] + 4.0 * (double)(d[3] + d[4]) + (fp32 ? 4.0 : 8.0) * (double)d[5];
    const double sec = kernel_ms * 1e-3;
    const double per_s = sec > 0.0 ? 1.0 / sec : 0.0;
    char buf[2048];
    snprintf(buf, sizeof buf,
             "{\"mcrt\":\"launch\",\"entry\":\"%s\",\"device\":%d,\"grid\":\"%s\",\"models\":%d,"
             "\"cells\":%lld,\"n_lambda\":%d,\"instruments\":%d,\"precision\":\"%s\",\"learned\":%s,"
             "\"n_per_lambda\":%llu,\"first_id\":%llu,\"count\":%llu,\"seed\":%llu,"
             "\"packets\":%llu,\"events\":%llu,\"prop_cells\":%llu,\"locate_cells\":%llu,"
             "\"peel_cells\":%llu,\"peel_adds\":%llu,\"peel_dropped\":%llu,\"capped\":%llu,"
             "\"guard\":%llu,\"nonfinite\":%llu,\"kernel_ms\":%.9g,\"packets_per_s\":%.9g,"
             "\"deposits_per_s\":%.9g,\"algorithmic_bytes\":%.9g,\"achieved_GBps\":%.9g,"
             "\"hbm_frac\":%.9g,\"rc\":%d}\n",
             entry, s0->ctx->device, s0->medium->grid->type == kOctree ? "octree" : "cartesian", n, cells, n_lambda,
             n_ins, fp32 ? "fp32" : "fp64", s0->prop ? "true" : "false", (unsigned long long)n_per_lambda,
             (unsigned long long)first_id, (unsigned long long)count, (unsigned long long)seed, d[0], d[1], d[2],
             d[3], d[4], d[5], d[6], d[7], d[8], d[9], kernel_ms, (double)d[0] * per_s,
             (double)(d[2] + d[5]) * per_s, bytes, bytes * per_s * 1e-9, bytes * per_s * 1e-9 / kHbmPeakGBs, rc);
    std::lock_guard<std::mutex> lock(g_log_mu);
    const char *path = std::getenv("MCRT_LOG_FILE");
    if (path && *path) {
        if (FILE *f = std::fopen(path, "a")) {
            std::fputs(buf, f);
            std::fclose(f);
        }
    } else {
        std::fputs(buf, stderr);
        std::fflush(stderr);
    }
}

} // namespace

// Definitions of the functions declared extern "C" in mcrt.h (they keep C
// linkage from that declaration).

const char *mcrt_last_error(void) { return g_err.c_str(); }

void mcrt_options_default(mcrt_options *opt)
{
    if (!opt) return;
    opt->precision = MCRT_FP32;
    opt->w_min = 1e-6;
    opt->event_cap = 10000;
    opt->tau_peel_max = HUGE_VAL;
    opt->chunk = 0;
    opt->waves_per_cu = 0;
    opt->threshold = 0;
    opt->top_level = -1;
    opt->brick[0] = opt->brick[1] = opt->brick[2] = -1;
    opt->queue_order = MCRT_QUEUE_PAIRED;
    opt->chunk_shift = 0;
    opt->deposit_slots = 0;
}

int mcrt_context_create(int device, void *stream, mcrt_context **out)
{
    if (!out) return fail(MCRT_EINVAL, "context_create: out is NULL");
    *out = nullptr;
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(MCRT_EINVAL, "context_create: no such device");
    HIP_TRY(hipSetDevice(device));
    // the device address of this device's allocation-free scratch, once
    const hipError_t se = noalloc_scratch_setup(device);
    if (se != hipSuccess)
        return fail(MCRT_EDEVICE, std::string("context_create: scratch address: ") + hipGetErrorString(se));
    int ncu = 0;
    HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device));
    auto *c = new mcrt_context;
    c->device = device;
    c->stream = (hipStream_t)stream;
    c->n_cu = ncu > 0 ? ncu : 1;
    *out = c;
    return MCRT_OK;
}

void mcrt_context_destroy(mcrt_context *ctx) { delete ctx; }

int mcrt_grid_create_cartesian(mcrt_context *ctx, const double box[6], const int32_t n[3], mcrt_grid **out)
{
    if (!out) return fail(MCRT_EINVAL, "grid_create_cartesian: out is NULL");
    *out = nullptr;
    if (!ctx || !box || !n) return fail(MCRT_EINVAL, "grid_create_cartesian: NULL argument");
    if (!finite_box(box)) return fail(MCRT_EINVAL, "grid_create_cartesian: box must have min < max, finite");
    int64_t cells = 1;
    for (int a = 0; a < 3; ++a) {
        if (n[a] <= 0) return fail(MCRT_EINVAL, "grid_create_cartesian: cell counts must be positive");
        cells *= n[a];
    }
    if (cells >= (int64_t(1) << 31)) return fail(MCRT_EINVAL, "grid_create_cartesian: more than 2^31-1 cells");
    auto *g = new mcrt_grid;
    g->ctx = ctx;
    g->type = kCartesian;
    std::memcpy(g->box, box, sizeof(g->box));
    for (int a = 0; a < 3; ++a) g->n[a] = n[a];
    g->n_cells = cells;
    *out = g;
    return MCRT_OK;
}

int mcrt_grid_create_octree(mcrt_context *ctx, const double box[6], int64_t n_nodes, const int32_t *first_child,
                            mcrt_grid **out)
{
    if (!out) return fail(MCRT_EINVAL, "grid_create_octree: out is NULL");
    *out = nullptr;
    if (!ctx || !box || !first_child) return fail(MCRT_EINVAL, "grid_create_octree: NULL argument");
    if (!finite_box(box)) return fail(MCRT_EINVAL, "grid_create_octree: box must have min < max, finite");
    if (n_nodes <= 0 || n_nodes >= (int64_t(1) << 27)) return fail(MCRT_EINVAL, "grid_create_octree: node count out of range");
    int64_t leaves = 0;
    for (int64_t i = 0; i < n_nodes; ++i)
        if (first_child[i] < 0) leaves++;
    std::vector<int32_t> node;
    std::string err;
    int depth = encode_octree(n_nodes, first_child, leaves, node, err);
    if (depth < 0) return fail(MCRT_EINVAL, "grid_create_octree: " + err);
    auto *g = new mcrt_grid;
    g->ctx = ctx;
    g->type = kOctree;
    std::memcpy(g->box, box, sizeof(g->box));
    g->depth = depth;
    for (int a = 0; a < 3; ++a) g->n[a] = 1 << depth;
    g->n_cells = leaves;
    g->first_child.assign(first_child, first_child + n_nodes);
    *out = g;
    return MCRT_OK;
}

void mcrt_grid_destroy(mcrt_grid *grid) { delete grid; }

int mcrt_medium_create(mcrt_grid *grid, const float *density, int32_t n_lambda, const double *lambda_um,
                       const double *kappa, const double *albedo, const double *g, mcrt_medium **out)
{
    if (!out) return fail(MCRT_EINVAL, "medium_create: out is NULL");
    *out = nullptr;
    if (!grid || !density || !kappa || !albedo || !g) return fail(MCRT_EINVAL, "medium_create: NULL argument");
    if (n_lambda <= 0 || n_lambda > (1 << 20)) return fail(MCRT_EINVAL, "medium_create: n_lambda out of range");
    for (int64_t i = 0; i < grid->n_cells; ++i)
        if (!(density[i] >= 0.0f) || !std::isfinite(density[i]))
            return fail(MCRT_EINVAL, "medium_create: densities must be finite and non-negative");
    for (int l = 0; l < n_lambda; ++l) {
        if (!(kappa[l] >= 0.0) || !std::isfinite(kappa[l])) return fail(MCRT_EINVAL, "medium_create: kappa must be finite, >= 0");
        if (!(albedo[l] >= 0.0 && albedo[l] <= 1.0)) return fail(MCRT_EINVAL, "medium_create: albedo must lie in [0, 1]");
        if (!(g[l] > -1.0 && g[l] < 1.0)) return fail(MCRT_EINVAL, "medium_create: g must lie in (-1, 1)");
    }
    auto *m = new mcrt_medium;
    m->grid = grid;
    m->density.assign(density, density + grid->n_cells);
    m->n_lambda = n_lambda;
    m->kappa.assign(kappa, kappa + n_lambda);
    m->albedo.assign(albedo, albedo + n_lambda);
    m->g.assign(g, g + n_lambda);
    if (lambda_um) {
        for (int l = 0; l < n_lambda; ++l)
            if (!(lambda_um[l] > 0.0) || !std::isfinite(lambda_um[l])) {
                delete m;
                return fail(MCRT_EINVAL, "medium_create: wavelengths must be positive");
            }
        m->lambda_um.assign(lambda_um, lambda_um + n_lambda);
    }
    *out = m;
    return MCRT_OK;
}

void mcrt_medium_destroy(mcrt_medium *medium) { delete medium; }

static int check_lum(int32_t n_lambda, const double *L)
{
    if (n_lambda <= 0 || !L) return fail(MCRT_EINVAL, "source: n_lambda must be positive and L non-NULL");
    for (int l = 0; l < n_lambda; ++l)
        if (!(L[l] >= 0.0) || !std::isfinite(L[l])) return fail(MCRT_EINVAL, "source: luminosities must be finite, >= 0");
    return MCRT_OK;
}

int mcrt_source_create_point(mcrt_context *ctx, const double pos[3], int32_t aniso, int32_t n_lambda, const double *L,
                             mcrt_source **out)
{
    if (!out) return fail(MCRT_EINVAL, "source_create_point: out is NULL");
    *out = nullptr;
    if (!ctx || !pos) return fail(MCRT_EINVAL, "source_create_point: NULL argument");
    if (aniso != 0 && aniso != 1) return fail(MCRT_EINVAL, "source_create_point: aniso must be 0 or 1");
    int rc = check_lum(n_lambda, L);
    if (rc) return rc;
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(pos[a])) return fail(MCRT_EINVAL, "source_create_point: position must be finite");
    auto *s = new mcrt_source;
    s->ctx = ctx;
    s->type = aniso ? kPointAniso : kPointIso;
    std::memcpy(s->pos, pos, sizeof(s->pos));
    s->L.assign(L, L + n_lambda);
    *out = s;
    return MCRT_OK;
}

int mcrt_source_create_expdisk(mcrt_context *ctx, double hR, double zs, int32_t n_lambda, const double *L,
                               mcrt_source **out)
{
    if (!out) return fail(MCRT_EINVAL, "source_create_expdisk: out is NULL");
    *out = nullptr;
    if (!ctx) return fail(MCRT_EINVAL, "source_create_expdisk: NULL context");
    if (!(hR > 0.0) || !(zs > 0.0) || !std::isfinite(hR) || !std::isfinite(zs))
        return fail(MCRT_EINVAL, "source_create_expdisk: scales must be positive");
    int rc = check_lum(n_lambda, L);
    if (rc) return rc;
    auto *s = new mcrt_source;
    s->ctx = ctx;
    s->type = kExpDisk;
    s->hR = hR;
    s->zs = zs;
    s->L.assign(L, L + n_lambda);
    *out = s;
    return MCRT_OK;
}

void mcrt_source_destroy(mcrt_source *src) { delete src; }

int mcrt_instrument_create(mcrt_context *ctx, double incl_deg, double azim_deg, double distance, const double fov[2],
                           const int32_t npix[2], mcrt_instrument **out)
{
    if (!out) return fail(MCRT_EINVAL, "instrument_create: out is NULL");
    *out = nullptr;
    if (!ctx || !fov || !npix) return fail(MCRT_EINVAL, "instrument_create: NULL argument");
    if (!(distance > 0.0) || !std::isfinite(distance)) return fail(MCRT_EINVAL, "instrument_create: distance must be positive");
    if (!std::isfinite(incl_deg) || !std::isfinite(azim_deg)) return fail(MCRT_EINVAL, "instrument_create: angles must be finite");
    for (int a = 0; a < 2; ++a) {
        if (!(fov[a] > 0.0) || !std::isfinite(fov[a])) return fail(MCRT_EINVAL, "instrument_create: field of view must be positive");
        if (npix[a] <= 0 || npix[a] > 65536) return fail(MCRT_EINVAL, "instrument_create: pixel counts must be in 1 .. 65536");
    }
    auto *i = new mcrt_instrument;
    i->ctx = ctx;
    i->h = HostInstrument{incl_deg, azim_deg, distance, {fov[0], fov[1]}, {npix[0], npix[1]}};
    *out = i;
    return MCRT_OK;
}

void mcrt_instrument_destroy(mcrt_instrument *ins) { delete ins; }

static void sim_free_device(mcrt_sim *s)
{
    dev_free(s->d_density);
    dev_free(s->d_node);
    dev_free(s->d_top);
    dev_free(s->d_optics);
    dev_free(s->d_optics_base);
    dev_free(s->d_lum);
    dev_free(s->d_ins);
    for (int j = 0; j < kMaxIns; ++j) {
        dev_free(s->d_col[j]);
        s->d_col[j] = nullptr;
    }
    s->d_density = nullptr;
    s->d_node = nullptr;
    s->d_top = nullptr;
    s->d_optics = nullptr;
    s->d_optics_base = nullptr;
    s->d_lum = nullptr;
    s->d_ins = nullptr;
}

void mcrt_sim_destroy(mcrt_sim *sim)
{
    if (!sim) return;
    (void)hipSetDevice(sim->ctx->device);
    sim_free_device(sim);
    delete sim;
}

template <typename Real> static int upload_instruments(mcrt_sim *s)
{
    std::vector<InsDesc<Real>> d((size_t)std::max(s->n_ins, 1));
    const mcrt_grid *g = s->medium->grid;
    // octree lattice column maps need the encoded tree (depth <= 10: at most
    // 2^30 lattice cells per map)
    std::vector<int32_t> onode;
    if (g->type == kOctree && s->depth <= kMaxColumnDepth) {
        std::string err;
        if (encode_octree((int64_t)g->first_child.size(), g->first_child.data(), g->n_cells, onode, err) < 0)
            return fail(MCRT_EINVAL, "sim_create: " + err);
    }
    for (int j = 0; j < s->n_ins; ++j) {
        make_ins_desc<Real>(s->ins[j], s->ins_offset[j], d[j], s->inv4pid2[j]);
        const int code = (g->type == kCartesian || !onode.empty()) ? axis_code(s->ins[j]) : -1;
        if (code < 0) continue;
        std::vector<Real> Sr;
        if (g->type == kCartesian) {
            std::vector<double> S;
            column_map(s->medium->density.data(), g->n, g->box, code, s->bs, s->sh, s->nb, s->n_store, S);
            Sr.assign(S.begin(), S.end());
        } else {
            octree_column_map<Real>(onode, s->depth, g->n_cells, s->medium->density.data(), g->box, code, Sr);
        }
        int rc = dev_alloc(&s->d_col[j], Sr.size() * sizeof(Real));
        if (rc) return rc;
        HIP_TRY(hipMemcpy(s->d_col[j], Sr.data(), Sr.size() * sizeof(Real), hipMemcpyHostToDevice));
        d[j].col = (const Real *)s->d_col[j];
        d[j].col_axis = code;
    }
    int rc = dev_alloc(&s->d_ins, d.size() * sizeof(InsDesc<Real>));
    if (rc) return rc;
    HIP_TRY(hipMemcpy(s->d_ins, d.data(), d.size() * sizeof(InsDesc<Real>), hipMemcpyHostToDevice));
    const int nl = s->medium->n_lambda;
    rc = dev_alloc(&s->d_optics, (size_t)nl * sizeof(Optics<Real>));
    // device copies the allocation-free run prepares its optics from
    std::vector<Optics<Real>> base((size_t)nl);
    for (int l = 0; l < nl; ++l) {
        base[l].kappa = (Real)s->medium->kappa[l];
        base[l].albedo = (Real)s->medium->albedo[l];
        base[l].g = (Real)s->medium->g[l];
        base[l].L0 = Real(0);
        base[l].lamf = (Real)s->lamf[l];
    }
    if (!rc) rc = dev_alloc(&s->d_optics_base, (size_t)nl * sizeof(Optics<Real>));
    if (!rc) rc = dev_alloc((void **)&s->d_lum, (size_t)nl * sizeof(double));
    if (rc) return rc;
    HIP_TRY(hipMemcpy(s->d_optics_base, base.data(), base.size() * sizeof(Optics<Real>), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(s->d_lum, s->source->L.data(), (size_t)nl * sizeof(double), hipMemcpyHostToDevice));
    return MCRT_OK;
}

int mcrt_sim_create(mcrt_context *ctx, mcrt_medium *medium, mcrt_source *source, mcrt_instrument *const *ins,
                    int32_t n_ins, const mcrt_options *opt, mcrt_sim **out)
{
    if (!out) return fail(MCRT_EINVAL, "sim_create: out is NULL");
    *out = nullptr;
    if (!ctx || !medium || !source) return fail(MCRT_EINVAL, "sim_create: NULL argument");
    if (n_ins < 0 || n_ins > kMaxIns || (n_ins > 0 && !ins))
        return fail(MCRT_EINVAL, "sim_create: 0 .. 8 instruments");
    if ((int)source->L.size() != medium->n_lambda)
        return fail(MCRT_EINVAL, "sim_create: source and medium disagree on n_lambda");
    mcrt_options o;
    mcrt_options_default(&o);
    if (opt) o = *opt;
    if (o.precision != MCRT_FP32 && o.precision != MCRT_FP64_VALIDATE)
        return fail(MCRT_EINVAL, "sim_create: unknown precision");
    if (!(o.w_min >= 0.0) || !(o.tau_peel_max > 0.0) || o.event_cap < 1)
        return fail(MCRT_EINVAL, "sim_create: w_min >= 0, tau_peel_max > 0, event_cap >= 1 required");
    if (o.chunk < 0 || o.waves_per_cu < 0 || o.waves_per_cu > 32 || o.threshold < 0 || o.threshold > 64 ||
        o.chunk_shift < -6 || o.chunk_shift > 6 || (o.deposit_slots != 0 && o.deposit_slots != 8 &&
                                                    o.deposit_slots != 16))
        return fail(MCRT_EINVAL, "sim_create: tuning values out of range");
    if (o.queue_order != MCRT_QUEUE_COST && o.queue_order != MCRT_QUEUE_CALLER && o.queue_order != MCRT_QUEUE_PAIRED)
        return fail(MCRT_EINVAL, "sim_create: unknown queue order");
    if (o.brick[0] >= 0 || o.brick[1] >= 0 || o.brick[2] >= 0) {
        if (o.brick[0] < 0 || o.brick[1] < 0 || o.brick[2] < 0 || o.brick[0] + o.brick[1] + o.brick[2] != 5)
            return fail(MCRT_EINVAL, "sim_create: brick log2 sizes must be >= 0 and sum to 5");
    }
    HIP_TRY(hipSetDevice(ctx->device));
    auto *s = new mcrt_sim;
    s->ctx = ctx;
    s->medium = medium;
    s->source = source;
    s->n_ins = n_ins;
    s->opt = o;
    long long off = 0;
    for (int j = 0; j < n_ins; ++j) {
        if (!ins[j]) {
            delete s;
            return fail(MCRT_EINVAL, "sim_create: NULL instrument");
        }
        s->ins[j] = ins[j]->h;
        s->ins_offset[j] = off;
        off += (long long)medium->n_lambda * ins[j]->h.npix[0] * ins[j]->h.npix[1];
    }
    s->image_elems = off;
    const mcrt_grid *g = medium->grid;
    feature_constants(g->box, medium->density.data(), g->n_cells,
                      medium->lambda_um.empty() ? nullptr : medium->lambda_um.data(), medium->n_lambda, s->r_out,
                      s->rho_mean, s->lamf);
    std::vector<float> stored;
    const float *dens = medium->density.data();
    s->n_store = g->n_cells;
    if (g->type == kCartesian) {
        double cs[3];
        for (int a = 0; a < 3; ++a) cs[a] = (g->box[3 + a] - g->box[a]) / (double)g->n[a];
        choose_bricks(cs, g->n, s->bs, s->sh, s->nb, s->n_store);
        if (o.brick[0] >= 0) {
            s->n_store = 32;
            for (int a = 0; a < 3; ++a) {
                s->bs[a] = o.brick[a];
                s->nb[a] = (g->n[a] + (1 << s->bs[a]) - 1) >> s->bs[a];
                s->n_store *= s->nb[a];
            }
            default_shifts(s->bs, s->sh);
        }
        if (s->n_store >= (1ll << 31)) {
            delete s;
            return fail(MCRT_EINVAL, "sim_create: bricked grid exceeds 2^31 cells");
        }
        stored.assign((size_t)s->n_store, 0.0f);
        for (int iz = 0; iz < g->n[2]; ++iz)
            for (int iy = 0; iy < g->n[1]; ++iy)
                for (int ix = 0; ix < g->n[0]; ++ix)
                    stored[(size_t)store_index_host(s->bs, s->sh, s->nb, ix, iy, iz)] =
                        dens[ix + (size_t)g->n[0] * (iy + (size_t)g->n[1] * iz)];
        dens = stored.data();
    }
    int rc = dev_alloc((void **)&s->d_density, (size_t)s->n_store * sizeof(float));
    if (!rc) {
        hipError_t e = hipMemcpy(s->d_density, dens, (size_t)s->n_store * sizeof(float), hipMemcpyHostToDevice);
        if (e != hipSuccess) rc = fail(MCRT_EDEVICE, std::string("density upload: ") + hipGetErrorString(e));
    }
    if (!rc && g->type == kOctree) {
        std::vector<int32_t> node;
        std::string err;
        int depth = encode_octree((int64_t)g->first_child.size(), g->first_child.data(), g->n_cells, node, err);
        s->depth = depth;
        s->top_level = o.top_level >= 0 ? std::min(o.top_level, depth) : std::min(depth, 7);
        std::vector<uint64_t> top, blocks;
        if (!build_walk(node, depth, s->top_level, dens, top, blocks, err)) rc = fail(MCRT_EINVAL, err);
        if (blocks.empty()) blocks.assign(1, 0);
        if (!rc) rc = dev_alloc((void **)&s->d_node, blocks.size() * sizeof(uint64_t));
        if (!rc) rc = dev_alloc((void **)&s->d_top, top.size() * sizeof(uint64_t));
        if (!rc) {
            hipError_t e = hipMemcpy(s->d_node, blocks.data(), blocks.size() * sizeof(uint64_t), hipMemcpyHostToDevice);
            if (e == hipSuccess) e = hipMemcpy(s->d_top, top.data(), top.size() * sizeof(uint64_t), hipMemcpyHostToDevice);
            if (e != hipSuccess) rc = fail(MCRT_EDEVICE, std::string("octree upload: ") + hipGetErrorString(e));
        }
    }
    if (!rc) rc = o.precision == MCRT_FP32 ? upload_instruments<float>(s) : upload_instruments<double>(s);
    if (rc) {
        sim_free_device(s);
        delete s;
        return rc;
    }
    *out = s;
    return MCRT_OK;
}

int mcrt_sim_info(const mcrt_sim *sim, int64_t *n_cells, int32_t *n_lambda, int32_t *n_ins)
{
    if (!sim) return fail(MCRT_EINVAL, "sim_info: NULL sim");
    if (n_cells) *n_cells = sim->medium->grid->n_cells;
    if (n_lambda) *n_lambda = sim->medium->n_lambda;
    if (n_ins) *n_ins = sim->n_ins;
    return MCRT_OK;
}

static size_t image_bytes(const mcrt_sim *s)
{
    return (size_t)s->image_elems * (s->opt.precision == MCRT_FP32 ? sizeof(float) : sizeof(double));
}

static size_t table_elems(const mcrt_sim *s) { return (size_t)s->n_store * (size_t)s->medium->n_lambda; }

void mcrt_result_destroy(mcrt_result *res)
{
    if (!res) return;
    (void)hipSetDevice(res->sim->ctx->device);
    dev_free(res->d_table);
    dev_free(res->d_images);
    dev_free(res->d_energy);
    dev_free(res->d_stats);
    dev_free(res->d_counter);
    delete res;
}

int mcrt_result_zero(mcrt_result *res)
{
    if (!res) return fail(MCRT_EINVAL, "result_zero: NULL result");
    const mcrt_sim *s = res->sim;
    HIP_TRY(hipSetDevice(s->ctx->device));
    hipStream_t st = s->ctx->stream;
    HIP_TRY(launch_fill_zero(res->d_table, table_elems(s) * sizeof(double), st));
    HIP_TRY(launch_fill_zero(res->d_images, image_bytes(s), st));
    HIP_TRY(launch_fill_zero(res->d_energy, 4 * sizeof(double), st));
    HIP_TRY(launch_fill_zero(res->d_stats, kNumStats * sizeof(unsigned long long), st));
    HIP_TRY(hipStreamSynchronize(st));
    res->kernel_ms = 0.0;
    std::fill(res->seen, res->seen + kNumStats, 0ull);
    return MCRT_OK;
}

int mcrt_result_create(mcrt_sim *sim, mcrt_result **out)
{
    if (!out) return fail(MCRT_EINVAL, "result_create: out is NULL");
    *out = nullptr;
    if (!sim) return fail(MCRT_EINVAL, "result_create: NULL sim");
    HIP_TRY(hipSetDevice(sim->ctx->device));
    auto *r = new mcrt_result;
    r->sim = sim;
    int rc = dev_alloc((void **)&r->d_table, table_elems(sim) * sizeof(double));
    if (!rc) rc = dev_alloc(&r->d_images, image_bytes(sim));
    if (!rc) rc = dev_alloc((void **)&r->d_energy, 4 * sizeof(double));
    if (!rc) rc = dev_alloc((void **)&r->d_stats, kNumStats * sizeof(unsigned long long));
    if (!rc) rc = dev_alloc((void **)&r->d_counter, sizeof(unsigned long long));
    if (!rc) rc = mcrt_result_zero(r);
    if (rc) {
        std::string msg = g_err;
        mcrt_result_destroy(r);
        g_err = msg;
        return rc;
    }
    *out = r;
    return MCRT_OK;
}

template <typename Real, typename ImgT, int G>
static int run_impl(mcrt_sim *s, uint64_t n_per_lambda, uint64_t first_id, uint64_t count, uint64_t seed,
                    mcrt_result *r, mcrt_histories *hist = nullptr, const mcrt_dust *dust = nullptr,
                    void *scratch = nullptr)
{
    const mcrt_medium *m = s->medium;
    const mcrt_grid *g = m->grid;
    hipStream_t st = s->ctx->stream;
    if (scratch) {
        // allocation-free: counter and optics in the device's scratch array,
        // prepared on the device (no host buffer, no copy from the host)
        HIP_TRY(launch_noalloc_setup<Real>(scratch, (const Optics<Real> *)s->d_optics_base, s->d_lum, m->n_lambda,
                                           n_per_lambda, st));
    } else {
        std::vector<Optics<Real>> optics((size_t)m->n_lambda);
        for (int l = 0; l < m->n_lambda; ++l) {
            optics[l].kappa = (Real)m->kappa[l];
            optics[l].albedo = (Real)m->albedo[l];
            optics[l].g = (Real)m->g[l];
            optics[l].L0 = (Real)((dust ? dust->L[l] : s->source->L[l]) / (double)n_per_lambda);
            optics[l].lamf = (Real)s->lamf[l];
        }
        HIP_TRY(hipMemcpyAsync(s->d_optics, optics.data(), optics.size() * sizeof(Optics<Real>),
                               hipMemcpyHostToDevice, st));
        HIP_TRY(launch_fill_zero(r->d_counter, sizeof(unsigned long long), st));
    }

    TransportArgs<Real, ImgT, G> a{};
    View<Real, ImgT, G> &v = a.view;
    for (int c = 0; c < 3; ++c) {
        v.bs[c] = s->bs[c];
        v.sh[c] = s->sh[c];
        v.nb[c] = s->nb[c];
        v.n[c] = g->n[c];
        v.lo[c] = (Real)g->box[c];
        v.hi[c] = (Real)g->box[3 + c];
        v.cs[c] = (Real)((g->box[3 + c] - g->box[c]) / (double)g->n[c]);
        v.ics[c] = (Real)((double)g->n[c] / (g->box[3 + c] - g->box[c]));
    }
    v.depth = s->depth;
    v.top_level = s->top_level;
    v.density = s->d_density;
    v.node = s->d_node;
    v.top = s->d_top;
    v.n_cells = g->n_cells;
    v.n_store = s->n_store;
    v.n_lambda = m->n_lambda;
    v.optics = nullptr;
    v.src_type = dust ? (int)kDust : s->source->type;
    if (dust) {
        v.dust_cdf = dust->d_cdf;
        v.dust_guide = dust->d_guide;
        v.dust_K = dust->K;
        v.dust_leaf = dust->d_leaf;
    }
    for (int c = 0; c < 3; ++c) v.src_pos[c] = (Real)s->source->pos[c];
    v.hR = (Real)s->source->hR;
    v.zs = (Real)s->source->zs;
    v.n_ins = s->n_ins;
    v.ins = nullptr;
    v.table = r->d_table;
    v.images = (ImgT *)r->d_images;
    v.w_min = (Real)s->opt.w_min;
    v.event_cap = s->opt.event_cap;
    v.tau_peel_max = (Real)s->opt.tau_peel_max;
    v.octree_guard = 16 * 3 * (1 << s->depth) + 64;
    v.key0 = (uint32_t)(seed & 0xffffffffu);
    v.key1 = (uint32_t)(seed >> 32);
    v.model = 0;
    v.r_out = (Real)s->r_out;
    v.rho_mean = (Real)s->rho_mean;
    if (s->prop) {
        v.learned = 1;
        v.alpha = (Real)s->alpha;
        v.mlp64 = s->prop->d_theta64;
        a.mlp_frags = s->prop->d_frags;
        a.mlp_bias = s->prop->d_bias;
    }
    if (hist) {
        v.hist = (Real *)hist->d_hist;
        v.hist_total = (Real *)hist->d_total;
        v.hist_events = hist->events;
    }
    a.optics = scratch ? (const Optics<Real> *)((const unsigned char *)scratch + kNoAllocHeader)
                       : (const Optics<Real> *)s->d_optics;
    a.ins = (const InsDesc<Real> *)s->d_ins;
    a.count = count;
    a.first_id = first_id;
    a.total = count * (uint64_t)m->n_lambda;
    int wpc = s->opt.waves_per_cu > 0 ? s->opt.waves_per_cu : 16;
    uint64_t waves = (uint64_t)s->ctx->n_cu * (uint64_t)wpc;
    // default chunk: 256 packets, smaller for small launches so that every
    // persistent wave gets work (never below 32)
    uint64_t auto_chunk = a.total / waves;
    auto_chunk = auto_chunk < 32 ? 32 : (auto_chunk > 256 ? 256 : auto_chunk);
    a.chunk = (uint32_t)(s->opt.chunk > 0 ? (uint64_t)s->opt.chunk : shifted_chunk(auto_chunk, s->opt.chunk_shift));
    a.threshold = s->opt.threshold > 0 ? s->opt.threshold : 16;
    a.counter = scratch ? (unsigned long long *)scratch : r->d_counter;
    a.energy = r->d_energy;
    a.stats = r->d_stats;
    uint64_t chunks = (a.total + a.chunk - 1) / a.chunk;
    if (waves > chunks) waves = chunks;
    int grid = (int)((waves + (kBlock / 64) - 1) / (kBlock / 64));
    if (grid < 1) grid = 1;

    auto launch = [&]() -> hipError_t {
        if constexpr (sizeof(Real) == 4 && G == kCartesian) return launch_transport_f32c(a, grid, st);
        else if constexpr (sizeof(Real) == 4) return launch_transport_f32o(a, grid, st);
        else if constexpr (G == kCartesian) return launch_transport_f64c(a, grid, st);
        else return launch_transport_f64o(a, grid, st);
    };
    if (scratch) {
        // no events (creating them allocates): the launch is not timed
        HIP_TRY(launch());
        HIP_TRY(hipStreamSynchronize(st));
        r->kernel_ms = 0.0;
    } else {
        EventPair ev;
        HIP_TRY(hipEventCreate(&ev.e0));
        HIP_TRY(hipEventCreate(&ev.e1));
        HIP_TRY(hipEventRecord(ev.e0, st));
        HIP_TRY(launch());
        HIP_TRY(hipEventRecord(ev.e1, st));
        HIP_TRY(hipEventSynchronize(ev.e1));
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, ev.e0, ev.e1));
        r->kernel_ms = ms;
    }
    unsigned long long stats[kNumStats];
    Counters delta;
    HIP_TRY(hipMemcpy(stats, r->d_stats, sizeof(stats), hipMemcpyDeviceToHost));
    const int rc = launch_outcome(r, stats, delta.v);
    if (!scratch)
        log_launch(hist ? "proposal_collect" : (dust ? "run_dust_into" : "run_into"), &s, 1, &delta, n_per_lambda,
                   first_id, count, seed, r->kernel_ms, rc);
    return rc;
}

namespace {
struct BusyGuard {
    std::atomic<int> &flag;
    bool owned;
    explicit BusyGuard(std::atomic<int> &f) : flag(f)
    {
        int expect = 0;
        owned = flag.compare_exchange_strong(expect, 1);
    }
    ~BusyGuard()
    {
        if (owned) flag.store(0);
    }
};
} // namespace

int mcrt_run_into(mcrt_sim *sim, uint64_t n_per_lambda, uint64_t first_id, uint64_t count, uint64_t seed,
                  mcrt_result *res)
{
    if (!sim || !res) return fail(MCRT_EINVAL, "run_into: NULL sim or result");
    if (res->sim != sim) return fail(MCRT_EINVAL, "run_into: result belongs to another sim");
    if (n_per_lambda == 0 || n_per_lambda > (uint64_t(1) << 32))
        return fail(MCRT_EINVAL, "run_into: n_per_lambda must be in 1 .. 2^32");
    if (first_id > n_per_lambda || count > n_per_lambda - first_id)
        return fail(MCRT_EINVAL, "run_into: id range exceeds n_per_lambda");
    BusyGuard guard(sim->busy);
    if (!guard.owned) return fail(MCRT_EBUSY, "run_into: the simulation is already running");
    if (count == 0) return MCRT_OK;
    HIP_TRY(hipSetDevice(sim->ctx->device));
    const bool oct = sim->medium->grid->type == kOctree;
    if (sim->opt.precision == MCRT_FP32) {
        if (oct) return run_impl<float, float, kOctree>(sim, n_per_lambda, first_id, count, seed, res);
        return run_impl<float, float, kCartesian>(sim, n_per_lambda, first_id, count, seed, res);
    }
    if (oct) return run_impl<double, double, kOctree>(sim, n_per_lambda, first_id, count, seed, res);
    return run_impl<double, double, kCartesian>(sim, n_per_lambda, first_id, count, seed, res);
}

int mcrt_run_into_noalloc(mcrt_sim *sim, uint64_t n_per_lambda, uint64_t first_id, uint64_t count, uint64_t seed,
                          mcrt_result *res)
{
    if (!sim || !res) return fail(MCRT_EINVAL, "run_into_noalloc: NULL sim or result");
    if (res->sim != sim) return fail(MCRT_EINVAL, "run_into_noalloc: result belongs to another sim");
    if (n_per_lambda == 0 || n_per_lambda > (uint64_t(1) << 32))
        return fail(MCRT_EINVAL, "run_into_noalloc: n_per_lambda must be in 1 .. 2^32");
    if (first_id > n_per_lambda || count > n_per_lambda - first_id)
        return fail(MCRT_EINVAL, "run_into_noalloc: id range exceeds n_per_lambda");
    if (sim->medium->n_lambda > kNoAllocMaxLambda)
        return fail(MCRT_EINVAL, "run_into_noalloc: at most 4096 wavelengths (the scratch array's size)");
    BusyGuard guard(sim->busy);
    if (!guard.owned) return fail(MCRT_EBUSY, "run_into_noalloc: the simulation is already running");
    if (count == 0) return MCRT_OK;
    HIP_TRY(hipSetDevice(sim->ctx->device));
    void *scratch = noalloc_scratch(sim->ctx->device);
    if (!scratch) return fail(MCRT_EDEVICE, "run_into_noalloc: no scratch address for this device");
    const bool oct = sim->medium->grid->type == kOctree;
    if (sim->opt.precision == MCRT_FP32) {
        if (oct) return run_impl<float, float, kOctree>(sim, n_per_lambda, first_id, count, seed, res, nullptr,
                                                         nullptr, scratch);
        return run_impl<float, float, kCartesian>(sim, n_per_lambda, first_id, count, seed, res, nullptr, nullptr,
                                                  scratch);
    }
    if (oct) return run_impl<double, double, kOctree>(sim, n_per_lambda, first_id, count, seed, res, nullptr,
                                                       nullptr, scratch);
    return run_impl<double, double, kCartesian>(sim, n_per_lambda, first_id, count, seed, res, nullptr, nullptr,
                                                scratch);
}

// ---------------------------------------------------------------------------
// Dust emission phase (Section 3.2): emission of a Cartesian sim's cells from
// the absorbed luminosity of one or more of its results, and runs of dust
// packets.
// ---------------------------------------------------------------------------
void mcrt_dust_params_default(mcrt_dust_params *p)
{
    if (!p) return;
    p->T0 = 20.0;
    p->beta = 2.0;
}

void mcrt_dust_destroy(mcrt_dust *d)
{
    if (!d) return;
    (void)hipSetDevice(d->sim->ctx->device);
    dev_free(d->d_cdf);
    dev_free(d->d_guide);
    dev_free(d->d_T);
    dev_free(d->d_leaf);
    delete d;
}

int mcrt_dust_create(mcrt_sim *sim, const mcrt_result *const *absorbed, int32_t n, const mcrt_dust_params *params,
                     mcrt_dust **out)
{
    if (!sim || !out || (n > 0 && !absorbed)) return fail(MCRT_EINVAL, "dust_create: NULL argument");
    *out = nullptr;
    if (n < 1 || n > 4) return fail(MCRT_EINVAL, "dust_create: between 1 and 4 absorption results");
    const mcrt_medium *m = sim->medium;
    const mcrt_grid *g = m->grid;
    if ((int)m->lambda_um.size() != m->n_lambda)
        return fail(MCRT_EINVAL, "dust_create: the medium was created without wavelengths");
    // results of sim, or of another sim on the device whose table has the
    // same layout (e.g. an FP64 validation run of the same scene)
    auto same_layout = [&](const mcrt_sim *o) {
        if (o == sim) return true;
        const mcrt_grid *og = o->medium->grid;
        bool same = o->ctx->device == sim->ctx->device && og->type == g->type && og->n_cells == g->n_cells &&
                    o->medium->n_lambda == m->n_lambda && o->n_store == sim->n_store;
        for (int a = 0; a < 3; ++a)
            same = same && og->n[a] == g->n[a] && o->bs[a] == sim->bs[a] && o->sh[a] == sim->sh[a] &&
                   o->nb[a] == sim->nb[a];
        return same;
    };
    for (int i = 0; i < n; ++i) {
        if (!absorbed[i]) return fail(MCRT_EINVAL, "dust_create: NULL result");
        if (!same_layout(absorbed[i]->sim))
            return fail(MCRT_EINVAL, "dust_create: result of a sim with another table layout or device");
    }
    mcrt_dust_params p;
    mcrt_dust_params_default(&p);
    if (params) p = *params;
    if (!(p.T0 > 0.0) || !std::isfinite(p.T0) || !(p.beta > -4.0) || !std::isfinite(p.beta))
        return fail(MCRT_EINVAL, "dust_create: T0 must be positive and beta > -4");
    if (g->n_cells >= (int64_t(1) << 31)) return fail(MCRT_EINVAL, "dust_create: too many cells");
    if (m->n_lambda > 65535) return fail(MCRT_EINVAL, "dust_create: at most 65535 wavelengths");
    HIP_TRY(hipSetDevice(sim->ctx->device));
    hipStream_t st = sim->ctx->stream;
    const int nl = m->n_lambda;
    const long long nc = g->n_cells;
    mcrt_dust *d = new mcrt_dust();
    d->sim = sim;
    d->params = p;
    d->K = (int)std::min<long long>(std::max<long long>(nc / 16, 1), 1 << 16);
    // bin widths between the geometric means of neighbouring wavelengths
    std::vector<double> kw((size_t)nl);
    const std::vector<double> &lam = m->lambda_um;
    for (int l = 0; l < nl; ++l) {
        double w;
        if (nl == 1) {
            w = lam[0];
        } else {
            const double lo = l > 0 ? std::sqrt(lam[l - 1] * lam[l]) : lam[0] * lam[0] / std::sqrt(lam[0] * lam[1]);
            const double hi = l + 1 < nl ? std::sqrt(lam[l] * lam[l + 1])
                                         : lam[nl - 1] * lam[nl - 1] / std::sqrt(lam[nl - 2] * lam[nl - 1]);
            w = hi - lo;
        }
        kw[l] = m->kappa[l] * (1.0 - m->albedo[l]) * w;
    }
    DustGrid dg{};
    dg.n_cells = nc;
    dg.n_store = sim->n_store;
    dg.n_lambda = nl;
    for (int a = 0; a < 3; ++a) {
        dg.n[a] = g->n[a];
        dg.bs[a] = sim->bs[a];
        dg.sh[a] = sim->sh[a];
        dg.nb[a] = sim->nb[a];
    }
    int rc = MCRT_OK;
    if (g->type == kOctree) {
        std::vector<int32_t> node, geo;
        std::string err;
        const int depth = encode_octree((int64_t)g->first_child.size(), g->first_child.data(), nc, node, err);
        if (depth < 0) rc = fail(MCRT_EINVAL, "dust_create: " + err);
        if (!rc) {
            leaf_geometry(node, depth, nc, geo);
            rc = dev_alloc((void **)&d->d_leaf, geo.size() * sizeof(int32_t));
            if (!rc) {
                hipError_t e = hipMemcpy(d->d_leaf, geo.data(), geo.size() * sizeof(int32_t), hipMemcpyHostToDevice);
                if (e != hipSuccess) rc = fail(MCRT_EDEVICE, std::string("dust_create: ") + hipGetErrorString(e));
            }
        }
        dg.leaf = d->d_leaf;
    }
    DustTables tabs{};
    tabs.n = n;
    for (int i = 0; i < n; ++i) tabs.t[i] = absorbed[i]->d_table;
    const int blocks = dust_blocks(sim->n_store), tiles = dust_scan_tiles(nc);
    double *d_abs = nullptr, *d_part = nullptr, *d_lam = nullptr, *d_kw = nullptr, *d_tiles = nullptr;
    if (!rc) rc = dev_alloc((void **)&d->d_cdf, (size_t)nl * (size_t)nc * sizeof(double));
    if (!rc) rc = dev_alloc((void **)&d->d_guide, (size_t)nl * (size_t)d->K * sizeof(int));
    if (!rc) rc = dev_alloc((void **)&d->d_T, (size_t)nc * sizeof(double));
    if (!rc) rc = dev_alloc((void **)&d_abs, (size_t)sim->n_store * sizeof(double));
    if (!rc) rc = dev_alloc((void **)&d_part, 2 * (size_t)blocks * sizeof(double));
    if (!rc) rc = dev_alloc((void **)&d_lam, (size_t)nl * sizeof(double));
    if (!rc) rc = dev_alloc((void **)&d_kw, (size_t)nl * sizeof(double));
    if (!rc) rc = dev_alloc((void **)&d_tiles, (size_t)nl * (size_t)tiles * sizeof(double));
    hipError_t e = hipSuccess;
    std::vector<double> part(2 * (size_t)blocks);
    if (!rc) {
        e = hipMemcpyAsync(d_lam, lam.data(), (size_t)nl * sizeof(double), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(d_kw, kw.data(), (size_t)nl * sizeof(double), hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = launch_dust_absorbed(dg, tabs, sim->d_density, d_abs, d_part, d_part + blocks, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(part.data(), d_part, part.size() * sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
    }
    if (!rc && e == hipSuccess) {
        double absorbed_total = 0.0, mass = 0.0;
        for (int b = 0; b < blocks; ++b) {
            absorbed_total += part[(size_t)b];
            mass += part[(size_t)blocks + b];
        }
        const double u0 = mass > 0.0 ? absorbed_total / mass : 0.0;
        e = launch_dust_emission(dg, d_abs, sim->d_density, d_lam, d_kw, u0, p.T0, p.beta, d->d_T, d->d_cdf, st);
        if (e == hipSuccess) e = launch_dust_scan(d->d_cdf, nc, nl, d_tiles, st);
        if (e == hipSuccess) e = launch_dust_guide(d->d_cdf, nc, d->K, nl, d->d_guide, st);
        d->L.assign((size_t)nl, 0.0);
        for (int l = 0; l < nl && e == hipSuccess; ++l)
            e = hipMemcpyAsync(&d->L[(size_t)l], d->d_cdf + (size_t)l * (size_t)nc + (size_t)(nc - 1), sizeof(double),
                               hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
    }
    dev_free(d_abs);
    dev_free(d_part);
    dev_free(d_lam);
    dev_free(d_kw);
    dev_free(d_tiles);
    if (!rc && e != hipSuccess) rc = fail(MCRT_EDEVICE, std::string("dust_create: ") + hipGetErrorString(e));
    if (rc) {
        mcrt_dust_destroy(d);
        return rc;
    }
    *out = d;
    return MCRT_OK;
}

int mcrt_dust_luminosity(const mcrt_dust *d, double *L, size_t count)
{
    if (!d || !L) return fail(MCRT_EINVAL, "dust_luminosity: NULL argument");
    if (count < d->L.size()) return fail(MCRT_EINVAL, "dust_luminosity: output buffer too small");
    std::copy(d->L.begin(), d->L.end(), L);
    return MCRT_OK;
}

int mcrt_dust_temperature(const mcrt_dust *d, double *T, size_t count)
{
    if (!d || !T) return fail(MCRT_EINVAL, "dust_temperature: NULL argument");
    const size_t nc = (size_t)d->sim->medium->grid->n_cells;
    if (count < nc) return fail(MCRT_EINVAL, "dust_temperature: output buffer too small");
    HIP_TRY(hipSetDevice(d->sim->ctx->device));
    HIP_TRY(hipMemcpyAsync(T, d->d_T, nc * sizeof(double), hipMemcpyDefault, d->sim->ctx->stream));
    HIP_TRY(hipStreamSynchronize(d->sim->ctx->stream));
    return MCRT_OK;
}

int mcrt_run_dust_into(mcrt_sim *sim, const mcrt_dust *dust, uint64_t n_per_lambda, uint64_t first_id,
                       uint64_t count, uint64_t seed, mcrt_result *res)
{
    if (!sim || !dust || !res) return fail(MCRT_EINVAL, "run_dust_into: NULL argument");
    if (dust->sim != sim || res->sim != sim) return fail(MCRT_EINVAL, "run_dust_into: dust or result of another sim");
    if (sim->prop) return fail(MCRT_EINVAL, "run_dust_into: the learned proposal is for point sources");
    if (n_per_lambda == 0 || n_per_lambda > (uint64_t(1) << 32))
        return fail(MCRT_EINVAL, "run_dust_into: n_per_lambda must be in 1 .. 2^32");
    if (first_id > n_per_lambda || count > n_per_lambda - first_id)
        return fail(MCRT_EINVAL, "run_dust_into: id range exceeds n_per_lambda");
    BusyGuard guard(sim->busy);
    if (!guard.owned) return fail(MCRT_EBUSY, "run_dust_into: the simulation is already running");
    if (count == 0) return MCRT_OK;
    HIP_TRY(hipSetDevice(sim->ctx->device));
    const bool oct = sim->medium->grid->type == kOctree;
    if (sim->opt.precision == MCRT_FP32) {
        if (oct) return run_impl<float, float, kOctree>(sim, n_per_lambda, first_id, count, seed, res, nullptr, dust);
        return run_impl<float, float, kCartesian>(sim, n_per_lambda, first_id, count, seed, res, nullptr, dust);
    }
    if (oct) return run_impl<double, double, kOctree>(sim, n_per_lambda, first_id, count, seed, res, nullptr, dust);
    return run_impl<double, double, kCartesian>(sim, n_per_lambda, first_id, count, seed, res, nullptr, dust);
}

int mcrt_dust_self_absorption(mcrt_sim *sim, const mcrt_result *stellar, const mcrt_dust_params *params,
                              uint64_t n_per_lambda, uint64_t seed, int32_t max_cycles, double tol, mcrt_dust **dust_out,
                              mcrt_result **result_out, int32_t *cycles_done)
{
    if (!sim || !stellar || !dust_out || !result_out) return fail(MCRT_EINVAL, "dust_self_absorption: NULL argument");
    *dust_out = nullptr;
    *result_out = nullptr;
    if (max_cycles < 1 || !(tol >= 0.0)) return fail(MCRT_EINVAL, "dust_self_absorption: max_cycles >= 1, tol >= 0");
    mcrt_dust *dust = nullptr;
    mcrt_result *prev = nullptr;
    double Lprev = 0.0;
    int rc = MCRT_OK, k = 0;
    for (k = 1; k <= max_cycles; ++k) {
        const mcrt_result *src[2] = {stellar, prev};
        mcrt_dust *dk = nullptr;
        rc = mcrt_dust_create(sim, src, prev ? 2 : 1, params, &dk);
        if (rc) break;
        mcrt_dust_destroy(dust);
        dust = dk;
        mcrt_result *rk = nullptr;
        rc = mcrt_result_create(sim, &rk);
        if (rc) break;
        rc = mcrt_run_dust_into(sim, dust, n_per_lambda, 0, n_per_lambda, seed + (uint64_t)(k - 1), rk);
        mcrt_result_destroy(prev);
        prev = rk;
        if (rc && !soft_code(rc)) break;
        double L = 0.0;
        for (double x : dust->L) L += x;
        const bool converged = k > 1 && std::fabs(L - Lprev) <= tol * L;
        Lprev = L;
        if (converged) break;
    }
    if (rc && !soft_code(rc)) {
        mcrt_dust_destroy(dust);
        mcrt_result_destroy(prev);
        return rc;
    }
    *dust_out = dust;
    *result_out = prev;
    if (cycles_done) *cycles_done = k > max_cycles ? max_cycles : k;
    return rc;
}

template <typename Real, typename ImgT>
static int batch_impl(mcrt_sim *const *sims, int32_t n, const uint64_t *npl, uint64_t seed, mcrt_result *const *res)
{
    mcrt_sim *s0 = sims[0];
    hipStream_t st = s0->ctx->stream;
    // default chunk: large, since a wave drains its lanes whenever its next
    // chunk belongs to another model -- total / (16 x waves), in 256 .. 16384
    uint64_t total_packets = 0;
    for (int i = 0; i < n; ++i) total_packets += npl[i] * (uint64_t)sims[i]->medium->n_lambda;
    const int wpc0 = s0->opt.waves_per_cu > 0 ? s0->opt.waves_per_cu : 16;
    uint64_t auto_chunk = total_packets / (16ull * (uint64_t)s0->ctx->n_cu * (uint64_t)wpc0);
    auto_chunk = auto_chunk < 256 ? 256 : (auto_chunk > 16384 ? 16384 : auto_chunk);
    const uint32_t chunk =
        (uint32_t)(s0->opt.chunk > 0 ? (uint64_t)s0->opt.chunk : shifted_chunk(auto_chunk, s0->opt.chunk_shift));
    // Queue order: by estimated cost (packets x wavelengths x cells along the
    // axes) the most and least expensive alternating (default: on a batch of
    // 256 uneven models 1.5 % faster than longest-processing-time order and
    // 4.5 % faster than a random caller order), or most expensive first, or
    // the caller's order.  The model index in the random streams stays the
    // position in the caller's list.
    std::vector<int> order((size_t)n);
    for (int i = 0; i < n; ++i) order[(size_t)i] = i;
    auto cost = [&](int i) {
        const mcrt_grid *g = sims[i]->medium->grid;
        return (double)npl[i] * sims[i]->medium->n_lambda * (double)(g->n[0] + g->n[1] + g->n[2]);
    };
    if (s0->opt.queue_order != MCRT_QUEUE_CALLER)
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
    if (s0->opt.queue_order == MCRT_QUEUE_PAIRED) {
        std::vector<int> paired;
        paired.reserve((size_t)n);
        for (int lo = 0, hi = n - 1; lo <= hi; ++lo, --hi) {
            paired.push_back(order[(size_t)lo]);
            if (hi != lo) paired.push_back(order[(size_t)hi]);
        }
        order.swap(paired);
    }
    std::vector<ModelDesc<Real, ImgT>> md((size_t)n);
    uint64_t chunk0 = 0;
    for (int q = 0; q < n; ++q) {
        const int i = order[(size_t)q];
        mcrt_sim *s = sims[i];
        const mcrt_medium *m = s->medium;
        const mcrt_grid *g = m->grid;
        std::vector<Optics<Real>> optics((size_t)m->n_lambda);
        for (int l = 0; l < m->n_lambda; ++l)
            optics[l] = Optics<Real>{(Real)m->kappa[l], (Real)m->albedo[l], (Real)m->g[l],
                                     (Real)(s->source->L[l] / (double)npl[i])};
        HIP_TRY(hipMemcpyAsync(s->d_optics, optics.data(), optics.size() * sizeof(Optics<Real>), hipMemcpyHostToDevice, st));
        ModelDesc<Real, ImgT> &d = md[(size_t)q];
        d = ModelDesc<Real, ImgT>{};
        View<Real, ImgT, kCartesian> &v = d.view;
        for (int c = 0; c < 3; ++c) {
            v.bs[c] = s->bs[c];
            v.sh[c] = s->sh[c];
            v.nb[c] = s->nb[c];
            v.n[c] = g->n[c];
            v.lo[c] = (Real)g->box[c];
            v.hi[c] = (Real)g->box[3 + c];
            v.cs[c] = (Real)((g->box[3 + c] - g->box[c]) / (double)g->n[c]);
            v.ics[c] = (Real)((double)g->n[c] / (g->box[3 + c] - g->box[c]));
            v.src_pos[c] = (Real)s->source->pos[c];
        }
        v.density = s->d_density;
        v.n_cells = g->n_cells;
        v.n_store = s->n_store;
        v.n_lambda = m->n_lambda;
        v.src_type = s->source->type;
        v.hR = (Real)s->source->hR;
        v.zs = (Real)s->source->zs;
        v.n_ins = s->n_ins;
        v.table = res[i]->d_table;
        v.images = (ImgT *)res[i]->d_images;
        v.w_min = (Real)s->opt.w_min;
        v.event_cap = s->opt.event_cap;
        v.tau_peel_max = (Real)s->opt.tau_peel_max;
        v.octree_guard = 64;
        v.key0 = (uint32_t)(seed & 0xffffffffu);
        v.key1 = (uint32_t)(seed >> 32);
        v.model = (uint32_t)i;
        d.optics = (const Optics<Real> *)s->d_optics;
        d.ins = (const InsDesc<Real> *)s->d_ins;
        v.optics = d.optics; // the batch kernel reads optics and frames from global memory
        v.ins = d.ins;
        d.count = npl[i];
        d.first_id = 0;
        d.total = npl[i] * (uint64_t)m->n_lambda;
        d.chunk0 = chunk0;
        d.energy = res[i]->d_energy;
        d.stats = res[i]->d_stats;
        chunk0 += (d.total + chunk - 1) / chunk;
    }
    DevPtr dmd;
    int rc = dev_alloc(&dmd.p, md.size() * sizeof(ModelDesc<Real, ImgT>));
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(dmd.p, md.data(), md.size() * sizeof(ModelDesc<Real, ImgT>), hipMemcpyHostToDevice, st));
    HIP_TRY(launch_fill_zero(res[0]->d_counter, sizeof(unsigned long long), st));
    BatchArgs<Real, ImgT> a{};
    a.models = (const ModelDesc<Real, ImgT> *)dmd.p;
    a.n_models = n;
    a.total_chunks = chunk0;
    a.chunk = chunk;
    a.threshold = s0->opt.threshold > 0 ? s0->opt.threshold : 24;
    a.counter = res[0]->d_counter;
    int wpc = s0->opt.waves_per_cu > 0 ? s0->opt.waves_per_cu : 16;
    uint64_t waves = (uint64_t)s0->ctx->n_cu * (uint64_t)wpc;
    if (waves > chunk0) waves = chunk0;
    int grid = (int)((waves + (kBlock / 64) - 1) / (kBlock / 64));
    if (grid < 1) grid = 1;
    EventPair ev;
    HIP_TRY(hipEventCreate(&ev.e0));
    HIP_TRY(hipEventCreate(&ev.e1));
    HIP_TRY(hipEventRecord(ev.e0, st));
    hipError_t le;
    if constexpr (sizeof(Real) == 4) le = launch_batch_f32(a, grid, st, s0->opt.deposit_slots == 8 ? 8 : 16);
    else le = launch_batch_f64(a, grid, st);
    HIP_TRY(le);
    HIP_TRY(hipEventRecord(ev.e1, st));
    HIP_TRY(hipEventSynchronize(ev.e1));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, ev.e0, ev.e1));
    int worst = MCRT_OK;
    std::vector<Counters> deltas((size_t)n);
    uint64_t requested = 0;
    for (int i = 0; i < n; ++i) {
        res[i]->kernel_ms = ms;
        unsigned long long stt[kNumStats];
        HIP_TRY(hipMemcpy(stt, res[i]->d_stats, sizeof(stt), hipMemcpyDeviceToHost));
        const int oc = launch_outcome(res[i], stt, deltas[(size_t)i].v);
        if (oc == MCRT_ENONFINITE || (oc == MCRT_ELIMIT && worst == MCRT_OK)) worst = oc;
        requested += npl[i] * (uint64_t)sims[i]->medium->n_lambda;
    }
    // n_per_lambda and count of a batch line: the packets of all models
    log_launch("batch_run_into", sims, n, deltas.data(), requested, 0, requested, seed, ms, worst);
    if (worst == MCRT_ENONFINITE)
        return fail(MCRT_ENONFINITE, "packets whose luminosity became NaN or infinite were ended (see "
                                     "stats.nonfinite); the other packets' results are valid");
    if (worst == MCRT_ELIMIT) return fail(MCRT_ELIMIT, "packets hit the event cap (results valid; see stats.capped)");
    return MCRT_OK;
}

int mcrt_batch_run_into(mcrt_sim *const *sims, int32_t n, const uint64_t *n_per_lambda, uint64_t seed,
                        mcrt_result *const *results)
{
    if (!sims || !n_per_lambda || !results || n <= 0) return fail(MCRT_EINVAL, "batch_run_into: NULL argument or n <= 0");
    for (int i = 0; i < n; ++i) {
        if (!sims[i] || !results[i] || results[i]->sim != sims[i])
            return fail(MCRT_EINVAL, "batch_run_into: result " + std::to_string(i) + " does not belong to its sim");
        if (sims[i]->ctx != sims[0]->ctx || sims[i]->opt.precision != sims[0]->opt.precision)
            return fail(MCRT_EINVAL, "batch_run_into: sims must share context and precision");
        if (sims[i]->medium->grid->type != kCartesian)
            return fail(MCRT_EINVAL, "batch_run_into: batched runs take Cartesian grids");
        if (sims[i]->prop) return fail(MCRT_EINVAL, "batch_run_into: batched runs use plain direction sampling");
        if (n_per_lambda[i] == 0 || n_per_lambda[i] > (uint64_t(1) << 32))
            return fail(MCRT_EINVAL, "batch_run_into: n_per_lambda must be in 1 .. 2^32");
    }
    std::vector<std::unique_ptr<BusyGuard>> guards;
    for (int i = 0; i < n; ++i) {
        guards.emplace_back(new BusyGuard(sims[i]->busy));
        if (!guards.back()->owned) return fail(MCRT_EBUSY, "batch_run_into: a simulation is already running (or listed twice)");
    }
    HIP_TRY(hipSetDevice(sims[0]->ctx->device));
    if (sims[0]->opt.precision == MCRT_FP32) return batch_impl<float, float>(sims, n, n_per_lambda, seed, results);
    return batch_impl<double, double>(sims, n, n_per_lambda, seed, results);
}

int mcrt_sim_set_tuning(mcrt_sim *sim, const mcrt_tuning *t)
{
    if (!sim || !t) return fail(MCRT_EINVAL, "sim_set_tuning: NULL argument");
    if (t->chunk < 0 || t->waves_per_cu <= 0 || t->waves_per_cu > 32 || t->threshold <= 0 || t->threshold > 64 ||
        t->chunk_shift < -6 || t->chunk_shift > 6 || (t->deposit_slots != 0 && t->deposit_slots != 8 &&
                                                       t->deposit_slots != 16))
        return fail(MCRT_EINVAL, "sim_set_tuning: values out of range");
    sim->opt.chunk = t->chunk;
    sim->opt.chunk_shift = t->chunk_shift;
    sim->opt.waves_per_cu = t->waves_per_cu;
    sim->opt.threshold = t->threshold;
    sim->opt.deposit_slots = t->deposit_slots;
    return MCRT_OK;
}

static std::string tune_key(mcrt_sim *const *sims, int32_t n)
{
    int64_t cells = 0;
    int nl = 0, nins = 0;
    for (int i = 0; i < n; ++i) {
        cells += sims[i]->medium->grid->n_cells;
        nl = std::max(nl, sims[i]->medium->n_lambda);
        nins = std::max(nins, sims[i]->n_ins);
    }
    int lc = 0;
    while ((int64_t(1) << lc) < cells) lc++;
    char buf[256];
    std::snprintf(buf, sizeof(buf), "grid=%s prec=%s models=%d cells=2^%d lambda=%d ins=%d",
                  sims[0]->medium->grid->type == kOctree ? "octree" : "cartesian",
                  sims[0]->opt.precision == MCRT_FP32 ? "fp32" : "fp64", n, lc, nl, nins);
    return buf;
}

int mcrt_autotune(mcrt_sim *const *sims, int32_t n, const uint64_t *trial_packets, uint64_t seed,
                  const char *cache_path, mcrt_tuning *best)
{
    if (!sims || n <= 0 || !trial_packets || !best) return fail(MCRT_EINVAL, "autotune: NULL argument or n <= 0");
    LogMute mute; // trial launches stay out of the run log
    const std::string key = tune_key(sims, n);
    if (cache_path) {
        std::FILE *f = std::fopen(cache_path, "r");
        if (f) {
            char line[512];
            while (std::fgets(line, sizeof(line), f)) {
                char *bar = std::strchr(line, '|');
                if (!bar) continue;
                *bar = 0;
                mcrt_tuning t{};
                if (key == line && std::sscanf(bar + 1, "%d %d %d %lf %lf %d %d", &t.chunk, &t.waves_per_cu,
                                               &t.threshold, &t.kernel_ms, &t.default_ms, &t.chunk_shift,
                                               &t.deposit_slots) >= 4) {
                    std::fclose(f);
                    t.from_cache = 1;
                    for (int i = 0; i < n; ++i) {
                        int rc = mcrt_sim_set_tuning(sims[i], &t);
                        if (rc) return rc;
                    }
                    *best = t;
                    return MCRT_OK;
                }
            }
            std::fclose(f);
        }
    }
    std::vector<mcrt_result *> res((size_t)n, nullptr);
    auto cleanup = [&]() {
        for (auto *r : res) mcrt_result_destroy(r);
    };
    for (int i = 0; i < n; ++i) {
        int rc = mcrt_result_create(sims[i], &res[(size_t)i]);
        if (rc) {
            cleanup();
            return rc;
        }
    }
    auto trial = [&](const mcrt_tuning &t, double &ms) -> int {
        for (int i = 0; i < n; ++i) {
            int rc = mcrt_sim_set_tuning(sims[i], &t);
            if (rc) return rc;
        }
        int rc;
        if (n == 1) rc = mcrt_run_into(sims[0], trial_packets[0], 0, trial_packets[0], seed, res[0]);
        else rc = mcrt_batch_run_into(sims, n, trial_packets, seed, res.data());
        if (rc != MCRT_OK && !soft_code(rc)) return rc;
        ms = res[0]->kernel_ms;
        return MCRT_OK;
    };
    // start from the library's own defaults (sims[0]'s options; chunk 0 = the
    // automatic chunk), so the search can only keep or beat them
    const mcrt_options &o0 = sims[0]->opt;
    const mcrt_tuning dflt{o0.chunk, o0.waves_per_cu > 0 ? o0.waves_per_cu : 16,
                           o0.threshold > 0 ? o0.threshold : (n == 1 ? 16 : 24), 0.0, 0, 0.0, o0.chunk_shift,
                           o0.deposit_slots > 0 ? o0.deposit_slots : 16};
    mcrt_tuning cur = dflt;
    double ms = 0.0;
    int rc = trial(cur, ms); // warm-up
    if (!rc) rc = trial(cur, ms);
    if (rc) {
        cleanup();
        return rc;
    }
    cur.kernel_ms = ms;
    // the chunk as a multiple of the automatic chunk, which scales with the
    // launch: a short trial then has the full launch's chunks per wave
    const int shifts[] = {-3, -2, -1, 0, 1, 2, 3};
    const int thresholds[] = {8, 16, 24, 32, 48};
    const int waves[] = {8, 12, 16};
    const int slots[] = {8, 16}; // the batch kernel's deposit tile (FP32 batches only)
    const int passes = n > 1 && o0.precision == MCRT_FP32 ? 4 : 3;
    auto same = [](const mcrt_tuning &x, const mcrt_tuning &y) {
        return x.chunk == y.chunk && x.chunk_shift == y.chunk_shift && x.threshold == y.threshold &&
               x.waves_per_cu == y.waves_per_cu && x.deposit_slots == y.deposit_slots;
    };
    for (int pass = 0; pass < passes && !rc; ++pass) {
        const int *vals = pass == 0 ? shifts : pass == 1 ? thresholds : pass == 2 ? waves : slots;
        int nv = pass == 0 ? 7 : pass == 1 ? 5 : pass == 2 ? 3 : 2;
        for (int k = 0; k < nv; ++k) {
            mcrt_tuning t = cur;
            if (pass == 0) {
                t.chunk = 0;
                t.chunk_shift = vals[k];
            } else if (pass == 1) {
                t.threshold = vals[k];
            } else if (pass == 2) {
                t.waves_per_cu = vals[k];
            } else {
                t.deposit_slots = vals[k];
            }
            if (same(t, cur)) continue;
            rc = trial(t, ms);
            if (rc) break;
            if (ms < cur.kernel_ms) {
                cur = t;
                cur.kernel_ms = ms;
            }
        }
    }
    // confirmation: the pick and the defaults twice more each, alternating;
    // the pick is kept only if its best time beats the defaults' best time
    double best_pick = cur.kernel_ms, best_dflt = ms;
    {
        double m = 0.0;
        best_dflt = 1e300;
        for (int r = 0; r < 2 && !rc; ++r) {
            rc = trial(dflt, m);
            if (!rc) best_dflt = std::min(best_dflt, m);
            if (!rc && !same(cur, dflt)) {
                rc = trial(cur, m);
                if (!rc) best_pick = std::min(best_pick, m);
            }
        }
        if (same(cur, dflt)) best_pick = std::min(best_pick, best_dflt);
    }
    if (!rc) {
        if (best_pick >= best_dflt) {
            cur = dflt;
            best_pick = best_dflt;
        }
        cur.kernel_ms = best_pick;
        cur.default_ms = best_dflt;
    }
    cleanup();
    if (rc) return rc;
    for (int i = 0; i < n; ++i) {
        rc = mcrt_sim_set_tuning(sims[i], &cur);
        if (rc) return rc;
    }
    cur.from_cache = 0;
    *best = cur;
    if (cache_path) {
        std::FILE *f = std::fopen(cache_path, "a");
        if (f) {
            std::fprintf(f, "%s|%d %d %d %.6f %.6f %d %d\n", key.c_str(), cur.chunk, cur.waves_per_cu,
                         cur.threshold, cur.kernel_ms, cur.default_ms, cur.chunk_shift, cur.deposit_slots);
            std::fclose(f);
        }
    }
    return MCRT_OK;
}

int mcrt_run_range(mcrt_sim *sim, uint64_t n_per_lambda, uint64_t first_id, uint64_t count, uint64_t seed,
                   mcrt_result **out)
{
    if (!out) return fail(MCRT_EINVAL, "run_range: out is NULL");
    *out = nullptr;
    mcrt_result *r = nullptr;
    int rc = mcrt_result_create(sim, &r);
    if (rc) return rc;
    rc = mcrt_run_into(sim, n_per_lambda, first_id, count, seed, r);
    if (rc != MCRT_OK && !soft_code(rc)) {
        std::string msg = g_err;
        mcrt_result_destroy(r);
        g_err = msg;
        return rc;
    }
    *out = r;
    return rc;
}

int mcrt_run(mcrt_sim *sim, uint64_t n_per_lambda, uint64_t seed, mcrt_result **out)
{
    return mcrt_run_range(sim, n_per_lambda, 0, n_per_lambda, seed, out);
}

int mcrt_result_absorption(const mcrt_result *res, double *out, size_t count)
{
    if (!res || !out) return fail(MCRT_EINVAL, "result_absorption: NULL argument");
    const mcrt_sim *s = res->sim;
    const mcrt_grid *g = s->medium->grid;
    const int64_t nc = g->n_cells;
    const int nl = s->medium->n_lambda;
    if (count < (size_t)nc * (size_t)nl) return fail(MCRT_EINVAL, "result_absorption: output buffer too small");
    const bool bricked = g->type == kCartesian;
    HIP_TRY(hipSetDevice(s->ctx->device));
    hipStream_t st = s->ctx->stream;
    int64_t block = std::max<int64_t>(1, ((int64_t)1 << 25) / nl); // cells per pass (<= 256 MB)
    if (block > nc) block = nc;
    double *tmp = nullptr;
    int rc = dev_alloc((void **)&tmp, (size_t)block * nl * sizeof(double));
    if (rc) return rc;
    for (int64_t c0 = 0; c0 < nc; c0 += block) {
        int64_t n = std::min(block, nc - c0);
        hipError_t e = launch_table_readback(res->d_table, tmp, s->n_store, nl, g->n, bricked ? s->bs : nullptr, s->sh, s->nb, c0, n, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(out + c0 * nl, tmp, (size_t)n * nl * sizeof(double), hipMemcpyDefault, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            dev_free(tmp);
            return fail(MCRT_EDEVICE, std::string("result_absorption: ") + hipGetErrorString(e));
        }
    }
    dev_free(tmp);
    return MCRT_OK;
}

int mcrt_result_image(const mcrt_result *res, int32_t ins, double *out, size_t count)
{
    if (!res || !out) return fail(MCRT_EINVAL, "result_image: NULL argument");
    const mcrt_sim *s = res->sim;
    if (ins < 0 || ins >= s->n_ins) return fail(MCRT_EINVAL, "result_image: no such instrument");
    int64_t n = (int64_t)s->medium->n_lambda * s->ins[ins].npix[0] * s->ins[ins].npix[1];
    if (count < (size_t)n) return fail(MCRT_EINVAL, "result_image: output buffer too small");
    HIP_TRY(hipSetDevice(s->ctx->device));
    hipStream_t st = s->ctx->stream;
    double *tmp = nullptr;
    int rc = dev_alloc((void **)&tmp, (size_t)n * sizeof(double));
    if (rc) return rc;
    hipError_t e;
    if (s->opt.precision == MCRT_FP32)
        e = launch_image_scale<float>((const float *)res->d_images + s->ins_offset[ins], tmp, n, s->inv4pid2[ins], st);
    else
        e = launch_image_scale<double>((const double *)res->d_images + s->ins_offset[ins], tmp, n, s->inv4pid2[ins], st);
    if (e == hipSuccess) e = hipMemcpyAsync(out, tmp, (size_t)n * sizeof(double), hipMemcpyDefault, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    dev_free(tmp);
    if (e != hipSuccess) return fail(MCRT_EDEVICE, std::string("result_image: ") + hipGetErrorString(e));
    return MCRT_OK;
}

int mcrt_result_sed(const mcrt_result *res, int32_t ins, double *out, size_t count)
{
    if (!res || !out) return fail(MCRT_EINVAL, "result_sed: NULL argument");
    const mcrt_sim *s = res->sim;
    if (ins < 0 || ins >= s->n_ins) return fail(MCRT_EINVAL, "result_sed: no such instrument");
    const int nl = s->medium->n_lambda;
    if (count < (size_t)nl) return fail(MCRT_EINVAL, "result_sed: output buffer too small");
    const int64_t npix = (int64_t)s->ins[ins].npix[0] * s->ins[ins].npix[1];
    HIP_TRY(hipSetDevice(s->ctx->device));
    hipStream_t st = s->ctx->stream;
    double *tmp = nullptr;
    int rc = dev_alloc((void **)&tmp, (size_t)nl * sizeof(double));
    if (rc) return rc;
    hipError_t e;
    if (s->opt.precision == MCRT_FP32)
        e = launch_sed<float>((const float *)res->d_images + s->ins_offset[ins], tmp, nl, npix, s->inv4pid2[ins], st);
    else
        e = launch_sed<double>((const double *)res->d_images + s->ins_offset[ins], tmp, nl, npix, s->inv4pid2[ins], st);
    if (e == hipSuccess) e = hipMemcpyAsync(out, tmp, (size_t)nl * sizeof(double), hipMemcpyDefault, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    dev_free(tmp);
    if (e != hipSuccess) return fail(MCRT_EDEVICE, std::string("result_sed: ") + hipGetErrorString(e));
    return MCRT_OK;
}

int mcrt_result_write(const mcrt_result *res, int32_t ins, const char *fits_path, const char *sed_path)
{
    if (!res) return fail(MCRT_EINVAL, "result_write: NULL result");
    const mcrt_sim *s = res->sim;
    if (ins < 0 || ins >= s->n_ins) return fail(MCRT_EINVAL, "result_write: no such instrument");
    const int nl = s->medium->n_lambda;
    if ((int)s->medium->lambda_um.size() != nl)
        return fail(MCRT_EINVAL, "result_write: the medium was created without wavelengths");
    const int64_t nx = s->ins[ins].npix[0], ny = s->ins[ins].npix[1];
    int rc = MCRT_OK;
    if (fits_path) {
        std::vector<double> cube((size_t)(nl * nx * ny));
        rc = mcrt_result_image(res, ins, cube.data(), cube.size());
        if (!rc) rc = mcrt_fits_cube_create(fits_path, nx, ny, nl, s->medium->lambda_um.data());
        if (!rc) rc = mcrt_fits_cube_write_slices(fits_path, nx, ny, nl, 0, nl, cube.data());
    }
    if (!rc && sed_path) {
        std::vector<double> sed((size_t)nl);
        rc = mcrt_result_sed(res, ins, sed.data(), sed.size());
        if (!rc) rc = mcrt_sed_write_text(sed_path, nl, s->medium->lambda_um.data(), sed.data());
    }
    return rc;
}

int mcrt_result_energy(const mcrt_result *res, double *emitted, double *absorbed, double *escaped, double *truncated)
{
    if (!res) return fail(MCRT_EINVAL, "result_energy: NULL result");
    HIP_TRY(hipSetDevice(res->sim->ctx->device));
    double e[4];
    HIP_TRY(hipMemcpy(e, res->d_energy, sizeof(e), hipMemcpyDeviceToHost));
    if (emitted) *emitted = e[0];
    if (absorbed) *absorbed = e[1];
    if (escaped) *escaped = e[2];
    if (truncated) *truncated = e[3];
    return MCRT_OK;
}

int mcrt_result_stats(const mcrt_result *res, mcrt_stats *stats)
{
    if (!res || !stats) return fail(MCRT_EINVAL, "result_stats: NULL argument");
    HIP_TRY(hipSetDevice(res->sim->ctx->device));
    unsigned long long s[kNumStats];
    HIP_TRY(hipMemcpy(s, res->d_stats, sizeof(s), hipMemcpyDeviceToHost));
    stats->packets = s[0];
    stats->events = s[1];
    stats->prop_cells = s[2];
    stats->locate_cells = s[3];
    stats->peel_cells = s[4];
    stats->peel_adds = s[5];
    stats->peel_dropped = s[6];
    stats->capped = s[7];
    stats->guard = s[8];
    stats->nonfinite = s[9];
    stats->kernel_ms = res->kernel_ms;
    return MCRT_OK;
}


// ---------------------------------------------------------------------------
// Learned direction proposal
// ---------------------------------------------------------------------------

namespace {

void proposal_free(mcrt_proposal *p)
{
    dev_free(p->d_theta);
    dev_free(p->d_m);
    dev_free(p->d_v);
    dev_free(p->d_frags);
    dev_free(p->d_bias);
    dev_free(p->d_theta64);
}

void histories_free(mcrt_histories *h)
{
    dev_free(h->d_hist);
    dev_free(h->d_total);
    dev_free(h->d_X);
    dev_free(h->d_KP);
    dev_free(h->d_C);
}

// Seeded uniform fan-in initialisation: weights U(-b, b), b = scale sqrt(6 / fan_in),
// from a 64-bit linear congruential stream; biases zero.
void init_params(uint64_t seed, float scale, std::vector<float> &theta)
{
    theta.assign((size_t)kMlpParams, 0.0f);
    uint64_t x = seed * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
    auto uni = [&x]() {
        x = x * 6364136223846793005ull + 1442695040888963407ull;
        return (double)(x >> 11) * 0x1p-53;
    };
    struct Blk {
        int off, n, fan;
    } blk[3] = {{0, 9 * 64, 9}, {640, 64 * 64, 64}, {4800, 64 * 40, 64}};
    for (auto &b : blk) {
        double bound = scale * std::sqrt(6.0 / b.fan);
        for (int i = 0; i < b.n; ++i) theta[(size_t)(b.off + i)] = (float)((2.0 * uni() - 1.0) * bound);
    }
}

int proposal_repack(mcrt_proposal *p)
{
    hipStream_t st = p->ctx->stream;
    HIP_TRY(launch_proposal_pack(p->d_theta, p->d_frags, p->d_bias, p->d_theta64, st));
    HIP_TRY(hipStreamSynchronize(st));
    return MCRT_OK;
}

// Device scratch of one gradient pass.
struct GradScratch {
    float *partial = nullptr;
    double *loss_partial = nullptr;
    ~GradScratch()
    {
        dev_free(partial);
        dev_free(loss_partial);
    }
};

int grad_waves(const mcrt_context *ctx, int64_t m)
{
    int64_t w = (m + 63) / 64;
    int64_t cap = 2 * (int64_t)ctx->n_cu;
    if (w > cap) w = cap;
    return (int)std::max<int64_t>(w, 1);
}

} // namespace

int mcrt_proposal_create(mcrt_context *ctx, const mcrt_mlp_desc *desc, mcrt_proposal **out)
{
    if (!out) return fail(MCRT_EINVAL, "proposal_create: out is NULL");
    *out = nullptr;
    if (!ctx || !desc) return fail(MCRT_EINVAL, "proposal_create: NULL argument");
    if (desc->n_in != 9 || desc->n_hidden != 64 || desc->n_out != 40)
        return fail(MCRT_EINVAL, "proposal_create: only the 9 -> 64 -> 64 -> 40 network is supported");
    if (!(desc->init_scale >= 0.0f) || !std::isfinite(desc->init_scale))
        return fail(MCRT_EINVAL, "proposal_create: init_scale must be finite and >= 0");
    HIP_TRY(hipSetDevice(ctx->device));
    auto *p = new mcrt_proposal;
    p->ctx = ctx;
    int rc = dev_alloc((void **)&p->d_theta, kMlpParams * sizeof(float));
    if (!rc) rc = dev_alloc((void **)&p->d_m, kMlpParams * sizeof(float));
    if (!rc) rc = dev_alloc((void **)&p->d_v, kMlpParams * sizeof(float));
    if (!rc) rc = dev_alloc((void **)&p->d_frags, kFragAllElems * sizeof(uint16_t));
    if (!rc) rc = dev_alloc((void **)&p->d_bias, 176 * sizeof(float));
    if (!rc) rc = dev_alloc((void **)&p->d_theta64, kMlpParams * sizeof(double));
    if (rc) {
        proposal_free(p);
        delete p;
        return rc;
    }
    std::vector<float> theta;
    init_params(desc->init_seed, desc->init_scale, theta);
    rc = mcrt_proposal_set_params(p, theta.data(), theta.size());
    if (rc) {
        std::string msg = g_err;
        proposal_free(p);
        delete p;
        g_err = msg;
        return rc;
    }
    *out = p;
    return MCRT_OK;
}

void mcrt_proposal_destroy(mcrt_proposal *p)
{
    if (!p) return;
    (void)hipSetDevice(p->ctx->device);
    proposal_free(p);
    delete p;
}

int mcrt_proposal_set_params(mcrt_proposal *p, const float *theta, size_t count)
{
    if (!p || !theta) return fail(MCRT_EINVAL, "proposal_set_params: NULL argument");
    if (count != (size_t)kMlpParams) return fail(MCRT_EINVAL, "proposal_set_params: count must be 7400");
    BusyGuard guard(p->busy);
    if (!guard.owned) return fail(MCRT_EBUSY, "proposal_set_params: the proposal is in use");
    HIP_TRY(hipSetDevice(p->ctx->device));
    hipStream_t st = p->ctx->stream;
    HIP_TRY(hipMemcpyAsync(p->d_theta, theta, kMlpParams * sizeof(float), hipMemcpyDefault, st));
    HIP_TRY(launch_fill_zero(p->d_m, kMlpParams * sizeof(float), st));
    HIP_TRY(launch_fill_zero(p->d_v, kMlpParams * sizeof(float), st));
    p->step = 0;
    return proposal_repack(p);
}

int mcrt_proposal_get_params(const mcrt_proposal *p, float *theta, size_t count)
{
    if (!p || !theta) return fail(MCRT_EINVAL, "proposal_get_params: NULL argument");
    if (count < (size_t)kMlpParams) return fail(MCRT_EINVAL, "proposal_get_params: count must be >= 7400");
    HIP_TRY(hipSetDevice(p->ctx->device));
    HIP_TRY(hipMemcpyAsync(theta, p->d_theta, kMlpParams * sizeof(float), hipMemcpyDefault, p->ctx->stream));
    HIP_TRY(hipStreamSynchronize(p->ctx->stream));
    return MCRT_OK;
}

int mcrt_proposal_get_weights(const mcrt_proposal *p, uint16_t *bf16, size_t count)
{
    if (!p || !bf16) return fail(MCRT_EINVAL, "proposal_get_weights: NULL argument");
    if (count < (size_t)kMlpParams) return fail(MCRT_EINVAL, "proposal_get_weights: count must be >= 7400");
    std::vector<float> theta((size_t)kMlpParams);
    int rc = mcrt_proposal_get_params(p, theta.data(), theta.size());
    if (rc) return rc;
    std::vector<uint16_t> w((size_t)kMlpParams);
    for (int i = 0; i < kMlpParams; ++i) {
        float r = Bf16<float>::round(theta[(size_t)i]);
        uint32_t b;
        std::memcpy(&b, &r, sizeof b);
        w[(size_t)i] = (uint16_t)(b >> 16);
    }
    HIP_TRY(hipMemcpy(bf16, w.data(), w.size() * sizeof(uint16_t), hipMemcpyDefault));
    return MCRT_OK;
}

int mcrt_proposal_forward(mcrt_proposal *p, const float *X, int64_t n, float *out)
{
    if (!p || (n > 0 && (!X || !out))) return fail(MCRT_EINVAL, "proposal_forward: NULL argument");
    if (n < 0 || n > (int64_t(1) << 34)) return fail(MCRT_EINVAL, "proposal_forward: n out of range");
    if (n == 0) return MCRT_OK;
    HIP_TRY(hipSetDevice(p->ctx->device));
    hipStream_t st = p->ctx->stream;
    float *dX = nullptr, *dO = nullptr;
    int rc = dev_alloc((void **)&dX, (size_t)n * 9 * sizeof(float));
    if (!rc) rc = dev_alloc((void **)&dO, (size_t)n * 40 * sizeof(float));
    hipError_t e = hipSuccess;
    if (!rc) {
        e = hipMemcpyAsync(dX, X, (size_t)n * 9 * sizeof(float), hipMemcpyDefault, st);
        if (e == hipSuccess) e = launch_proposal_forward(p->d_frags, p->d_bias, dX, n, dO, st);
        if (e == hipSuccess) e = hipMemcpyAsync(out, dO, (size_t)n * 40 * sizeof(float), hipMemcpyDefault, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
    }
    dev_free(dX);
    dev_free(dO);
    if (rc) return rc;
    if (e != hipSuccess) return fail(MCRT_EDEVICE, std::string("proposal_forward: ") + hipGetErrorString(e));
    return MCRT_OK;
}

// One pass of the gradient kernel over device samples, summed by the Adam
// kernel (update = 0) or followed by an Adam step (update = 1).
static int grad_pass(mcrt_proposal *p, const float *dX, const float *dKP, const float *dC, int64_t n, int64_t m,
                     int random, uint64_t seed, float scale, const AdamArgs &adam_in, GradScratch &scr)
{
    hipStream_t st = p->ctx->stream;
    const int waves = grad_waves(p->ctx, m);
    if (!scr.partial) {
        int rc = dev_alloc((void **)&scr.partial, (size_t)waves * kGradStrideFloats * sizeof(float));
        if (!rc) rc = dev_alloc((void **)&scr.loss_partial, (size_t)waves * sizeof(double));
        if (rc) return rc;
    }
    GradArgs g{};
    g.frags = p->d_frags;
    g.bias = p->d_bias;
    g.X = dX;
    g.KP = dKP;
    g.C = dC;
    g.n = n;
    g.m = m;
    g.random = random;
    g.key0 = (uint32_t)(seed & 0xffffffffu);
    g.key1 = (uint32_t)(seed >> 32);
    g.step = (uint32_t)adam_in.step;
    g.scale = scale;
    g.partial = scr.partial;
    g.loss_partial = scr.loss_partial;
    HIP_TRY(launch_proposal_grad(g, waves, st));
    HIP_TRY(launch_proposal_adam(scr.partial, waves, scr.loss_partial, adam_in, st));
    return MCRT_OK;
}

int mcrt_proposal_grad(mcrt_proposal *p, const float *X, const float *KP, const float *C, int64_t n, double *loss,
                       float *grad)
{
    if (!p || !X || !KP || !C || !grad) return fail(MCRT_EINVAL, "proposal_grad: NULL argument");
    if (n <= 0 || n > (int64_t(1) << 31)) return fail(MCRT_EINVAL, "proposal_grad: n must be in 1 .. 2^31");
    BusyGuard guard(p->busy);
    if (!guard.owned) return fail(MCRT_EBUSY, "proposal_grad: the proposal is in use");
    HIP_TRY(hipSetDevice(p->ctx->device));
    hipStream_t st = p->ctx->stream;
    std::vector<float> hc((size_t)n);
    HIP_TRY(hipMemcpy(hc.data(), C, (size_t)n * sizeof(float), hipMemcpyDefault));
    double csum = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (!(hc[(size_t)i] >= 0.0f) || !std::isfinite(hc[(size_t)i]))
            return fail(MCRT_EINVAL, "proposal_grad: weights must be finite and >= 0");
        csum += hc[(size_t)i];
    }
    if (!(csum > 0.0)) return fail(MCRT_EINVAL, "proposal_grad: the weights sum to zero");
    float *dX = nullptr, *dKP = nullptr, *dC = nullptr, *dG = nullptr;
    double *dL = nullptr;
    int rc = dev_alloc((void **)&dX, (size_t)n * 9 * sizeof(float));
    if (!rc) rc = dev_alloc((void **)&dKP, (size_t)n * 3 * sizeof(float));
    if (!rc) rc = dev_alloc((void **)&dC, (size_t)n * sizeof(float));
    if (!rc) rc = dev_alloc((void **)&dG, kMlpParams * sizeof(float));
    if (!rc) rc = dev_alloc((void **)&dL, sizeof(double));
    if (!rc) {
        hipError_t e = hipMemcpyAsync(dX, X, (size_t)n * 9 * sizeof(float), hipMemcpyDefault, st);
        if (e == hipSuccess) e = hipMemcpyAsync(dKP, KP, (size_t)n * 3 * sizeof(float), hipMemcpyDefault, st);
        if (e == hipSuccess) e = hipMemcpyAsync(dC, hc.data(), (size_t)n * sizeof(float), hipMemcpyHostToDevice, st);
        if (e != hipSuccess) rc = fail(MCRT_EDEVICE, std::string("proposal_grad: ") + hipGetErrorString(e));
    }
    if (!rc) {
        GradScratch scr;
        AdamArgs a{};
        a.step = 1;
        a.update = 0;
        a.grad_out = dG;
        a.loss_out = dL;
        rc = grad_pass(p, dX, dKP, dC, n, n, 0, 0, (float)(1.0 / csum), a, scr);
        if (!rc) {
            hipError_t e = hipMemcpyAsync(grad, dG, kMlpParams * sizeof(float), hipMemcpyDefault, st);
            double l = 0.0;
            if (e == hipSuccess) e = hipMemcpyAsync(&l, dL, sizeof(double), hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) rc = fail(MCRT_EDEVICE, std::string("proposal_grad: ") + hipGetErrorString(e));
            if (loss) *loss = l;
        }
    }
    dev_free(dX);
    dev_free(dKP);
    dev_free(dC);
    dev_free(dG);
    dev_free(dL);
    return rc;
}

void mcrt_train_opts_default(mcrt_train_opts *o)
{
    if (!o) return;
    o->epochs = 2;
    o->batch = 16384;
    o->lr = 1e-3f;
    o->beta1 = 0.9f;
    o->beta2 = 0.999f;
    o->eps = 1e-8f;
    o->seed = 1;
}

int mcrt_proposal_train(mcrt_proposal *p, const mcrt_histories *h, const mcrt_train_opts *opt, double *final_loss)
{
    if (!p || !h) return fail(MCRT_EINVAL, "proposal_train: NULL argument");
    if (h->ctx != p->ctx) return fail(MCRT_EINVAL, "proposal_train: proposal and histories of different contexts");
    mcrt_train_opts o;
    mcrt_train_opts_default(&o);
    if (opt) o = *opt;
    if (o.epochs < 0 || o.batch < 64 || o.batch > (1 << 24) || !(o.lr > 0.0f) || !(o.beta1 >= 0.0f && o.beta1 < 1.0f) ||
        !(o.beta2 >= 0.0f && o.beta2 < 1.0f) || !(o.eps > 0.0f))
        return fail(MCRT_EINVAL, "proposal_train: epochs >= 0, batch in 64 .. 2^24, lr > 0, betas in [0, 1), eps > 0");
    if (h->n_samples <= 0 || !(h->c_sum > 0.0)) return fail(MCRT_EINVAL, "proposal_train: no training samples");
    BusyGuard guard(p->busy);
    if (!guard.owned) return fail(MCRT_EBUSY, "proposal_train: the proposal is in use");
    HIP_TRY(hipSetDevice(p->ctx->device));
    hipStream_t st = p->ctx->stream;
    const int64_t steps = (int64_t)o.epochs * ((h->n_samples + o.batch - 1) / o.batch);
    const float scale = (float)((double)h->n_samples / (h->c_sum * (double)o.batch));
    GradScratch scr;
    double *dL = nullptr;
    int rc = dev_alloc((void **)&dL, sizeof(double));
    if (rc) return rc;
    for (int64_t k = 0; k < steps && !rc; ++k) {
        AdamArgs a{};
        a.theta = p->d_theta;
        a.m = p->d_m;
        a.v = p->d_v;
        a.lr = o.lr;
        a.b1 = o.beta1;
        a.b2 = o.beta2;
        a.eps = o.eps;
        a.step = ++p->step;
        a.update = 1;
        a.loss_out = dL;
        rc = grad_pass(p, h->d_X, h->d_KP, h->d_C, h->n_samples, o.batch, 1, o.seed, scale, a, scr);
        if (!rc) {
            hipError_t e = launch_proposal_pack(p->d_theta, p->d_frags, p->d_bias, p->d_theta64, st);
            if (e != hipSuccess) rc = fail(MCRT_EDEVICE, std::string("proposal_train: ") + hipGetErrorString(e));
        }
    }
    double l = 0.0;
    if (!rc) {
        hipError_t e = hipMemcpyAsync(&l, dL, sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = fail(MCRT_EDEVICE, std::string("proposal_train: ") + hipGetErrorString(e));
    }
    dev_free(dL);
    if (!rc && final_loss) *final_loss = steps > 0 ? l : 0.0;
    return rc;
}

int mcrt_proposal_eval(mcrt_proposal *p, const mcrt_histories *h, double *loss)
{
    if (!p || !h || !loss) return fail(MCRT_EINVAL, "proposal_eval: NULL argument");
    if (h->ctx != p->ctx) return fail(MCRT_EINVAL, "proposal_eval: proposal and histories of different contexts");
    if (h->n_samples <= 0 || !(h->c_sum > 0.0)) return fail(MCRT_EINVAL, "proposal_eval: no samples");
    BusyGuard guard(p->busy);
    if (!guard.owned) return fail(MCRT_EBUSY, "proposal_eval: the proposal is in use");
    HIP_TRY(hipSetDevice(p->ctx->device));
    GradScratch scr;
    double *dL = nullptr;
    int rc = dev_alloc((void **)&dL, sizeof(double));
    if (rc) return rc;
    AdamArgs a{};
    a.step = 1;
    a.update = 0;
    a.loss_out = dL;
    rc = grad_pass(p, h->d_X, h->d_KP, h->d_C, h->n_samples, h->n_samples, 0, 0, (float)(1.0 / h->c_sum), a, scr);
    double l = 0.0;
    if (!rc) {
        hipError_t e = hipMemcpyAsync(&l, dL, sizeof(double), hipMemcpyDeviceToHost, p->ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(p->ctx->stream);
        if (e != hipSuccess) rc = fail(MCRT_EDEVICE, std::string("proposal_eval: ") + hipGetErrorString(e));
    }
    dev_free(dL);
    if (!rc) *loss = l;
    return rc;
}

int mcrt_sim_set_proposal(mcrt_sim *sim, mcrt_proposal *p, double alpha)
{
    if (!sim) return fail(MCRT_EINVAL, "sim_set_proposal: NULL sim");
    BusyGuard guard(sim->busy);
    if (!guard.owned) return fail(MCRT_EBUSY, "sim_set_proposal: the simulation is running");
    if (!p) {
        sim->prop = nullptr;
        return MCRT_OK;
    }
    if (p->ctx != sim->ctx) return fail(MCRT_EINVAL, "sim_set_proposal: proposal of another context");
    if (!(alpha > 0.0 && alpha <= 1.0)) return fail(MCRT_EINVAL, "sim_set_proposal: alpha must lie in (0, 1]");
    if (sim->medium->lambda_um.empty())
        return fail(MCRT_EINVAL, "sim_set_proposal: the medium needs wavelengths (lambda_um) for the features");
    sim->prop = p;
    sim->alpha = alpha;
    return MCRT_OK;
}

int mcrt_proposal_collect(mcrt_sim *sim, uint64_t n_per_lambda, uint64_t first_id, uint64_t count, uint64_t seed,
                          int32_t max_events, mcrt_result *res, mcrt_histories **out)
{
    if (!out) return fail(MCRT_EINVAL, "proposal_collect: out is NULL");
    *out = nullptr;
    if (!sim || !res) return fail(MCRT_EINVAL, "proposal_collect: NULL sim or result");
    if (res->sim != sim) return fail(MCRT_EINVAL, "proposal_collect: result belongs to another sim");
    if (sim->prop) return fail(MCRT_EINVAL, "proposal_collect: histories come from plain runs (detach the proposal)");
    if (sim->medium->lambda_um.empty())
        return fail(MCRT_EINVAL, "proposal_collect: the medium needs wavelengths (lambda_um) for the features");
    if (max_events < 1 || max_events > 4096) return fail(MCRT_EINVAL, "proposal_collect: max_events in 1 .. 4096");
    if (n_per_lambda == 0 || n_per_lambda > (uint64_t(1) << 32) || first_id > n_per_lambda ||
        count > n_per_lambda - first_id || count == 0)
        return fail(MCRT_EINVAL, "proposal_collect: bad packet range");
    const uint64_t npk = count * (uint64_t)sim->medium->n_lambda;
    if (npk > (uint64_t(1) << 32)) return fail(MCRT_EINVAL, "proposal_collect: at most 2^32 packets per collection");
    BusyGuard guard(sim->busy);
    if (!guard.owned) return fail(MCRT_EBUSY, "proposal_collect: the simulation is already running");
    HIP_TRY(hipSetDevice(sim->ctx->device));
    hipStream_t st = sim->ctx->stream;
    auto *h = new mcrt_histories;
    h->ctx = sim->ctx;
    h->fp64 = sim->opt.precision == MCRT_FP64_VALIDATE;
    h->n_packets = (int64_t)npk;
    h->events = max_events;
    const size_t rb = h->fp64 ? sizeof(double) : sizeof(float);
    const size_t hist_bytes = (size_t)npk * (size_t)max_events * kHistFloats * rb;
    int rc = dev_alloc(&h->d_hist, hist_bytes);
    if (!rc) rc = dev_alloc(&h->d_total, (size_t)npk * rb);
    if (!rc) {
        hipError_t e = launch_fill_zero(h->d_hist, hist_bytes, st);
        if (e == hipSuccess) e = launch_fill_zero(h->d_total, (size_t)npk * rb, st);
        if (e != hipSuccess) rc = fail(MCRT_EDEVICE, std::string("proposal_collect: ") + hipGetErrorString(e));
    }
    int run_rc = MCRT_OK;
    if (!rc) {
        const bool oct = sim->medium->grid->type == kOctree;
        if (!h->fp64) {
            run_rc = oct ? run_impl<float, float, kOctree>(sim, n_per_lambda, first_id, count, seed, res, h)
                         : run_impl<float, float, kCartesian>(sim, n_per_lambda, first_id, count, seed, res, h);
        } else {
            run_rc = oct ? run_impl<double, double, kOctree>(sim, n_per_lambda, first_id, count, seed, res, h)
                         : run_impl<double, double, kCartesian>(sim, n_per_lambda, first_id, count, seed, res, h);
        }
        if (run_rc != MCRT_OK && !soft_code(run_rc)) rc = run_rc;
    }
    // compaction into training samples
    uint32_t *d_count = nullptr;
    uint64_t *d_off = nullptr, *d_bs = nullptr, *d_tot = nullptr;
    double *d_csum = nullptr;
    if (!rc) {
        const int64_t nb = ((int64_t)npk + 1023) / 1024;
        rc = dev_alloc((void **)&d_count, (size_t)npk * sizeof(uint32_t));
        if (!rc) rc = dev_alloc((void **)&d_off, (size_t)npk * sizeof(uint64_t));
        if (!rc) rc = dev_alloc((void **)&d_bs, (size_t)nb * sizeof(uint64_t));
        if (!rc) rc = dev_alloc((void **)&d_tot, sizeof(uint64_t));
        if (!rc) rc = dev_alloc((void **)&d_csum, sizeof(double));
    }
    if (!rc) {
        uint64_t ns = 0;
        hipError_t e = launch_hist_count(h->d_hist, h->d_total, h->fp64, (int64_t)npk, max_events, d_count, d_off,
                                         d_bs, d_tot, st);
        if (e == hipSuccess) e = hipMemcpyAsync(&ns, d_tot, sizeof(ns), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = fail(MCRT_EDEVICE, std::string("proposal_collect: ") + hipGetErrorString(e));
        h->n_samples = (int64_t)ns;
        if (!rc && ns > 0) {
            rc = dev_alloc((void **)&h->d_X, (size_t)ns * 9 * sizeof(float));
            if (!rc) rc = dev_alloc((void **)&h->d_KP, (size_t)ns * 3 * sizeof(float));
            if (!rc) rc = dev_alloc((void **)&h->d_C, (size_t)ns * sizeof(float));
            if (!rc) {
                e = launch_hist_write(h->d_hist, h->d_total, h->fp64, (int64_t)npk, max_events, d_off, h->d_X,
                                      h->d_KP, h->d_C, st);
                if (e == hipSuccess) e = launch_sum_f32(h->d_C, (int64_t)ns, d_csum, st);
                if (e == hipSuccess) e = hipMemcpyAsync(&h->c_sum, d_csum, sizeof(double), hipMemcpyDeviceToHost, st);
                if (e == hipSuccess) e = hipStreamSynchronize(st);
                if (e != hipSuccess) rc = fail(MCRT_EDEVICE, std::string("proposal_collect: ") + hipGetErrorString(e));
            }
        }
    }
    dev_free(d_count);
    dev_free(d_off);
    dev_free(d_bs);
    dev_free(d_tot);
    dev_free(d_csum);
    if (rc) {
        std::string msg = g_err;
        histories_free(h);
        delete h;
        g_err = msg;
        return rc;
    }
    *out = h;
    return run_rc;
}

int mcrt_histories_info(const mcrt_histories *h, int64_t *n_packets, int32_t *max_events, int64_t *n_samples,
                        double *weight_sum)
{
    if (!h) return fail(MCRT_EINVAL, "histories_info: NULL histories");
    if (n_packets) *n_packets = h->n_packets;
    if (max_events) *max_events = h->events;
    if (n_samples) *n_samples = h->n_samples;
    if (weight_sum) *weight_sum = h->c_sum;
    return MCRT_OK;
}

int mcrt_histories_records(const mcrt_histories *h, double *records, size_t count, double *totals,
                           size_t count_totals)
{
    if (!h || !records || !totals) return fail(MCRT_EINVAL, "histories_records: NULL argument");
    const size_t nrec = (size_t)h->n_packets * (size_t)h->events * kHistFloats;
    if (count < nrec || count_totals < (size_t)h->n_packets)
        return fail(MCRT_EINVAL, "histories_records: output buffer too small");
    HIP_TRY(hipSetDevice(h->ctx->device));
    if (h->fp64) {
        HIP_TRY(hipMemcpy(records, h->d_hist, nrec * sizeof(double), hipMemcpyDefault));
        HIP_TRY(hipMemcpy(totals, h->d_total, (size_t)h->n_packets * sizeof(double), hipMemcpyDefault));
        return MCRT_OK;
    }
    std::vector<float> a(nrec), b((size_t)h->n_packets);
    HIP_TRY(hipMemcpy(a.data(), h->d_hist, nrec * sizeof(float), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(b.data(), h->d_total, b.size() * sizeof(float), hipMemcpyDeviceToHost));
    std::vector<double> da(a.begin(), a.end()), db(b.begin(), b.end());
    HIP_TRY(hipMemcpy(records, da.data(), nrec * sizeof(double), hipMemcpyDefault));
    HIP_TRY(hipMemcpy(totals, db.data(), db.size() * sizeof(double), hipMemcpyDefault));
    return MCRT_OK;
}

int mcrt_histories_samples(const mcrt_histories *h, float *X, float *KP, float *C, size_t n)
{
    if (!h || !X || !KP || !C) return fail(MCRT_EINVAL, "histories_samples: NULL argument");
    if (n < (size_t)h->n_samples) return fail(MCRT_EINVAL, "histories_samples: output buffers too small");
    if (h->n_samples == 0) return MCRT_OK;
    HIP_TRY(hipSetDevice(h->ctx->device));
    HIP_TRY(hipMemcpy(X, h->d_X, (size_t)h->n_samples * 9 * sizeof(float), hipMemcpyDefault));
    HIP_TRY(hipMemcpy(KP, h->d_KP, (size_t)h->n_samples * 3 * sizeof(float), hipMemcpyDefault));
    HIP_TRY(hipMemcpy(C, h->d_C, (size_t)h->n_samples * sizeof(float), hipMemcpyDefault));
    return MCRT_OK;
}

void mcrt_histories_destroy(mcrt_histories *h)
{
    if (!h) return;
    (void)hipSetDevice(h->ctx->device);
    histories_free(h);
    delete h;
}
