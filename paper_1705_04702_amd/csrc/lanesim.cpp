// lanesim.cpp -- serial host instantiation of the transport lane logic
// (transport_core.h), packet after packet in (wavelength, id) order, with
// plain additions in place of the device atomics.
//
// TEST HARNESS: it lets the CPU test suite check the kernel's per-lane code
// (march, event processing, sampling, scene setup) without a GPU.  It is not
// used by the library or its Python binding.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

namespace mcrt {
using std::atanh;
using std::cos;
using std::exp;
using std::expm1;
using std::fabs;
using std::floor;
using std::log;
using std::log1p;
using std::sin;
using std::sqrt;
} // namespace mcrt

#define MCRT_HD inline
#include "transport_core.h"
#include "scene_setup.h"

using namespace mcrt;

namespace {
struct HostSink {
    static constexpr bool kLearn = true, kHist = true; // chosen at run time
    void deposit(double *table, long long slab, int cell, double v)
    {
        if (v != 0.0) table[slab + cell] += v;
    }
    template <typename L, typename T> void pixel(L &, T *images, long long idx, T v) { images[idx] += v; }
};
} // namespace

extern "C" {

typedef struct {
    int32_t grid_type;
    double box[6];
    int32_t n[3];
    int64_t n_nodes;
    const int32_t *first_child;
    int64_t n_cells;
    const float *density;
    int32_t n_lambda;
    const double *kappa, *albedo, *g, *L;
    int32_t src_type;
    double src_pos[3];
    double hR, zs;
    int32_t n_ins;
    const double *ins_geom;   // [n_ins][5] incl, azim, distance, fov_x, fov_y
    const int32_t *ins_npix;  // [n_ins][2]
    double w_min;
    int64_t event_cap;
    double tau_peel_max;
    int32_t precision;        // 0 FP32, 1 FP64
    int32_t top_level;        // -1 default
    uint32_t model;           // fourth word of the Philox counter
    const double *lambda_um;  // wavelengths (learned features), may be NULL
    const double *mlp;        // network parameters (bf16 weights) or NULL: plain sampling
    double alpha;             // weight of the physical distribution in the proposal
} ls_scene;

typedef struct {
    double *table;   // [n_cells][n_lambda]
    double *images;  // concatenated [n_lambda][ny][nx] per instrument, flux
    double *energy;  // [4]
    uint64_t *stats; // [10]
    double *hist;       // [packets][hist_events][14] or NULL
    double *hist_total; // [packets]
    int32_t hist_events;
} ls_out;

}

template <typename Real, int G>
static int run(const ls_scene *s, uint64_t npl, uint64_t first, uint64_t count, uint64_t seed, ls_out *o)
{
    View<Real, Real, G> v{};
    std::vector<int32_t> node;
    std::vector<uint64_t> top, blocks;
    int depth = 0;
    if (s->grid_type == kOctree) {
        std::string err;
        depth = encode_octree(s->n_nodes, s->first_child, s->n_cells, node, err);
        if (depth < 0) return -2;
        v.top_level = s->top_level >= 0 ? (s->top_level < depth ? s->top_level : depth) : (depth < 7 ? depth : 7);
        if (!build_walk(node, depth, v.top_level, s->density, top, blocks, err)) return -2;
        if (blocks.empty()) blocks.assign(1, 0);
        for (int a = 0; a < 3; ++a) v.n[a] = 1 << depth;
    } else {
        for (int a = 0; a < 3; ++a) v.n[a] = s->n[a];
    }
    v.depth = depth;
    for (int a = 0; a < 3; ++a) {
        v.lo[a] = (Real)s->box[a];
        v.hi[a] = (Real)s->box[3 + a];
        v.cs[a] = (Real)((s->box[3 + a] - s->box[a]) / (double)v.n[a]);
        v.ics[a] = (Real)((double)v.n[a] / (s->box[3 + a] - s->box[a]));
    }
    std::vector<float> stored;
    v.n_store = s->n_cells;
    if (G == kCartesian) {
        double cs[3];
        for (int a = 0; a < 3; ++a) cs[a] = (s->box[3 + a] - s->box[a]) / (double)v.n[a];
        long long ns;
        choose_bricks(cs, v.n, v.bs, v.sh, v.nb, ns);
        v.n_store = ns;
        stored.assign((size_t)ns, 0.0f);
        for (int iz = 0; iz < v.n[2]; ++iz)
            for (int iy = 0; iy < v.n[1]; ++iy)
                for (int ix = 0; ix < v.n[0]; ++ix)
                    stored[(size_t)store_index_host(v.bs, v.sh, v.nb, ix, iy, iz)] =
                        s->density[ix + (size_t)v.n[0] * (iy + (size_t)v.n[1] * iz)];
        v.density = stored.data();
    } else {
        v.density = s->density;
    }
    v.node = (const unsigned long long *)blocks.data();
    v.top = (const unsigned long long *)top.data();
    v.n_cells = s->n_cells;
    v.n_lambda = s->n_lambda;
    std::vector<Optics<Real>> optics((size_t)s->n_lambda);
    double r_out = 0.0, rho_mean = 0.0;
    std::vector<double> lamf;
    feature_constants(s->box, s->density, s->n_cells, s->lambda_um, s->n_lambda, r_out, rho_mean, lamf);
    for (int l = 0; l < s->n_lambda; ++l)
        optics[l] = Optics<Real>{(Real)s->kappa[l], (Real)s->albedo[l], (Real)s->g[l], (Real)(s->L[l] / (double)npl),
                                 (Real)lamf[l]};
    v.optics = optics.data();
    v.src_type = s->src_type;
    for (int a = 0; a < 3; ++a) v.src_pos[a] = (Real)s->src_pos[a];
    v.hR = (Real)s->hR;
    v.zs = (Real)s->zs;
    v.n_ins = s->n_ins;
    std::vector<InsDesc<Real>> ins((size_t)(s->n_ins > 0 ? s->n_ins : 1));
    std::vector<double> inv4pid2((size_t)(s->n_ins > 0 ? s->n_ins : 1));
    std::vector<std::vector<Real>> cols((size_t)(s->n_ins > 0 ? s->n_ins : 1));
    long long off = 0;
    for (int j = 0; j < s->n_ins; ++j) {
        const double *gm = s->ins_geom + 5 * j;
        HostInstrument h{gm[0], gm[1], gm[2], {gm[3], gm[4]}, {s->ins_npix[2 * j], s->ins_npix[2 * j + 1]}};
        make_ins_desc<Real>(h, off, ins[j], inv4pid2[j]);
        off += (long long)s->n_lambda * h.npix[0] * h.npix[1];
        const int code = (G == kCartesian || depth <= kMaxColumnDepth) ? axis_code(h) : -1;
        if (code >= 0) {
            if (G == kCartesian) {
                std::vector<double> S;
                int n3[3] = {s->n[0], s->n[1], s->n[2]};
                column_map(s->density, n3, s->box, code, v.bs, v.sh, v.nb, v.n_store, S);
                cols[j].assign(S.begin(), S.end());
            } else {
                std::vector<int32_t> onode;
                std::string err;
                if (encode_octree(s->n_nodes, s->first_child, s->n_cells, onode, err) < 0) return -2;
                octree_column_map<Real>(onode, depth, s->n_cells, s->density, s->box, code, cols[j]);
            }
            ins[j].col = cols[j].data();
            ins[j].col_axis = code;
        }
    }
    v.ins = ins.data();
    std::vector<double> table((size_t)v.n_store * s->n_lambda, 0.0);
    std::vector<Real> images((size_t)(off > 0 ? off : 1), Real(0));
    v.table = table.data();
    v.images = images.data();
    v.w_min = (Real)s->w_min;
    v.event_cap = s->event_cap;
    v.tau_peel_max = (Real)s->tau_peel_max;
    v.octree_guard = 16 * 3 * (1 << depth) + 64;
    v.key0 = (uint32_t)(seed & 0xffffffffu);
    v.key1 = (uint32_t)(seed >> 32);
    v.model = s->model;
    v.learned = s->mlp != nullptr;
    v.alpha = (Real)s->alpha;
    std::vector<double> mlp64;
    if (s->mlp) {
        std::vector<float> theta(s->mlp, s->mlp + kMlpParams); // FP32 master values
        mlp_params_f64(theta.data(), mlp64);
        v.mlp64 = mlp64.data();
    }
    v.r_out = (Real)r_out;
    v.rho_mean = (Real)rho_mean;
    std::vector<Real> hist, hist_total;
    if (o->hist && !s->mlp) {
        hist.assign((size_t)count * s->n_lambda * o->hist_events * kHistFloats, Real(0));
        hist_total.assign((size_t)count * s->n_lambda, Real(0));
        v.hist = hist.data();
        v.hist_total = hist_total.data();
        v.hist_events = o->hist_events;
    }

    HostSink sink;
    Tally ty{};
    for (int l = 0; l < s->n_lambda; ++l) {
        for (uint64_t i = first; i < first + count; ++i) {
            Lane<Real> ln{};
            launch<HostSink>(v, ln, ty, (uint32_t)l, (uint32_t)i, (uint32_t)((uint64_t)l * count + (i - first)));
            settle(v, ln, ty, sink);
            while (ln.mode != kDead || ln.parked) {
                if (ln.parked) {
                    resolve_direction_scalar<HostSink>(v, ln, ty);
                    if (!ln.marching) settle(v, ln, ty, sink);
                    continue;
                }
                march_step(v, ln, ty, sink);
                if (!ln.marching) settle(v, ln, ty, sink);
            }
        }
    }
    for (int64_t c = 0; c < s->n_cells; ++c) {
        long long sc = c;
        if (G == kCartesian) {
            int ix = (int)(c % v.n[0]), iy = (int)((c / v.n[0]) % v.n[1]), iz = (int)(c / ((int64_t)v.n[0] * v.n[1]));
            sc = store_index_host(v.bs, v.sh, v.nb, ix, iy, iz);
        }
        for (int l = 0; l < s->n_lambda; ++l) o->table[c * s->n_lambda + l] = table[(size_t)l * v.n_store + sc];
    }
    for (int j = 0; j < s->n_ins; ++j) {
        long long n = (long long)s->n_lambda * s->ins_npix[2 * j] * s->ins_npix[2 * j + 1];
        for (long long q = 0; q < n; ++q) o->images[ins[j].offset + q] = (double)images[ins[j].offset + q] * inv4pid2[j];
    }
    o->energy[0] = ty.emitted;
    o->energy[1] = ty.absorbed;
    o->energy[2] = ty.escaped;
    o->energy[3] = ty.truncated;
    uint64_t st[10] = {ty.packets, ty.events, ty.prop_cells, ty.locate_cells, ty.peel_cells,
                       ty.peel_adds, ty.peel_dropped, ty.capped, ty.guard, ty.nonfinite};
    std::memcpy(o->stats, st, sizeof(st));
    for (size_t q = 0; q < hist.size(); ++q) o->hist[q] = (double)hist[q];
    for (size_t q = 0; q < hist_total.size(); ++q) o->hist_total[q] = (double)hist_total[q];
    return 0;
}

extern "C" int ls_run(const ls_scene *s, uint64_t n_per_lambda, uint64_t first_id, uint64_t count, uint64_t seed,
                      ls_out *out)
{
    if (!s || !out || n_per_lambda == 0 || first_id + count > n_per_lambda) return -1;
    if (s->mlp && !s->lambda_um) return -1;
    if (out->hist && (!out->hist_total || out->hist_events < 1)) return -1;
    if (s->grid_type == kOctree) {
        if (s->precision == 1) return run<double, kOctree>(s, n_per_lambda, first_id, count, seed, out);
        return run<float, kOctree>(s, n_per_lambda, first_id, count, seed, out);
    }
    if (s->precision == 1) return run<double, kCartesian>(s, n_per_lambda, first_id, count, seed, out);
    return run<float, kCartesian>(s, n_per_lambda, first_id, count, seed, out);
}
