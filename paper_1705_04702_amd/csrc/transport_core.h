// transport_core.h -- per-lane logic of the Monte Carlo photon-packet life
// cycle (stellar emission phase of the hybrid-parallel SKIRT paper, Section
// 3.2; accumulation as in Section 5.2 "Lockfree additions").
//
// Everything here acts on ONE packet held in registers by one lane; the
// persistent wave scheduler (transport_kernel.h) decides when each lane
// steps its ray march and when it processes the end of a march.  The header
// is written against a policy `Sink` that performs the shared-table and image
// additions (hardware atomics on the GPU), so the same lane code can also be
// instantiated serially for host-side checking.  The includer defines MCRT_HD
// (function qualifiers) before including this file.
//
// Templates are instantiated for Real = float (production: FP32 transport,
// FP64 table totals and energy sums) and Real = double (validation mode,
// same operation order as an FP64 reference, no contraction).
#pragma once

#include <stdint.h>

#include "det_math.h"

namespace mcrt {

constexpr int kMaxIns = 8;        // instruments per simulation
constexpr int kMaxLdsLambda = 128; // per-wavelength optics staged in LDS (more: read from global memory)

enum Mode : int {
    kDead = 0,      // no packet (needs a refill)
    kPeelEmit = 1,  // emission peel-off march towards instrument j
    kProp = 2,      // propagation march with continuous absorption
    kLocate = 3,    // second march to the forced interaction point
    kPeelScat = 4,  // scattering peel-off march towards instrument j
    kLaunched = 5,  // launched, first march not yet begun
    kNewDir = 6,    // direction chosen by the learned proposal, propagation not yet begun
};
// A lane waiting for the learned proposal to pick its next direction has
// mode kDead with `parked` set: the event loop stops there exactly as for a
// finished packet, and the kernel hands it to the proposal instead of
// refilling it.

constexpr int kMlpParams = 7400; // 9 -> 64 -> 64 -> 40
constexpr int kHistFloats = 14;  // features (9), new direction (3), luminosity, flux so far

enum GridType : int { kCartesian = 0, kOctree = 1 };
enum SourceType : int { kPointIso = 0, kPointAniso = 1, kExpDisk = 2, kDust = 3 };

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): counter (block, packet, wavelength,
// model), key (seed low, seed high).  Slot s of a packet uses block s/2 and
// the word pair (2(s%2), 2(s%2)+1) as (high, low).
// ---------------------------------------------------------------------------
struct U4 {
    uint32_t x, y, z, w;
};

MCRT_HD U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    return U4{c0, c1, c2, c3};
}

// Open-interval uniforms from a (high, low) word pair.
template <typename Real> struct Uni;
template <> struct Uni<float> {
    MCRT_HD static float from(uint32_t hi, uint32_t) { return ((float)(hi >> 9) + 0.5f) * 0x1p-23f; }
};
template <> struct Uni<double> {
    MCRT_HD static double from(uint32_t hi, uint32_t lo)
    {
        uint64_t w = ((uint64_t)hi << 32) | (uint64_t)lo;
        return ((double)(w >> 12) + 0.5) * 0x1p-52;
    }
};

struct Stream {
    uint32_t k0, k1, packet, lambda, model;
    // the two uniforms of block b: slots 2b and 2b+1
    template <typename Real> MCRT_HD void pair(uint32_t block, Real &a, Real &b) const
    {
        U4 o = philox(block, packet, lambda, model, k0, k1);
        a = Uni<Real>::from(o.x, o.y);
        b = Uni<Real>::from(o.z, o.w);
    }
    template <typename Real> MCRT_HD Real slot(uint32_t s) const
    {
        U4 o = philox(s >> 1, packet, lambda, model, k0, k1);
        return (s & 1u) ? Uni<Real>::from(o.z, o.w) : Uni<Real>::from(o.x, o.y);
    }
};

// ---------------------------------------------------------------------------
// Scene views
// ---------------------------------------------------------------------------
template <typename Real> struct InsDesc {
    Real kobs[3], ex[3], ey[3];
    Real half_fovx, half_fovy, pixx, pixy; // pixel size = fov / npix
    int nx, ny;
    long long offset; // first image element of this instrument
    Real inv4pid2;    // flux per unit of image accumulation
    // Line of sight along a grid axis, so a peel-off's optical depth needs no
    // march.  Cartesian grids: col[store(c)] = sum of density x path length
    // over the cells beyond c up to the boundary; octree grids (depth <= 10):
    // col[x + N (y + N z)] = the same sum over lattice cells from (x, y, z)
    // itself.  col_axis = 2 axis + (k < 0), -1 (col == nullptr) otherwise
    const Real *col;
    int col_axis;
};

template <typename Real> struct Optics {
    Real kappa, albedo, g, L0, lamf; // lamf: wavelength feature of the proposal
};

template <typename Real, typename ImgT, int G> struct View {
    // grid
    int n[3];       // cells per axis (Cartesian) or lattice size 2^depth (octree)
    int depth;      // octree maximum depth
    int top_level;  // octree: level of the dense top table
    Real lo[3], hi[3], cs[3];
    Real ics[3]; // 1 / cs (FP32 octree steps multiply; FP64 divides)
    const float *density; // Cartesian: per stored cell; octree: per leaf (the walk's entries carry it too)
    // octree: the leaf walk's blocks of 64 entries and its top table; an entry's
    // low word is a leaf (bit 31, level, cell) or a block index, a leaf's high
    // word its density's FP32 bits
    const unsigned long long *node;
    const unsigned long long *top;
    long long n_cells;
    // Cartesian storage layout: bricks of 2^bs[0] x 2^bs[1] x 2^bs[2] = 32 cells,
    // nb[] bricks per axis; n_store = cells per wavelength slice incl. padding
    int bs[3], nb[3], sh[3]; // in-brick index: sum_a (c_a mod 2^bs_a) << sh_a
    long long n_store;
    // per wavelength
    int n_lambda;
    const Optics<Real> *optics;
    // source
    int src_type;
    Real src_pos[3];
    Real hR, zs;
    // dust emission (kDust): per wavelength the running sums of the cells'
    // emission in natural cell order (octree: leaf order) [n_lambda][n_cells], and a guide
    // of dust_K entries per wavelength: guide[k] = first cell whose running
    // sum exceeds k total / K
    const double *dust_cdf;
    const int *dust_guide;
    int dust_K;
    const int *dust_leaf; // octree: per leaf (origin x, y, z on the 2^depth lattice, level)
    // instruments
    int n_ins;
    const InsDesc<Real> *ins;
    // outputs
    double *table;  // [n_lambda][n_store]
    ImgT *images;   // [n_ins][n_lambda][ny][nx], flux * 4 pi d^2
    // options
    Real w_min;
    long long event_cap;
    Real tau_peel_max;
    int octree_guard;
    uint32_t key0, key1, model;
    // learned proposal (learned = 0: plain sampling)
    int learned;
    Real alpha;
    const double *mlp64;  // FP64 copy of the parameters (bf16 values) for the scalar network
    Real r_out, rho_mean; // feature scales
    // plain-run histories (hist == nullptr: not recorded)
    Real *hist;           // [slot][hist_events][kHistFloats]
    Real *hist_total;     // [slot]
    int hist_events;
};

// Per-lane tallies, reduced once per wave at the end of the kernel.
struct Tally {
    double emitted, absorbed, escaped, truncated;
    uint32_t packets, events, prop_cells, locate_cells, peel_cells, peel_adds, peel_dropped, capped, guard;
    uint32_t nonfinite; // packets ended because their luminosity became NaN or infinite
};

template <typename Real> struct Lane {
    Real r[3], k[3];    // packet position and direction
    Real d[3], id3[3];  // march direction and its reciprocal
    Real tn0, tn1, tn2; // Cartesian: ray parameter of the next plane per axis
    Real t;             // ray parameter at the start of the current segment
    Real L, L0;         // current luminosity, launch luminosity
    Real wpeel;         // peel-off luminosity times phase
    Real E, tau, wabs, tau_int;
    Real a_t0, a_tau, a_kr, a_ds; // locate: last segment with positive optical depth
    Optics<Real> opt;
    int c0, c1, c2;     // cell index (Cartesian) or lattice cursor (octree)
    int mode, j, nseg, steps;
    long long e;
    uint32_t id, lam;
    uint32_t slot;      // packet index in the launch (histories)
    Real rho_star;      // density of the interaction cell
    Real flux;          // image flux produced so far (histories)
    long long pix;      // pending pixel add (index, -1: none) for the wave-level combine
    Real pval;
    bool marching, found, dropped, emis_dir, parked;
};

// Per-axis fields are separate scalars (not arrays): stores through a
// runtime axis index would move the lane state to scratch memory.  These
// accessors are only called with compile-time axis numbers.
template <typename Real> MCRT_HD int &cidx(Lane<Real> &ln, int a) { return a == 0 ? ln.c0 : (a == 1 ? ln.c1 : ln.c2); }
template <typename Real> MCRT_HD int cidx(const Lane<Real> &ln, int a) { return a == 0 ? ln.c0 : (a == 1 ? ln.c1 : ln.c2); }
template <typename Real> MCRT_HD Real &tnx(Lane<Real> &ln, int a) { return a == 0 ? ln.tn0 : (a == 1 ? ln.tn1 : ln.tn2); }

// ---------------------------------------------------------------------------
// Precision traits: FP64 divides exactly like the reference; FP32 multiplies
// by the reciprocal of the direction.
// ---------------------------------------------------------------------------
template <typename Real> struct Prec;
template <> struct Prec<float> {
    MCRT_HD static float over_k(float num, float k, float ik) { return num * ik; }
    MCRT_HD static float inf() { return __builtin_huge_valf(); }
};
template <> struct Prec<double> {
    MCRT_HD static double over_k(double num, double k, double) { return num / k; }
    MCRT_HD static double inf() { return __builtin_huge_val(); }
};

template <typename Real> MCRT_HD Real rmax(Real a, Real b) { return a > b ? a : b; }

// Element i of a device buffer named by a view (a device allocation, never
// LDS: the optics and instrument tables, which the kernels may stage in LDS,
// do not go through here).  Saying so keeps the load a global one where the
// view itself was read from memory (the batched kernel), which the compiler
// would otherwise issue as a flat load.
template <typename T> MCRT_HD T gload(const T *p, long long i)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return ((const __attribute__((address_space(1))) T *)p)[i];
#else
    return p[i];
#endif
}

// Storage position of Cartesian cell (ix, iy, iz): bricks of 32 cells shaped
// to the cells' aspect ratio, so that successive cells of a ray tend to share
// cache lines of the density and table arrays.
// Octree top table: the cubes of the top level in tiles of 4 x 4 x 4 (256
// bytes, each half one 128-byte line), so that the consecutive cubes of a
// ray in any direction tend to share lines; linear below level 2.
MCRT_HD int top_index(int x, int y, int z, int top_level)
{
    if (top_level < 2) return (((z << top_level) + y) << top_level) + x;
    const int tl = top_level - 2;
    const int tile = ((((z >> 2) << tl) + (y >> 2)) << tl) + (x >> 2);
    return (tile << 6) + ((z & 3) << 4) + ((y & 3) << 2) + (x & 3);
}

template <typename Real, typename ImgT, int G>
MCRT_HD int store_index(const View<Real, ImgT, G> &v, int ix, int iy, int iz)
{
    int brick = (ix >> v.bs[0]) + v.nb[0] * ((iy >> v.bs[1]) + v.nb[1] * (iz >> v.bs[2]));
    int in = ((ix & ((1 << v.bs[0]) - 1)) << v.sh[0]) + ((iy & ((1 << v.bs[1]) - 1)) << v.sh[1]) +
             ((iz & ((1 << v.bs[2]) - 1)) << v.sh[2]);
    return brick * 32 + in;
}

// Elementary functions: the device math library in FP32; in FP64 the
// fixed-sequence implementations of det_math.h.
template <typename Real> struct Math;
template <> struct Math<float> {
    MCRT_HD static float e_exp(float x) { return exp(x); }
    MCRT_HD static float e_expm1(float x) { return expm1(x); }
    MCRT_HD static float e_log(float x) { return log(x); }
    MCRT_HD static float e_log1p(float x) { return log1p(x); }
    MCRT_HD static float e_atanh(float x) { return atanh(x); }
    MCRT_HD static void e_sincos(float x, float &s, float &c)
    {
        s = sin(x);
        c = cos(x);
    }
};
template <> struct Math<double> {
    MCRT_HD static double e_exp(double x) { return dm::exp(x); }
    MCRT_HD static double e_expm1(double x) { return dm::expm1(x); }
    MCRT_HD static double e_log(double x) { return dm::log(x); }
    MCRT_HD static double e_log1p(double x) { return dm::log1p(x); }
    MCRT_HD static double e_atanh(double x) { return dm::atanh(x); }
    MCRT_HD static void e_sincos(double x, double &s, double &c) { dm::sincos(x, s, c); }
};

// Slice containing coordinate p; a point on a plane that the ray leaves
// downwards belongs to the slice below.
template <typename Real> MCRT_HD int slice_index(Real p, Real lo, Real cs, int n, Real k)
{
    Real q = floor((p - lo) / cs);
    int i;
    if (q < Real(0)) i = 0;
    else if (q > Real(n - 1)) i = n - 1;
    else i = (int)q;
    if (p == lo + (Real)i * cs && k < Real(0)) i -= 1;
    return i;
}

// Start of the ray r + t d (t >= 0) in the grid box: t0 and slice indices.
template <typename Real, typename ImgT, int G>
MCRT_HD bool ray_start(const View<Real, ImgT, G> &v, const Real r[3], const Real d[3], Real &t0, int idx[3])
{
    bool inside = true;
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if (!(r[a] >= v.lo[a] && r[a] <= v.hi[a])) inside = false;
    if (inside) {
        t0 = Real(0);
#pragma unroll
        for (int a = 0; a < 3; ++a) idx[a] = slice_index(r[a], v.lo[a], v.cs[a], v.n[a], d[a]);
    } else {
        Real tn = -Prec<Real>::inf(), tf = Prec<Real>::inf();
        int entry = -1;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (d[a] == Real(0)) {
                if (r[a] < v.lo[a] || r[a] > v.hi[a]) return false;
            } else {
                Real t1 = (v.lo[a] - r[a]) / d[a];
                Real t2 = (v.hi[a] - r[a]) / d[a];
                Real nr = t1 < t2 ? t1 : t2;
                Real fr = t1 < t2 ? t2 : t1;
                if (nr > tn) {
                    tn = nr;
                    entry = a;
                }
                if (fr < tf) tf = fr;
            }
        }
        if (entry < 0 || tn > tf || tf < Real(0) || tn < Real(0)) return false;
        t0 = tn;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (a == entry) {
                idx[a] = d[a] > Real(0) ? 0 : v.n[a] - 1;
            } else {
                Real p = r[a] + tn * d[a];
                idx[a] = slice_index(p, v.lo[a], v.cs[a], v.n[a], d[a]);
            }
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if (idx[a] < 0 || idx[a] >= v.n[a]) return false;
    return true;
}

template <typename Real, typename ImgT, int G>
MCRT_HD Real plane_t(const View<Real, ImgT, G> &v, const Lane<Real> &ln, int a, int j)
{
    return Prec<Real>::over_k(v.lo[a] + (Real)j * v.cs[a] - ln.r[a], ln.d[a], ln.id3[a]);
}

template <typename Real, typename ImgT, int G>
MCRT_HD Real next_plane_t(const View<Real, ImgT, G> &v, const Lane<Real> &ln, int a)
{
    if (ln.d[a] > Real(0)) return plane_t(v, ln, a, cidx(ln, a) + 1);
    if (ln.d[a] < Real(0)) return plane_t(v, ln, a, cidx(ln, a));
    return Prec<Real>::inf();
}

// Begins a march from the packet position along direction dir.
template <typename Real, typename ImgT, int G>
MCRT_HD void begin_march(const View<Real, ImgT, G> &v, Lane<Real> &ln, const Real dir[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        ln.d[a] = dir[a];
        ln.id3[a] = dir[a] != Real(0) ? Real(1) / dir[a] : Real(0);
    }
    ln.nseg = 0;
    ln.steps = 0;
    ln.tau = Real(0);
    Real t0;
    int idx[3];
    ln.marching = ray_start(v, ln.r, ln.d, t0, idx);
    ln.c0 = idx[0];
    ln.c1 = idx[1];
    ln.c2 = idx[2];
    ln.t = t0;
    if constexpr (G == kCartesian) {
        if (ln.marching) {
            ln.tn0 = next_plane_t(v, ln, 0);
            ln.tn1 = next_plane_t(v, ln, 1);
            ln.tn2 = next_plane_t(v, ln, 2);
        }
    }
}

// ---------------------------------------------------------------------------
// One segment of the march: finds the cell and its path length, then applies
// the mode's action (deposit, optical-depth sum, interaction search).
// ---------------------------------------------------------------------------
// One geometric step of the march: the cell the ray is in, where it leaves
// it, and the lattice state advanced to the next cell.  Needs no density, so
// several steps can be taken before their density loads complete.  Returns
// true when the ray leaves the grid after this segment.
template <typename Real, typename ImgT, int G>
MCRT_HD bool geo_step(const View<Real, ImgT, G> &v, Lane<Real> &ln, Tally &ty, int &cell, Real &te, float &rho)
{
    bool exits = false;
    if constexpr (G == kCartesian) {
        Real tmin = ln.tn0;
        int am = 0;
        if (ln.tn1 < tmin) {
            tmin = ln.tn1;
            am = 1;
        }
        if (ln.tn2 < tmin) {
            tmin = ln.tn2;
            am = 2;
        }
        te = rmax(tmin, ln.t);
        cell = store_index(v, ln.c0, ln.c1, ln.c2);
        if constexpr (sizeof(Real) == 4) {
            // FP32: branch-free -- the lanes of a wave step different axes.
            // Each axis' next crossing is computed and kept only on the axis
            // stepped (an axis with d = 0 is never stepped: its crossing
            // stays at infinity).
            const int u0 = ln.d[0] > Real(0) ? 1 : 0, u1 = ln.d[1] > Real(0) ? 1 : 0,
                      u2 = ln.d[2] > Real(0) ? 1 : 0;
            ln.c0 += am == 0 ? 2 * u0 - 1 : 0;
            ln.c1 += am == 1 ? 2 * u1 - 1 : 0;
            ln.c2 += am == 2 ? 2 * u2 - 1 : 0;
            exits = (unsigned)ln.c0 >= (unsigned)v.n[0] || (unsigned)ln.c1 >= (unsigned)v.n[1] ||
                    (unsigned)ln.c2 >= (unsigned)v.n[2];
            const Real p0 = plane_t(v, ln, 0, ln.c0 + u0), p1 = plane_t(v, ln, 1, ln.c1 + u1),
                       p2 = plane_t(v, ln, 2, ln.c2 + u2);
            ln.tn0 = am == 0 ? p0 : ln.tn0;
            ln.tn1 = am == 1 ? p1 : ln.tn1;
            ln.tn2 = am == 2 ? p2 : ln.tn2;
            return exits;
        }
        // explicit per-axis branches (a loop over `a == am` gets folded into a
        // runtime-indexed store, which would move the arrays to scratch)
        if (am == 0) {
            ln.c0 += ln.d[0] > Real(0) ? 1 : -1;
            exits = ln.c0 < 0 || ln.c0 >= v.n[0];
            if (!exits) ln.tn0 = next_plane_t(v, ln, 0);
        } else if (am == 1) {
            ln.c1 += ln.d[1] > Real(0) ? 1 : -1;
            exits = ln.c1 < 0 || ln.c1 >= v.n[1];
            if (!exits) ln.tn1 = next_plane_t(v, ln, 1);
        } else {
            ln.c2 += ln.d[2] > Real(0) ? 1 : -1;
            exits = ln.c2 < 0 || ln.c2 >= v.n[2];
            if (!exits) ln.tn2 = next_plane_t(v, ln, 2);
        }
    } else {
        // locate the leaf holding lattice point ci: dense top table, then one
        // load per two levels (blocks of 4 x 4 x 4 sub-cubes)
        const int sh = v.depth - v.top_level;
        unsigned long long e64 = v.top[top_index(ln.c0 >> sh, ln.c1 >> sh, ln.c2 >> sh, v.top_level)];
        uint32_t e = (uint32_t)e64;
        int lv = v.top_level;
        while (!(e >> 31)) {
            const int s = v.depth - 1 - lv;
            const int i = (((ln.c0 << 1) >> s) & 3) + 4 * (((ln.c1 << 1) >> s) & 3) + 16 * (((ln.c2 << 1) >> s) & 3);
            e64 = v.node[((long long)e << 6) + i];
            e = (uint32_t)e64;
            lv += 2;
        }
        const int level = (int)((e >> 27) & 15u);
        cell = (int)(e & ((1u << 27) - 1));
        rho = __builtin_bit_cast(float, (uint32_t)(e64 >> 32));
        const int size = 1 << (v.depth - level);
        int o[3];
        Real tn[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            o[a] = cidx(ln, a) & ~(size - 1);
            const Real t = plane_t(v, ln, a, ln.d[a] > Real(0) ? o[a] + size : o[a]);
            tn[a] = ln.d[a] != Real(0) ? t : Prec<Real>::inf();
        }
        Real tmin = tn[0];
        int am = 0;
        if (tn[1] < tmin) {
            tmin = tn[1];
            am = 1;
        }
        if (tn[2] < tmin) {
            tmin = tn[2];
            am = 2;
        }
        te = rmax(tmin, ln.t);
        // the stepped axis moves to the next cube; the others take the
        // lattice cell of the exit point, clamped to the leaf (selects: the
        // lanes of a wave step different axes)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int hi = o[a] + size - 1;
            const int q = ln.d[a] > Real(0) ? hi + 1 : o[a] - 1;
            const Real p = ln.r[a] + te * ln.d[a];
            // truncation, then the clamp into [o, hi]: the same as floor
            // then the clamp, since o >= 0 (p stays within the leaf up to
            // rounding, so the conversion never overflows)
            const int t = (int)Prec<Real>::over_k(p - v.lo[a], v.cs[a], v.ics[a]);
            const int qi = t < o[a] ? o[a] : (t > hi ? hi : t);
            exits = exits || (a == am && (unsigned)q >= (unsigned)v.n[a]);
            cidx(ln, a) = a == am ? q : qi;
        }
        if (++ln.steps >= v.octree_guard) {
            exits = true;
            ty.guard++;
        }
    }
    return exits;
}

// Applies one segment (cell, start, length, density) to the lane's march:
// continuous-absorption deposit, interaction search or optical-depth sum.
// Returns true when the march stops here (interaction found, peel-off cut).
template <typename Real, typename ImgT, int G, typename Sink>
MCRT_HD bool apply_segment(const View<Real, ImgT, G> &v, Lane<Real> &ln, Tally &ty, Sink &sink, int cell,
                           Real t_start, Real ds, float rho)
{
    ln.nseg++;
    const Real kr = ln.opt.kappa * (Real)rho;
    const Real dtau = kr * ds;
    const Real tprev = ln.tau;
    ln.tau = tprev + dtau;
    if (ln.mode == kProp) {
        Real x = -Math<Real>::e_expm1(-dtau);
        Real A = ln.wabs * ln.E * x;
        sink.deposit(v.table, (long long)ln.lam * v.n_store, cell, (double)A);
        ty.absorbed += (double)A;
        ln.E = ln.E * (Real(1) - x);
        ty.prop_cells++;
        return false;
    }
    // interaction search and peel-off depth, written as selects: the lanes of
    // a wave mix both
    const bool loc = ln.mode == kLocate;
    const bool save = loc && dtau > Real(0); // last segment with positive depth
    ln.a_t0 = save ? t_start : ln.a_t0;
    ln.a_tau = save ? tprev : ln.a_tau;
    ln.a_kr = save ? kr : ln.a_kr;
    ln.a_ds = save ? ds : ln.a_ds;
    ln.rho_star = save ? (Real)rho : ln.rho_star;
    ty.locate_cells += loc ? 1u : 0u;
    ty.peel_cells += loc ? 0u : 1u;
    const bool hit = ln.tau >= (loc ? ln.tau_int : v.tau_peel_max);
    ln.found = ln.found || (hit && loc);
    ln.dropped = ln.dropped || (hit && !loc);
    return hit;
}

// K segments of the march: K geometric steps, then (Cartesian) K independent
// density loads in flight together, then the segments applied in order (the
// same operations in the same order as one segment at a time).  A Cartesian
// step is pure arithmetic, so it also runs past the ray's exit (its results
// are not used) rather than branching; every load reads a valid cell.  An
// octree step's walk entry carries the leaf's density.
template <int K, typename Real, typename ImgT, int G, typename Sink>
MCRT_HD void march_batch(const View<Real, ImgT, G> &v, Lane<Real> &ln, Tally &ty, Sink &sink)
{
    int cell[K];
    Real ts[K], ds[K];
    float rho[K];
    bool ok[K];
    bool more = true;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        ok[k] = more;
        cell[k] = 0;
        rho[k] = 0.0f;
        ts[k] = ln.t;
        ds[k] = Real(0);
        if (G == kCartesian || more) {
            Real te;
            bool exits = geo_step(v, ln, ty, cell[k], te, rho[k]);
            ds[k] = te - ln.t;
            ln.t = te;
            more = more && !exits;
        }
    }
    // Cartesian: the densities of the K cells, loaded together; an octree
    // step found its leaf's density in the walk entry
    if constexpr (G == kCartesian) {
#pragma unroll
        for (int k = 0; k < K; ++k) rho[k] = gload(v.density, ok[k] ? cell[k] : 0);
    }
    bool stop = false;
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (ok[k] && !stop) stop = apply_segment(v, ln, ty, sink, cell[k], ts[k], ds[k], rho[k]);
    if (stop || !more) ln.marching = false;
}

// Segments per march iteration: the Cartesian step is pure arithmetic, so
// four loads can be put in flight; the octree step itself reads the tree.
template <int G> struct BatchOf {
    static constexpr int value = G == kCartesian ? 4 : 2;
};

template <typename Real, typename ImgT, int G, typename Sink>
MCRT_HD void march_step(const View<Real, ImgT, G> &v, Lane<Real> &ln, Tally &ty, Sink &sink)
{
    march_batch<BatchOf<G>::value>(v, ln, ty, sink);
}

// ---------------------------------------------------------------------------
// Event processing between marches.
// ---------------------------------------------------------------------------
template <typename Real> MCRT_HD Real hg_phase(Real g, Real mu)
{
    Real num = Real(1) - g * g;
    Real den = Real(1) + g * g - Real(2) * g * mu;
    return num / (den * sqrt(den));
}

template <typename Real> MCRT_HD Real hg_sample(Real g, Real u)
{
    Real mu;
    if (fabs(g) >= Real(1e-6)) {
        Real q = (Real(1) - g * g) / (Real(1) - g + Real(2) * g * u);
        mu = (Real(1) + g * g - q * q) / (Real(2) * g);
    } else {
        mu = Real(2) * u - Real(1);
    }
    if (mu < Real(-1)) mu = Real(-1);
    if (mu > Real(1)) mu = Real(1);
    return mu;
}

template <typename Real>
MCRT_HD void rotate_about_pole(Real a, Real b, Real c, Real mu, Real st, Real cp, Real sp, Real &x, Real &y, Real &z)
{
    Real s = sqrt(Real(1) - c * c);
    x = mu * a + st * (a * c * cp - b * sp) / s;
    y = mu * b + st * (b * c * cp + a * sp) / s;
    z = mu * c - st * s * cp;
}

// New direction at polar cosine mu and azimuth phi about k (the x axis
// replaces z as the azimuth reference within 0.00447 rad of the z axis).
template <typename Real> MCRT_HD void rotate(Real k[3], Real mu, Real phi)
{
    Real st = sqrt(rmax(Real(0), Real(1) - mu * mu));
    Real sp, cp;
    Math<Real>::e_sincos(phi, sp, cp);
    Real x, y, z;
    if (fabs(k[2]) < Real(0.99999)) {
        rotate_about_pole(k[0], k[1], k[2], mu, st, cp, sp, x, y, z);
    } else {
        Real px, py, pz;
        rotate_about_pole(k[1], k[2], k[0], mu, st, cp, sp, py, pz, px);
        x = px;
        y = py;
        z = pz;
    }
    Real nrm = sqrt(x * x + y * y + z * z);
    k[0] = x / nrm;
    k[1] = y / nrm;
    k[2] = z / nrm;
}

template <typename Real> struct Consts {
    MCRT_HD static Real two_pi() { return Real(6.283185307179586476925286766559); }
};

template <typename Real, typename ImgT, int G>
MCRT_HD Stream stream_of(const View<Real, ImgT, G> &v, const Lane<Real> &ln)
{
    return Stream{v.key0, v.key1, ln.id, ln.lam, v.model};
}

// Optical depth to the boundary along axis A from the lane's march start:
// the start cell from the start point to its exit face, then the column
// beyond it (Cartesian grids).
template <int A, typename Real, typename ImgT, int G>
MCRT_HD Real column_tau(const View<Real, ImgT, G> &v, const Lane<Real> &ln, const Real *col)
{
    const Real tn = A == 0 ? ln.tn0 : (A == 1 ? ln.tn1 : ln.tn2);
    const int cell = store_index(v, ln.c0, ln.c1, ln.c2);
    return ln.opt.kappa * ((Real)gload(v.density, cell) * (tn - ln.t) + gload(col, cell));
}

// Octree grids: optical depth to the boundary along lattice axis A from the
// march start, from the cumulative column at lattice resolution (col[c] =
// density x width summed from lattice cell c itself to the boundary on the
// observer's side): the next cell's column plus the part of this cell's
// (their difference) still to cross.
template <int A, typename Real, typename ImgT, int G>
MCRT_HD Real octree_column_tau(const View<Real, ImgT, G> &v, const Lane<Real> &ln, const Real *col)
{
    const long long N = v.n[0];
    const long long idx = (long long)ln.c0 + N * ((long long)ln.c1 + N * (long long)ln.c2);
    const int c = A == 0 ? ln.c0 : (A == 1 ? ln.c1 : ln.c2);
    const bool neg = ln.d[A] < Real(0);
    const long long stride = A == 0 ? 1 : (A == 1 ? N : N * N);
    const bool has_next = (unsigned)(neg ? c - 1 : c + 1) < (unsigned)N;
    const Real Sc = gload(col, idx);
    const Real Sn = gload(col, has_next ? (neg ? idx - stride : idx + stride) : idx);
    const Real Snext = has_next ? Sn : Real(0);
    Real f = Prec<Real>::over_k(plane_t(v, ln, A, neg ? c : c + 1) - ln.t, v.cs[A], v.ics[A]);
    f = f < Real(0) ? Real(0) : (f > Real(1) ? Real(1) : f);
    return ln.opt.kappa * (Snext + (Sc - Snext) * f);
}

template <typename Real, typename ImgT, int G>
MCRT_HD void begin_peel(const View<Real, ImgT, G> &v, Lane<Real> &ln, int j, bool emission)
{
    ln.mode = emission ? kPeelEmit : kPeelScat;
    ln.j = j;
    ln.dropped = false;
    const InsDesc<Real> &in = v.ins[j];
    Real w;
    if (emission) {
        Real s = v.src_type == kPointAniso ? Real(2) * fabs(in.kobs[2]) : Real(1);
        w = ln.L0 * s;
    } else {
        Real mu = ln.k[0] * in.kobs[0] + ln.k[1] * in.kobs[1] + ln.k[2] * in.kobs[2];
        w = ln.L * hg_phase(ln.opt.g, mu);
    }
    ln.wpeel = w;
    begin_march(v, ln, in.kobs);
    if constexpr (G == kCartesian) {
        if (in.col != nullptr && ln.marching) {
            // optical depth to the boundary along the axis: this cell from the
            // start point to its exit face, then the column beyond it
            // per-axis copies with compile-time axis numbers: a runtime choice
            // among the lane's per-axis fields would move the lane to scratch
            const int a = in.col_axis >> 1;
            Real tau;
            if (a == 0) tau = column_tau<0>(v, ln, in.col);
            else if (a == 1) tau = column_tau<1>(v, ln, in.col);
            else tau = column_tau<2>(v, ln, in.col);
            ln.tau = tau;
            ln.dropped = tau >= v.tau_peel_max;
            ln.nseg = 1;
            ln.marching = false;
        }
    } else {
        if (in.col != nullptr && ln.marching) {
            const int a = in.col_axis >> 1;
            Real tau;
            if (a == 0) tau = octree_column_tau<0>(v, ln, in.col);
            else if (a == 1) tau = octree_column_tau<1>(v, ln, in.col);
            else tau = octree_column_tau<2>(v, ln, in.col);
            ln.tau = tau;
            ln.dropped = tau >= v.tau_peel_max;
            ln.nseg = 1;
            ln.marching = false;
        }
    }
}

template <typename Real, typename ImgT, int G>
MCRT_HD void begin_prop(const View<Real, ImgT, G> &v, Lane<Real> &ln)
{
    ln.mode = kProp;
    ln.wabs = (Real(1) - ln.opt.albedo) * ln.L;
    ln.E = Real(1);
    begin_march(v, ln, ln.k);
}

template <typename Real, typename ImgT, int G>
MCRT_HD void begin_locate(const View<Real, ImgT, G> &v, Lane<Real> &ln)
{
    ln.mode = kLocate;
    ln.found = false;
    begin_march(v, ln, ln.k);
}

// ---------------------------------------------------------------------------
// Learned direction proposal and plain-run histories
// ---------------------------------------------------------------------------
template <typename Real> struct Bf16;
template <> struct Bf16<float> {
    // nearest-even rounding to bfloat16, returned as float
    MCRT_HD static float round(float x)
    {
        uint32_t b;
        __builtin_memcpy(&b, &x, sizeof b);
        b = ((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16) << 16;
        float r;
        __builtin_memcpy(&r, &b, sizeof r);
        return r;
    }
};
template <> struct Bf16<double> {
    MCRT_HD static double round(double x) { return (double)Bf16<float>::round((float)x); }
};

// Which optional features a kernel variant carries is a compile-time
// property of its sink (Sink::kLearn, Sink::kHist); the View's runtime fields
// then select them.  Variants without a feature compile without its code.
template <typename Sink, typename Real, typename ImgT, int G> MCRT_HD bool learned_on(const View<Real, ImgT, G> &v)
{
    return Sink::kLearn && v.learned != 0;
}
template <typename Sink, typename Real, typename ImgT, int G> MCRT_HD bool hist_on(const View<Real, ImgT, G> &v)
{
    return Sink::kHist && v.hist != nullptr;
}

// Packet end: the total image flux of the packet goes to the histories.
template <typename Sink, typename Real, typename ImgT, int G>
MCRT_HD void end_packet(const View<Real, ImgT, G> &v, Lane<Real> &ln)
{
    ln.mode = kDead;
    ln.marching = false;
    if (hist_on<Sink>(v)) v.hist_total[ln.slot] = ln.flux;
}

// Features: position / r_out, incoming direction (zero at emission), the
// wavelength feature, log10 of the interaction cell's density over the mean
// (zero at emission), event flag.
template <typename Real, typename ImgT, int G>
MCRT_HD void event_features(const View<Real, ImgT, G> &v, const Lane<Real> &ln, bool scattering, Real f[9])
{
    const Real inv_ln10 = Real(0.43429448190325182765);
    for (int a = 0; a < 3; ++a) f[a] = ln.r[a] / v.r_out;
    for (int a = 0; a < 3; ++a) f[3 + a] = scattering ? ln.k[a] : Real(0);
    f[6] = ln.opt.lamf;
    f[7] = scattering ? Math<Real>::e_log(ln.rho_star / v.rho_mean) * inv_ln10 : Real(0);
    f[8] = scattering ? Real(1) : Real(0);
}

template <typename Real, typename ImgT, int G>
MCRT_HD void record_event(const View<Real, ImgT, G> &v, const Lane<Real> &ln, long long e, const Real f[9],
                          const Real kp[3], Real L)
{
    if (!v.hist || e >= v.hist_events) return;
    Real *h = v.hist + ((long long)ln.slot * v.hist_events + e) * kHistFloats;
    for (int i = 0; i < 9; ++i) h[i] = f[i];
    for (int i = 0; i < 3; ++i) h[9 + i] = kp[i];
    h[12] = L;
    h[13] = ln.flux;
}

// The proposal network one sample at a time: bf16-rounded inputs and hidden
// activations, sums over the inputs in order, then the bias.
template <typename Real>
MCRT_HD void mlp_forward_scalar(const double *theta, const Real f[9], Real out[40])
{
    const double *W1 = theta, *b1 = W1 + 9 * 64, *W2 = b1 + 64, *b2 = W2 + 64 * 64;
    const double *W3 = b2 + 64, *b3 = W3 + 64 * 40;
    Real x[9], h1[64], h2[64];
    for (int k = 0; k < 9; ++k) x[k] = Bf16<Real>::round(f[k]);
    for (int j = 0; j < 64; ++j) {
        Real acc = Real(0);
        for (int k = 0; k < 9; ++k) acc = acc + x[k] * (Real)W1[k * 64 + j];
        Real z = acc + (Real)b1[j];
        h1[j] = Bf16<Real>::round(z > Real(0) ? z : Real(0));
    }
    for (int j = 0; j < 64; ++j) {
        Real acc = Real(0);
        for (int k = 0; k < 64; ++k) acc = acc + h1[k] * (Real)W2[k * 64 + j];
        Real z = acc + (Real)b2[j];
        h2[j] = Bf16<Real>::round(z > Real(0) ? z : Real(0));
    }
    for (int j = 0; j < 40; ++j) {
        Real acc = Real(0);
        for (int k = 0; k < 64; ++k) acc = acc + h2[k] * (Real)W3[k * 40 + j];
        out[j] = acc + (Real)b3[j];
    }
}

template <typename Real> struct Consts4 {
    MCRT_HD static Real four_pi() { return Real(12.566370614359172953850573533118); }
};

// Direction from the proposal q = alpha p_phys + (1 - alpha) sum_j pi_j vMF_j
// given the network outputs o[40]; the packet carries W = p_phys / q.  Then the
// next propagation (after a scattering: the event count and cap first).  The
// outputs are turned into the mixture in place (o[j] = pi_j, o[8+3j..] = mu_j,
// o[32+j] = kappa_j), so o may be a row of a shared-memory tile.
template <typename Sink, typename Real, typename ImgT, int G, typename Ptr>
MCRT_HD void apply_proposal(const View<Real, ImgT, G> &v, Lane<Real> &ln, Tally &ty, Ptr o)
{
    Real mx = o[0];
    for (int j = 1; j < 8; ++j)
        if (o[j] > mx) mx = o[j];
    Real sum = Real(0);
    for (int j = 0; j < 8; ++j) {
        Real e = Math<Real>::e_exp(o[j] - mx);
        o[j] = e;
        sum = sum + e;
    }
    for (int j = 0; j < 8; ++j) {
        o[j] = o[j] / sum;
        Real a = o[8 + 3 * j], b = o[9 + 3 * j], c = o[10 + 3 * j];
        Real nrm = sqrt(a * a + b * b + c * c);
        if (nrm > Real(0)) {
            o[8 + 3 * j] = a / nrm;
            o[9 + 3 * j] = b / nrm;
            o[10 + 3 * j] = c / nrm;
        } else {
            o[8 + 3 * j] = Real(0);
            o[9 + 3 * j] = Real(0);
            o[10 + 3 * j] = Real(1);
        }
        Real sj = o[32 + j];
        Real sp = Math<Real>::e_log1p(Math<Real>::e_exp(-fabs(sj))) + (sj > Real(0) ? sj : Real(0));
        Real k = sp + Real(1e-3);
        if (k < Real(1e-3)) k = Real(1e-3);
        if (k > Real(1e3)) k = Real(1e3);
        o[32 + j] = k;
    }
    Stream st = stream_of(v, ln);
    const bool emis = ln.emis_dir;
    // u1: slot 5 (emission) or 8e+1; u2, u3: slots 6, 7 or 8e+2, 8e+3 (one Philox block)
    Real u1 = st.template slot<Real>(emis ? 5u : (uint32_t)(8 * ln.e + 1));
    Real u2, u3;
    st.template pair<Real>(emis ? 3u : (uint32_t)(4 * ln.e + 1), u2, u3);
    Real kp[3];
    if (u3 < v.alpha) {
        if (emis) {
            Real m;
            if (v.src_type == kPointAniso) m = u1 < Real(0.5) ? sqrt(Real(2) * u1) : -sqrt(Real(2) * u1 - Real(1));
            else m = Real(2) * u1 - Real(1);
            Real phi = Consts<Real>::two_pi() * u2;
            Real s = sqrt(rmax(Real(0), Real(1) - m * m));
            Real sphi, cphi;
            Math<Real>::e_sincos(phi, sphi, cphi);
            kp[0] = s * cphi;
            kp[1] = s * sphi;
            kp[2] = m;
        } else {
            kp[0] = ln.k[0];
            kp[1] = ln.k[1];
            kp[2] = ln.k[2];
            rotate(kp, hg_sample(ln.opt.g, u1), Consts<Real>::two_pi() * u2);
        }
    } else {
        Real w = (u3 - v.alpha) / (Real(1) - v.alpha), c = Real(0);
        int j = 7;
        for (int i = 0; i < 8; ++i) {
            c = c + o[i];
            if (w < c) {
                j = i;
                break;
            }
        }
        Real kj = o[32 + j];
        Real cw = Real(1) + Math<Real>::e_log(u1 + (Real(1) - u1) * Math<Real>::e_exp(Real(-2) * kj)) / kj;
        if (cw < Real(-1)) cw = Real(-1);
        if (cw > Real(1)) cw = Real(1);
        kp[0] = o[8 + 3 * j];
        kp[1] = o[9 + 3 * j];
        kp[2] = o[10 + 3 * j];
        rotate(kp, cw, Consts<Real>::two_pi() * u2);
    }
    Real pphys;
    if (emis) {
        Real S = v.src_type == kPointAniso ? Real(2) * fabs(kp[2]) : Real(1);
        pphys = S / Consts4<Real>::four_pi();
    } else {
        Real cosang = ln.k[0] * kp[0] + ln.k[1] * kp[1] + ln.k[2] * kp[2];
        pphys = hg_phase(ln.opt.g, cosang) / Consts4<Real>::four_pi();
    }
    Real qv = Real(0);
    for (int j = 0; j < 8; ++j) {
        Real kj = o[32 + j];
        Real dot = o[8 + 3 * j] * kp[0] + o[9 + 3 * j] * kp[1] + o[10 + 3 * j] * kp[2];
        Real fj = kj / (Consts<Real>::two_pi() * -Math<Real>::e_expm1(Real(-2) * kj)) *
                  Math<Real>::e_exp(kj * (dot - Real(1)));
        qv = qv + o[j] * fj;
    }
    Real q = v.alpha * pphys + (Real(1) - v.alpha) * qv;
    ln.parked = false;
    const Real Lin = emis ? ln.L0 : ln.L;
    ln.L = Lin * (pphys / q);
    // a network that outputs NaN or infinity (diverged parameters) gives a
    // non-finite weight, and a non-finite direction always does: the packet
    // ends, counted, before the direction is marched; its luminosity before
    // the weight is truncated, as at the event cap
    if (!__builtin_isfinite(ln.L)) {
        ty.truncated += (double)Lin;
        ty.nonfinite++;
        end_packet<Sink>(v, ln);
        return;
    }
    ln.k[0] = kp[0];
    ln.k[1] = kp[1];
    ln.k[2] = kp[2];
    if (!emis) ln.e = ln.e + 1;
    ln.mode = kNewDir; // the event loop starts the propagation (or applies the cap)
    ln.marching = false;
}

// Scattering: new HG direction (or the learned proposal), then the next
// propagation (or the event cap).
template <typename Sink, typename Real, typename ImgT, int G>
MCRT_HD void scatter(const View<Real, ImgT, G> &v, Lane<Real> &ln, Tally &ty)
{
    if (learned_on<Sink>(v)) {
        ln.mode = kDead;
        ln.parked = true;
        ln.emis_dir = false;
        ln.marching = false;
        return;
    }
    Real f[9];
    if (hist_on<Sink>(v)) event_features(v, ln, true, f);
    Stream st = stream_of(v, ln);
    Real u1 = st.template slot<Real>((uint32_t)(8 * ln.e + 1));
    Real u2 = st.template slot<Real>((uint32_t)(8 * ln.e + 2));
    Real mu = hg_sample(ln.opt.g, u1);
    Real phi = Consts<Real>::two_pi() * u2;
    rotate(ln.k, mu, phi);
    if (hist_on<Sink>(v)) record_event(v, ln, ln.e, f, ln.k, ln.L);
    ln.e = ln.e + 1;
    if (ln.e > v.event_cap) {
        ty.truncated += (double)ln.L;
        ty.capped++;
        end_packet<Sink>(v, ln);
        return;
    }
    begin_prop(v, ln);
}

// After the emission peel-offs: the emission direction (already sampled, or
// left to the learned proposal for point sources), then the first propagation.
// Point sources take the learned proposal at emission; extended sources
// (disk, dust) sample their own emission direction.
template <typename Real, typename ImgT, int G> MCRT_HD bool point_source(const View<Real, ImgT, G> &v)
{
    return v.src_type == kPointIso || v.src_type == kPointAniso;
}

// Dust emission: the first cell (natural order) whose running sum exceeds
// u times the wavelength's total.  The guide brackets the answer between
// guide[k - 1] and guide[k + 2], k = floor(x K / total), then bisection.
template <typename Real, typename ImgT, int G>
MCRT_HD long long dust_cell(const View<Real, ImgT, G> &v, uint32_t lam, double u)
{
    const long long n = v.n_cells;
    const double *cdf = v.dust_cdf + (long long)lam * n;
    const double total = cdf[n - 1];
    if (!(total > 0.0)) return n - 1;
    const double x = u * total;
    const int K = v.dust_K;
    const int *guide = v.dust_guide + (long long)lam * K;
    const double step = total / (double)K;
    double q = x / step;
    int k = q < (double)K ? (int)q : K - 1;
    long long lo = k > 0 ? guide[k - 1] : 0;
    long long hi = k + 2 < K ? guide[k + 2] : n - 1;
    while (lo < hi) {
        const long long mid = lo + (hi - lo) / 2;
        if (cdf[mid] > x) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

template <typename Sink, typename Real, typename ImgT, int G>
MCRT_HD void emission_done(const View<Real, ImgT, G> &v, Lane<Real> &ln)
{
    if (learned_on<Sink>(v) && point_source(v)) {
        ln.mode = kDead;
        ln.parked = true;
        ln.emis_dir = true;
        ln.marching = false;
        return;
    }
    if (hist_on<Sink>(v)) {
        Real f[9];
        event_features(v, ln, false, f);
        record_event(v, ln, 0, f, ln.k, ln.L0);
    }
    begin_prop(v, ln);
}

// Launches packet (lam, id): position, direction, emission peel-offs.
template <typename Sink, typename Real, typename ImgT, int G>
MCRT_HD void launch(const View<Real, ImgT, G> &v, Lane<Real> &ln, Tally &ty, uint32_t lam, uint32_t id,
                    uint32_t slot)
{
    ln.lam = lam;
    ln.id = id;
    ln.slot = slot;
    ln.flux = Real(0);
    ln.emis_dir = false;
    ln.parked = false;
    ln.opt = v.optics[lam]; // (LDS or device memory: a generic load)
    Stream st = stream_of(v, ln);
    // dust sources exist in the plain kernels only
    constexpr bool kDustOn = !Sink::kLearn && !Sink::kHist;
    if (kDustOn && v.src_type == kDust) {
        // the emitting cell, then a uniform point inside it
        Real u0, u1, u2, u3;
        st.template pair<Real>(0, u0, u1);
        st.template pair<Real>(1, u2, u3);
        const long long m = dust_cell(v, lam, (double)u0);
        if constexpr (G == kCartesian) {
            const long long nxy = (long long)v.n[0] * v.n[1];
            const int ix = (int)(m % v.n[0]), iy = (int)((m / v.n[0]) % v.n[1]), iz = (int)(m / nxy);
            ln.r[0] = v.lo[0] + ((Real)ix + u1) * v.cs[0];
            ln.r[1] = v.lo[1] + ((Real)iy + u2) * v.cs[1];
            ln.r[2] = v.lo[2] + ((Real)iz + u3) * v.cs[2];
        } else {
            const int *lf = v.dust_leaf + 4 * m;
            const Real size = (Real)(1 << (v.depth - lf[3]));
            ln.r[0] = v.lo[0] + ((Real)lf[0] + u1 * size) * v.cs[0];
            ln.r[1] = v.lo[1] + ((Real)lf[1] + u2 * size) * v.cs[1];
            ln.r[2] = v.lo[2] + ((Real)lf[2] + u3 * size) * v.cs[2];
        }
    } else if (v.src_type == kExpDisk) {
        Real u0, u1, u2, u3;
        st.template pair<Real>(0, u0, u1);
        st.template pair<Real>(1, u2, u3);
        Real R = -v.hR * Math<Real>::e_log(u0 * u1);
        Real phi = Consts<Real>::two_pi() * u2;
        Real z = v.zs * Math<Real>::e_atanh(Real(2) * u3 - Real(1));
        Real sphi, cphi;
        Math<Real>::e_sincos(phi, sphi, cphi);
        ln.r[0] = R * cphi;
        ln.r[1] = R * sphi;
        ln.r[2] = z;
    } else {
        ln.r[0] = v.src_pos[0];
        ln.r[1] = v.src_pos[1];
        ln.r[2] = v.src_pos[2];
    }
    if (!(learned_on<Sink>(v) && point_source(v))) {
        Real u4, u5, u6, u7;
        st.template pair<Real>(2, u4, u5);
        st.template pair<Real>(3, u6, u7);
        Real mu;
        if (v.src_type == kPointAniso) mu = u5 < Real(0.5) ? sqrt(Real(2) * u5) : -sqrt(Real(2) * u5 - Real(1));
        else mu = Real(2) * u5 - Real(1);
        Real phi = Consts<Real>::two_pi() * u6;
        Real s = sqrt(rmax(Real(0), Real(1) - mu * mu));
        Real sphi, cphi;
        Math<Real>::e_sincos(phi, sphi, cphi);
        ln.k[0] = s * cphi;
        ln.k[1] = s * sphi;
        ln.k[2] = mu;
    }
    ln.L0 = ln.opt.L0;
    ln.L = ln.L0;
    ln.e = 1;
    ty.emitted += (double)ln.L0;
    ty.packets++;
    ln.marching = false;
    // a packet without luminosity (a wavelength the source does not emit at)
    // would add zero everywhere: it ends at launch
    ln.mode = ln.L0 > Real(0) ? kLaunched : kDead;
}

// Handles the end of a march; leaves the lane marching again, dead, or
// waiting for the learned proposal.
template <typename Real, typename ImgT, int G, typename Sink>
MCRT_HD void finish_march(const View<Real, ImgT, G> &v, Lane<Real> &ln, Tally &ty, Sink &sink)
{
    if (ln.mode == kLaunched) {
        if (v.n_ins > 0) begin_peel(v, ln, 0, true);
        else emission_done<Sink>(v, ln);
        return;
    }
    if (Sink::kLearn && ln.mode == kNewDir) {
        if (ln.e > v.event_cap) {
            ty.truncated += (double)ln.L;
            ty.capped++;
            end_packet<Sink>(v, ln);
            return;
        }
        begin_prop(v, ln);
        return;
    }
    if (ln.mode == kPeelEmit || ln.mode == kPeelScat) {
        const InsDesc<Real> &in = v.ins[ln.j];
        if (ln.dropped) {
            ty.peel_dropped++;
        } else {
            Real x = ln.r[0] * in.ex[0] + ln.r[1] * in.ex[1] + ln.r[2] * in.ex[2];
            Real y = ln.r[0] * in.ey[0] + ln.r[1] * in.ey[1] + ln.r[2] * in.ey[2];
            Real px = floor((x + in.half_fovx) / in.pixx);
            Real py = floor((y + in.half_fovy) / in.pixy);
            if (px >= Real(0) && px < Real(in.nx) && py >= Real(0) && py < Real(in.ny)) {
                long long idx = in.offset + ((long long)ln.lam * in.ny + (long long)py) * in.nx + (long long)px;
                Real val = ln.wpeel * Math<Real>::e_exp(-ln.tau);
                sink.pixel(ln, v.images, idx, (ImgT)val);
                if (hist_on<Sink>(v)) ln.flux = ln.flux + val * in.inv4pid2;
                ty.peel_adds++;
            }
        }
        int j = ln.j + 1;
        bool emission = ln.mode == kPeelEmit;
        if (j < v.n_ins) {
            begin_peel(v, ln, j, emission);
        } else if (emission) {
            emission_done<Sink>(v, ln);
        } else {
            scatter<Sink>(v, ln, ty);
        }
        return;
    }
    if (ln.mode == kProp) {
        const Real Epath = ln.E;
        // L * Epath is finite exactly when both factors are (Epath <= 1): a
        // packet whose luminosity or transmission went NaN or infinite ends
        // here, counted, before it feeds another tally
        const Real esc = ln.L * Epath;
        if (!__builtin_isfinite(esc)) {
            ty.nonfinite++;
            end_packet<Sink>(v, ln);
            return;
        }
        ty.escaped += (double)esc;
        if (ln.nseg == 0 || ln.opt.albedo == Real(0) || ln.tau == Real(0)) {
            end_packet<Sink>(v, ln);
            return;
        }
        Real Ls = ln.opt.albedo * ln.L * (Real(1) - Epath);
        if (Ls < v.w_min * ln.L0) {
            ty.truncated += (double)Ls;
            end_packet<Sink>(v, ln);
            return;
        }
        Stream st = stream_of(v, ln);
        Real u = st.template slot<Real>((uint32_t)(8 * ln.e + 0));
        ln.tau_int = -Math<Real>::e_log1p(-u * (Real(1) - Epath));
        ln.L = Ls;
        begin_locate(v, ln);
        return;
    }
    if (ln.mode == kLocate) {
        Real inside = (ln.tau_int - ln.a_tau) / ln.a_kr;
        if (inside < Real(0)) inside = Real(0);
        if (inside > ln.a_ds) inside = ln.a_ds;
        Real dist = ln.a_t0 + inside;
        ln.r[0] = ln.r[0] + ln.k[0] * dist;
        ln.r[1] = ln.r[1] + ln.k[1] * dist;
        ln.r[2] = ln.r[2] + ln.k[2] * dist;
        ty.events++;
        if (v.n_ins > 0) begin_peel(v, ln, 0, false);
        else scatter<Sink>(v, ln, ty);
        return;
    }
    end_packet<Sink>(v, ln);
}

template <typename Real, typename ImgT, int G, typename Sink>
MCRT_HD void settle(const View<Real, ImgT, G> &v, Lane<Real> &ln, Tally &ty, Sink &sink)
{
    while (!ln.marching && ln.mode != kDead) finish_march(v, ln, ty, sink);
}

// One sample at a time: features, network, proposal (host simulator and the
// FP64 validation kernel; the FP32 kernel evaluates the network per wave).
// Leaves the lane marching, dead, or with a finished march to settle.
template <typename Sink, typename Real, typename ImgT, int G>
MCRT_HD void resolve_direction_scalar(const View<Real, ImgT, G> &v, Lane<Real> &ln, Tally &ty)
{
    Real f[9], o[40];
    event_features(v, ln, !ln.emis_dir, f);
    mlp_forward_scalar(v.mlp64, f, o);
    apply_proposal<Sink>(v, ln, ty, (Real *)o);
}

} // namespace mcrt
