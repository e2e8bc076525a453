// scene_setup.h -- host-side preparation of the per-simulation constants the
// transport lanes read: instrument frames, per-wavelength optics and the
// octree node encoding.  Shared by the C-ABI library and the host lane
// simulator so both see identical constants.
#pragma once

#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

namespace mcrt {

struct HostInstrument {
    double incl_deg, azim_deg, distance, fov[2];
    int32_t npix[2];
};

// Distant observer frame (parallel projection): k_obs towards the observer,
// sky basis e_x = (-sin a, cos a, 0), e_y = (-cos i cos a, -cos i sin a, sin i).
template <typename Real>
inline void make_ins_desc(const HostInstrument &h, long long offset, InsDesc<Real> &o, double &inv4pid2)
{
    const double pi = 3.14159265358979323846;
    double i = h.incl_deg * pi / 180.0, a = h.azim_deg * pi / 180.0;
    double si = std::sin(i), ci = std::cos(i), sa = std::sin(a), ca = std::cos(a);
    double kobs[3] = {si * ca, si * sa, ci};
    double ex[3] = {-sa, ca, 0.0};
    double ey[3] = {-ci * ca, -ci * sa, si};
    for (int c = 0; c < 3; ++c) {
        o.kobs[c] = (Real)kobs[c];
        o.ex[c] = (Real)ex[c];
        o.ey[c] = (Real)ey[c];
    }
    o.half_fovx = (Real)(0.5 * h.fov[0]);
    o.half_fovy = (Real)(0.5 * h.fov[1]);
    o.pixx = (Real)(h.fov[0] / (double)h.npix[0]);
    o.pixy = (Real)(h.fov[1] / (double)h.npix[1]);
    o.nx = h.npix[0];
    o.ny = h.npix[1];
    o.offset = offset;
    inv4pid2 = 1.0 / (4.0 * pi * h.distance * h.distance);
    o.inv4pid2 = (Real)inv4pid2;
    o.col = nullptr;
    o.col_axis = -1;
}

// Line of sight along a grid axis: one component exactly +-1, the others
// below 1e-12 (cos 90 deg evaluates to 6e-17).  Returns 2 axis + (k < 0), or
// -1.  A ray that drifts by less than 1e-12 of its length off the axis
// crosses no other plane inside the grid (unless it starts within that
// distance of one).
inline int axis_code(const HostInstrument &h)
{
    const double pi = 3.14159265358979323846;
    double i = h.incl_deg * pi / 180.0, a = h.azim_deg * pi / 180.0;
    double k[3] = {std::sin(i) * std::cos(a), std::sin(i) * std::sin(a), std::cos(i)};
    for (int ax = 0; ax < 3; ++ax) {
        if (std::fabs(k[ax]) != 1.0) continue;
        bool ok = true;
        for (int b = 0; b < 3; ++b)
            if (b != ax && std::fabs(k[b]) > 1e-12) ok = false;
        if (ok) return 2 * ax + (k[ax] < 0.0 ? 1 : 0);
    }
    return -1;
}

// Parameters of the proposal network as the FP64 scalar network reads them:
// FP32 master values, weights rounded to bfloat16 (nearest even), biases kept.
// Layout: W1 [9][64], b1 [64], W2 [64][64], b2 [64], W3 [64][40], b3 [40].
inline void mlp_params_f64(const float *theta, std::vector<double> &out)
{
    out.assign((size_t)kMlpParams, 0.0);
    const int w1 = 0, b1 = 9 * 64, w2 = b1 + 64, b2 = w2 + 64 * 64, w3 = b2 + 64, b3 = w3 + 64 * 40;
    for (int i = 0; i < kMlpParams; ++i) {
        bool weight = (i < b1) || (i >= w2 && i < b2) || (i >= w3 && i < b3);
        out[(size_t)i] = weight ? (double)Bf16<float>::round(theta[i]) : (double)theta[i];
    }
    (void)w1;
}

// Constants of the learned proposal's features: r_out = half the largest box
// side, the mean cell density (sequential FP64 sum in cell order) and, per
// wavelength, (log l - log l_min) / (log l_max - log l_min), 0 for a single
// wavelength.
inline void feature_constants(const double box[6], const float *density, long long n_cells,
                              const double *lambda_um, int n_lambda, double &r_out, double &rho_mean,
                              std::vector<double> &lamf)
{
    double side = 0.0;
    for (int a = 0; a < 3; ++a)
        if (box[3 + a] - box[a] > side) side = box[3 + a] - box[a];
    r_out = 0.5 * side;
    double sum = 0.0;
    for (long long m = 0; m < n_cells; ++m) sum = sum + (double)density[m];
    rho_mean = sum / (double)n_cells;
    lamf.assign((size_t)n_lambda, 0.0);
    if (!lambda_um || n_lambda <= 0) return;
    double lmin = lambda_um[0], lmax = lambda_um[0];
    for (int l = 1; l < n_lambda; ++l) {
        if (lambda_um[l] < lmin) lmin = lambda_um[l];
        if (lambda_um[l] > lmax) lmax = lambda_um[l];
    }
    for (int l = 0; l < n_lambda; ++l)
        lamf[l] = lmax > lmin ? (std::log(lambda_um[l]) - std::log(lmin)) / (std::log(lmax) - std::log(lmin)) : 0.0;
}

// Encodes an octree given as first_child (-1 for leaves, children contiguous
// in the order c = bx + 2 by + 4 bz) into node values: >= 0 first child,
// < 0 -(leaf + 1), leaves numbered in depth-first order.  Returns the depth,
// or -1 with a message if the tree is malformed.
inline int encode_octree(int64_t n_nodes, const int32_t *first_child, int64_t n_cells,
                         std::vector<int32_t> &node, std::string &err)
{
    if (n_nodes <= 0 || n_nodes >= (int64_t(1) << 27)) {
        err = "octree: node count out of range (1 .. 2^27-1)";
        return -1;
    }
    node.assign((size_t)n_nodes, 0);
    std::vector<uint8_t> seen((size_t)n_nodes, 0);
    std::vector<std::pair<int64_t, int>> stack;
    stack.reserve(1024);
    stack.push_back({0, 0});
    seen[0] = 1;
    int64_t next_leaf = 0;
    int depth = 0;
    while (!stack.empty()) {
        auto [nd, level] = stack.back();
        stack.pop_back();
        int32_t fc = first_child[nd];
        if (fc < 0) {
            node[(size_t)nd] = (int32_t)(-(next_leaf + 1));
            next_leaf++;
            if (level > depth) depth = level;
        } else {
            if ((int64_t)fc + 7 >= n_nodes || fc <= nd) {
                err = "octree: first_child out of range";
                return -1;
            }
            if (level + 1 > 15) {
                err = "octree: depth exceeds 15";
                return -1;
            }
            node[(size_t)nd] = fc;
            for (int c = 7; c >= 0; --c) {
                if (seen[(size_t)fc + c]) {
                    err = "octree: node reachable twice";
                    return -1;
                }
                seen[(size_t)fc + c] = 1;
                stack.push_back({(int64_t)fc + c, level + 1});
            }
        }
    }
    if (next_leaf != n_cells) {
        err = "octree: leaf count does not match the density array";
        return -1;
    }
    for (int64_t i = 0; i < n_nodes; ++i)
        if (!seen[(size_t)i]) {
            err = "octree: unreachable node";
            return -1;
        }
    return depth;
}

// The leaf walk of the transport kernel.  A dense top table at level
// top_level, then blocks of 64 entries that each cover the two levels below an
// internal node (4 x 4 x 4 sub-cubes, index i + 4 j + 16 k): one dependent
// load per two tree levels.  An entry is 64 bits: its low word is either a
// leaf, 1 << 31 | (level << 27) | cell, or the index of the next block (below
// 2^25); a leaf's high word holds the bits of the leaf's FP32 density, so the
// load that finds the leaf also brings its density (no load from a separate
// density array, whose line would be one more request per step).  A leaf one
// level below the node fills its 8 sub-cubes; a node one level above the
// deepest leaves gets a block whose lower sub-cube bit is a copy (the walk
// reads it as 0).  Returns false (with a message) if the blocks would not fit
// 32-bit indices.
inline uint64_t walk_leaf(int level, int32_t val, const float *density)
{
    const uint32_t cell = (uint32_t)(-val - 1);
    uint32_t rho;
    std::memcpy(&rho, density + cell, sizeof(rho));
    return ((uint64_t)rho << 32) | (1u << 31) | ((uint32_t)level << 27) | cell;
}

// Position of a top-level cube in the top table: 4 x 4 x 4 tiles (the
// device's top_index), linear below level 2.
inline int top_index_host(int x, int y, int z, int top_level)
{
    if (top_level < 2) return (((z << top_level) + y) << top_level) + x;
    const int tl = top_level - 2;
    const int tile = ((((z >> 2) << tl) + (y >> 2)) << tl) + (x >> 2);
    return (tile << 6) + ((z & 3) << 4) + ((y & 3) << 2) + (x & 3);
}

inline bool build_walk(const std::vector<int32_t> &node, int depth, int top_level, const float *density,
                       std::vector<uint64_t> &top, std::vector<uint64_t> &blocks, std::string &err)
{
    blocks.clear();
    // block of internal node nd at level L; returns its index
    std::vector<std::pair<int32_t, int>> work; // (node, level) of blocks still to fill
    auto new_block = [&](int32_t nd, int level) -> uint32_t {
        const size_t b = blocks.size() / 64;
        blocks.resize(blocks.size() + 64, 0);
        work.push_back({nd, level});
        return (uint32_t)b;
    };
    auto fill = [&](size_t b, int32_t nd, int level) {
        for (int k = 0; k < 4; ++k)
            for (int j = 0; j < 4; ++j)
                for (int i = 0; i < 4; ++i) {
                    const int c1 = (i >> 1) + 2 * (j >> 1) + 4 * (k >> 1);
                    const int32_t m1 = node[(size_t)nd] + c1;
                    const int32_t e1 = node[(size_t)m1];
                    uint64_t e;
                    if (e1 < 0) {
                        e = walk_leaf(level + 1, e1, density);
                    } else {
                        const int c2 = (i & 1) + 2 * (j & 1) + 4 * (k & 1);
                        const int32_t m2 = e1 + c2;
                        const int32_t e2 = node[(size_t)m2];
                        e = e2 < 0 ? walk_leaf(level + 2, e2, density) : new_block(m2, level + 2);
                    }
                    blocks[b * 64 + (size_t)(i + 4 * j + 16 * k)] = e;
                }
    };
    const int T = 1 << top_level;
    top.assign((size_t)T * T * T, 0);
    std::vector<int32_t> block_of((size_t)node.size(), -1);
    for (int bz = 0; bz < T; ++bz)
        for (int by = 0; by < T; ++by)
            for (int bx = 0; bx < T; ++bx) {
                int32_t nd = 0;
                int level = 0;
                while (level < top_level && node[(size_t)nd] >= 0) {
                    int bit = top_level - 1 - level;
                    int child = ((bx >> bit) & 1) + 2 * ((by >> bit) & 1) + 4 * ((bz >> bit) & 1);
                    nd = node[(size_t)nd] + child;
                    level++;
                }
                const int32_t val = node[(size_t)nd];
                uint64_t e;
                if (val < 0) {
                    e = walk_leaf(level, val, density);
                } else {
                    if (block_of[(size_t)nd] < 0) block_of[(size_t)nd] = (int32_t)new_block(nd, level);
                    e = (uint64_t)(uint32_t)block_of[(size_t)nd];
                }
                top[(size_t)top_index_host(bx, by, bz, top_level)] = e;
            }
    (void)depth;
    for (size_t w = 0; w < work.size(); ++w) {
        if (blocks.size() >= (size_t(1) << 31)) {
            err = "octree: walk blocks exceed 2^31 entries";
            return false;
        }
        const auto [nd, level] = work[w];
        fill(w, nd, level);
    }
    return true;
}

// Per leaf of an encoded octree (leaf order): its cube's origin on the
// finest lattice (2^depth per axis) and its level, 4 ints per leaf.
inline void leaf_geometry(const std::vector<int32_t> &node, int depth, int64_t n_leaves, std::vector<int32_t> &geo)
{
    geo.assign((size_t)n_leaves * 4, 0);
    struct Item {
        int32_t nd;
        int level;
        int32_t x, y, z; // origin in units of the node's own size
    };
    std::vector<Item> stack;
    stack.push_back({0, 0, 0, 0, 0});
    while (!stack.empty()) {
        const Item it = stack.back();
        stack.pop_back();
        const int32_t v = node[(size_t)it.nd];
        if (v < 0) {
            const int64_t leaf = -(int64_t)v - 1;
            const int sh = depth - it.level;
            geo[(size_t)leaf * 4 + 0] = it.x << sh;
            geo[(size_t)leaf * 4 + 1] = it.y << sh;
            geo[(size_t)leaf * 4 + 2] = it.z << sh;
            geo[(size_t)leaf * 4 + 3] = it.level;
        } else {
            for (int c = 0; c < 8; ++c)
                stack.push_back({v + c, it.level + 1, 2 * it.x + (c & 1), 2 * it.y + ((c >> 1) & 1),
                                 2 * it.z + ((c >> 2) & 1)});
        }
    }
}

// Brick shape for the Cartesian storage layout: 32 cells per brick (one
// 128-byte line of FP32 densities); within a brick each axis's cell bits are
// contiguous, in = sum_a (c_a mod 2^bs_a) << sh_a.  The first 8 cells of a
// brick are one 64-byte line of the FP64 table, and the transport kernel
// issues a ray's consecutive deposits together, so the line is made as close
// to a physical cube as possible: its 3 bits go one at a time to the axis of
// smallest physical extent cs_a 2^bs_a (ties: the lower axis); the other 2
// bits go to the axis of smallest extent after that, which is placed last in
// the index so the line stays the first 8 cells.  No axis gets more bits than
// its own extent needs (rounded up to a power of two) unless the whole grid
// is smaller than a brick (then x is padded).
inline void choose_bricks(const double cs[3], const int n[3], int bs[3], int sh[3], int nb[3], long long &n_store)
{
    int lim[3];
    for (int a = 0; a < 3; ++a) {
        bs[a] = 0;
        sh[a] = 0;
        lim[a] = 0;
        while ((1 << lim[a]) < n[a]) lim[a]++;
    }
    auto pick = [&]() {
        int best = -1;
        double ext = 0.0;
        for (int a = 0; a < 3; ++a) {
            double e = cs[a] * (double)(1 << bs[a]);
            if (bs[a] < lim[a] && (best < 0 || e < ext)) {
                best = a;
                ext = e;
            }
        }
        return best < 0 ? 0 : best; // grid smaller than a brick: pad along x
    };
    for (int k = 0; k < 3; ++k) bs[pick()]++;
    const int last = pick();
    for (int k = 0; k < 2; ++k) bs[last]++;
    int pos = 0;
    for (int a = 0; a < 3; ++a)
        if (a != last) {
            sh[a] = pos;
            pos += bs[a];
        }
    sh[last] = pos;
    n_store = 32;
    for (int a = 0; a < 3; ++a) {
        nb[a] = (n[a] + (1 << bs[a]) - 1) >> bs[a];
        n_store *= nb[a];
    }
}

// Shifts of an explicitly requested brick shape: x fastest, then y, then z.
inline void default_shifts(const int bs[3], int sh[3])
{
    sh[0] = 0;
    sh[1] = bs[0];
    sh[2] = bs[0] + bs[1];
}

inline long long store_index_host(const int bs[3], const int sh[3], const int nb[3], int ix, int iy, int iz)
{
    long long brick = (ix >> bs[0]) + (long long)nb[0] * ((iy >> bs[1]) + (long long)nb[1] * (iz >> bs[2]));
    int in = ((ix & ((1 << bs[0]) - 1)) << sh[0]) + ((iy & ((1 << bs[1]) - 1)) << sh[1]) +
             ((iz & ((1 << bs[2]) - 1)) << sh[2]);
    return brick * 32 + in;
}

// Column map of a line of sight along +-axis (code = 2 axis + (k < 0)): for
// every cell, the sum of density x cell width over the cells beyond it in the
// direction of sight, up to the grid boundary (FP64, storage order; planes at
// lo + j (hi - lo) / n).  The optical depth from a point in cell c to the
// boundary is then kappa (rho_c d + S_c), d the distance to c's exit face.
inline void column_map(const float *density, const int n[3], const double box[6], int code, const int bs[3],
                       const int sh[3], const int nb[3], long long n_store, std::vector<double> &S)
{
    const int a = code >> 1;
    const bool neg = (code & 1) != 0;
    const int u = (a + 1) % 3, w = (a + 2) % 3;
    const double cs = (box[3 + a] - box[a]) / (double)n[a];
    S.assign((size_t)n_store, 0.0);
    for (int iw = 0; iw < n[w]; ++iw)
        for (int iu = 0; iu < n[u]; ++iu) {
            double acc = 0.0;
            for (int s = 0; s < n[a]; ++s) {
                const int ia = neg ? s : n[a] - 1 - s; // from the far end of the line of sight
                int c[3];
                c[a] = ia;
                c[u] = iu;
                c[w] = iw;
                S[(size_t)store_index_host(bs, sh, nb, c[0], c[1], c[2])] = acc;
                const double lo = box[a] + (double)ia * cs, hi = box[a] + (double)(ia + 1) * cs;
                acc = acc + (double)density[c[0] + (size_t)n[0] * (c[1] + (size_t)n[1] * c[2])] * (hi - lo);
            }
        }
}

// Octree grids, line of sight along a lattice axis (code = 2 axis + (k < 0),
// as axis_code): S[x + N (y + N z)] (N = 2^depth lattice cells per axis) =
// sum of density x width over the lattice cells from (x, y, z) itself up to
// the boundary on the observer's side (every lattice cell of a leaf has the
// leaf's density).  A peel-off from a point of lattice cell c then has the
// optical depth kappa (S[c'] + (S[c] - S[c']) f), c' the next lattice cell
// towards the observer (S = 0 past the boundary) and f the fraction of c's
// width still to cross: two reads instead of a march through the leaves.
template <typename Real>
inline void octree_column_map(const std::vector<int32_t> &node, int depth, int64_t n_leaves, const float *density,
                              const double box[6], int code, std::vector<Real> &S)
{
    const int a = code >> 1;
    const bool neg = (code & 1) != 0;
    const int64_t N = int64_t(1) << depth;
    std::vector<int32_t> geo;
    leaf_geometry(node, depth, n_leaves, geo);
    std::vector<float> lat((size_t)(N * N * N), 0.0f);
    for (int64_t l = 0; l < n_leaves; ++l) {
        const int64_t x0 = geo[(size_t)l * 4], y0 = geo[(size_t)l * 4 + 1], z0 = geo[(size_t)l * 4 + 2];
        const int64_t size = int64_t(1) << (depth - geo[(size_t)l * 4 + 3]);
        const float rho = density[l];
        for (int64_t z = z0; z < z0 + size; ++z)
            for (int64_t y = y0; y < y0 + size; ++y)
                for (int64_t x = x0; x < x0 + size; ++x) lat[(size_t)(x + N * (y + N * z))] = rho;
    }
    const int u = (a + 1) % 3, w = (a + 2) % 3;
    int64_t st[3] = {1, N, N * N};
    const double cs = (box[3 + a] - box[a]) / (double)N;
    S.assign((size_t)(N * N * N), Real(0));
    for (int64_t iw = 0; iw < N; ++iw)
        for (int64_t iu = 0; iu < N; ++iu) {
            double acc = 0.0;
            for (int64_t s = 0; s < N; ++s) {
                const int64_t ia = neg ? s : N - 1 - s; // from the observer's side of the grid inwards
                const int64_t idx = ia * st[a] + iu * st[u] + iw * st[w];
                const double lo = box[a] + (double)ia * cs, hi = box[a] + (double)(ia + 1) * cs;
                acc = acc + (double)lat[(size_t)idx] * (hi - lo);
                S[(size_t)idx] = (Real)acc;
            }
        }
}

// Largest octree depth whose lattice column maps are built (8^10 cells).
constexpr int kMaxColumnDepth = 10;

} // namespace mcrt
