/*
 * mcrt_oracle.c -- plain serial FP64 oracle of the Monte Carlo photon-packet
 * life cycle described in the hybrid-parallel SKIRT paper, Section 3.2
 * ("Stellar emission phase"): each packet is launched, propagated through the
 * dust grid, loses luminosity continuously by absorption into the
 * per-cell, per-wavelength absorbed-luminosity table (Section 5.2, the
 * DustSystem::absorb / ParallelTable description), is forced to interact,
 * peels off luminosity towards every instrument at emission (Fig. 2 caption)
 * and at every scattering event, and is followed until only a negligible part
 * of its launch luminosity remains.
 *
 * TEST INFRASTRUCTURE ONLY (see mcrt_oracle.h).  The paper names the
 * acceleration techniques (peel-off, continuous absorption, forced
 * scattering; Section 1) without giving their formulas; this file writes out
 * the standard estimator those names denote, step by step in the order the
 * method takes them, with no blocking, fusion or reordering.  The readings
 * taken where the paper is silent are listed with the design notes.
 *
 * Compiled with -O2 -ffp-contract=off (no fused multiply-add), FP64 only.
 */
#include "mcrt_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as  */
/* easy as 1, 2, 3", SC'11, Section 4): 10 rounds of the Philox S-P network  */
/* on a 128-bit counter with a 64-bit key, the key bumped by the Weyl        */
/* constants between rounds.                                                 */
/* ------------------------------------------------------------------------ */

static void mulhilo32(uint32_t a, uint32_t b, uint32_t *hi, uint32_t *lo)
{
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    *lo = (uint32_t)p;
}

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint32_t hi0, lo0, hi1, lo1;
        mulhilo32(M0, c0, &hi0, &lo0);
        mulhilo32(M1, c2, &hi1, &lo1);
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Slot s of a packet's stream: Philox block floor(s/2), output words
 * 2(s mod 2) (high) and 2(s mod 2)+1 (low).  Counter = (block, packet,
 * wavelength, model); key = (low 32 bits of the seed, high 32 bits). */
static void slot_words(uint64_t seed, uint32_t packet, uint32_t lambda, uint32_t model,
                       uint32_t slot, uint32_t *hi, uint32_t *lo)
{
    uint32_t ctr[4] = {slot / 2u, packet, lambda, model};
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    uint32_t out[4];
    or_philox4x32_10(ctr, key, out);
    uint32_t w = 2u * (slot % 2u);
    *hi = out[w];
    *lo = out[w + 1];
}

/* Uniform in the open interval (0, 1) from the top 52 bits of the slot's
 * 64-bit word: ((w >> 12) + 1/2) * 2^-52. */
double or_uniform64(uint64_t seed, uint32_t packet, uint32_t lambda, uint32_t model, uint32_t slot)
{
    uint32_t hi, lo;
    slot_words(seed, packet, lambda, model, slot, &hi, &lo);
    uint64_t w = ((uint64_t)hi << 32) | (uint64_t)lo;
    return ((double)(w >> 12) + 0.5) * 0x1p-52;
}

/* Single-precision variant: ((hi >> 9) + 1/2) * 2^-23. */
float or_uniform32(uint64_t seed, uint32_t packet, uint32_t lambda, uint32_t model, uint32_t slot)
{
    uint32_t hi, lo;
    slot_words(seed, packet, lambda, model, slot, &hi, &lo);
    return ((float)(hi >> 9) + 0.5f) * 0x1p-23f;
}


/* ------------------------------------------------------------------------ */
/* Elementary functions with an explicitly specified operation sequence, so  */
/* that FP64 results do not depend on the platform's math library:           */
/* Cody & Waite additive argument reduction (W. J. Cody and W. Waite,        */
/* "Software Manual for the Elementary Functions", 1980) followed by         */
/* truncated Taylor series in Horner form; the logarithm through the series  */
/* of 2 atanh(s), s = (m - 1)/(m + 1); log1p through the correction of       */
/* Goldberg, "What every computer scientist should know about floating-point */
/* arithmetic" (1991), Theorem 4.  Each is within a few ulp of the exact     */
/* value (pinned against the C library in the tests).                         */
/* ------------------------------------------------------------------------ */

static const double LN2_HI = 0x1.62e42fee00000p-1;  /* ln 2 to 32 bits */
static const double LN2_LO = 0x1.a39ef35793c76p-33; /* ln 2 - LN2_HI */
static const double INV_LN2 = 0x1.71547652b82fep+0;
static const double SQRT2 = 0x1.6a09e667f3bcdp+0;
static const double PIO2_1 = 0x1.921fb54400000p+0;  /* pi/2 to 33 bits */
static const double PIO2_2 = 0x1.0b4611a600000p-34; /* next 33 bits */
static const double PIO2_3 = 0x1.3198a2e037073p-69; /* remainder */
static const double TWO_OVER_PI = 0x1.45f306dc9c883p-1;

/* 1/j!, j = 0 .. 22 */
static const double INV_FACT[23] = {
    1.0, 1.0, 0x1.0000000000000p-1, 0x1.5555555555555p-3, 0x1.5555555555555p-5,
    0x1.1111111111111p-7, 0x1.6c16c16c16c17p-10, 0x1.a01a01a01a01ap-13, 0x1.a01a01a01a01ap-16,
    0x1.71de3a556c734p-19, 0x1.27e4fb7789f5cp-22, 0x1.ae64567f544e4p-26, 0x1.1eed8eff8d898p-29,
    0x1.6124613a86d09p-33, 0x1.93974a8c07c9dp-37, 0x1.ae7f3e733b81fp-41, 0x1.ae7f3e733b81fp-45,
    0x1.952c77030ad4ap-49, 0x1.6827863b97d97p-53, 0x1.2f49b46814157p-57, 0x1.e542ba4020225p-62,
    0x1.71b8ef6dcf572p-66, 0x1.0ce396db7f853p-70};

/* 1/(2j+1), j = 0 .. 11 */
static const double INV_ODD[12] = {
    1.0, 0x1.5555555555555p-2, 0x1.999999999999ap-3, 0x1.2492492492492p-3, 0x1.c71c71c71c71cp-4,
    0x1.745d1745d1746p-4, 0x1.3b13b13b13b14p-4, 0x1.1111111111111p-4, 0x1.e1e1e1e1e1e1ep-5,
    0x1.af286bca1af28p-5, 0x1.8618618618618p-5, 0x1.642c8590b2164p-5};

static double pow2i(int j) /* 2^j for -1022 <= j <= 1023 */
{
    uint64_t b = (uint64_t)(j + 1023) << 52;
    double d;
    memcpy(&d, &b, sizeof d);
    return d;
}

/* p * 2^k with at most one rounding (into the subnormal range) */
static double scale2(double p, int k)
{
    if (k > 1023) return p * pow2i(1023) * pow2i(k - 1023);
    if (k < -1022) return p * pow2i(-1022) * pow2i(k + 1022);
    return p * pow2i(k);
}

double or_exp(double x)
{
    if (x != x) return x;
    if (x > 709.782712893384) return INFINITY;
    if (x < -745.2) return 0.0;
    double kd = floor(x * INV_LN2 + 0.5);
    double r = (x - kd * LN2_HI) - kd * LN2_LO;
    /* e^r = sum_{j=0}^{13} r^j / j!,  |r| <= 0.3466 */
    double p = INV_FACT[13];
    for (int j = 12; j >= 0; --j) p = p * r + INV_FACT[j];
    return scale2(p, (int)kd);
}

double or_expm1(double x)
{
    if (x != x) return x;
    if (fabs(x) < 1.0) {
        /* x * sum_{j=0}^{21} x^j / (j+1)!,  |x| < 1 */
        double p = INV_FACT[22];
        for (int j = 21; j >= 1; --j) p = p * x + INV_FACT[j];
        return x * p;
    }
    return or_exp(x) - 1.0;
}

double or_log(double x)
{
    if (x != x || x < 0.0) return NAN;
    if (x == 0.0) return -INFINITY;
    if (x == INFINITY) return x;
    int e = 0;
    if (x < 0x1p-1022) {
        x = x * 0x1p54;
        e = -54;
    }
    uint64_t b;
    memcpy(&b, &x, sizeof b);
    e += (int)((b >> 52) & 0x7ff) - 1023;
    b = (b & 0x000fffffffffffffull) | (0x3ffull << 52);
    double m;
    memcpy(&m, &b, sizeof m); /* m in [1, 2) */
    if (m > SQRT2) {
        m = m * 0.5;
        e += 1;
    }
    double f = m - 1.0;
    double s = f / (2.0 + f);
    double s2 = s * s;
    /* log m = 2 s sum_{j=0}^{11} s^(2j) / (2j+1) */
    double q = INV_ODD[11];
    for (int j = 10; j >= 0; --j) q = q * s2 + INV_ODD[j];
    double lm = 2.0 * s * q;
    double de = (double)e;
    return de * LN2_HI + (de * LN2_LO + lm);
}

double or_log1p(double x)
{
    if (x != x) return x;
    if (x == -1.0) return -INFINITY;
    if (x < -1.0) return NAN;
    double u = 1.0 + x;
    if (u == 1.0) return x;
    return or_log(u) * (x / (u - 1.0));
}

/* atanh |x| = log1p(2|x| / (1 - |x|)) / 2, odd symmetry */
double or_atanh(double x)
{
    double ax = fabs(x);
    double h = 0.5 * or_log1p((2.0 * ax) / (1.0 - ax));
    return x < 0.0 ? -h : h;
}

void or_sincos(double x, double *sn, double *cs)
{
    double q = floor(x * TWO_OVER_PI + 0.5);
    double r = ((x - q * PIO2_1) - q * PIO2_2) - q * PIO2_3;
    double r2 = r * r;
    /* sin r = r sum_{j=0}^{9} (-1)^j r^(2j) / (2j+1)!,
     * cos r = sum_{j=0}^{10} (-1)^j r^(2j) / (2j)!,  |r| <= pi/4 */
    double ps = -INV_FACT[19];
    for (int j = 8; j >= 0; --j) ps = (j % 2 ? -INV_FACT[2 * j + 1] : INV_FACT[2 * j + 1]) + r2 * ps;
    double pc = INV_FACT[20];
    for (int j = 9; j >= 0; --j) pc = (j % 2 ? -INV_FACT[2 * j] : INV_FACT[2 * j]) + r2 * pc;
    double sr = r * ps, cr = pc;
    long long n = (long long)q;
    int quad = (int)(((n % 4) + 4) % 4);
    if (quad == 0) { *sn = sr; *cs = cr; }
    else if (quad == 1) { *sn = cr; *cs = -sr; }
    else if (quad == 2) { *sn = -sr; *cs = -cr; }
    else { *sn = -cr; *cs = sr; }
}

/* ------------------------------------------------------------------------ */
/* Geometry: the dust grid and the ray march.                               */
/* ------------------------------------------------------------------------ */

typedef struct {
    const or_scene *s;
    /* octree derived data */
    int depth;          /* maximum leaf depth D */
    int64_t lattice;    /* 2^D */
    int64_t *leaf_of_node; /* leaf index (depth-first order) or -1 */
    int *leaf_level;       /* per leaf: its level */
    int64_t *leaf_org;     /* per leaf: lattice origin (3 per leaf, lattice 2^D) */
} geom;

typedef struct {
    int64_t *cell;
    double *tend;       /* ray parameter at the end of the segment */
    int64_t n, cap;
    double t0;          /* ray parameter where the first segment starts */
} seglist;

static int seg_push(seglist *sl, int64_t cell, double tend)
{
    if (sl->n == sl->cap) {
        int64_t nc = sl->cap ? 2 * sl->cap : 256;
        int64_t *c = (int64_t *)realloc(sl->cell, (size_t)nc * sizeof(int64_t));
        if (!c) return -1;
        sl->cell = c;
        double *t = (double *)realloc(sl->tend, (size_t)nc * sizeof(double));
        if (!t) return -1;
        sl->tend = t;
        sl->cap = nc;
    }
    sl->cell[sl->n] = cell;
    sl->tend[sl->n] = tend;
    sl->n++;
    return 0;
}

static void seg_free(seglist *sl)
{
    free(sl->cell);
    free(sl->tend);
    memset(sl, 0, sizeof(*sl));
}

/* Builds the octree derived data: maximum depth and depth-first leaf order
 * (children visited in the order c = bx + 2 by + 4 bz). */
static int geom_init(geom *g, const or_scene *s)
{
    memset(g, 0, sizeof(*g));
    g->s = s;
    if (s->grid_type != OR_GRID_OCTREE) return 0;
    int64_t nn = s->n_nodes;
    g->leaf_of_node = (int64_t *)malloc((size_t)nn * sizeof(int64_t));
    int64_t *stack_node = (int64_t *)malloc((size_t)(nn + 8) * sizeof(int64_t));
    int *stack_level = (int *)malloc((size_t)(nn + 8) * sizeof(int));
    /* node origins in units of the node's own level: child c of a node at
     * (x, y, z) sits at (2x + bx, 2y + by, 2z + bz) */
    int64_t *stack_org = (int64_t *)malloc((size_t)(nn + 8) * 3 * sizeof(int64_t));
    g->leaf_level = (int *)malloc((size_t)(s->n_cells > 0 ? s->n_cells : 1) * sizeof(int));
    int64_t *org_at_level = (int64_t *)malloc((size_t)(s->n_cells > 0 ? s->n_cells : 1) * 3 * sizeof(int64_t));
    if (!g->leaf_of_node || !stack_node || !stack_level || !stack_org || !g->leaf_level || !org_at_level) {
        free(stack_node);
        free(stack_level);
        free(stack_org);
        free(org_at_level);
        return -1;
    }
    for (int64_t i = 0; i < nn; ++i) g->leaf_of_node[i] = -1;
    int64_t top = 0, next_leaf = 0;
    int maxdepth = 0;
    stack_node[top] = 0;
    stack_level[top] = 0;
    stack_org[0] = stack_org[1] = stack_org[2] = 0;
    top++;
    while (top > 0) {
        top--;
        int64_t node = stack_node[top];
        int level = stack_level[top];
        const int64_t ox = stack_org[3 * top], oy = stack_org[3 * top + 1], oz = stack_org[3 * top + 2];
        int32_t fc = s->first_child[node];
        if (fc < 0) {
            if (next_leaf < s->n_cells) {
                g->leaf_level[next_leaf] = level;
                org_at_level[3 * next_leaf] = ox;
                org_at_level[3 * next_leaf + 1] = oy;
                org_at_level[3 * next_leaf + 2] = oz;
            }
            g->leaf_of_node[node] = next_leaf++;
            if (level > maxdepth) maxdepth = level;
        } else {
            for (int c = 7; c >= 0; --c) {
                stack_node[top] = (int64_t)fc + c;
                stack_level[top] = level + 1;
                stack_org[3 * top] = 2 * ox + (c & 1);
                stack_org[3 * top + 1] = 2 * oy + ((c >> 1) & 1);
                stack_org[3 * top + 2] = 2 * oz + ((c >> 2) & 1);
                top++;
            }
        }
    }
    free(stack_node);
    free(stack_level);
    free(stack_org);
    g->depth = maxdepth;
    g->lattice = (int64_t)1 << maxdepth;
    if (next_leaf != s->n_cells) {
        free(org_at_level);
        return -1;
    }
    /* origins on the finest lattice */
    for (int64_t m = 0; m < s->n_cells; ++m)
        for (int a = 0; a < 3; ++a) org_at_level[3 * m + a] <<= (maxdepth - g->leaf_level[m]);
    g->leaf_org = org_at_level;
    return 0;
}

static void geom_free(geom *g)
{
    free(g->leaf_of_node);
    free(g->leaf_level);
    free(g->leaf_org);
    g->leaf_of_node = NULL;
    g->leaf_level = NULL;
    g->leaf_org = NULL;
}

/* Index of the grid slice containing coordinate p along an axis with origin
 * lo, spacing d and n slices; a point exactly on a plane that the ray leaves
 * towards lower coordinates belongs to the slice below the plane. */
static int64_t slice_index(double p, double lo, double d, int64_t n, double k)
{
    int64_t i = (int64_t)floor((p - lo) / d);
    if (i < 0) i = 0;
    if (i > n - 1) i = n - 1;
    if (p == lo + (double)i * d && k < 0.0) i -= 1;
    return i;
}

/* Finds where the ray r + t k (t >= 0) starts inside the box: t0 and the
 * slice indices along each axis (spacing d[a], n[a] slices).  Returns 0 if
 * the ray misses the box or leaves it immediately. */
static int ray_start(const double box[6], const double d[3], const int64_t n[3],
                     const double r[3], const double k[3], double *t0, int64_t idx[3])
{
    const double *lo = box, *hi = box + 3;
    int inside = 1;
    for (int a = 0; a < 3; ++a)
        if (!(r[a] >= lo[a] && r[a] <= hi[a])) inside = 0;
    if (inside) {
        *t0 = 0.0;
        for (int a = 0; a < 3; ++a) idx[a] = slice_index(r[a], lo[a], d[a], n[a], k[a]);
    } else {
        double tn = -INFINITY, tf = INFINITY;
        int entry = -1;
        for (int a = 0; a < 3; ++a) {
            if (k[a] == 0.0) {
                if (r[a] < lo[a] || r[a] > hi[a]) return 0;
            } else {
                double t1 = (lo[a] - r[a]) / k[a];
                double t2 = (hi[a] - r[a]) / k[a];
                double near = t1 < t2 ? t1 : t2;
                double far = t1 < t2 ? t2 : t1;
                if (near > tn) {
                    tn = near;
                    entry = a;
                }
                if (far < tf) tf = far;
            }
        }
        if (entry < 0 || tn > tf || tf < 0.0 || tn < 0.0) return 0;
        *t0 = tn;
        for (int a = 0; a < 3; ++a) {
            if (a == entry) {
                idx[a] = k[a] > 0.0 ? 0 : n[a] - 1;
            } else {
                double p = r[a] + tn * k[a];
                idx[a] = slice_index(p, lo[a], d[a], n[a], k[a]);
            }
        }
    }
    for (int a = 0; a < 3; ++a)
        if (idx[a] < 0 || idx[a] >= n[a]) return 0;
    return 1;
}

/* Ray parameter where the ray crosses the plane lo + j d of axis a. */
static double plane_t(double lo, double d, int64_t j, double r, double k)
{
    return (lo + (double)j * d - r) / k;
}

/* Cartesian grid: 3-D digital differential analyser.  At each step the axis
 * whose next plane is nearest is stepped (ties to the lowest axis); plane
 * crossings are recomputed from the original ray origin every step. */
static int march_cartesian(const geom *g, const double r[3], const double k[3], seglist *sl)
{
    const or_scene *s = g->s;
    int64_t n[3] = {s->n[0], s->n[1], s->n[2]};
    double d[3];
    for (int a = 0; a < 3; ++a) d[a] = (s->box[3 + a] - s->box[a]) / (double)n[a];
    sl->n = 0;
    sl->t0 = 0.0;
    int64_t idx[3];
    double t;
    if (!ray_start(s->box, d, n, r, k, &t, idx)) return 0;
    sl->t0 = t;
    for (;;) {
        double tn[3];
        for (int a = 0; a < 3; ++a) {
            if (k[a] > 0.0) tn[a] = plane_t(s->box[a], d[a], idx[a] + 1, r[a], k[a]);
            else if (k[a] < 0.0) tn[a] = plane_t(s->box[a], d[a], idx[a], r[a], k[a]);
            else tn[a] = INFINITY;
        }
        int am = 0;
        if (tn[1] < tn[am]) am = 1;
        if (tn[2] < tn[am]) am = 2;
        double te = tn[am] > t ? tn[am] : t;
        int64_t cell = idx[0] + n[0] * (idx[1] + n[1] * idx[2]);
        if (seg_push(sl, cell, te)) return -1;
        t = te;
        idx[am] += k[am] > 0.0 ? 1 : -1;
        if (idx[am] < 0 || idx[am] >= n[am]) break;
    }
    return 0;
}

/* Octree: walk on the integer lattice of the deepest level.  The current
 * lattice point is located by descending from the root; the leaf's exit
 * plane is found as in the Cartesian march; the next lattice point lies just
 * across the exit face, with the in-face coordinates taken from the exit
 * point and clamped into the current leaf. */
static int march_octree(const geom *g, const double r[3], const double k[3], seglist *sl)
{
    const or_scene *s = g->s;
    int64_t N = g->lattice;
    int64_t n[3] = {N, N, N};
    double d[3];
    for (int a = 0; a < 3; ++a) d[a] = (s->box[3 + a] - s->box[a]) / (double)N;
    sl->n = 0;
    sl->t0 = 0.0;
    int64_t c[3];
    double t;
    if (!ray_start(s->box, d, n, r, k, &t, c)) return 0;
    sl->t0 = t;
    int64_t guard = 16 * 3 * N + 64;
    for (int64_t step = 0; step < guard; ++step) {
        int64_t node = 0;
        int level = 0;
        while (s->first_child[node] >= 0) {
            int bit = g->depth - 1 - level;
            int64_t child = ((c[0] >> bit) & 1) + 2 * ((c[1] >> bit) & 1) + 4 * ((c[2] >> bit) & 1);
            node = (int64_t)s->first_child[node] + child;
            level++;
        }
        int64_t size = (int64_t)1 << (g->depth - level);
        int64_t o[3];
        for (int a = 0; a < 3; ++a) o[a] = c[a] - (c[a] % size);
        double tn[3];
        for (int a = 0; a < 3; ++a) {
            if (k[a] > 0.0) tn[a] = plane_t(s->box[a], d[a], o[a] + size, r[a], k[a]);
            else if (k[a] < 0.0) tn[a] = plane_t(s->box[a], d[a], o[a], r[a], k[a]);
            else tn[a] = INFINITY;
        }
        int am = 0;
        if (tn[1] < tn[am]) am = 1;
        if (tn[2] < tn[am]) am = 2;
        double te = tn[am] > t ? tn[am] : t;
        if (seg_push(sl, g->leaf_of_node[node], te)) return -1;
        t = te;
        int64_t nc[3];
        for (int a = 0; a < 3; ++a) {
            if (a == am) {
                nc[a] = k[a] > 0.0 ? o[a] + size : o[a] - 1;
            } else {
                double p = r[a] + te * k[a];
                int64_t q = (int64_t)floor((p - s->box[a]) / d[a]);
                if (q < o[a]) q = o[a];
                if (q > o[a] + size - 1) q = o[a] + size - 1;
                nc[a] = q;
            }
        }
        if (nc[am] < 0 || nc[am] >= N) return 0;
        c[0] = nc[0]; c[1] = nc[1]; c[2] = nc[2];
    }
    return -2; /* the walk did not leave the grid: malformed octree */
}

static int march(const geom *g, const double r[3], const double k[3], seglist *sl)
{
    if (g->s->grid_type == OR_GRID_OCTREE) return march_octree(g, r, k, sl);
    return march_cartesian(g, r, k, sl);
}

int64_t or_march(const or_scene *scene, const double r[3], const double k[3],
                 int64_t *cells, double *lengths, int64_t max_seg)
{
    geom g;
    if (geom_init(&g, scene)) {
        geom_free(&g);
        return -1;
    }
    seglist sl;
    memset(&sl, 0, sizeof(sl));
    int rc = march(&g, r, k, &sl);
    int64_t n = sl.n;
    if (rc || n > max_seg) {
        n = -1;
    } else {
        double prev = sl.t0;
        for (int64_t i = 0; i < n; ++i) {
            cells[i] = sl.cell[i];
            lengths[i] = sl.tend[i] - prev;
            prev = sl.tend[i];
        }
    }
    seg_free(&sl);
    geom_free(&g);
    return n;
}

/* ------------------------------------------------------------------------ */
/* Phase function and direction sampling.                                    */
/* ------------------------------------------------------------------------ */

/* Henyey-Greenstein phase function, normalised to average 1 over the sphere. */
double or_hg_phase(double g, double mu)
{
    double num = 1.0 - g * g;
    double den = 1.0 + g * g - 2.0 * g * mu;
    return num / (den * sqrt(den));
}

/* Inverse-CDF sample of the cosine of the HG scattering angle. */
double or_hg_sample(double g, double u)
{
    double mu;
    if (fabs(g) >= 1e-6) {
        double q = (1.0 - g * g) / (1.0 - g + 2.0 * g * u);
        mu = (1.0 + g * g - q * q) / (2.0 * g);
    } else {
        mu = 2.0 * u - 1.0;
    }
    if (mu < -1.0) mu = -1.0;
    if (mu > 1.0) mu = 1.0;
    return mu;
}

/* Direction at polar cosine mu and azimuth phi about k.  The azimuth is
 * measured from the plane of k and the z axis; when k is within 0.00447 rad
 * of the z axis (|k_z| >= 0.99999) the x axis serves instead, applying the
 * same formula to the cyclically permuted components (y, z, x). */
static void rotate_about_pole(double a, double b, double c, double mu, double st,
                              double cp, double sp, double *x, double *y, double *z)
{
    double s = sqrt(1.0 - c * c);
    *x = mu * a + st * (a * c * cp - b * sp) / s;
    *y = mu * b + st * (b * c * cp + a * sp) / s;
    *z = mu * c - st * s * cp;
}

void or_rotate(const double k[3], double mu, double phi, double out[3])
{
    double st = sqrt(fmax(0.0, 1.0 - mu * mu));
    double sp, cp;
    or_sincos(phi, &sp, &cp);
    double x, y, z;
    if (fabs(k[2]) < 0.99999) {
        rotate_about_pole(k[0], k[1], k[2], mu, st, cp, sp, &x, &y, &z);
    } else {
        double py, pz, px;
        rotate_about_pole(k[1], k[2], k[0], mu, st, cp, sp, &py, &pz, &px);
        x = px;
        y = py;
        z = pz;
    }
    double nrm = sqrt(x * x + y * y + z * z);
    out[0] = x / nrm;
    out[1] = y / nrm;
    out[2] = z / nrm;
}


/* ------------------------------------------------------------------------ */
/* Learned direction proposal: MLP 9 -> 64 -> 64 -> 40 (ReLU) giving an      */
/* 8-lobe von Mises-Fisher mixture, mixed with the physical distribution.    */
/* ------------------------------------------------------------------------ */

static const double INV_LN10 = 0.43429448190325182765;

/* nearest-even to float32, then nearest-even to bfloat16 */
static double bf16_round(double x)
{
    float f = (float)x;
    uint32_t b;
    memcpy(&b, &f, sizeof b);
    uint32_t lsb = (b >> 16) & 1u;
    b = ((b + 0x7FFFu + lsb) >> 16) << 16;
    memcpy(&f, &b, sizeof f);
    return (double)f;
}

/* z_j = sum_k x_k W[k][j] (k in order, from 0) + b_j */
static void affine(const double *x, int nin, const double *W, const double *b, int nout, double *z)
{
    for (int j = 0; j < nout; ++j) {
        double acc = 0.0;
        for (int k = 0; k < nin; ++k) acc = acc + x[k] * W[k * nout + j];
        z[j] = acc + b[j];
    }
}

void or_mlp_forward(const double *theta, const double f[9], double out[40])
{
    const double *W1 = theta, *b1 = W1 + 9 * 64, *W2 = b1 + 64, *b2 = W2 + 64 * 64;
    const double *W3 = b2 + 64, *b3 = W3 + 64 * 40;
    double x[9], z[64], h1[64], h2[64];
    for (int k = 0; k < 9; ++k) x[k] = bf16_round(f[k]);
    affine(x, 9, W1, b1, 64, z);
    for (int j = 0; j < 64; ++j) h1[j] = bf16_round(z[j] > 0.0 ? z[j] : 0.0);
    affine(h1, 64, W2, b2, 64, z);
    for (int j = 0; j < 64; ++j) h2[j] = bf16_round(z[j] > 0.0 ? z[j] : 0.0);
    affine(h2, 64, W3, b3, 40, out);
}

typedef struct {
    double pi[8], mu[8][3], kappa[8];
} mixture;

static void mixture_from(const double o[40], mixture *m)
{
    double mx = o[0];
    for (int j = 1; j < 8; ++j)
        if (o[j] > mx) mx = o[j];
    double e[8], sum = 0.0;
    for (int j = 0; j < 8; ++j) {
        e[j] = or_exp(o[j] - mx);
        sum = sum + e[j];
    }
    for (int j = 0; j < 8; ++j) {
        m->pi[j] = e[j] / sum;
        double a = o[8 + 3 * j], b = o[9 + 3 * j], c = o[10 + 3 * j];
        double nrm = sqrt(a * a + b * b + c * c);
        if (nrm > 0.0) {
            m->mu[j][0] = a / nrm;
            m->mu[j][1] = b / nrm;
            m->mu[j][2] = c / nrm;
        } else {
            m->mu[j][0] = 0.0;
            m->mu[j][1] = 0.0;
            m->mu[j][2] = 1.0;
        }
        double s = o[32 + j];
        double sp = or_log1p(or_exp(-fabs(s))) + (s > 0.0 ? s : 0.0);
        double k = sp + 1e-3;
        if (k < 1e-3) k = 1e-3;
        if (k > 1e3) k = 1e3;
        m->kappa[j] = k;
    }
}

/* density of the vMF part at direction kp */
static double mixture_vmf_pdf(const mixture *m, const double kp[3])
{
    double q = 0.0;
    for (int j = 0; j < 8; ++j) {
        double k = m->kappa[j];
        double dot = m->mu[j][0] * kp[0] + m->mu[j][1] * kp[1] + m->mu[j][2] * kp[2];
        double f = k / (2.0 * OR_PI * -or_expm1(-2.0 * k)) * or_exp(k * (dot - 1.0));
        q = q + m->pi[j] * f;
    }
    return q;
}

/* With probability 1 - alpha (selector u3) a direction from the vMF part:
 * lobe by the cumulative weights at (u3 - alpha)/(1 - alpha), cosine to its
 * mean by the inverse CDF at u1, azimuth 2 pi u2.  Returns 1 if it sampled,
 * 0 if the caller must draw from the physical distribution with (u1, u2). */
static int mixture_sample(const mixture *m, double alpha, double u1, double u2, double u3, double kp[3])
{
    if (u3 < alpha) return 0;
    double v = (u3 - alpha) / (1.0 - alpha), c = 0.0;
    int j = 7;
    for (int i = 0; i < 8; ++i) {
        c = c + m->pi[i];
        if (v < c) {
            j = i;
            break;
        }
    }
    double k = m->kappa[j];
    double w = 1.0 + or_log(u1 + (1.0 - u1) * or_exp(-2.0 * k)) / k;
    if (w < -1.0) w = -1.0;
    if (w > 1.0) w = 1.0;
    or_rotate(m->mu[j], w, 2.0 * OR_PI * u2, kp);
    return 1;
}

/* ------------------------------------------------------------------------ */
/* The packet life cycle.                                                    */
/* ------------------------------------------------------------------------ */

typedef struct {
    double kobs[3], ex[3], ey[3];
    double fovx, fovy, inv4pid2;
    int64_t nx, ny;
    int64_t offset; /* first element of this instrument in the image array */
} instr;

typedef struct {
    /* per-packet second-moment scratch: dense accumulators with touched lists */
    double *acc;
    int64_t *touched;
    int64_t ntouched;
    double *m2;
} moment_buf;

/* Every contribution is non-negative, so an element is untouched exactly
 * while its accumulator is zero; zero contributions are skipped. */
static void moment_add(moment_buf *mb, int64_t idx, double v)
{
    if (!mb->m2 || v == 0.0) return;
    if (mb->acc[idx] == 0.0) mb->touched[mb->ntouched++] = idx;
    mb->acc[idx] += v;
}

static void moment_flush(moment_buf *mb)
{
    if (!mb->m2) return;
    for (int64_t i = 0; i < mb->ntouched; ++i) {
        int64_t idx = mb->touched[i];
        mb->m2[idx] += mb->acc[idx] * mb->acc[idx];
        mb->acc[idx] = 0.0;
    }
    mb->ntouched = 0;
}

typedef struct {
    const or_scene *s;
    geom g;
    instr *ins;
    seglist sl;
    or_out *out;
    moment_buf mt, mi;
    uint64_t seed;
    uint32_t model;
    double flux;     /* image flux produced so far by the current packet */
} runctx;

/* Optical depth from r along k to the grid boundary. */
static int optical_depth(runctx *c, const double r[3], const double k[3], double kappa, double *tau)
{
    int rc = march(&c->g, r, k, &c->sl);
    if (rc) return rc;
    double prev = c->sl.t0, sum = 0.0;
    for (int64_t n = 0; n < c->sl.n; ++n) {
        double ds = c->sl.tend[n] - prev;
        prev = c->sl.tend[n];
        sum += kappa * (double)c->s->density[c->sl.cell[n]] * ds;
    }
    c->out->stats.peel_cells += (uint64_t)c->sl.n;
    *tau = sum;
    return 0;
}

/* Peel-off: the luminosity lum, weighted by the probability per unit solid
 * angle (phase, normalised to average 1) of leaving towards the observer and
 * by the transmission exp(-tau) along the way, lands as flux
 * lum * phase * exp(-tau) / (4 pi d^2) in the pixel that r projects onto. */
static int peel(runctx *c, int ell, const double r[3], double lum, double phase,
                double kappa, int j)
{
    const instr *in = &c->ins[j];
    double tau;
    int rc = optical_depth(c, r, in->kobs, kappa, &tau);
    if (rc) return rc;
    if (tau >= c->s->tau_peel_max) {
        c->out->stats.peel_dropped++;
        return 0;
    }
    double x = r[0] * in->ex[0] + r[1] * in->ex[1] + r[2] * in->ex[2];
    double y = r[0] * in->ey[0] + r[1] * in->ey[1] + r[2] * in->ey[2];
    double px = floor((x + 0.5 * in->fovx) / (in->fovx / (double)in->nx));
    double py = floor((y + 0.5 * in->fovy) / (in->fovy / (double)in->ny));
    if (px < 0.0 || px >= (double)in->nx || py < 0.0 || py >= (double)in->ny) return 0;
    double flux = lum * phase * or_exp(-tau) * in->inv4pid2;
    int64_t idx = in->offset + ((int64_t)ell * in->ny + (int64_t)py) * in->nx + (int64_t)px;
    c->out->images[idx] += flux;
    c->flux += flux;
    moment_add(&c->mi, idx, flux);
    c->out->stats.peel_adds++;
    return 0;
}

static double source_phase(const or_scene *s, const double kobs[3])
{
    if (s->source_type == OR_SRC_POINT_ANISO) return 2.0 * fabs(kobs[2]);
    return 1.0;
}

/* Event features: position / r_out (3), incoming direction (3, zero at
 * emission), wavelength feature, log10 of the cell density over the mean
 * (0 at emission), event flag (0 emission, 1 scattering). */
static void event_features(const or_scene *s, int ell, const double r[3], const double *kin, double rho,
                           double f[9])
{
    for (int a = 0; a < 3; ++a) f[a] = r[a] / s->r_out;
    for (int a = 0; a < 3; ++a) f[3 + a] = kin ? kin[a] : 0.0;
    f[6] = s->lam_feature[ell];
    f[7] = kin ? or_log(rho / s->rho_mean) * INV_LN10 : 0.0;
    f[8] = kin ? 1.0 : 0.0;
}

static void record_event(runctx *c, int64_t slot, int64_t e, const double f[9], const double kp[3], double L)
{
    or_out *o = c->out;
    if (!o->hist || e >= o->hist_events) return;
    double *h = o->hist + (slot * o->hist_events + e) * 14;
    for (int i = 0; i < 9; ++i) h[i] = f[i];
    for (int i = 0; i < 3; ++i) h[9 + i] = kp[i];
    h[12] = L;
    h[13] = c->flux;
}

static int one_packet(runctx *c, int ell, uint32_t id, double L0, int64_t slot)
{
    const or_scene *s = c->s;
    or_out *o = c->out;
    const double kappa = s->kappa[ell], albedo = s->albedo[ell], g = s->hg_g[ell];
#define U(slot) or_uniform64(c->seed, id, (uint32_t)ell, c->model, (uint32_t)(slot))
    /* a packet without luminosity adds zero to every tally: it ends at launch */
    if (!(L0 > 0.0)) {
        o->stats.packets++;
        return 0;
    }
    /* launch */
    double r[3], k[3];
    if (s->source_type == OR_SRC_EXPDISK) {
        double R = -s->disk_hR * or_log(U(0) * U(1));
        double phi = 2.0 * OR_PI * U(2);
        double z = s->disk_zs * or_atanh(2.0 * U(3) - 1.0);
        double sphi, cphi;
        or_sincos(phi, &sphi, &cphi);
        r[0] = R * cphi;
        r[1] = R * sphi;
        r[2] = z;
    } else if (s->source_type == OR_SRC_DUST) {
        /* the emitting cell: the first whose running sum exceeds u times the
         * total (bisection), then a uniform point inside it */
        const double *cdf = s->dust_cdf + (int64_t)ell * s->n_cells;
        const double x = U(0) * cdf[s->n_cells - 1];
        int64_t lo = 0, hi = s->n_cells - 1;
        while (lo < hi) {
            int64_t mid = lo + (hi - lo) / 2;
            if (cdf[mid] > x) hi = mid;
            else lo = mid + 1;
        }
        if (s->grid_type == OR_GRID_OCTREE) {
            /* the leaf's cube on the 2^D lattice */
            const int64_t size = (int64_t)1 << (c->g.depth - c->g.leaf_level[lo]);
            for (int a = 0; a < 3; ++a) {
                double width = (s->box[3 + a] - s->box[a]) / (double)c->g.lattice;
                r[a] = s->box[a] + ((double)c->g.leaf_org[3 * lo + a] + U(1 + a) * (double)size) * width;
            }
        } else {
            int64_t idx[3] = {lo % s->n[0], (lo / s->n[0]) % s->n[1], lo / ((int64_t)s->n[0] * s->n[1])};
            for (int a = 0; a < 3; ++a) {
                double width = (s->box[3 + a] - s->box[a]) / (double)s->n[a];
                r[a] = s->box[a] + ((double)idx[a] + U(1 + a)) * width;
            }
        }
    } else {
        r[0] = s->src_pos[0];
        r[1] = s->src_pos[1];
        r[2] = s->src_pos[2];
    }
    c->flux = 0.0;
    o->energy[0] += L0;
    o->stats.packets++;
    /* emission peel-off */
    for (int j = 0; j < s->n_ins; ++j) {
        int rc = peel(c, ell, r, L0, source_phase(s, c->ins[j].kobs), kappa, j);
        if (rc) return rc;
    }
    /* emission direction: the source's angular distribution, or the learned
     * proposal (point sources) with weight p_phys / q */
    const int learned = s->mlp != NULL;
    double L = L0;
    int use_phys = 1;
    mixture mx;
    const int point = s->source_type == OR_SRC_POINT_ISO || s->source_type == OR_SRC_POINT_ANISO;
    if (learned && point) {
        double f[9], out[40];
        event_features(s, ell, r, NULL, 0.0, f);
        or_mlp_forward(s->mlp, f, out);
        mixture_from(out, &mx);
        use_phys = !mixture_sample(&mx, s->alpha, U(5), U(6), U(7), k);
    }
    if (use_phys) {
        double mu;
        if (s->source_type == OR_SRC_POINT_ANISO) {
            double u5 = U(5);
            mu = u5 < 0.5 ? sqrt(2.0 * u5) : -sqrt(2.0 * u5 - 1.0);
        } else {
            mu = 2.0 * U(5) - 1.0;
        }
        double phi = 2.0 * OR_PI * U(6);
        double st = sqrt(fmax(0.0, 1.0 - mu * mu));
        double sphi, cphi;
        or_sincos(phi, &sphi, &cphi);
        k[0] = st * cphi;
        k[1] = st * sphi;
        k[2] = mu;
    }
    if (learned && point) {
        double S = s->source_type == OR_SRC_POINT_ANISO ? 2.0 * fabs(k[2]) : 1.0;
        double pphys = S / (4.0 * OR_PI);
        double q = s->alpha * pphys + (1.0 - s->alpha) * mixture_vmf_pdf(&mx, k);
        L = L0 * (pphys / q);
    }
    if (!learned) {
        double f[9];
        event_features(s, ell, r, NULL, 0.0, f);
        record_event(c, slot, 0, f, k, L0);
    }
    int64_t e = 1;
    for (;;) {
        /* propagation to the boundary with continuous absorption */
        int rc = march(&c->g, r, k, &c->sl);
        if (rc) return rc;
        o->stats.prop_cells += (uint64_t)c->sl.n;
        const double wabs = (1.0 - albedo) * L;
        double E = 1.0, tau = 0.0, prev = c->sl.t0;
        for (int64_t n = 0; n < c->sl.n; ++n) {
            int64_t m = c->sl.cell[n];
            double ds = c->sl.tend[n] - prev;
            prev = c->sl.tend[n];
            double dtau = kappa * (double)s->density[m] * ds;
            double x = -or_expm1(-dtau);
            double A = wabs * E * x;
            int64_t ti = m * s->n_lambda + ell;
            o->table[ti] += A;
            moment_add(&c->mt, ti, A);
            o->energy[1] += A;
            E = E * (1.0 - x);
            tau = tau + dtau;
        }
        const double Epath = E;
        o->energy[2] += L * Epath;
        if (c->sl.n == 0 || albedo == 0.0 || tau == 0.0) break;
        /* scattered luminosity and termination */
        double Ls = albedo * L * (1.0 - Epath);
        if (Ls < s->w_min * L0) {
            o->energy[3] += Ls;
            break;
        }
        /* forced interaction point */
        double tau_int = -or_log1p(-U(8 * e + 0) * (1.0 - Epath));
        int64_t nstar = -1, nlast = -1;
        double taucum = 0.0, taustar_prev = 0.0, taulast_prev = 0.0;
        prev = c->sl.t0;
        double start_star = 0.0, start_last = 0.0;
        for (int64_t n = 0; n < c->sl.n; ++n) {
            int64_t m = c->sl.cell[n];
            double ds = c->sl.tend[n] - prev;
            double dtau = kappa * (double)s->density[m] * ds;
            double tprev = taucum;
            taucum = taucum + dtau;
            if (dtau > 0.0) {
                nlast = n;
                taulast_prev = tprev;
                start_last = prev;
            }
            if (taucum >= tau_int) {
                nstar = n;
                taustar_prev = tprev;
                start_star = prev;
                break;
            }
            prev = c->sl.tend[n];
        }
        if (nstar < 0) {
            nstar = nlast;
            taustar_prev = taulast_prev;
            start_star = start_last;
        }
        double rho_star;
        {
            int64_t m = c->sl.cell[nstar];
            rho_star = (double)s->density[m];
            double ds = c->sl.tend[nstar] - start_star;
            double inside = (tau_int - taustar_prev) / (kappa * (double)s->density[m]);
            if (inside < 0.0) inside = 0.0;
            if (inside > ds) inside = ds;
            double dist = start_star + inside;
            r[0] = r[0] + k[0] * dist;
            r[1] = r[1] + k[1] * dist;
            r[2] = r[2] + k[2] * dist;
        }
        o->stats.events++;
        /* scattering peel-off */
        for (int j = 0; j < s->n_ins; ++j) {
            const double *ko = c->ins[j].kobs;
            double cosang = k[0] * ko[0] + k[1] * ko[1] + k[2] * ko[2];
            rc = peel(c, ell, r, Ls, or_hg_phase(g, cosang), kappa, j);
            if (rc) return rc;
        }
        /* new direction: Henyey-Greenstein about k, or the learned proposal
         * with weight p_phys / q */
        double kn[3], f[9];
        event_features(s, ell, r, k, rho_star, f);
        int phys = 1;
        if (learned) {
            double out[40];
            or_mlp_forward(s->mlp, f, out);
            mixture_from(out, &mx);
            phys = !mixture_sample(&mx, s->alpha, U(8 * e + 1), U(8 * e + 2), U(8 * e + 3), kn);
        }
        if (phys) {
            double mus = or_hg_sample(g, U(8 * e + 1));
            double phis = 2.0 * OR_PI * U(8 * e + 2);
            or_rotate(k, mus, phis, kn);
        }
        if (learned) {
            double cosang = k[0] * kn[0] + k[1] * kn[1] + k[2] * kn[2];
            double pphys = or_hg_phase(g, cosang) / (4.0 * OR_PI);
            double q = s->alpha * pphys + (1.0 - s->alpha) * mixture_vmf_pdf(&mx, kn);
            L = Ls * (pphys / q);
        } else {
            L = Ls;
            record_event(c, slot, e, f, kn, Ls);
        }
        k[0] = kn[0];
        k[1] = kn[1];
        k[2] = kn[2];
        e = e + 1;
        if (e > s->event_cap) {
            o->energy[3] += L;
            o->stats.capped++;
            break;
        }
    }
#undef U
    if (c->out->hist_total) c->out->hist_total[slot] = c->flux;
    moment_flush(&c->mt);
    moment_flush(&c->mi);
    return 0;
}

static void instruments_init(const or_scene *s, instr *ins)
{
    int64_t off = 0;
    for (int j = 0; j < s->n_ins; ++j) {
        const double *gm = s->ins_geom + 5 * j;
        double i = gm[0] * OR_PI / 180.0, a = gm[1] * OR_PI / 180.0;
        double si = sin(i), ci = cos(i), sa = sin(a), ca = cos(a);
        instr *in = &ins[j];
        in->kobs[0] = si * ca;
        in->kobs[1] = si * sa;
        in->kobs[2] = ci;
        in->ex[0] = -sa;
        in->ex[1] = ca;
        in->ex[2] = 0.0;
        in->ey[0] = -ci * ca;
        in->ey[1] = -ci * sa;
        in->ey[2] = si;
        in->fovx = gm[3];
        in->fovy = gm[4];
        in->inv4pid2 = 1.0 / (4.0 * OR_PI * gm[2] * gm[2]);
        in->nx = s->ins_npix[2 * j];
        in->ny = s->ins_npix[2 * j + 1];
        in->offset = off;
        off += (int64_t)s->n_lambda * in->nx * in->ny;
    }
}

/* Feature constants of the learned proposal, from the scene. */
static void feature_constants(or_scene *s, double *lam_feature)
{
    double side = 0.0;
    for (int a = 0; a < 3; ++a)
        if (s->box[3 + a] - s->box[a] > side) side = s->box[3 + a] - s->box[a];
    s->r_out = 0.5 * side;
    double sum = 0.0;
    for (int64_t m = 0; m < s->n_cells; ++m) sum = sum + (double)s->density[m];
    s->rho_mean = sum / (double)s->n_cells;
    double lmin = s->lambda_um[0], lmax = s->lambda_um[0];
    for (int l = 1; l < s->n_lambda; ++l) {
        if (s->lambda_um[l] < lmin) lmin = s->lambda_um[l];
        if (s->lambda_um[l] > lmax) lmax = s->lambda_um[l];
    }
    for (int l = 0; l < s->n_lambda; ++l)
        lam_feature[l] = lmax > lmin ? (log(s->lambda_um[l]) - log(lmin)) / (log(lmax) - log(lmin)) : 0.0;
    s->lam_feature = lam_feature;
}

/* ---------------------------------------------------------------------------
 * Dust emission (Section 3.2, dust emission and self-absorption phases; the
 * paper's dust model files are not available, so a modified blackbody stands
 * in): every cell re-emits the luminosity it absorbed, with the spectral
 * shape kappa_abs B_lambda(T) dlambda and a temperature fixed by its heating.
 * ------------------------------------------------------------------------- */
double or_planck(double lambda_um, double T)
{
    const double h = 6.62607015e-34, c = 2.99792458e8, k = 1.380649e-23; /* SI, exact */
    const double lam = lambda_um * 1e-6;
    const double x = h * c / (lam * k * T);
    return 2.0 * h * c * c / (lam * lam * lam * lam * lam) / or_expm1(x);
}

void or_bin_widths(const double *lambda_um, int32_t n, double *width)
{
    if (n == 1) {
        width[0] = lambda_um[0];
        return;
    }
    /* bin edges: geometric means of neighbours; the outer edges mirror the
     * inner ones in log lambda */
    for (int32_t l = 0; l < n; ++l) {
        double lo = l > 0 ? sqrt(lambda_um[l - 1] * lambda_um[l])
                          : lambda_um[0] * lambda_um[0] / sqrt(lambda_um[0] * lambda_um[1]);
        double hi = l + 1 < n ? sqrt(lambda_um[l] * lambda_um[l + 1])
                              : lambda_um[n - 1] * lambda_um[n - 1] / sqrt(lambda_um[n - 2] * lambda_um[n - 1]);
        width[l] = hi - lo;
    }
}

int or_dust_emission(const or_scene *s, const double *table, double T0, double beta, double *T, double *emis)
{
    if (!s || !table || !T || !emis || !s->lambda_um || s->n_lambda < 1 || !(T0 > 0.0) || !(beta > -4.0)) return -1;
    const int64_t nc = s->n_cells;
    const int32_t nl = s->n_lambda;
    /* cell volumes: Cartesian cells all 1, an octree leaf at level L 8^-L
     * (the box's volume) -- only ratios of masses matter */
    geom g;
    if (geom_init(&g, s)) {
        geom_free(&g);
        return -1;
    }
    double *width = (double *)malloc((size_t)nl * sizeof(double));
    double *shape = (double *)malloc((size_t)nl * sizeof(double));
    double *cmass = (double *)malloc((size_t)nc * sizeof(double));
    or_bin_widths(s->lambda_um, nl, width);
    double mass = 0.0, absorbed = 0.0;
    for (int64_t m = 0; m < nc; ++m) {
        const double vol = s->grid_type == OR_GRID_OCTREE ? ldexp(1.0, -3 * g.leaf_level[m]) : 1.0;
        cmass[m] = (double)s->density[m] * vol;
        mass += cmass[m];
        for (int32_t l = 0; l < nl; ++l) absorbed += table[m * nl + l];
    }
    const double u0 = mass > 0.0 ? absorbed / mass : 0.0;
    for (int64_t m = 0; m < nc; ++m) {
        double La = 0.0;
        for (int32_t l = 0; l < nl; ++l) La += table[m * nl + l];
        const double mm = cmass[m];
        T[m] = 0.0;
        for (int32_t l = 0; l < nl; ++l) emis[m * nl + l] = 0.0;
        if (!(La > 0.0) || !(mm > 0.0) || !(u0 > 0.0)) continue;
        const double Tm = T0 * or_exp(or_log((La / mm) / u0) / (4.0 + beta));
        T[m] = Tm;
        double sum = 0.0;
        for (int32_t l = 0; l < nl; ++l) {
            shape[l] = s->kappa[l] * (1.0 - s->albedo[l]) * width[l] * or_planck(s->lambda_um[l], Tm);
            sum += shape[l];
        }
        if (!(sum > 0.0)) continue; /* nothing the grid's bins can carry */
        for (int32_t l = 0; l < nl; ++l) emis[m * nl + l] = La * (shape[l] / sum);
    }
    free(width);
    free(shape);
    free(cmass);
    geom_free(&g);
    return 0;
}

int or_run(const or_scene *s_in, uint64_t n_per_lambda, uint64_t first_id,
           uint64_t count, uint64_t seed, uint32_t model, or_out *out)
{
    if (!s_in || !out || n_per_lambda == 0 || first_id + count > n_per_lambda) return -1;
    if (s_in->mlp && !s_in->lambda_um) return -1;
    or_scene scene = *s_in;
    or_scene *s = &scene;
    double *lam_feature = (double *)calloc((size_t)(s->n_lambda > 0 ? s->n_lambda : 1), sizeof(double));
    if (s->lambda_um && s->n_lambda > 0) feature_constants(s, lam_feature);
    if (first_id + count > 0xffffffffull + 1ull) return -1;
    if (s->n_lambda <= 0 || s->n_cells <= 0 || s->n_ins < 0) return -1;
    if (s->source_type == OR_SRC_DUST && !s->dust_cdf) return -1;
    runctx c;
    memset(&c, 0, sizeof(c));
    c.s = s;
    c.out = out;
    c.seed = seed;
    c.model = model;
    if (geom_init(&c.g, s)) {
        geom_free(&c.g);
        return -2;
    }
    c.ins = (instr *)calloc((size_t)(s->n_ins > 0 ? s->n_ins : 1), sizeof(instr));
    instruments_init(s, c.ins);
    int64_t ntab = s->n_cells * s->n_lambda;
    int64_t nimg = 0;
    for (int j = 0; j < s->n_ins; ++j) nimg += (int64_t)s->n_lambda * c.ins[j].nx * c.ins[j].ny;
    if (out->table_m2) {
        c.mt.m2 = out->table_m2;
        c.mt.acc = (double *)calloc((size_t)ntab, sizeof(double));
        c.mt.touched = (int64_t *)malloc((size_t)ntab * sizeof(int64_t));
    }
    if (out->image_m2 && nimg > 0) {
        c.mi.m2 = out->image_m2;
        c.mi.acc = (double *)calloc((size_t)nimg, sizeof(double));
        c.mi.touched = (int64_t *)malloc((size_t)nimg * sizeof(int64_t));
    }
    int rc = 0;
    for (int ell = 0; ell < s->n_lambda && rc == 0; ++ell) {
        double L0 = s->lum[ell] / (double)n_per_lambda;
        for (uint64_t i = first_id; i < first_id + count; ++i) {
            rc = one_packet(&c, ell, (uint32_t)i, L0, (int64_t)ell * (int64_t)count + (int64_t)(i - first_id));
            if (rc) break;
        }
    }
    free(c.mt.acc);
    free(c.mt.touched);
    free(c.mi.acc);
    free(c.mi.touched);
    free(c.ins);
    free(lam_feature);
    seg_free(&c.sl);
    geom_free(&c.g);
    return rc ? -3 : 0;
}
