/*
 * mcrt_oracle.h -- serial FP64 CPU oracle for the Monte Carlo photon-packet
 * life cycle (stellar emission phase) of the hybrid-parallel SKIRT paper
 * (Verstocken et al. 2017, Section 3.2 "Stellar emission phase" and the
 * Fig. 2 caption; accumulation primitive of Section 5.2 "Lockfree additions").
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against an independent, plain, obviously-correct implementation.  Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no code, header, table or constant generator with the
 * GPU path.
 *
 * Everything is double precision, compiled without floating-point
 * contraction, serial, one packet at a time.
 */
#ifndef MCRT_ORACLE_H
#define MCRT_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_GRID_CARTESIAN = 0, OR_GRID_OCTREE = 1 };
enum { OR_SRC_POINT_ISO = 0, OR_SRC_POINT_ANISO = 1, OR_SRC_EXPDISK = 2, OR_SRC_DUST = 3 };

/* One scene.  All arrays are borrowed (the caller owns them). */
typedef struct {
    int32_t grid_type;          /* OR_GRID_* */
    double box[6];              /* xmin, ymin, zmin, xmax, ymax, zmax */
    int32_t n[3];               /* Cartesian cell counts */
    int64_t n_nodes;            /* octree node count */
    const int32_t *first_child; /* octree: index of child 0, -1 for a leaf */
    int64_t n_cells;            /* number of dust cells (leaves) */
    const float *density;       /* [n_cells] */
    int32_t n_lambda;
    const double *kappa;        /* [n_lambda] extinction per unit density */
    const double *albedo;       /* [n_lambda] */
    const double *hg_g;         /* [n_lambda] */
    int32_t source_type;        /* OR_SRC_* */
    double src_pos[3];          /* point sources */
    double disk_hR, disk_zs;    /* exponential disk */
    const double *lum;          /* [n_lambda] luminosity per wavelength bin */
    int32_t n_ins;
    const double *ins_geom;     /* [n_ins][5]: incl_deg, azim_deg, distance, fov_x, fov_y */
    const int32_t *ins_npix;    /* [n_ins][2]: nx, ny */
    double w_min;               /* termination fraction of the launch luminosity */
    int64_t event_cap;          /* maximum scattering events per packet */
    double tau_peel_max;        /* +inf: every peel-off counts (the definition); a finite value
                                   drops peel-offs whose optical depth reaches it */
    /* learned direction proposal (NULL mlp = plain sampling) */
    const double *mlp;          /* 7400 parameters, weights bfloat16-representable */
    double alpha;               /* weight of the physical component */
    const double *lambda_um;    /* [n_lambda] wavelengths (features) */
    /* derived by or_run: position feature scale (half the largest box side),
     * (log lambda - log lambda_min) / log range, mean cell density */
    double r_out;
    const double *lam_feature;
    double rho_mean;
    /* OR_SRC_DUST: [n_lambda][n_cells] running sums over the cells (natural
     * order ix + nx (iy + ny iz), or the leaf order) of the dust emission, from
     * or_dust_emission; lum[] holds each row's last element */
    const double *dust_cdf;
} or_scene;

typedef struct {
    uint64_t packets;
    uint64_t events;            /* forced interactions followed by a scattering */
    uint64_t prop_cells;        /* segments visited by propagation marches */
    uint64_t peel_cells;        /* segments visited by peel-off marches */
    uint64_t peel_adds;         /* pixel additions */
    uint64_t peel_dropped;      /* peel-offs cut by tau_peel_max */
    uint64_t capped;            /* packets that hit the event cap */
} or_stats;

/* Outputs of one run (all zeroed by the caller, accumulated by the oracle).
 * table:   [n_cells][n_lambda]   element (i, j) at i*n_lambda + j (Section 5.2,
 *          ParallelTable multithreading mode).
 * images:  concatenation over instruments of [n_lambda][ny][nx] fluxes.
 * energy:  [4] emitted, absorbed, escaped, truncated.
 * table_m2, image_m2: optional (NULL to skip) per-packet second moments,
 *          sum over packets of (per-packet contribution)^2.
 */
typedef struct {
    double *table;
    double *images;
    double *energy;
    double *table_m2;
    double *image_m2;
    or_stats stats;
    /* optional plain-run histories: per packet (launch order) and event e <
     * hist_events: 9 features, new direction (3), luminosity after the event,
     * image flux produced so far; hist_total: the packet's total image flux */
    double *hist;
    double *hist_total;
    int32_t hist_events;
} or_out;

/* Runs packet ids [first_id, first_id + count) of every wavelength, with the
 * per-packet luminosity L_lambda / n_per_lambda.  model is the fourth word of
 * the Philox counter.  Returns 0, or a negative value on invalid input. */
int or_run(const or_scene *scene, uint64_t n_per_lambda, uint64_t first_id,
           uint64_t count, uint64_t seed, uint32_t model, or_out *out);

/* Dust emission (stand-in for the dust emission and self-absorption phases
 * of Section 3.2): from the absorbed luminosity table [n_cells][n_lambda],
 * each cell's temperature T = T0 (u / u0)^(1 / (4 + beta)) with u = absorbed
 * luminosity per unit mass (mass = density x volume; octree leaves at level
 * L have volume 8^-L of the box) and u0 = total absorbed / total mass, and
 * its emission spread over the wavelength bins in proportion to kappa
 * (1 - albedo) B_lambda(T) dlambda (bin widths between the geometric means of
 * neighbouring wavelengths), so that every cell emits what it absorbed.
 * Writes T[n_cells] (0 where nothing is absorbed) and emis[n_cells][n_lambda].
 * Returns 0, or -1 on invalid input.  A dust packet starts at a uniform point
 * of its cell (Cartesian cell or octree leaf). */
int or_dust_emission(const or_scene *scene, const double *table, double T0, double beta, double *T,
                     double *emis);
/* Planck spectral radiance B_lambda(T) in W m^-2 m^-1 sr^-1, lambda in micron. */
double or_planck(double lambda_um, double T);
/* Widths of the wavelength bins around lambda_um[n] (n >= 1). */
void or_bin_widths(const double *lambda_um, int32_t n, double *width);

/* Building blocks exposed for the pin tests. */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double or_uniform64(uint64_t seed, uint32_t packet, uint32_t lambda, uint32_t model, uint32_t slot);
float or_uniform32(uint64_t seed, uint32_t packet, uint32_t lambda, uint32_t model, uint32_t slot);

/* Ray march: writes up to max_seg (cell, length) pairs; returns the number of
 * segments, or -1 if max_seg was too small. */
int64_t or_march(const or_scene *scene, const double r[3], const double k[3],
                 int64_t *cells, double *lengths, int64_t max_seg);

/* Elementary functions with a platform-independent operation sequence. */
double or_exp(double x);
double or_expm1(double x);
double or_log(double x);
double or_log1p(double x);
double or_atanh(double x);
void or_sincos(double x, double *s, double *c);

/* The proposal network on bfloat16-rounded inputs and activations, FP64
 * sums: f[9] -> out[40]. */
void or_mlp_forward(const double *theta, const double f[9], double out[40]);

/* Henyey-Greenstein phase function and sampler. */
double or_hg_phase(double g, double mu);
double or_hg_sample(double g, double u);
void or_rotate(const double k[3], double mu, double phi, double out[3]);

#ifdef __cplusplus
}
#endif

#endif
