/*
 * mcrt.h -- C-ABI of the MI355X photon-packet transport library.
 *
 * The library runs the stellar emission phase of a Monte Carlo dust
 * radiative-transfer simulation as described in the hybrid-parallel SKIRT
 * paper (Verstocken et al. 2017), Section 3.2 "Stellar emission phase": for
 * each wavelength a fixed number of photon packets is launched from the
 * primary source, propagated through the dust grid while it loses
 * luminosity continuously to absorption (written to the per-cell,
 * per-wavelength absorbed-luminosity table), forced to interact, scattered,
 * and peeled off towards every instrument at emission and at every
 * scattering event, until only a negligible part of its launch luminosity
 * remains.  The table is the "absorbed stellar luminosity" table of Fig. 2
 * and Section 5.2 (ParallelTable, element (i, j) = cell i, wavelength j);
 * additions to it are lock-free (Section 5.2 "Lockfree additions"), here as
 * hardware FP64 atomic adds.  The client needs only a handful of calls
 * (Section 5.1.1, "the client").
 *
 * Conventions
 *  - Every function returns MCRT_OK (0) or a negative MCRT_E* code; the
 *    thread-local message of the last failure is mcrt_last_error().  No C++
 *    exception crosses this boundary.
 *  - Handles are opaque, created and destroyed only by the library.  A
 *    handle must outlive every handle created from it (context > grid >
 *    medium > sim > result; source and instrument > sim).
 *  - Input arrays are host memory, copied at create time; the caller keeps
 *    ownership.
 *  - Result readers copy into a caller buffer that may be host memory or
 *    device memory on the context's device; `count` (elements) is checked and
 *    MCRT_EINVAL is returned if it is smaller than required.
 *  - All device work of a call runs on the context's stream; every call
 *    returns after that work has completed.
 *  - One run per simulation at a time: a second concurrent run on the same
 *    sim returns MCRT_EBUSY (the single-owner rule of the paper's
 *    ProcessManager, Section 5.1).
 *  - Units are arbitrary but consistent: lengths (grid box, distances, field
 *    of view) in one unit, kappa is extinction per unit density per unit
 *    length, luminosities per wavelength bin.
 *  - Run log (the paper's per-phase timing, Section 7, as one record per
 *    launch): with the environment variable MCRT_LOG set to a positive
 *    integer, every timed transport launch (mcrt_run_into, mcrt_run_range,
 *    mcrt_run, mcrt_batch_run_into, mcrt_run_dust_into and the dust cycles,
 *    mcrt_proposal_collect) appends one JSON line to the file named by
 *    MCRT_LOG_FILE, else to stderr: the entry point, the scene's shape
 *    (grid kind, cells, wavelengths, instruments; summed over a batch's
 *    models), precision, the id range, the counters of mcrt_stats that THIS
 *    launch added, the kernel time, and packets/s, deposits/s (propagation
 *    cells + pixel additions), the algorithmic HBM bytes (12 per
 *    propagation cell, 4 per interaction-search or peel-off cell, 4 (FP32)
 *    or 8 (FP64) per pixel addition), their rate in GB/s and its fraction of
 *    8 TB/s, and the return code.  Both variables are read at every launch.
 *    Autotuner trials and the untimed mcrt_run_into_noalloc are not logged.
 */
#ifndef MCRT_H
#define MCRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MCRT_OK 0
#define MCRT_EINVAL (-1)  /* invalid handle, argument or size */
#define MCRT_ENOMEM (-2)  /* device or host allocation failed */
#define MCRT_EDEVICE (-3) /* HIP runtime error */
#define MCRT_EBUSY (-4)   /* the simulation is already running */
#define MCRT_ELIMIT (-5)  /* packets hit the event cap; results are valid, see stats.capped */
#define MCRT_ENONFINITE (-6) /* packets whose luminosity became NaN or infinite were ended
                                (see stats.nonfinite); the other packets' results are valid */

/* FP32 transport, FP64 table totals and energy sums.  Luminosities travel
 * in FP32 and the images are FP32: a wavelength whose packet luminosity
 * (source or dust luminosity / n_per_lambda) is below FP32's normal range
 * (1.2e-38) is carried with fewer significant bits, and below 2^-150
 * (7e-46) its packets launch with zero luminosity and contribute nothing --
 * the far Wien tail of cold dust emission, say; the FP64 validation mode
 * keeps it. */
#define MCRT_FP32 0
#define MCRT_FP64_VALIDATE 1  /* FP64 throughout, no contraction */

#define MCRT_MAX_INSTRUMENTS 8

typedef struct mcrt_context mcrt_context;
typedef struct mcrt_grid mcrt_grid;
typedef struct mcrt_medium mcrt_medium;
typedef struct mcrt_source mcrt_source;
typedef struct mcrt_instrument mcrt_instrument;
typedef struct mcrt_sim mcrt_sim;
typedef struct mcrt_result mcrt_result;
typedef struct mcrt_proposal mcrt_proposal;
typedef struct mcrt_histories mcrt_histories;
typedef struct mcrt_dust mcrt_dust;

typedef struct {
    int32_t precision;     /* MCRT_FP32 or MCRT_FP64_VALIDATE */
    double w_min;          /* a packet ends once its scattered luminosity drops below
                              w_min times its launch luminosity ("negligible part",
                              Section 3.2); default 1e-6 */
    int64_t event_cap;     /* maximum scattering events per packet; default 10000 */
    double tau_peel_max;   /* default +infinity: every peel-off reaches its pixel, as the
                              estimator defines it (Section 3.2, peel-off).  A finite value
                              is an approximation the caller opts into: a peel-off march
                              stops once its optical depth reaches tau_peel_max and that
                              contribution is dropped, an error below exp(-tau_peel_max)
                              of the contribution (40: 4e-18, below FP32 resolution) */
    int32_t chunk;         /* packets per work-queue grab; 0 = default */
    int32_t waves_per_cu;  /* persistent waves per compute unit; 0 = default */
    int32_t threshold;     /* lanes that must finish a march before events run; 0 = default
                              (16; batches 24) */
    int32_t top_level;     /* octree top-table level; -1 = default */
    int32_t brick[3];      /* Cartesian storage bricks: log2 cells per axis, summing to 5
                              (32 cells per brick); {-1, -1, -1} = chosen from the cell
                              aspect ratio */
    int32_t queue_order;   /* batches (the first simulation's options): the order of the
                              models in the work queue, one of MCRT_QUEUE_*; default
                              MCRT_QUEUE_PAIRED.  A model's random streams are keyed by its
                              position in the caller's list, so no order changes a result,
                              only the launch's tail (Section 7.4, Fig. 14) */
    int32_t chunk_shift;   /* the automatic chunk (chunk = 0) times 2^chunk_shift, in
                              -6 .. 6; default 0.  The automatic chunk scales with the
                              launch, so a shift tuned on a short trial carries over to
                              the full launch */
    int32_t deposit_slots; /* FP32 batches (the first simulation's options): deposit slots
                              per lane in the wave's LDS tile, 8 (the tile is issued
                              after every march iteration) or 16 (after every other
                              one); 0 = default (16) */
} mcrt_options;

/* Batch queue orders (Section 5.2 assigners; Section 7.4 load-balance lesson). */
#define MCRT_QUEUE_COST 0   /* most expensive model first (longest processing time) */
#define MCRT_QUEUE_CALLER 1 /* the caller's order (the sequential assigner's blocks) */
#define MCRT_QUEUE_PAIRED 2 /* most and least expensive alternating (the suggested pairs;
                               the default) */

typedef struct {
    uint64_t packets;      /* packets launched */
    uint64_t events;       /* forced interactions followed by a scattering */
    uint64_t prop_cells;   /* cells crossed by propagation marches (with deposits) */
    uint64_t locate_cells; /* cells crossed while locating interaction points */
    uint64_t peel_cells;   /* cells crossed by peel-off marches */
    uint64_t peel_adds;    /* pixel additions */
    uint64_t peel_dropped; /* peel-offs cut by tau_peel_max */
    uint64_t capped;       /* packets that hit the event cap */
    uint64_t guard;        /* octree marches stopped by the step guard (0 for valid trees) */
    uint64_t nonfinite;    /* packets ended because their luminosity (or, with the learned
                              proposal, their weight) became NaN or infinite; a finite
                              scene gives 0 */
    double kernel_ms;      /* transport kernel time of the last run into this result */
} mcrt_stats;

/* Fills *opt with the defaults listed above. */
void mcrt_options_default(mcrt_options *opt);

/* The execution resources every later call runs on (the role of the
 * parallel engine's thread pool in Section 5.1.2 and 5.2.4, here one device
 * and one stream): binds a device (HIP ordinal) and a stream (a hipStream_t
 * such as torch's current_stream().cuda_stream, or NULL for the default
 * stream; the caller keeps it alive).  Errors: MCRT_EINVAL (no such device,
 * out NULL), MCRT_EDEVICE. */
int mcrt_context_create(int device, void *hip_stream_or_null, mcrt_context **out);
void mcrt_context_destroy(mcrt_context *ctx);

/* Dust grid (Section 3.2, setup phase).  Cartesian: box = {xmin, ymin, zmin,
 * xmax, ymax, zmax}, n cells per axis; cell index m = ix + nx (iy + ny iz),
 * planes at xmin + j (xmax - xmin) / nx. */
int mcrt_grid_create_cartesian(mcrt_context *ctx, const double box[6], const int32_t n[3],
                               mcrt_grid **out);
/* Octree: first_child[node] is the index of the node's first child or -1 for
 * a leaf; the 8 children are contiguous in the order c = bx + 2 by + 4 bz;
 * node 0 is the root (the whole box); leaves are numbered in depth-first
 * order; maximum depth 15, fewer than 2^27 nodes. */
int mcrt_grid_create_octree(mcrt_context *ctx, const double box[6], int64_t n_nodes,
                            const int32_t *first_child, mcrt_grid **out);
void mcrt_grid_destroy(mcrt_grid *grid);

/* Dust medium (the dust system of Section 3.2 over the grid of the setup
 * phase, with the wavelength grid of Section 7.2): density per cell (grid
 * order; FP32, >= 0), and per wavelength the extinction coefficient kappa
 * (per unit density and length, >= 0), the albedo (in [0, 1]) and the
 * Henyey-Greenstein asymmetry parameter g (in (-1, 1)).  lambda_um (micron,
 * increasing) may be NULL; the learned proposal, dust emission and the
 * writing phase need it.  Host arrays, copied.  Errors: MCRT_EINVAL for
 * values out of range or non-finite, MCRT_ENOMEM. */
int mcrt_medium_create(mcrt_grid *grid, const float *density, int32_t n_lambda,
                       const double *lambda_um, const double *kappa, const double *albedo,
                       const double *g, mcrt_medium **out);
void mcrt_medium_destroy(mcrt_medium *medium);

/* Primary sources with a-priori known emission (Section 3.2), luminosity L
 * per wavelength bin.  Point source at pos: aniso = 0 isotropic, 1 angular
 * distribution 2|cos theta| about the z axis.  Exponential disk: surface
 * density exp(-R/hR), vertical sech^2(z/zs), centred at the origin in the
 * z = 0 plane. */
int mcrt_source_create_point(mcrt_context *ctx, const double pos[3], int32_t aniso,
                             int32_t n_lambda, const double *L, mcrt_source **out);
int mcrt_source_create_expdisk(mcrt_context *ctx, double hR, double zs, int32_t n_lambda,
                               const double *L, mcrt_source **out);
void mcrt_source_destroy(mcrt_source *src);

/* Distant observer with parallel projection (the instrument table of
 * Section 3.2): viewing direction (sin i cos a, sin i sin a, cos i), sky
 * axes e_x = (-sin a, cos a, 0) and e_y = (-cos i cos a, -cos i sin a, sin i),
 * field of view fov[2] centred on the origin, npix[2] = {nx, ny} pixels.
 * Images hold flux L phase exp(-tau) / (4 pi distance^2) per pixel. */
int mcrt_instrument_create(mcrt_context *ctx, double incl_deg, double azim_deg, double distance,
                           const double fov[2], const int32_t npix[2], mcrt_instrument **out);
void mcrt_instrument_destroy(mcrt_instrument *ins);

/* Assembles a simulation of the stellar emission phase (Section 3.2: the
 * grid and dust system of the setup phase, the primary source, the
 * instruments) and uploads the scene to the device; the device copy is
 * read-only during runs (the per-run state lives in results).  opt may be
 * NULL for defaults.  The medium's and source's n_lambda must agree; at
 * most MCRT_MAX_INSTRUMENTS instruments.  Errors: MCRT_EINVAL, MCRT_ENOMEM,
 * MCRT_EDEVICE. */
int mcrt_sim_create(mcrt_context *ctx, mcrt_medium *medium, mcrt_source *source,
                    mcrt_instrument *const *ins, int32_t n_ins, const mcrt_options *opt,
                    mcrt_sim **out);
void mcrt_sim_destroy(mcrt_sim *sim);

/* A zeroed result (table, images, energy sums, stats) for the sim. */
int mcrt_result_create(mcrt_sim *sim, mcrt_result **out);
int mcrt_result_zero(mcrt_result *res);

/* Runs packet ids [first_id, first_id + count) of every wavelength, each
 * packet carrying L / n_per_lambda (a fixed number of packets per
 * wavelength, Section 3.2, stellar emission phase), and ADDS their
 * contributions to res.  Because absorbed luminosities add linearly
 * (Section 5.2.5) and every packet has its own counter-based random stream,
 * running disjoint id ranges into one result equals one run over their union
 * (resume, sharding).  Returns MCRT_ELIMIT (with valid results) if a packet
 * of THIS launch hit the event cap, MCRT_ENONFINITE if a packet of this
 * launch was ended for a non-finite luminosity (either is decided from the
 * counts this launch added, not from earlier launches into res); also
 * MCRT_EINVAL, MCRT_EBUSY, MCRT_EDEVICE. */
int mcrt_run_into(mcrt_sim *sim, uint64_t n_per_lambda, uint64_t first_id, uint64_t count,
                  uint64_t seed, mcrt_result *res);
/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): mcrt_run_into without
 * any allocation, copy from the host or event creation in the call.  Same
 * arguments, results, errors and return codes as mcrt_run_into (the same
 * kernels).  The launch's scratch -- the work-queue counter and the
 * per-wavelength optics staged for the launch -- lives in a fixed device
 * array of 164096 bytes per GPU that the library holds until the process
 * ends (its address is taken when the first context on that GPU is
 * created) and that every call on that GPU shares: the call prepares it on
 * the device, so nothing of an earlier call's contents leaks into a later
 * one, but calls that overlap on one GPU (from several threads or streams)
 * race on it and must not be made.  At most 4096 wavelengths (MCRT_EINVAL
 * beyond).  The kernel is not timed (stats.kernel_ms reads 0).  The caller
 * creates the sim and the result beforehand (those calls allocate). */
int mcrt_run_into_noalloc(mcrt_sim *sim, uint64_t n_per_lambda, uint64_t first_id, uint64_t count,
                          uint64_t seed, mcrt_result *res);
/* Convenience (Section 3.2, stellar emission phase: all n_per_lambda packets
 * of every wavelength): new result + run; *out is set (and owned by the
 * caller) on MCRT_OK, MCRT_ELIMIT and MCRT_ENONFINITE. */
int mcrt_run(mcrt_sim *sim, uint64_t n_per_lambda, uint64_t seed, mcrt_result **out);
/* Convenience: new result + run of an id range (one shard of the task
 * parallel mode of Section 4.2, which splits the packets of every wavelength
 * between processes); *out as for mcrt_run. */
int mcrt_run_range(mcrt_sim *sim, uint64_t n_per_lambda, uint64_t first_id, uint64_t count,
                   uint64_t seed, mcrt_result **out);

/* Batched run (the many-small-models use case of Section 3.1): sims[i]
 * (distinct Cartesian sims of one context and one precision) runs packet ids
 * [0, n_per_lambda[i]) of each of its wavelengths and adds them to
 * results[i] (created with mcrt_result_create for sims[i]), all in ONE
 * persistent launch.  The position i in the batch is the fourth word of the
 * packets' Philox counters, so results equal per-model runs with model = i.
 * Queue tuning (chunk, threshold, waves per CU) and the queue order come from
 * sims[0]'s options.
 * Returns MCRT_ELIMIT (with valid results) if any packet hit its event cap. */
int mcrt_batch_run_into(mcrt_sim *const *sims, int32_t n, const uint64_t *n_per_lambda, uint64_t seed,
                        mcrt_result *const *results);

/* Launch tuning of a sim (overrides its options' queue parameters; the work
 * distribution of Section 5.2.4: how many packets a thread takes per grab). */
typedef struct {
    int32_t chunk;        /* packets per work-queue grab; 0 = the automatic chunk */
    int32_t waves_per_cu; /* persistent waves per compute unit */
    int32_t threshold;    /* lanes that must finish a march before events run */
    double kernel_ms;     /* trial time of this setting (output of the tuner) */
    int32_t from_cache;   /* 1 if the tuner found the setting in its cache */
    double default_ms;    /* trial time of the library's defaults (output of the tuner) */
    int32_t chunk_shift;  /* with chunk = 0: the automatic chunk times 2^chunk_shift (-6 .. 6) */
    int32_t deposit_slots; /* FP32 batches: deposit tile of 8 or 16 slots per lane; 0 = default */
} mcrt_tuning;

int mcrt_sim_set_tuning(mcrt_sim *sim, const mcrt_tuning *t);

/* Autotuner: coordinate search, starting from sims[0]'s options (the
 * library's defaults unless set), over the chunk as a multiple of the
 * automatic chunk (chunk = 0, chunk_shift -3 .. 3: the automatic chunk
 * scales with the launch, so a setting tuned on a short trial keeps its
 * shape in the full launch), threshold {8..48}, waves per CU
 * {8, 12, 16} and, for FP32 batches, the deposit tile {8, 16} slots per
 * lane, with trial runs of trial_packets[i] packets per wavelength of
 * each sim (one sim: the single-model kernel; several: the batched kernel),
 * keeping the fastest; the pick and the defaults are then timed twice more
 * each and the pick is kept only if its best time beats the defaults' (both
 * times are returned).  Trials should be long enough to have the full
 * launch's shape (a launch's tail weighs more in a short trial).  With
 * cache_path (may be NULL) the
 * result is stored under a key describing the problem class (grid type,
 * precision, model count, cells, wavelengths, instruments) and reused on the
 * next call without trials.  The tuning is applied to every sim and returned
 * in *best.  Results do not depend on the tuning beyond the order of atomic
 * additions. */
int mcrt_autotune(mcrt_sim *const *sims, int32_t n, const uint64_t *trial_packets, uint64_t seed,
                  const char *cache_path, mcrt_tuning *best);

/* ------------------------------------------------------------------------
 * Learned direction proposal.  An extension of the interaction-direction
 * sampling of Section 3.2 (the paper itself samples directions from the
 * physical phase function): a small network maps the features of an
 * emission or scattering event -- position / r_out (r_out = half the largest
 * box side), incoming direction (zero at emission), the wavelength feature
 * (log l - log l_min) / (log l_max - log l_min), log10 of the interaction
 * cell's density over the mean cell density (zero at emission) and an event
 * flag (0 emission, 1 scattering) -- to an 8-lobe von Mises-Fisher mixture.
 * New directions are drawn from q = alpha p_phys + (1 - alpha) sum_j pi_j
 * vMF_j and the packet luminosity is multiplied by p_phys / q, so every
 * tally keeps its expectation.  Point sources use the proposal at emission
 * too; the disk source keeps its physical emission.
 * Network: 9 -> 64 -> 64 -> 40 with ReLU, outputs = 8 mixture logits, 8 x 3
 * raw lobe axes (normalised), 8 raw concentrations (kappa = clamp(softplus +
 * 1e-3, 1e-3, 1e3)).  Weights, inputs and hidden activations are bfloat16
 * (nearest even); sums FP32 on the matrix cores (FP64 in the FP64
 * validation transport).  Parameter layout (7400 floats): W1 [9][64]
 * (input-major), b1 [64], W2 [64][64], b2 [64], W3 [64][40], b3 [40].
 * ---------------------------------------------------------------------- */
#define MCRT_MLP_PARAMS 7400

typedef struct {
    int32_t n_in, n_hidden, n_out; /* must be 9, 64, 40 */
    uint64_t init_seed;            /* uniform fan-in initialisation, biases 0 */
    float init_scale;              /* weights U(-b, b), b = init_scale sqrt(6 / fan_in) */
} mcrt_mlp_desc;

int mcrt_proposal_create(mcrt_context *ctx, const mcrt_mlp_desc *desc, mcrt_proposal **out);
void mcrt_proposal_destroy(mcrt_proposal *p);
/* FP32 master parameters (host or device buffers, count = 7400); setting them
 * also resets the Adam state.  get_weights: the parameters rounded to
 * bfloat16 bit patterns (as the network uses the weights). */
int mcrt_proposal_set_params(mcrt_proposal *p, const float *theta, size_t count);
int mcrt_proposal_get_params(const mcrt_proposal *p, float *theta, size_t count);
int mcrt_proposal_get_weights(const mcrt_proposal *p, uint16_t *bf16, size_t count);
/* Network outputs on the matrix cores: X [n][9] -> out [n][40] (host or
 * device buffers). */
int mcrt_proposal_forward(mcrt_proposal *p, const float *X, int64_t n, float *out);
/* Weighted negative log-likelihood of the vMF part,
 * loss = -sum_e C_e log q_vMF(KP_e | X_e) / sum_e C_e, and its gradient
 * [7400] in the parameter layout, for n samples (features X [n][9],
 * directions KP [n][3], weights C [n] >= 0, not all zero; host or device
 * buffers).  The backward pass carries the output and pre-activation
 * gradients as bfloat16 high + low parts on the matrix cores. */
int mcrt_proposal_grad(mcrt_proposal *p, const float *X, const float *KP, const float *C, int64_t n,
                       double *loss, float *grad);

/* Attaches the proposal to a sim (p = NULL detaches).  alpha in (0, 1] is
 * the weight of the physical distribution (defensive mixture).  The medium
 * must have been created with wavelengths.  The proposal must outlive the
 * sim's runs; batched runs reject sims with a proposal. */
int mcrt_sim_set_proposal(mcrt_sim *sim, mcrt_proposal *p, double alpha);

/* Plain run (no proposal attached) of packet ids [first_id, first_id +
 * count) of every wavelength that ADDS to res like mcrt_run_into and also
 * records, per packet (slot = wavelength * count + id - first_id) and per
 * event e < max_events (e = 0 emission, e >= 1 scattering e): the 9
 * features, the direction taken (3), the luminosity after the event and the
 * image flux the packet had produced so far; plus each packet's total image
 * flux.  Training samples are the recorded events with weight C = (total -
 * flux so far) / luminosity > 0, in (slot, event) order.  At most 2^32
 * packets.  Returns MCRT_ELIMIT with valid histories if a packet hit the
 * event cap. */
int mcrt_proposal_collect(mcrt_sim *sim, uint64_t n_per_lambda, uint64_t first_id, uint64_t count,
                          uint64_t seed, int32_t max_events, mcrt_result *res, mcrt_histories **out);
int mcrt_histories_info(const mcrt_histories *h, int64_t *n_packets, int32_t *max_events,
                        int64_t *n_samples, double *weight_sum);
/* Raw records [packet][max_events][14] (zero for events not reached) and
 * packet totals, converted to double (host or device buffers). */
int mcrt_histories_records(const mcrt_histories *h, double *records, size_t count, double *totals,
                           size_t count_totals);
/* Training samples: X [n][9], KP [n][3], C [n] (host or device buffers). */
int mcrt_histories_samples(const mcrt_histories *h, float *X, float *KP, float *C, size_t n);
void mcrt_histories_destroy(mcrt_histories *h);

typedef struct {
    int32_t epochs;      /* passes over the samples (in minibatch draws) */
    int32_t batch;       /* samples per Adam step, drawn uniformly with replacement */
    float lr, beta1, beta2, eps;
    uint64_t seed;       /* minibatch draws */
} mcrt_train_opts;
void mcrt_train_opts_default(mcrt_train_opts *opt);
/* Adam on the FP32 master parameters for epochs * ceil(n_samples / batch)
 * steps (forward and backward on the matrix cores); *final_loss (may be
 * NULL) receives the last minibatch's loss.  The Adam state persists across
 * calls until mcrt_proposal_set_params. */
int mcrt_proposal_train(mcrt_proposal *p, const mcrt_histories *h, const mcrt_train_opts *opt,
                        double *final_loss);
/* Loss over all samples of h at the current parameters. */
int mcrt_proposal_eval(mcrt_proposal *p, const mcrt_histories *h, double *loss);

/* Absorbed luminosity table, out[i * n_lambda + j] for cell i and
 * wavelength j (Section 5.2, ParallelTable element (i, j)); count >=
 * n_cells * n_lambda. */
int mcrt_result_absorption(const mcrt_result *res, double *out, size_t count);
/* Image of instrument ins (its table of flux per pixel per wavelength, the
 * instrument of Section 3.2 that emission and scattering events peel off
 * onto; Section 5.2.6 for the wavelength-sliced data cube), layout
 * [lambda][y][x], flux units (L phase exp(-tau) / (4 pi d^2) summed per
 * pixel); FP64 copy of the FP32 production images; count >= n_lambda * ny *
 * nx; host or device buffer. */
int mcrt_result_image(const mcrt_result *res, int32_t ins, double *out, size_t count);
/* SED of instrument ins: out[l] = total flux of wavelength slice l (the sum
 * of its pixels, flux units, reduced on the device in FP64 in a fixed order);
 * count >= n_lambda.  (Section 3.2, writing: SEDs next to the data cubes.) */
int mcrt_result_sed(const mcrt_result *res, int32_t ins, double *out, size_t count);
/* Writing phase (Section 3.2): the data cube of instrument ins as a FITS file
 * (fits_path; layout as mcrt_fits_cube_create) and its SED as a text file
 * (sed_path, as mcrt_sed_write_text); either path may be NULL.  Needs the
 * medium's wavelengths (MCRT_EINVAL without them).  Files are overwritten. */
int mcrt_result_write(const mcrt_result *res, int32_t ins, const char *fits_path, const char *sed_path);

/* ---- Dust emission phase (Section 3.2: dust emission and self-absorption
 * phases).  The paper's dust model files are not available; a modified
 * blackbody stands in.  Cartesian and octree grids.
 *
 * A cell m that absorbed La(m) (summed over wavelengths) re-emits exactly
 * La(m), spread over the wavelength bins l in proportion to
 *     kappa_l (1 - albedo_l) dlambda_l B_lambda(lambda_l, T_m),
 * dlambda_l the bin width between the geometric means of neighbouring
 * wavelengths (outer edges mirrored in log lambda), B_lambda the Planck
 * function, and T_m = T0 (u_m / u0)^(1 / (4 + beta)) with
 * u_m = La(m) / mass(m), mass = density x volume (Cartesian cells 1, an
 * octree leaf at level L 8^-L of the box) and u0 = total absorbed / total
 * mass (the temperature of a grain whose emissivity goes as lambda^-beta, in
 * units where heating u0 gives T0).  Cells in natural order (octree: leaf
 * order).  Dust packets start at a uniform point of a cell drawn in proportion to its
 * emission at the packet's wavelength (Philox slot 0 for the cell, 1-3 for
 * the point, 5-6 for the isotropic direction), with L0 = the wavelength's
 * dust luminosity / n_per_lambda, and then follow the stellar packets' life
 * cycle (absorption, forced scattering, peel-offs). */
typedef struct {
    double T0;   /* temperature (K) at the mean heating; default 20 */
    double beta; /* emissivity index, > -4; default 2 */
} mcrt_dust_params;
void mcrt_dust_params_default(mcrt_dust_params *p);
/* Emission of sim's cells from the sum of the absorption tables of
 * absorbed[0 .. n-1] (1 <= n <= 4; results of sim, or of another sim on the
 * same device whose table has the same layout -- grid, wavelengths and
 * storage bricks -- such as an FP64 validation run of the same scene, so that
 * an FP32 sim can emit from a validated absorption; MCRT_EINVAL otherwise;
 * they must not be running).
 * Computed on the device in FP64 (a fixed-order reduction and scan: the same
 * result on every call); needs the medium's wavelengths.  The handle holds
 * n_lambda x n_cells FP64 running sums on the device until destroyed. */
int mcrt_dust_create(mcrt_sim *sim, const mcrt_result *const *absorbed, int32_t n, const mcrt_dust_params *params,
                     mcrt_dust **out);
/* Emitted luminosity per wavelength (count >= n_lambda). */
int mcrt_dust_luminosity(const mcrt_dust *dust, double *L, size_t count);
/* Cell temperatures in natural cell order (0 where nothing is absorbed);
 * count >= n_cells; host or device buffer. */
int mcrt_dust_temperature(const mcrt_dust *dust, double *T, size_t count);
void mcrt_dust_destroy(mcrt_dust *dust);
/* Runs dust packet ids [first_id, first_id + count) of every wavelength into
 * res, as mcrt_run_into (same errors; MCRT_EINVAL with a learned proposal). */
int mcrt_run_dust_into(mcrt_sim *sim, const mcrt_dust *dust, uint64_t n_per_lambda, uint64_t first_id,
                       uint64_t count, uint64_t seed, mcrt_result *res);
/* Self-absorption cycles: cycle k = 1, 2, ... emits from the stellar
 * absorption plus the previous cycle's dust absorption and runs n_per_lambda
 * dust packets per wavelength with seed + k - 1 into a fresh result; stops
 * after max_cycles or when the total dust luminosity changed by at most
 * tol relative to the previous cycle.  Returns the last cycle's emission and
 * result (owned by the caller) and the number of cycles run. */
int mcrt_dust_self_absorption(mcrt_sim *sim, const mcrt_result *stellar, const mcrt_dust_params *params,
                              uint64_t n_per_lambda, uint64_t seed, int32_t max_cycles, double tol,
                              mcrt_dust **dust_out, mcrt_result **result_out, int32_t *cycles_done);

/* ---- Output files (host only: no device is touched) ----
 * A data cube with one wavelength axis and two spatial axes whose wavelength
 * slices may be produced in pieces, as the wavelength-sliced data cube of
 * Section 5.2 (ParallelDatacube class).
 * mcrt_fits_cube_create writes a FITS file: a primary HDU with BITPIX -64 and
 * NAXIS1 = nx (x fastest), NAXIS2 = ny, NAXIS3 = n_lambda, all zero, and an
 * IMAGE extension WAVELENGTHS holding lambda_um[n_lambda] (micron).
 * mcrt_fits_cube_write_slices writes slices [first, first + count) of such a
 * file in place from slices[count][ny][nx] (host FP64, row-major); the file
 * must have been created with the same shape (MCRT_EINVAL otherwise).
 * Different slice ranges may be written by different callers, one at a time
 * per range; the caller keeps ownership of every array. */
int mcrt_fits_cube_create(const char *path, int64_t nx, int64_t ny, int32_t n_lambda, const double *lambda_um);
int mcrt_fits_cube_write_slices(const char *path, int64_t nx, int64_t ny, int32_t n_lambda, int32_t first,
                                int32_t count, const double *slices);
/* Text SED: two comment lines, then one line "lambda_um flux" per wavelength
 * (17 significant digits). */
int mcrt_sed_write_text(const char *path, int32_t n_lambda, const double *lambda_um, const double *sed);

/* Energy sums (FP64) of the packets run into res: emitted (the launch
 * luminosities), absorbed (the sum of the table, Section 3.2), escaped (the
 * transmitted part of every propagation) and truncated (luminosity of
 * packets ended once they kept only a negligible part of their launch
 * luminosity, Section 3.2, or at the event cap); emitted = absorbed +
 * escaped + truncated up to rounding (in expectation with the learned
 * proposal).  Any pointer may be NULL. */
int mcrt_result_energy(const mcrt_result *res, double *emitted, double *absorbed,
                       double *escaped, double *truncated);
/* Counters of the packets run into res (mcrt_stats) and the kernel time of
 * the last launch: the cells and pixels behind the per-packet work of
 * Section 3.2 (propagation, forced interaction, peel-offs). */
int mcrt_result_stats(const mcrt_result *res, mcrt_stats *stats);
void mcrt_result_destroy(mcrt_result *res);

/* Sizes of a simulation, for sizing result buffers. */
int mcrt_sim_info(const mcrt_sim *sim, int64_t *n_cells, int32_t *n_lambda, int32_t *n_ins);

/* Thread-local message describing the last failure of this thread (the
 * boundary reports errors by code and message, never by exception; the
 * client of Section 5.1.1 needs nothing else to use the library). */
const char *mcrt_last_error(void);

/* Memory-system microbenchmarks giving the transport kernel its roofline
 * denominators (random access is what bounds the method: the paper's
 * Section 1 calls Monte Carlo radiative transfer memory-bound with random
 * access patterns).  kind: 0 random 4-byte gathers, 1 random FP64 atomic adds
 * (device scope), 2 random FP64 atomic adds (workgroup scope), 3 random FP32
 * atomic adds, 4 streaming copy, 5 FP64 atomic adds in runs of 4 consecutive
 * elements, 6 FP64 atomic adds by groups of 8 lanes on one 64-byte line, 7 the
 * same by whole waves on 64 consecutive elements.  bytes = working-set size
 * (>= 4096), n_ops = operations.  *rate receives operations/s (bytes/s,
 * read + written, for the copy).  Allocates and frees its own buffers;
 * synchronises the device.  Errors: MCRT_EINVAL,
 * MCRT_ENOMEM, MCRT_EDEVICE (message in mcrt_microbench_error()). */
int mcrt_microbench(int device, int kind, uint64_t bytes, uint64_t n_ops, double *rate);
const char *mcrt_microbench_error(void);

#ifdef __cplusplus
}
#endif

#endif
