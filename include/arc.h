/*
 * arc.h -- C ABI of libarc, the gfx950 (MI355X) implementation of the adaptive HEALPix
 * ray-tracing radiative-transfer step of Hartley & Ricotti, "ARC: Adaptive
 * Ray-tracing with CUDA" (arXiv:1807.07094).
 *
 * One call to arc_trace casts rays from every point source through a uniform grid
 * (section 2.1, steps iii a-d; section 2.4), splits each ray into four HEALPix
 * children when its cross-section outgrows the cell, attenuates the photons of every
 * frequency bin by exp(-tau) at each cell crossing and deposits the photons lost in a
 * cell there (eq:ion, photon conserving), and returns per-cell photoionisation and
 * photoheating rates for HI, HeI and HeII (eq:ion with the in-bin species split;
 * section 2.8). arc_chem_step then advances each cell's ionisation state and
 * temperature (eq:diffeq, eq:anninos, section 2.7).
 *
 * Conventions
 *   - Every call returns an arc_status. No exception or abort crosses this ABI.
 *   - Grid arrays are device pointers owned by the caller, FP32, contiguous, laid out
 *     [nz][ny][nx] with x fastest. Positions and lengths are in cell units.
 *   - Source and bin tables are host pointers owned by the caller; they are read
 *     during the call only.
 *   - The context owns every internal buffer (opacity, fixed-point radiation field,
 *     ray queues, direction tables). One context per host thread.
 *   - Calls are blocking: they enqueue on the given stream (NULL = the default stream),
 *     then synchronise it before returning.
 *   - After ARC_E_DEVICE the context must be destroyed. After any other error it stays
 *     usable, and the contents of the outputs are unspecified.
 */
#ifndef ARC_H
#define ARC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t arc_status;
#define ARC_OK 0
#define ARC_E_ARG (-1)         /* null pointer, bad size or bad enum */
#define ARC_E_RANGE (-2)       /* value outside its domain: source off-grid or off the 2^-12
                                  lattice, n_H <= 0, a fraction outside [0,1], non-finite
                                  input, a bin with sigma_HI <= 0 */
#define ARC_E_NOMEM (-3)       /* device allocation failed */
#define ARC_E_DEVICE (-4)      /* HIP runtime error; destroy the context */
#define ARC_E_OVERFLOW (-5)    /* requested fixed-point unit cannot hold the field */
#define ARC_E_QUEUE (-6)       /* ray-queue capacity exceeded */
#define ARC_E_UNSUPPORTED (-7) /* valid but not implemented combination */
#define ARC_E_MISMATCH (-8)    /* autotuner: two launch shapes gave different fields */

typedef struct arc_ctx arc_ctx;

/* Create a context on HIP device `device`. */
arc_status arc_create(int32_t device, arc_ctx** out);
/* Release every buffer the context owns. NULL is ignored. */
void arc_destroy(arc_ctx* ctx);
/* Text of the last error on this context (never NULL; "" after success). */
const char* arc_last_error(const arc_ctx* ctx);

/* Uniform N^3 grid (section 2.3). Device pointers, caller-owned. */
typedef struct {
    int32_t nx, ny, nz;
    double cell_cm;     /* cell side L [cm] */
    double y_he;        /* n_He / n_H by number; 0 = hydrogen only */
    const float* n_h;   /* [ncell] hydrogen number density [cm^-3], > 0 */
    float* x_hi;        /* [ncell] n_HI / n_H in [0,1] */
    float* x_hei;       /* [ncell] n_HeI / n_He in [0,1] */
    float* x_heii;      /* [ncell] n_HeII / n_He in [0,1] */
    float* temp;        /* [ncell] temperature [K] (read and written by arc_chem_step) */
} arc_grid;

/* Point sources (section 2.1: source positions; section 2.4: photon rate per bin).
 * Host pointers. Positions must lie on the 2^-12 cell lattice inside [0, n).
 *
 * Optically thin approximation (section 2.6), optional. r_thin[i] > 0 (used rounded to
 * float, below 2^20 cells) is source i's thin radius R, normally the R_tau<0.1 measured by
 * the previous trace: every cell whose centre lies within R of the source receives the
 * point-source field S_b / (4 pi r^2) (r the centre's distance, at least half a cell), and
 * the source's rays start at radius R with zero optical depth (a ray whose split radius
 * does not lie beyond R splits at once, without a crossing). r_thin_out, if set, receives
 * each source's R_tau<0.1 of this trace: the least path length at which a ray's optical depth
 * in the bin of lowest photon energy reaches 0.1, a ray that leaves the grid (or starts
 * outside it) below 0.1 counting with its length there; +inf when no ray of the source
 * measures one. Either one needs ARC_PREC_FP32_COMP (else ARC_E_UNSUPPORTED); a radius that
 * is negative, not finite or not below 2^20 gives ARC_E_RANGE. */
typedef struct {
    int32_t n;
    const double* pos;  /* [n][3] x, y, z in cell units */
    const double* ndot; /* [n] ionising photons per second, escape fraction applied */
    const double* r_thin; /* [n] thin radius per source [cells], or NULL (no thin sphere) */
    double* r_thin_out; /* [n] out: R_tau<0.1 per source [cells], or NULL (not measured) */
} arc_sources;

/* Frequency bins (section 2.2): one frequency per bin standing for the bin-averaged
 * cross sections. Host pointers. 1 <= nbins <= 4. */
typedef struct {
    int32_t nbins;
    const double* frac;  /* [nbins] fraction of each source's photons in the bin, sum 1 */
    const double* e_erg; /* [nbins] photon energy [erg] */
    const double* sigma; /* [nbins][3] cross sections of HI, HeI, HeII [cm^2]; HI > 0 */
    const double* e_thr; /* [3] ionisation thresholds of HI, HeI, HeII [erg] */
} arc_freq_bins;

/* Arithmetic of the traversal (section 2.4 stepping and attenuation). */
#define ARC_PREC_FP32_COMP 0  /* FP32 with double-float path length and compensated tau */
#define ARC_PREC_FP32_PLAIN 1 /* FP32 with plain path length and tau sums */

/* Work schedule. Both give bitwise-identical fixed-point fields for the same precision. */
#define ARC_SCHED_PLAIN 0     /* per source, per HEALPix level launches (section 2.1 iii) */
#define ARC_SCHED_BATCHED 1   /* every source in one persistent launch with a device queue */
#define ARC_SCHED_BATCHED_TUNED 2 /* batched, with the launch shape the context's autotuner
                                     chose for this grid (tuned on first use, see arc_autotune);
                                     tune_* fields are ignored */

typedef struct {
    int32_t level0;        /* HEALPix level of the root rays (section 2.1: typically 1) */
    int32_t max_level;     /* last level that splits; < 0 = first level whose split radius
                              reaches the box diagonal */
    double rays_per_cell;  /* Phi: rays per cell-face area at the split radius (> 0) */
    double eps_term;       /* a ray ends once every bin is attenuated below eps_term (and
                              its last crossing had dtau >= 0.01 in every bin); the rest of
                              its photons are absorbed in that cell. 0 = never. */
    int32_t precision;     /* ARC_PREC_* */
    int32_t schedule;      /* ARC_SCHED_* */
    void* stream;          /* hipStream_t, NULL = default stream */
    int32_t tune_waves;    /* batched: waves per workgroup (0 = default) */
    int32_t tune_blocks;   /* batched: workgroups in the persistent grid (0 = default) */
    int32_t tune_refill;   /* batched: refill a wave once this many lanes idle (0 = 48) */
    int32_t tune_item_level; /* batched: HEALPix level whose rays become the persistent
                                launch's work items; earlier levels are traced level by
                                level (0 = five levels below the first). Lowered while the
                                rays of that level could exceed a sixth of the device
                                memory (48-byte records). */
    uint64_t* tree_out;    /* optional device array: every ray traced is appended as
                              (src << 32) | (level << 28) | pixel; NULL = off */
    int64_t tree_cap;      /* capacity of tree_out in entries */
    double u_j_override;   /* 0 = automatic fixed-point unit; > 0 forces this unit (tests) */
    int32_t graph;         /* batched schedules: 1 = record the call's launches in HIP graphs
                              once and replay them while every launch argument repeats
                              (same grid, buffers, sources' fixed-point scales, shape);
                              results are identical to 0 */
    int32_t correction;    /* geometric correction (section 2.5), ARC_CORR_*; needs
                              ARC_PREC_FP32_COMP (else ARC_E_UNSUPPORTED) */
    int32_t spill_cap;     /* batched: records of each wave's spill area in device memory, one
                              per split ray waiting with its four children (0 = 4096; < 0 =
                              ARC_E_ARG). Records that do not fit are dropped and the call
                              returns ARC_E_QUEUE. */
    int32_t tune_stack;    /* batched: split rays each wave's LDS stack holds before it spills
                              to memory: 64, 128 or 256 (0 = 64; else ARC_E_ARG) */
} arc_trace_params;

/* Geometric correction (section 2.5). D_edge: distance from a crossing's midpoint to the
 * nearest face of its cell; L_Pix: the ray's pixel width there, r sqrt(4 pi / N_pix). The
 * cell keeps f_c = 1/2 + D_edge / L_Pix of the crossing's photons when D_edge < L_Pix / 2
 * (eq:correction). ARC_CORR_CONSERVING also deposits the rest in the neighbour across that
 * face, at the neighbour's opacity (eq:correction2, the absorber ratio taken per bin as the
 * opacity ratio), so photons are conserved, whatever the ratio; the cell keeps the share
 * when that neighbour is outside the grid or has no absorber of the bin (zero opacity).
 * The moved photons are held in a second fixed-point field of two 64-bit limbs per bin
 * (units 2^20 u_J,b and 2^-12 u_J,b) and divided by the receiving cell's opacity when the
 * rates are formed. Faces within 1e-9 cell of each other count as tied (lower axis, then
 * lower face). The other two modes drop the removed share. */
#define ARC_CORR_NONE 0
#define ARC_CORR_FC 1           /* f_c alone */
#define ARC_CORR_CONSERVING 2   /* f_c plus the secondary deposit: the paper's choice */
#define ARC_CORR_FC_SQUARED 3   /* f_c squared alone */

/* Rates out: device pointers, caller-owned, each [3][ncell] (HI, HeI, HeII). */
typedef struct {
    float* gamma;  /* photoionisation rate per absorber [1/s] */
    float* heat;   /* photoheating rate per absorber [erg/s] */
} arc_rates;

/* Photon ledger of one trace, in photons emitted during dt (rates times dt). */
typedef struct {
    double emitted;        /* sum over sources of ndot * dt */
    double absorbed;       /* sum over cells and bins of deposited-field * opacity * dt */
    double escaped;        /* photons carried out of the grid */
    uint64_t crossings;    /* (ray, cell) segments: the unit of the throughput metric */
    uint64_t rays;         /* rays traced */
    uint64_t splits;       /* rays split into four children */
    uint64_t terminated;   /* rays ended by the attenuation criterion */
    uint64_t escaped_rays; /* rays that left the grid */
    uint64_t spills;       /* batched: records (a split ray's four children each) moved from
                              on-chip stacks to memory */
    int64_t tree_count;    /* rays appended to tree_out (may exceed tree_cap) */
    double u_j[4];         /* fixed-point unit of each bin [photons/s * cell] */
    double ms_trace;       /* device time of the trace kernels [ms] */
    double ms_total;       /* device time of the whole call [ms] */
    double ms_kernel;      /* batched: device time of the persistent trace kernel [ms] */
    double absorbed_thin;  /* part of `absorbed` deposited by the optically thin fill
                              (section 2.6); the rays alone conserve photons:
                              emitted = (absorbed - absorbed_thin) + escaped */
    uint64_t deposits;     /* fixed-point deposits issued as atomics, one per cell and merge
                              window after crossings of the same cell are summed on chip (each
                              covers the cell's bins in one memory request) */
    uint64_t kernel_crossings; /* batched: crossings of the persistent trace kernel alone */
    uint64_t kernel_deposits;  /* batched: deposits of the persistent trace kernel alone */
} arc_ledger;

/* One ray-tracing pass (a whole RT step's radiation field). `out` receives the rates;
 * `ledger` may be NULL. dt > 0 only scales the ledger. */
arc_status arc_trace(arc_ctx* ctx, const arc_grid* grid, const arc_sources* src,
                     const arc_freq_bins* bins, double dt, const arc_trace_params* params,
                     arc_rates* out, arc_ledger* ledger);

/* Launch shape of the batched schedule. */
typedef struct {
    int32_t waves;         /* waves per workgroup of the persistent launch (1, 2, 4, 8) */
    int32_t waves_per_cu;  /* resident waves per compute unit the grid is sized for */
    int32_t refill;        /* refill a wave once this many lanes idle */
    int32_t item_delta;    /* work-item level minus the first level (ARC_SCHED_BATCHED uses 5);
                              a trace lowers it under the memory bound of tune_item_level */
    double ms_best;        /* trace time of the chosen shape [ms] (tuning sources) */
    double ms_default;     /* trace time of the default shape [ms] (tuning sources) */
    int32_t candidates;    /* shapes timed */
    int32_t stack;         /* split rays per wave's LDS stack (64, 128, 256) */
} arc_tune_result;

/* Autotuner of the batched schedule (no paper counterpart: the paper traces one source
 * at a time). Times launch shapes of the batched tracer on the given sources (pass a
 * representative subset: every shape traces them all, twice) by coordinate descent over
 * the work-item level, waves per workgroup and per CU, the refill threshold and the depth
 * of the waves' LDS stacks. Every
 * shape's fixed-point field is checked against the first one's bit for bit (two 64-bit
 * checksums); a difference returns ARC_E_MISMATCH. The best shape is cached in the context
 * for this grid size, bin count, level range and precision, where ARC_SCHED_BATCHED_TUNED
 * finds it. params->schedule and tune_* are ignored. The field and rates afterwards are
 * those of the last shape timed. */
arc_status arc_autotune(arc_ctx* ctx, const arc_grid* grid, const arc_sources* src, const arc_freq_bins* bins,
                        double dt, const arc_trace_params* params, arc_rates* out, arc_tune_result* result);

/* Copy the fixed-point field of the last arc_trace, [nbins][ncell] int64 in units of
 * ledger.u_j[b], into the device array `dst` (caller-owned, nbins * ncell entries). If the
 * last trace used ARC_CORR_CONSERVING, dst must hold 3 * nbins * ncell entries: the field is
 * followed by the moved-photon field's low limb [nbins][ncell] (units 2^-12 u_j[b]) and its
 * high limb [nbins][ncell] (units 2^20 u_j[b]); a cell's rate field is then
 * J + (high 2^20 + low 2^-12) / kappa, kappa its opacity per cell length. */
arc_status arc_get_field(arc_ctx* ctx, int64_t* dst, int64_t count, void* stream);

/* Measurement only (no paper counterpart): the device's rate of the two random memory
 * requests a crossing makes, on the buffers of the last arc_trace (2 to 4 bins, else
 * ARC_E_ARG), for holding the trace kernel against. `items` random cells among the first
 * `cells` of the blocked layout (0 = all of them; a counter-based hash of the index and
 * `seed`) each take (1) one deposit: an int64 atomic add to every bin of the cell, issued by
 * adjacent lanes of one instruction as the tracer issues them, and (2) one 16-byte opacity
 * gather. Best of three timings of each, per second. Overwrites the fixed-point field
 * (arc_get_field then fails until the next trace). Blocks. */
arc_status arc_probe_requests(arc_ctx* ctx, int64_t items, int64_t cells, uint64_t seed, void* stream,
                              double* deposits_per_s, double* gathers_per_s);

/* FP32 HEALPix pixel centres of `level` (nested order) as used by the tracer, written
 * to the device array `dst` of 3 * 12 * 4^level floats (x, y, z per pixel). */
arc_status arc_healpix_dirs(arc_ctx* ctx, int32_t level, float* dst, void* stream);

/* Chemistry (section 2.7 and 2.8). */
#define ARC_CHEM_PLAIN 0      /* sub-cycled backward-difference solver in every cell */
#define ARC_CHEM_MLP_GATED 1  /* learned step where its gate accepts the cell, plain elsewhere */
#define ARC_CHEM_MLP_ONLY 2   /* learned step in every cell (evaluation of the network only) */

/* Learned chemistry: an 8 -> 64 -> 64 -> 2 network (ReLU; BF16 weights and activations, FP32
 * accumulation on the matrix cores) in place of the sub-cycled update of section 2.7. Inputs
 * (n_H, x_HI, T, Gamma_HI, dt, h, x_HeII, x_HeI), with h = H_HI x_HI + y (H_HeI x_HeI + H_HeII
 * x_HeII) the photoheating per hydrogen atom. Outputs: log10(T'/T) and the correction of
 * x_HI' to an exact exponential relaxation of x_HI with the recombination, collisional and
 * photoionisation rates of the start of the step. It does not predict helium; its gate
 * accepts a cell only when (1) the first five inputs fall inside the training range in a 8^5
 * occupancy bin with at least gate_min_count training samples, whose held-out error, taken
 * twice over, is <= gate_tol (the error of a sample is the larger of |x_HI' error| and
 * |T' error| / (10 T')), (2) the output temperature is physical, and (3) helium is close to
 * steady over dt. Other cells run the plain solver. */
typedef struct arc_mlp arc_mlp;

typedef struct {
    int32_t epochs;        /* passes over the training samples */
    int32_t batch;         /* minibatch size (multiple of 64 recommended) */
    double lr;             /* peak Adam learning rate (cosine decay to lr/20 over the run) */
    uint32_t seed;         /* initialisation and shuffling */
    double val_frac;       /* share of the samples held out for the gate (0 < v < 1) */
    void* stream;          /* hipStream_t, NULL = default stream */
    double y_he;           /* n_He / n_H of the samples' gas (for the x_HI baseline) */
    int32_t collisional;   /* the samples' solver included collisional ionisation */
} arc_train_params;

typedef struct {
    double val_rmse_x;     /* held-out RMS error of x_HI' */
    double val_rmse_logt;  /* held-out RMS error of log10 T' */
    double val_max_err;    /* held-out max of the per-sample gate error */
    int64_t n_train, n_val;
    int64_t bins_used;     /* occupancy bins holding training samples */
    double ms;             /* wall time of the training call [ms] */
} arc_train_report;

/* Create an untrained network owned by the caller (release with arc_mlp_destroy). */
arc_status arc_mlp_create(arc_ctx* ctx, arc_mlp** out);
void arc_mlp_destroy(arc_mlp* mlp);
/* Train on m device samples: X [m][8] = (n_H [cm^-3], x_HI, T [K], Gamma_HI [1/s], dt [s],
 * h [erg/s], x_HeII, x_HeI), Y [m][2] = (x_HI', T' [K]) from the plain solver. All inputs must be
 * finite with n_H, T, dt > 0. Fits the standardisation, trains, then calibrates the gate on
 * the held-out samples. */
arc_status arc_mlp_train(arc_ctx* ctx, arc_mlp* mlp, const float* X, const float* Y, int64_t m,
                         const arc_train_params* params, arc_train_report* report);
/* Network (weights, standardisation, gate) as a byte blob: with buf == NULL, *size
 * receives the size; otherwise buf must hold *size bytes. */
arc_status arc_mlp_save(const arc_mlp* mlp, void* buf, size_t* size);
arc_status arc_mlp_load(arc_mlp* mlp, const void* buf, size_t size);
/* Predictions for device samples X [m][8] (same units as training) into device P [m][2]
 * = (x_HI', T' [K]), without the gate. */
arc_status arc_mlp_predict(arc_ctx* ctx, const arc_mlp* mlp, const float* X, int64_t m, float* P, void* stream);

typedef struct {
    int32_t isothermal;    /* 1: temperature fixed */
    int32_t rates;         /* 0: fixed alpha_hii, no helium recombination or collisional
                              terms; 1: Hui & Gnedin (1997) case-B coefficients and cooling */
    int32_t collisional;   /* include collisional ionisation (rates == 1) */
    double alpha_hii;      /* [cm^3/s] for rates == 0 */
    double eps;            /* sub-cycle limit on fractional changes (paper: 0.1) */
    int32_t max_sub;       /* sub-cycle cap, then one backward step to the end */
    double t_floor;        /* minimum temperature [K] */
    int32_t mode;          /* ARC_CHEM_* */
    void* stream;          /* hipStream_t, NULL = default stream */
    const arc_mlp* mlp;    /* trained network for the MLP modes */
    double gate_tol;       /* MLP_GATED: largest accepted held-out bin error */
    int32_t gate_min_count; /* MLP_GATED: smallest accepted training count per bin */
    int32_t graph;         /* 1 = record the step's launches in HIP graphs once and replay them
                              while every launch argument repeats; results are identical to 0 */
} arc_chem_params;

typedef struct {
    int64_t cells;         /* cells updated */
    int64_t sub_total;     /* sub-cycles summed over cells */
    int32_t sub_max;       /* largest sub-cycle count of a cell */
    int64_t capped;        /* cells that reached max_sub */
    double ms;             /* device time [ms] */
    int64_t fallback;      /* MLP_GATED: cells handed to the plain solver */
    double ms_mlp;         /* MLP modes: device time of the network and gate [ms] */
} arc_chem_stats;

/* Advance x_hi, x_hei, x_heii and temp of `grid` in place over dt [s] with the rates
 * held constant. `stats` may be NULL. */
arc_status arc_chem_step(arc_ctx* ctx, const arc_grid* grid, const arc_rates* rates, double dt,
                         const arc_chem_params* params, arc_chem_stats* stats);

/* Adaptive RT time step (section 2.9) from the grid's current state and the rates of the
 * last trace. Per cell, ndot_HI = alpha_HII n_e n_HII - (Gamma_HI + k_HI n_e) n_HI, with the
 * coefficients `params` selects (rates, collisional, alpha_hii; the rest is ignored):
 *   *dt_n: min of eps n_HI / |ndot_HI| over cells with tau = n_HI sigma0 L > 0.5 (the
 *          neutral-fraction limit),
 *   *dt_i: min of eps / (sigma0 L |ndot_HI|) over all cells (the intensity limit),
 * with sigma0 = bins->sigma[0] (HI cross section of the softest bin) and L = cell_cm.
 * Cells with ndot_HI = 0 impose nothing; a minimum over no cell is +inf. eps > 0. Blocks
 * until both values are on the host (host pointers). */
arc_status arc_rt_timestep(arc_ctx* ctx, const arc_grid* grid, const arc_rates* rates,
                           const arc_freq_bins* bins, const arc_chem_params* params, double eps,
                           double* dt_n, double* dt_i);

/* arc_rt_timestep for callers that cannot allocate device memory or synchronise (code under
 * HIP graph capture, tight serving loops): the same minima, computed by the same kernels,
 * but held in a small static device array of the library (256 bytes per GPU, kept until
 * the process ends) instead of the context's memory, and written as doubles to the caller's
 * device array dt_out[2] = (dt_n, dt_i) in seconds, stream-ordered on params->stream; the
 * call neither allocates nor blocks. The array's size does not depend on the grid (two
 * words are used; grids are bounded as for every call, below 2^31 cells). All calls on one
 * GPU share its array: calls that overlap on one GPU (different streams without ordering)
 * race and must not be made. */
arc_status arc_rt_timestep_noalloc(arc_ctx* ctx, const arc_grid* grid, const arc_rates* rates,
                                   const arc_freq_bins* bins, const arc_chem_params* params, double eps,
                                   double* dt_out);

#ifdef __cplusplus
}
#endif
#endif
