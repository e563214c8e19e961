/*
 * arc_oracle.h -- plain FP64 CPU oracle for the adaptive HEALPix ray-tracing
 * radiative-transfer step of Hartley & Ricotti, "ARC: Adaptive Ray-tracing with
 * CUDA" (arXiv:1807.07094).
 *
 * TEST INFRASTRUCTURE ONLY. This code exists to check the GPU library against the
 * paper. Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
 * may load it. It shares no source with the GPU library and includes none of its
 * headers.
 *
 * Conventions
 *   - Grid arrays are [nz][ny][nx], x fastest; cell index c = x + nx*(y + ny*z).
 *   - Positions and path lengths are in cell units; cell_cm converts to cm.
 *   - Species index S: 0 = HI, 1 = HeI, 2 = HeII.
 *   - All arithmetic is IEEE double, single-threaded unless stated.
 */
#ifndef ARC_ORACLE_H
#define ARC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t nx, ny, nz;
    double cell_cm;          /* cell side L [cm] */
    double y_he;             /* n_He / n_H by number; 0 = hydrogen only */
    const float* n_h;        /* [ncell] hydrogen number density [cm^-3] */
    const float* x_hi;       /* [ncell] neutral hydrogen fraction */
    const float* x_hei;      /* [ncell] n_HeI / n_He */
    const float* x_heii;     /* [ncell] n_HeII / n_He */
} orc_grid;

typedef struct {
    int32_t n;
    const double* pos;       /* [n][3] cell units */
    const double* ndot;      /* [n] ionising photons per second */
    const double* r_thin;    /* [n] or NULL: optically thin radius of each source (section 2.6),
                                cells; used rounded to float. NULL = 0 for every source */
    double* r_thin_out;      /* [n] or NULL: out: each source's new R_tau<0.1 from this trace */
} orc_sources;

typedef struct {
    int32_t nbins;
    const double* frac;      /* [nbins] photon fraction of each bin, sums to 1 */
    const double* e_erg;     /* [nbins] photon energy of each bin [erg] */
    const double* sigma;     /* [nbins][3] cross sections HI, HeI, HeII [cm^2] */
    const double* e_thr;     /* [3] ionisation thresholds HI, HeI, HeII [erg] */
} orc_bins;

typedef struct {
    int32_t level0;          /* HEALPix level of the root rays */
    int32_t max_level;       /* <0: smallest level whose split radius exceeds the box diagonal */
    double rays_per_cell;    /* Phi: rays per cell-face area at the split radius */
    double eps_term;         /* terminate when every bin is attenuated below this; 0 = never */
    int32_t correction;      /* geometric correction (section 2.5): 0 none; 1 f_c (eq:correction);
                                2 f_c plus the photon-conserving secondary deposit
                                (eq:correction2); 3 f_c squared. Not with the direct rates. */
} orc_params;

typedef struct {
    double emitted;          /* sum of source rates [photons/s] */
    double absorbed_trace;   /* photons absorbed, summed along the rays [photons/s] */
    double escaped;          /* photons that left the box [photons/s] */
    uint64_t crossings;      /* (ray, cell) segments */
    uint64_t rays;           /* rays traced */
    uint64_t splits;         /* rays that split into four children */
    uint64_t terminated;     /* rays ended by the attenuation criterion */
    uint64_t escaped_rays;   /* rays that left the box */
    int64_t tree_count;      /* rays recorded (may exceed tree_cap) */
    double absorbed_thin;    /* photons absorbed by the optically thin fill, sum J_fill kappa [photons/s] */
} orc_ledger;

/* HEALPix, nested scheme (Gorski et al. 2005, ApJ 622, 759). */
int64_t orc_npix(int32_t level);
void orc_healpix_vec(int32_t level, int64_t pix, double v[3]);

/* Split radius of a level-`level` ray, in cell units, and the automatic top level. */
double orc_t_split(double rays_per_cell, int32_t level);
int32_t orc_auto_max_level(int32_t nx, int32_t ny, int32_t nz, double rays_per_cell);

/* Cell-by-cell walk of one ray x(t) = xs + t*d for t in [t0, t_end) (t_end < 0: no end).
 * Writes up to `cap` (cell index, segment length) pairs; returns the number of segments
 * (which may exceed cap). *how = 0 left the box, 1 reached t_end, 2 started outside. */
int64_t orc_walk(int32_t nx, int32_t ny, int32_t nz, const double xs[3], const double d[3],
                 double t0, double t_end, int64_t* cells, double* ds, int64_t cap, int32_t* how);

/* One ray-tracing pass over all sources (section 2.1 steps iii a-d, section 2.4), with the
 * optically thin approximation of section 2.6 for sources with r_thin > 0: cells whose centre
 * lies within R of the source receive S_b / (4 pi r^2) of field (r the centre's distance in
 * cells, at least 1/2), and the source's rays start at radius R with zero optical depth (a ray
 * whose level's split radius is not beyond R splits at once, without a crossing). With
 * r_thin_out, each source's R_tau<0.1 is measured: the least path length at which a ray's
 * optical depth in the softest bin (lowest energy) reaches 0.1, a path that leaves the box
 * below 0.1 counting with its length at the box face.
 *   J      [nbins][ncell] out: sum over crossings of P_b * ds * g(dtau_b)   [photons/s * cells]
 *   gdir   [3][ncell] out or NULL: photoionisation rate per absorber summed directly in the
 *          form of eq:ion with the in-bin species split (for checking the J route)
 *   tree   [tree_cap] out or NULL: (src << 32) | (level << 28) | pix of every ray traced
 * Returns 0, or -1 on bad arguments / allocation failure. */
int32_t orc_trace(const orc_grid* g, const orc_sources* s, const orc_bins* b, const orc_params* p,
                  double* J, double* gdir, uint64_t* tree, int64_t tree_cap, orc_ledger* led);

/* orc_trace with the sources split over nthreads host threads (source i on thread
 * i mod nthreads), adding into the one field J with atomic compare-and-swap additions:
 * equal to orc_trace up to the order of the floating-point additions. No direct rates or
 * ray tree. For timing the oracle on every core of a host. */
int32_t orc_trace_mt(const orc_grid* g, const orc_sources* s, const orc_bins* b, const orc_params* p, double* J,
                     int32_t nthreads, orc_ledger* led);

/* Rates from J (eq:ion per bin with the species split, section 2.8 heating):
 *   gamma[S][c] = sum_b sigma_{b,S} J_b[c] / L^2                      [1/s]
 *   heat[S][c]  = sum_b sigma_{b,S} (E_b - E_S)^+ J_b[c] / L^2        [erg/s]
 *   *absorbed   = sum_c sum_b J_b[c] * kappa_b[c]                      [photons/s] */
void orc_finalize(const orc_grid* g, const orc_bins* b, const double* J,
                  double* gamma, double* heat, double* absorbed);

typedef struct {
    int32_t isothermal;      /* 1: temperature held fixed */
    int32_t rates;           /* 0: fixed alpha_hii, no helium/collisional terms; 1: Hui & Gnedin 1997 case B */
    int32_t collisional;     /* include collisional ionisation (rates == 1) */
    double alpha_hii;        /* case-B HII recombination coefficient for rates == 0 [cm^3/s] */
    double eps;              /* sub-cycle fractional-change limit */
    int32_t max_sub;         /* sub-cycle cap; then one backward step to the end */
    double t_floor;          /* minimum temperature [K] */
} orc_chem_params;

/* Sub-cycled backward-difference chemistry and energy update (eq:diffeq, eq:anninos,
 * section 2.7 sub-cycle step, section 2.8). Rates are held constant over dt.
 * x_* and temp are read from the float state and written to the double outputs.
 * nsub [ncell] (or NULL) receives the sub-cycle count; flags bit 0 = hit the cap. */
void orc_chem(int64_t ncell, double y_he, const float* n_h,
              const float* x_hi, const float* x_hei, const float* x_heii, const float* temp,
              const double* gamma, const double* heat, double dt, const orc_chem_params* cp,
              double* x_hi_out, double* x_hei_out, double* x_heii_out, double* temp_out,
              int32_t* nsub, int32_t* flags);

/* Adaptive RT time step (section 2.9) from the current state and rates. Per cell,
 * ndot_HI = alpha_HII n_e n_HII - (Gamma_HI + k_HI n_e) n_HI (the chemistry's source term
 * at the start of a step, with the coefficients of cp); then
 *   dt_n = eps n_HI / |ndot_HI| over cells with tau = n_HI sigma0 L > 0.5,
 *   dt_I = eps / (sigma0 L |ndot_HI|) over every cell,
 * sigma0 being the HI cross section of the softest bin. Cells with ndot_HI = 0 impose
 * nothing; a minimum over no cell is +inf. */
void orc_timestep(int64_t ncell, double y_he, double cell_cm, const float* n_h, const float* x_hi,
                  const float* x_hei, const float* x_heii, const float* temp, const double* gamma_hi,
                  const orc_chem_params* cp, double sigma0, double eps, double* dt_n, double* dt_i);

/* Rate coefficients at temperature T (Hui & Gnedin 1997 fits), exposed for pinning.
 * out: [0] alpha_HII [1] alpha_HeII (incl. dielectronic) [2] alpha_HeIII
 *      [3] k_HI [4] k_HeI [5] k_HeII (collisional ionisation)   all cm^3/s */
void orc_rate_coeffs(double T, double out[6]);

/* Cooling coefficients at temperature T [erg cm^3 s^-1], exposed for pinning:
 *   [0] HII [1] HeII [2] HeIII recombination cooling, [3] HeII dielectronic cooling,
 *   [4] HI [5] HeII collisional excitation, [6] bremsstrahlung per Z^2 of the ion. */
void orc_cooling_coeffs(double T, double out[7]);
/* Cooling rate per volume [erg cm^-3 s^-1] of a gas with these number densities. */
double orc_cooling(double T, double ne, double nhi, double nhii, double nhei, double nheii, double nheiii,
                   int collisional);

#ifdef __cplusplus
}
#endif
#endif
