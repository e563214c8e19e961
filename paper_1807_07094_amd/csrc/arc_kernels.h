// arc_kernels.h -- launch wrappers of libarc's kernels (host-callable).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "arc_device.h"

namespace arc {

struct OpacityArgs {
    int nb;
    int nx, ny, nz, nbx8, nby8, nbz8;
    uint32_t ncell;
    double L, y;
    double sigma[kMaxBins][3];
    const float *n_h, *x_hi, *x_hei, *x_heii;
    float* kappa1;
    float4* kappa4;
    unsigned long long* J;
    unsigned long long* M;     // moved-photon field of the conserving correction, or null
    int nbp;
    int* errflag;
};

struct FinalizeArgs {
    int nb, nbp;
    int nx, ny, nz, nbx8, nby8, nbz8;
    uint32_t ncell;
    double gam[kMaxBins][3];   // u_J,b sigma_bS / L^2
    double hea[kMaxBins][3];   // u_J,b sigma_bS (E_b - E_S)^+ / L^2
    double uj[kMaxBins];
    const unsigned long long* J;
    const unsigned long long* M;  // moved-photon field (two limbs per bin), or null
    const float* kappa1;
    const float4* kappa4;
    float *gamma, *heat;       // [3][ncell]
    double* absorbed;          // sum_c sum_b u_J J kappa
};

// Section 2.6 fill of the optically thin spheres.
struct ThinFillArgs {
    int nb, nbp, nsrc, parts;  // parts: blocks per source
    int nx, ny, nz, nbx8, nby8;
    const double *pos, *ndot, *r_thin;
    double coef[kMaxBins];     // frac_b / (4 pi u_J,b)
    double uj[kMaxBins];
    unsigned long long* J;
    const float* kappa1;
    const float4* kappa4;
    double* absorbed_thin;     // sum of the fill's deposits times u_J kappa
};

struct ChemArgs {
    uint32_t ncell;
    double y;
    const float* n_h;
    float *x_hi, *x_hei, *x_heii, *temp;
    const float *gamma, *heat;
    double dt;
    int isothermal, rates, collisional, max_sub;
    double alpha_hii, eps, t_floor;
    unsigned long long* stats;  // [0] sub total, [1] capped, [2] max, [3] cells updated
    uint32_t* chunk_counter;    // zero before the launch
    // optional: update only the cells whose bit is set, bit (c mod 64) of word c / 64
    const unsigned long long* mask;
};

hipError_t launch_zero_u64(unsigned long long* p, size_t n, hipStream_t s);
hipError_t launch_zero_f64(double* p, size_t n, hipStream_t s);
hipError_t launch_set_u32(uint32_t* p, uint32_t v, hipStream_t s);
hipError_t launch_snapshot_counters(unsigned long long* counters, hipStream_t s);
// out[0] = sum J[i], out[1] = sum J[i] (2i + 1), both mod 2^64; out must be zeroed first.
hipError_t launch_field_checksum(const unsigned long long* J, size_t n, unsigned long long* out, hipStream_t s);
hipError_t launch_opacity(const OpacityArgs& a, hipStream_t s);
hipError_t launch_healpix(int level, float4* out, hipStream_t s);
hipError_t launch_sources(int n, const double* pos, const double* ndot, const double* r_thin,
                          const double* frac_over_12uj, int nb, SourceRec* out, hipStream_t s);
hipError_t launch_thin_fill(const ThinFillArgs& a, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t n, uint32_t v, hipStream_t s);
// Root rays of sources first_src .. first_src + nsrc - 1, or of order[0 .. nsrc) if order
// is given (source k's rays are contiguous, in pixel order).
hipError_t launch_seed_roots(uint32_t first_src, uint32_t nsrc, int level0, const uint32_t* order, RayRec* out,
                             hipStream_t s);
// n_in_dev (optional) holds the ray count on the device; n_in bounds it and sizes the grid.
// fam_out: a split ray writes one family record (its own id and depth) instead of its four
// children, for the persistent launch.
hipError_t launch_trace_rays(const TraceArgs& A, int prec, const RayRec* in, const uint32_t* n_in_dev, uint32_t n_in,
                             RayRec* out, uint32_t* n_out, uint32_t out_cap, int fam_out, hipStream_t s);
// fam: the work items are family records (four rays each), else single rays. stack_cap:
// split rays each wave's LDS stack holds (64, 128 or 256).
hipError_t launch_trace_persistent(const TraceArgs& A, int prec, const RayRec* items, const uint32_t* n_items,
                                   uint32_t* head, RayRec* spill, uint32_t spill_cap, int blocks, int waves,
                                   int refill, int fam, int stack_cap, hipStream_t s);
int persistent_max_waves();
hipError_t launch_finalize(const FinalizeArgs& a, hipStream_t s);
hipError_t launch_probe_deposits(unsigned long long* J, int nbp, int nb, uint64_t ncell, uint64_t items,
                                 uint64_t seed, int cus, hipStream_t s);
hipError_t launch_probe_gathers(const float4* kappa, uint64_t ncell, uint64_t items, uint64_t seed, float* sink,
                                int cus, hipStream_t s);
hipError_t launch_get_field(const unsigned long long* J, const unsigned long long* M, int nb, int nbp, int nx, int ny,
                            int nbx8, int nby8, uint32_t ncell, long long* dst, hipStream_t s);
// cus: compute units of the device (the solver launches resident waves only)
hipError_t launch_chem(const ChemArgs& a, int cus, hipStream_t s);

// Section 2.9 time-step limits: out[0] = min dt_n, out[1] = min dt_I as the bit patterns of
// non-negative doubles (+inf when no cell constrains); reset with launch_timestep_reset.
struct TimestepArgs {
    uint32_t ncell;
    double y, cell_cm, sigma0, eps;
    const float *n_h, *x_hi, *x_hei, *x_heii, *temp;
    const float* gamma_hi;
    int rates, collisional;
    double alpha_hii;
    unsigned long long* out;
};
hipError_t launch_timestep_reset(unsigned long long* out, hipStream_t s);
hipError_t launch_timestep(const TimestepArgs& a, int cus, hipStream_t s);
hipError_t launch_timestep_publish(const unsigned long long* bits, double* out, hipStream_t s);

}  // namespace arc
