// arc_api.hip -- host side of libarc: the C ABI of include/arc.h.
//
// Validation, fixed-point unit selection, buffer ownership and the two tracing
// schedules. Every per-cell and per-ray step runs in the kernels of arc_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "arc.h"
#include "arc_kernels.h"
#include "arc_mlp_host.h"

using namespace arc;

struct arc_ctx {
    int device = 0;
    int cus = 0;
    std::string err;
    // grid-sized buffers
    size_t ncell_cap = 0;
    int nbp_cap = 0;
    void* kappa = nullptr;             // float or float4 per cell
    size_t kappa_bytes = 0;
    unsigned long long* J = nullptr;   // [cell][nbp]
    size_t J_bytes = 0;
    unsigned long long* M = nullptr;   // conserving correction: moved photons, [cell][2][nbp]
    size_t M_bytes = 0;
    // source table
    SourceRec* src = nullptr;
    double* src_pos = nullptr;
    double* src_ndot = nullptr;
    uint32_t* src_order = nullptr;
    double* src_rthin = nullptr;       // optically thin radius per source (section 2.6)
    uint32_t* r_out = nullptr;         // measured R_tau<0.1 per source (FP32 bits)
    int src_cap = 0;
    // HEALPix centres, levels 0..dirs_levels-1
    float4* dirs = nullptr;
    int dirs_levels = 0;
    long long dir_off[kMaxLevels] = {0};
    // ray arrays (per-level schedule) and work queue (batched)
    RayRec* rays[2] = {nullptr, nullptr};
    size_t rcap[2] = {0, 0};   // records each ray buffer holds
    size_t item_bytes = 0;     // bound on the larger ray buffer of the batched schedule [bytes]
    RayRec* spill = nullptr;
    size_t spill_entries = 0;
    // small device scalars
    unsigned long long* counters = nullptr;  // kNumCounters
    double* acc = nullptr;                    // [0..3] escaped per bin, [4] absorbed
    uint32_t* u32 = nullptr;                  // [0] n_out, [1] queue head
    int* errflag = nullptr;
    unsigned long long* chem_stats = nullptr;  // [0..3] chemistry statistics, [4] work counter
    unsigned long long* reject = nullptr;     // learned step: cells for the plain solver, a bit each
    size_t reject_cap = 0;                    // words
    hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    bool timed_kernel = false;  // ev[4], ev[5] bracket the dominant trace kernel
    // last trace
    int last_nb = 0, last_nbp = 0, last_nx = 0, last_ny = 0, last_nbx8 = 0, last_nby8 = 0;
    size_t last_ncell = 0;
    bool last_moved = false;  // the last trace filled M
    bool have_field = false;
    // replayed launches of the batched schedule: [0] set-up, [1] the first levels, [2] the
    // persistent trace, [3] the rates; valid while the launch arguments equal graph_key
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t gexec[4] = {nullptr, nullptr, nullptr, nullptr};
    std::vector<unsigned char> graph_key;
    // the chemistry step's stages (statistics, network, solver), same scheme
    hipGraphExec_t cexec[3] = {nullptr, nullptr, nullptr};
    std::vector<unsigned char> chem_key;
    unsigned long long* sums = nullptr;  // field checksums of the autotuner
    unsigned long long* static_scratch = nullptr;  // this device's copy of `scratch`
    struct Tuned {
        int nx, ny, nz, nb, level0, lmax, precision;
        arc_tune_result shape;
    };
    std::vector<Tuned> tuned;
};

// Scratch of the allocation-free entry point (arc_rt_timestep_noalloc): a file-scope device
// array, one copy per GPU, held until the process ends. Host code never passes its name to
// a kernel (on the host the name is a stand-in, not a device address): each context
// resolves the device's copy once, at creation, with hipGetSymbolAddress, and uses that.
constexpr int kStaticScratchWords = 32;  // 256 bytes
constexpr int kTimestepScratchWords = 2; // the two grid minima of section 2.9
static __device__ __align__(256) unsigned long long scratch[kStaticScratchWords];

namespace {

arc_status fail(arc_ctx* c, arc_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return s;
}

#define HIP_TRY(ctx, expr)                                                                        \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return fail(ctx, e_ == hipErrorOutOfMemory ? ARC_E_NOMEM : ARC_E_DEVICE, "%s: %s (%s:%d)", \
                        #expr, hipGetErrorString(e_), __FILE__, __LINE__);                        \
    } while (0)

template <typename T>
hipError_t grow(T** p, size_t* cap_bytes, size_t need_bytes)
{
    if (*p && *cap_bytes >= need_bytes) return hipSuccess;
    if (*p) {
        hipError_t e = hipFree(*p);
        if (e != hipSuccess) return e;
        *p = nullptr;
        *cap_bytes = 0;
    }
    hipError_t e = hipMalloc((void**)p, need_bytes);
    if (e == hipSuccess) *cap_bytes = need_bytes;
    return e;
}

bool on_lattice(double v) { return std::isfinite(v) && std::floor(v * 4096.0) == v * 4096.0; }

// Split radius of each level, rounded once to float (pi r^2 / (3 4^l) = 1 / Phi).
float split_base(double phi) { return (float)std::sqrt(3.0 / (M_PI * phi)); }

int auto_max_level(int nx, int ny, int nz, double phi)
{
    const double diag = std::sqrt((double)nx * nx + (double)ny * ny + (double)nz * nz);
    const float base = split_base(phi);
    int l = 0;
    while ((double)std::ldexp(base, l) < diag && l < 40) ++l;
    return l;
}

arc_status check_grid(arc_ctx* c, const arc_grid* g)
{
    if (!g || !g->n_h || !g->x_hi || !g->x_hei || !g->x_heii) return fail(c, ARC_E_ARG, "null grid pointer");
    if (g->nx <= 0 || g->ny <= 0 || g->nz <= 0) return fail(c, ARC_E_ARG, "grid dimensions must be positive");
    if (g->nx > 2048 || g->ny > 2048 || g->nz > 2048)
        return fail(c, ARC_E_UNSUPPORTED, "grid dimensions above 2048 are not supported");
    const double ncell = (double)g->nx * g->ny * g->nz;
    if (ncell > 2147483647.0) return fail(c, ARC_E_UNSUPPORTED, "more than 2^31-1 cells");
    if (!(g->cell_cm > 0) || !std::isfinite(g->cell_cm)) return fail(c, ARC_E_RANGE, "cell_cm must be finite and > 0");
    if (!(g->y_he >= 0) || !std::isfinite(g->y_he)) return fail(c, ARC_E_RANGE, "y_he must be finite and >= 0");
    return ARC_OK;
}

arc_status check_bins(arc_ctx* c, const arc_freq_bins* b)
{
    if (!b || !b->frac || !b->e_erg || !b->sigma || !b->e_thr) return fail(c, ARC_E_ARG, "null bin pointer");
    if (b->nbins < 1 || b->nbins > kMaxBins) return fail(c, ARC_E_ARG, "nbins must be 1..4");
    double sum = 0;
    for (int k = 0; k < b->nbins; ++k) {
        if (!(b->frac[k] >= 0) || !std::isfinite(b->frac[k])) return fail(c, ARC_E_RANGE, "frac[%d] invalid", k);
        if (!(b->e_erg[k] > 0) || !std::isfinite(b->e_erg[k])) return fail(c, ARC_E_RANGE, "e_erg[%d] invalid", k);
        if (!(b->sigma[3 * k] > 0) || !std::isfinite(b->sigma[3 * k]))
            return fail(c, ARC_E_RANGE, "sigma_HI of bin %d must be > 0", k);
        for (int s = 1; s < 3; ++s)
            if (!(b->sigma[3 * k + s] >= 0) || !std::isfinite(b->sigma[3 * k + s]))
                return fail(c, ARC_E_RANGE, "sigma[%d][%d] invalid", k, s);
        sum += b->frac[k];
    }
    if (std::fabs(sum - 1.0) > 1e-6) return fail(c, ARC_E_RANGE, "bin fractions sum to %.9g, not 1", sum);
    for (int s = 0; s < 3; ++s)
        if (!(b->e_thr[s] > 0) || !std::isfinite(b->e_thr[s])) return fail(c, ARC_E_RANGE, "e_thr[%d] invalid", s);
    return ARC_OK;
}

arc_status check_sources(arc_ctx* c, const arc_sources* s, const arc_grid* g)
{
    if (!s) return fail(c, ARC_E_ARG, "null sources");
    if (s->n < 0) return fail(c, ARC_E_ARG, "negative source count");
    if (s->n > 0 && (!s->pos || !s->ndot)) return fail(c, ARC_E_ARG, "null source arrays");
    const int dims[3] = {g->nx, g->ny, g->nz};
    for (int i = 0; i < s->n; ++i) {
        for (int a = 0; a < 3; ++a) {
            const double v = s->pos[3 * i + a];
            if (!on_lattice(v)) return fail(c, ARC_E_RANGE, "source %d coordinate %d is not on the 2^-12 lattice", i, a);
            if (!(v >= 0.0 && v < (double)dims[a])) return fail(c, ARC_E_RANGE, "source %d lies outside the grid", i);
        }
        if (!(s->ndot[i] > 0) || !std::isfinite(s->ndot[i])) return fail(c, ARC_E_RANGE, "source %d ndot invalid", i);
    }
    return ARC_OK;
}

arc_status ensure_dirs(arc_ctx* c, int levels, hipStream_t st)
{
    if (levels <= c->dirs_levels) return ARC_OK;
    long long off[kMaxLevels];
    long long total = 0;
    for (int l = 0; l < levels; ++l) {
        off[l] = total;
        total += 12ll << (2 * l);
    }
    float4* nd = nullptr;
    HIP_TRY(c, hipMalloc((void**)&nd, (size_t)total * sizeof(float4)));
    for (int l = 0; l < levels; ++l) {
        hipError_t e = launch_healpix(l, nd + off[l], st);
        if (e != hipSuccess) {
            (void)hipFree(nd);
            return fail(c, ARC_E_DEVICE, "healpix launch: %s", hipGetErrorString(e));
        }
    }
    HIP_TRY(c, hipStreamSynchronize(st));
    if (c->dirs) HIP_TRY(c, hipFree(c->dirs));
    c->dirs = nd;
    c->dirs_levels = levels;
    for (int l = 0; l < levels; ++l) c->dir_off[l] = off[l];
    return ARC_OK;
}

}  // namespace

namespace arc {
int ctx_device(const arc_ctx* c) { return c->device; }
arc_status ctx_fail(arc_ctx* c, arc_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return s;
}
}  // namespace arc

extern "C" {

arc_status arc_create(int32_t device, arc_ctx** out)
{
    if (!out) return ARC_E_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return ARC_E_DEVICE;
    if (hipSetDevice(device) != hipSuccess) return ARC_E_DEVICE;
    arc_ctx* c = new (std::nothrow) arc_ctx();
    if (!c) return ARC_E_NOMEM;
    c->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        delete c;
        return ARC_E_DEVICE;
    }
    c->cus = prop.multiProcessorCount;
    c->item_bytes = prop.totalGlobalMem / 6;
    // this device's copy of the static scratch (the device is current)
    if (hipGetSymbolAddress((void**)&c->static_scratch, HIP_SYMBOL(scratch)) != hipSuccess || !c->static_scratch) {
        delete c;
        return ARC_E_DEVICE;
    }
    bool ok = hipMalloc((void**)&c->counters, kNumCounters * sizeof(unsigned long long)) == hipSuccess &&
              hipMalloc((void**)&c->acc, 8 * sizeof(double)) == hipSuccess &&
              hipMalloc((void**)&c->u32, 4 * sizeof(uint32_t)) == hipSuccess &&
              hipMalloc((void**)&c->errflag, sizeof(int)) == hipSuccess &&
              hipMalloc((void**)&c->chem_stats, 5 * sizeof(unsigned long long)) == hipSuccess &&
              hipMalloc((void**)&c->sums, 2 * sizeof(unsigned long long)) == hipSuccess;
    for (int i = 0; i < 6 && ok; ++i) ok = hipEventCreate(&c->ev[i]) == hipSuccess;
    if (!ok) {
        arc_destroy(c);
        return ARC_E_NOMEM;
    }
    *out = c;
    return ARC_OK;
}

void arc_destroy(arc_ctx* c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    void* bufs[] = {c->kappa, c->J, c->M, c->src, c->src_pos, c->src_ndot, c->src_order, c->src_rthin, c->r_out,
                    c->dirs, c->rays[0], c->rays[1], c->spill, c->counters, c->acc, c->u32, c->errflag,
                    c->chem_stats, c->reject};
    for (void* p : bufs)
        if (p) (void)hipFree(p);
    for (int i = 0; i < 6; ++i)
        if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
    for (int i = 0; i < 4; ++i)
        if (c->gexec[i]) (void)hipGraphExecDestroy(c->gexec[i]);
    for (int i = 0; i < 3; ++i)
        if (c->cexec[i]) (void)hipGraphExecDestroy(c->cexec[i]);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->sums) (void)hipFree(c->sums);
    delete c;
}

const char* arc_last_error(const arc_ctx* c) { return c ? c->err.c_str() : "null context"; }

}  // extern "C"

namespace {

// Everything one trace launches with. Zero-filled before use so that its bytes (padding
// included) can serve as the key of the recorded graphs.
struct TracePlan {
    int nb, nbp, lmax;
    size_t ncell;
    int nbx8, nby8, nbz8;
    double uj[kMaxBins];
    double sum_ndot;
    int nsrc;
    double src_scale[kMaxBins];  // frac_b / (12 u_J,b)
    OpacityArgs oa;
    TraceArgs A;
    FinalizeArgs fa;
    ThinFillArgs tf;
    int thin;        // optically thin approximation in use (section 2.6)
    int precision;
    // batched schedule
    int waves, blocks, refill, litem;
    int stack;          // split rays per wave's LDS stack
    int spill_cap_req;  // records of each wave's spill area (0: 4096)
    double n_roots;
    size_t cap[2];  // records of rays0 / rays1
    uint32_t spill_cap;
    RayRec* rays0;
    RayRec* rays1;
    RayRec* spill;
    uint32_t* u32;
    const uint32_t* order;  // sources by decreasing photon rate (work-queue order)
};

// Validation, fixed-point units, buffers and launch arguments shared by both schedules.
arc_status plan_trace(arc_ctx* c, const arc_grid* g, const arc_sources* s, const arc_freq_bins* b, double dt,
                      const arc_trace_params* p, const arc_rates* out, TracePlan& P)
{
    std::memset(&P, 0, sizeof P);
    arc_status rc;
    if ((rc = check_grid(c, g)) != ARC_OK) return rc;
    if ((rc = check_bins(c, b)) != ARC_OK) return rc;
    if ((rc = check_sources(c, s, g)) != ARC_OK) return rc;
    if (!p) return fail(c, ARC_E_ARG, "null params");
    if (!out || !out->gamma || !out->heat) return fail(c, ARC_E_ARG, "null rate outputs");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(c, ARC_E_RANGE, "dt must be finite and > 0");
    if (!(p->rays_per_cell > 0) || !std::isfinite(p->rays_per_cell)) return fail(c, ARC_E_RANGE, "rays_per_cell must be > 0");
    if (!(p->eps_term >= 0 && p->eps_term < 1)) return fail(c, ARC_E_RANGE, "eps_term must be in [0,1)");
    if (p->precision != ARC_PREC_FP32_COMP && p->precision != ARC_PREC_FP32_PLAIN) return fail(c, ARC_E_ARG, "bad precision");
    if (p->schedule != ARC_SCHED_PLAIN && p->schedule != ARC_SCHED_BATCHED && p->schedule != ARC_SCHED_BATCHED_TUNED)
        return fail(c, ARC_E_ARG, "bad schedule");
    const int lmax = p->max_level < 0 ? auto_max_level(g->nx, g->ny, g->nz, p->rays_per_cell) : p->max_level;
    if (p->level0 < 0 || p->level0 > lmax) return fail(c, ARC_E_ARG, "level0 must be in [0, max_level]");
    if (lmax > 12) return fail(c, ARC_E_UNSUPPORTED, "max_level %d > 12 (pixel ids are 28-bit)", lmax);
    if (!(p->u_j_override >= 0)) return fail(c, ARC_E_ARG, "u_j_override must be >= 0");
    if (p->tree_out && p->tree_cap < 0) return fail(c, ARC_E_ARG, "tree_cap < 0");
    if (p->correction < ARC_CORR_NONE || p->correction > ARC_CORR_FC_SQUARED)
        return fail(c, ARC_E_ARG, "bad correction mode %d", p->correction);
    if (p->correction != ARC_CORR_NONE && p->precision != ARC_PREC_FP32_COMP)
        return fail(c, ARC_E_UNSUPPORTED, "the geometric correction needs ARC_PREC_FP32_COMP");
    if (p->spill_cap < 0) return fail(c, ARC_E_ARG, "spill_cap must be >= 0");
    if (p->tune_stack != 0 && p->tune_stack != 64 && p->tune_stack != 128 && p->tune_stack != 256)
        return fail(c, ARC_E_ARG, "tune_stack must be 0, 64, 128 or 256");
    // optically thin approximation (section 2.6): per-source start radii and/or the measured
    // R_tau<0.1
    bool thin = s->r_thin_out != nullptr;
    double max_r = 0.0;
    if (s->r_thin)
        for (int i = 0; i < s->n; ++i) {
            const double r = s->r_thin[i];
            if (!(r >= 0.0) || !(r < 1048576.0))
                return fail(c, ARC_E_RANGE, "r_thin[%d] must be finite, >= 0 and below 2^20 cells", i);
            thin = thin || r > 0.0;
            max_r = std::max(max_r, (double)(float)r);
        }
    if (thin && p->precision != ARC_PREC_FP32_COMP)
        return fail(c, ARC_E_UNSUPPORTED, "the optically thin approximation needs ARC_PREC_FP32_COMP");

    hipStream_t st = (hipStream_t)p->stream;
    HIP_TRY(c, hipSetDevice(c->device));
    const int nb = b->nbins;
    const int nbp = nb == 1 ? 1 : (nb == 2 ? 2 : 4);
    const size_t ncell = (size_t)g->nx * g->ny * g->nz;
    const int nbx8 = (g->nx + 7) / 8, nby8 = (g->ny + 7) / 8, nbz8 = (g->nz + 7) / 8;
    const size_t nblocked = (size_t)nbx8 * nby8 * nbz8 * 512;  // cells of the blocked layout
    if (nblocked > 2147483648ull) return fail(c, ARC_E_UNSUPPORTED, "blocked grid exceeds 2^31 cells");
    P.nb = nb;
    P.nbp = nbp;
    P.lmax = lmax;
    P.ncell = ncell;
    P.nbx8 = nbx8;
    P.nby8 = nby8;
    P.nbz8 = nbz8;
    P.nsrc = s->n;
    P.precision = p->precision;
    P.thin = thin ? 1 : 0;
    P.spill_cap_req = p->spill_cap;

    // Fixed-point unit per bin. One source deposits at most sqrt(3) S_b into a cell
    // (the photon rate through any sphere is at most S_b and a cell is at most sqrt(3)
    // long), plus a remainder below eps_term S_b sqrt(3) / 0.01 on termination, plus with
    // the optically thin fill at most S_b / pi (r >= 1/2). The sum over sources therefore
    // stays below 2^62 units. With the conserving correction a cell also receives into its
    // field at most half of each of its six neighbours' deposits times the opacity ratio
    // kMovedRatioJ: 1 + 6 * 16 / 2 = 49 times the bound (larger ratios move photons into the
    // moved-photon field, counted in the same unit: all of them together are at most the
    // photons emitted).
    for (int k = 0; k < kMaxBins; ++k) P.uj[k] = 1.0;
    for (int i = 0; i < s->n; ++i) P.sum_ndot += s->ndot[i];
    const double corr_factor = p->correction == ARC_CORR_CONSERVING ? 1.0 + 6.0 * (double)kMovedRatioJ / 2.0 : 1.0;
    for (int k = 0; k < nb; ++k) {
        const double bound = (std::sqrt(3.0) + p->eps_term * std::sqrt(3.0) / (double)kDtauTermMin +
                              (thin ? 1.0 / M_PI : 0.0)) *
                             P.sum_ndot * b->frac[k] * (1.0 + 1e-6) * corr_factor;
        const double need = bound / 4611686018427387904.0;  // 2^62
        if (p->u_j_override > 0) {
            if (p->u_j_override < need)
                return fail(c, ARC_E_OVERFLOW, "fixed-point unit %.6g too small for bin %d (needs >= %.6g)",
                            p->u_j_override, k, need);
            P.uj[k] = p->u_j_override;
        } else {
            P.uj[k] = need > 0 ? need : 1.0;
        }
        P.src_scale[k] = b->frac[k] / (12.0 * P.uj[k]);
    }

    // Buffers.
    {
        const size_t kb = nblocked * (nb == 1 ? sizeof(float) : sizeof(float4));
        HIP_TRY(c, grow(&c->kappa, &c->kappa_bytes, kb));
        HIP_TRY(c, grow(&c->J, &c->J_bytes, nblocked * nbp * sizeof(unsigned long long)));
        if (p->correction == ARC_CORR_CONSERVING)
            HIP_TRY(c, grow(&c->M, &c->M_bytes, nblocked * 2 * nbp * sizeof(unsigned long long)));
        if (s->n > c->src_cap) {
            void* old[] = {c->src, c->src_pos, c->src_ndot, c->src_order, c->src_rthin, c->r_out};
            for (void* q : old)
                if (q) HIP_TRY(c, hipFree(q));
            c->src = nullptr;
            c->src_pos = c->src_ndot = c->src_rthin = nullptr;
            c->src_order = c->r_out = nullptr;
            c->src_cap = 0;
            HIP_TRY(c, hipMalloc((void**)&c->src, s->n * sizeof(SourceRec)));
            HIP_TRY(c, hipMalloc((void**)&c->src_pos, s->n * 3 * sizeof(double)));
            HIP_TRY(c, hipMalloc((void**)&c->src_ndot, s->n * sizeof(double)));
            HIP_TRY(c, hipMalloc((void**)&c->src_order, s->n * sizeof(uint32_t)));
            HIP_TRY(c, hipMalloc((void**)&c->src_rthin, s->n * sizeof(double)));
            HIP_TRY(c, hipMalloc((void**)&c->r_out, s->n * sizeof(uint32_t)));
            c->src_cap = s->n;
        }
    }
    if ((rc = ensure_dirs(c, lmax + 1, st)) != ARC_OK) return rc;

    OpacityArgs& oa = P.oa;
    oa.nb = nb;
    oa.nx = g->nx;
    oa.ny = g->ny;
    oa.nz = g->nz;
    oa.nbx8 = nbx8;
    oa.nby8 = nby8;
    oa.nbz8 = nbz8;
    oa.ncell = (uint32_t)ncell;
    oa.L = g->cell_cm;
    oa.y = g->y_he;
    for (int k = 0; k < nb; ++k)
        for (int sp = 0; sp < 3; ++sp) oa.sigma[k][sp] = b->sigma[3 * k + sp];
    oa.n_h = g->n_h;
    oa.x_hi = g->x_hi;
    oa.x_hei = g->x_hei;
    oa.x_heii = g->x_heii;
    oa.kappa1 = nb == 1 ? (float*)c->kappa : nullptr;
    oa.kappa4 = nb == 1 ? nullptr : (float4*)c->kappa;
    oa.J = c->J;
    oa.M = p->correction == ARC_CORR_CONSERVING ? c->M : nullptr;
    oa.nbp = nbp;
    oa.errflag = c->errflag;

    TraceArgs& A = P.A;
    A.nx = g->nx;
    A.ny = g->ny;
    A.nz = g->nz;
    A.nb = nb;
    A.nbx8 = nbx8;
    A.nby8 = nby8;
    A.level0 = p->level0;
    A.lmax = lmax;
    const float base = split_base(p->rays_per_cell);
    for (int l = 0; l < kMaxLevels; ++l) A.tsplit[l] = l < lmax ? std::ldexp(base, l) : INFINITY;
    A.tau_term = p->eps_term > 0 ? (float)(-std::log(p->eps_term)) : INFINITY;
    A.kappa1 = oa.kappa1;
    A.kappa4 = oa.kappa4;
    A.J = c->J;
    A.nbp = nbp;
    A.src = c->src;
    A.dirs = c->dirs;
    for (int l = 0; l < kMaxLevels; ++l) A.dir_off[l] = l < c->dirs_levels ? c->dir_off[l] : 0;
    A.esc = c->acc;
    A.counters = c->counters;
    A.tree = (unsigned long long*)p->tree_out;
    A.tree_cap = p->tree_out ? p->tree_cap : 0;
    A.corr = p->correction;
    A.M = oa.M;
    // softest bin: the lowest photon energy (the first of equal ones)
    A.ksoft = 0;
    for (int k = 1; k < nb; ++k)
        if (b->e_erg[k] < b->e_erg[A.ksoft]) A.ksoft = k;
    A.r_out = thin ? c->r_out : nullptr;

    FinalizeArgs& fa = P.fa;
    fa.nb = nb;
    fa.nbp = nbp;
    fa.nx = g->nx;
    fa.ny = g->ny;
    fa.nz = g->nz;
    fa.nbx8 = nbx8;
    fa.nby8 = nby8;
    fa.nbz8 = nbz8;
    fa.ncell = (uint32_t)ncell;
    const double L2 = g->cell_cm * g->cell_cm;
    for (int k = 0; k < nb; ++k) {
        fa.uj[k] = P.uj[k];
        for (int sp = 0; sp < 3; ++sp) {
            fa.gam[k][sp] = P.uj[k] * b->sigma[3 * k + sp] / L2;
            const double excess = b->e_erg[k] - b->e_thr[sp];
            fa.hea[k][sp] = excess > 0 ? P.uj[k] * b->sigma[3 * k + sp] * excess / L2 : 0.0;
        }
    }
    fa.J = c->J;
    fa.M = oa.M;
    fa.kappa1 = oa.kappa1;
    fa.kappa4 = oa.kappa4;
    fa.gamma = out->gamma;
    fa.heat = out->heat;
    fa.absorbed = c->acc + 4;

    if (thin) {
        ThinFillArgs& tf = P.tf;
        tf.nb = nb;
        tf.nbp = nbp;
        tf.nsrc = s->r_thin && max_r > 0.0 ? s->n : 0;
        // blocks per source: about 8192 cells of the largest bounding box each, a power of two
        const double box = std::pow(2.0 * max_r + 2.0, 3.0);
        int parts = 1;
        while (parts < 1024 && (double)parts * 8192.0 < box) parts *= 2;
        tf.parts = parts;
        tf.nx = g->nx;
        tf.ny = g->ny;
        tf.nz = g->nz;
        tf.nbx8 = nbx8;
        tf.nby8 = nby8;
        tf.pos = c->src_pos;
        tf.ndot = c->src_ndot;
        tf.r_thin = c->src_rthin;
        for (int k = 0; k < nb; ++k) {
            tf.coef[k] = b->frac[k] / (4.0 * M_PI * P.uj[k]);
            tf.uj[k] = P.uj[k];
        }
        tf.J = c->J;
        tf.kappa1 = oa.kappa1;
        tf.kappa4 = oa.kappa4;
        tf.absorbed_thin = c->acc + 5;
    }
    return ARC_OK;
}

// Default work-item level: five levels below the first. The levels above it are traced
// level by level (all rays of a level in one launch, no stacks); below it a subtree is
// small enough for its wave's LDS stack, so rays seldom spill to memory (1024^3 x 16384
// sources: item level 4 -> 6 took the persistent launch from 1440 to 990 ms and the spills
// from 1.4e8 to 4e5). Lowered while the larger ray buffer would exceed item_bytes.
constexpr int kDefaultItemDepth = 5;

// Default refill threshold of the persistent launch: a wave refills once 48 of its lanes are
// idle, so that many rays, mostly children of the same splits, start together and their merged
// deposits make fewer atomics (1024^3 x 16384 sources from the generated state, merge windows
// of two segments: refill at 32, 48 and 64 idle lanes, 0.283, 0.273 and 0.261 deposit items per
// crossing, 744, 718 and 712 ms; windows of four: 48 and 64, 686 and 696 ms, the wider merge
// costing more issue per crossing than the last atomics it saves).
constexpr int kDefaultRefill = 48;

// Default depth of each wave's LDS stack: 64 split rays (2 KB), a full split round of the
// wave; deeper stacks spill less but hold fewer waves per compute unit.
constexpr int kDefaultStack = 64;

// Records of a ray buffer, without keeping its contents.
hipError_t grow_rays(arc_ctx* c, int i, size_t n)
{
    size_t bytes = c->rcap[i] * sizeof(RayRec);
    const hipError_t e = grow(&c->rays[i], &bytes, n * sizeof(RayRec));
    c->rcap[i] = bytes / sizeof(RayRec);
    return e;
}

// Launch shape of the batched schedule and the buffers it needs. item_level: the HEALPix
// level whose rays are the persistent launch's work items (0: the default depth); it is
// clamped to [level0, lmax] and to the memory bound.
arc_status shape_batched(arc_ctx* c, TracePlan& P, int waves, int blocks, int refill, int item_level, int stack)
{
    if (stack != 64 && stack != 128 && stack != 256) return fail(c, ARC_E_ARG, "LDS stack depth must be 64, 128 or 256");
    if (waves != 1 && waves != 2 && waves != 4 && waves != 8) return fail(c, ARC_E_ARG, "tune_waves must be 1, 2, 4 or 8");
    if (blocks < 1) return fail(c, ARC_E_ARG, "tune_blocks must be >= 1");
    const int level0 = P.A.level0, lmax = P.lmax;
    const uint32_t npix0 = 12u << (2 * level0);
    const double n_roots = (double)P.nsrc * npix0;
    // rays of level l at most (every ray reaches it)
    auto rays_at = [&](int l) { return n_roots * std::ldexp(1.0, 2 * (l - level0)); };
    int litem = item_level > 0 ? item_level : level0 + kDefaultItemDepth;
    litem = std::max(level0, std::min(lmax, litem));
    while (litem > level0 &&
           (rays_at(litem) > (double)0xFFFFFFF0u || rays_at(litem) * sizeof(RayRec) > (double)c->item_bytes))
        --litem;
    if (rays_at(litem) > (double)0xFFFFFFF0u) return fail(c, ARC_E_UNSUPPORTED, "too many work items");
    // buffer b holds the levels l with (l - level0) % 2 == b: the count of its deepest one
    size_t need[2] = {1, 1};
    for (int l = level0; l <= litem; ++l)
        need[(l - level0) & 1] = std::max(need[(l - level0) & 1], (size_t)rays_at(l));
    for (int i = 0; i < 2; ++i)
        if (need[i] > c->rcap[i]) HIP_TRY(c, grow_rays(c, i, need[i]));
    const uint32_t spill_cap = P.spill_cap_req > 0 ? (uint32_t)P.spill_cap_req : 4096u;
    const size_t spill_need = (size_t)blocks * waves * spill_cap;
    if (spill_need > c->spill_entries) {
        size_t cap_bytes = c->spill_entries * sizeof(RayRec);
        HIP_TRY(c, grow(&c->spill, &cap_bytes, spill_need * sizeof(RayRec)));
        c->spill_entries = spill_need;
    }
    P.waves = waves;
    P.blocks = blocks;
    P.refill = std::max(1, std::min(64, refill));
    P.stack = stack;
    P.litem = litem;
    P.n_roots = n_roots;
    P.cap[0] = c->rcap[0];
    P.cap[1] = c->rcap[1];
    P.spill_cap = spill_cap;
    P.rays0 = c->rays[0];
    P.rays1 = c->rays[1];
    P.spill = c->spill;
    P.u32 = c->u32;
    P.order = c->src_order;
    return ARC_OK;
}

// Stage 0: counters, opacity (section 2.2 cross sections times densities) and the
// source table.
hipError_t enqueue_common(arc_ctx* c, const TracePlan& P, hipStream_t st)
{
    hipError_t e;
    if ((e = launch_zero_u64(c->counters, kNumCounters, st)) != hipSuccess) return e;
    if ((e = launch_zero_f64(c->acc, 8, st)) != hipSuccess) return e;
    if ((e = launch_set_u32((uint32_t*)c->errflag, 0u, st)) != hipSuccess) return e;
    if ((e = launch_opacity(P.oa, st)) != hipSuccess) return e;
    if (P.nsrc > 0 && (e = launch_sources(P.nsrc, c->src_pos, c->src_ndot, P.thin ? c->src_rthin : nullptr,
                                          P.src_scale, P.nb, c->src, st)) != hipSuccess)
        return e;
    if (P.thin) {
        // no ray measured yet: R_tau<0.1 = +inf
        if ((e = launch_fill_u32(c->r_out, (uint32_t)P.nsrc, 0x7F800000u, st)) != hipSuccess) return e;
        if ((e = launch_thin_fill(P.tf, st)) != hipSuccess) return e;
    }
    return hipSuccess;
}

// Stage 1 (batched): the root rays of every source and the levels traced level by level
// before the persistent launch.
hipError_t enqueue_levels(const TracePlan& P, hipStream_t st)
{
    hipError_t e;
    if (P.nsrc == 0) return hipSuccess;
    if ((e = launch_seed_roots(0, (uint32_t)P.nsrc, P.A.level0, P.order, P.rays0, st)) != hipSuccess) return e;
    uint32_t* cnt = P.u32 + 2;  // [2], [3]: ray counts of consecutive levels
    if ((e = launch_set_u32(cnt, (uint32_t)P.n_roots, st)) != hipSuccess) return e;
    size_t bound = (size_t)P.n_roots;
    int cur = 0;
    RayRec* r[2] = {P.rays0, P.rays1};
    for (int l = P.A.level0; l < P.litem; ++l) {
        uint32_t* cin = cnt + ((l - P.A.level0) & 1);
        uint32_t* cout = cnt + ((l - P.A.level0 + 1) & 1);
        if ((e = launch_set_u32(cout, 0u, st)) != hipSuccess) return e;
        const uint32_t out_cap = (uint32_t)std::min<size_t>(P.cap[1 - cur], 0xFFFFFFF0u);
        // the last level leaves family records: the work items of the persistent launch
        const int fam_out = l + 1 == P.litem ? 1 : 0;
        if ((e = launch_trace_rays(P.A, P.precision, r[cur], cin, (uint32_t)bound, r[1 - cur], cout, out_cap, fam_out,
                                   st)) != hipSuccess)
            return e;
        bound *= 4;
        cur = 1 - cur;
    }
    if ((e = launch_snapshot_counters(P.A.counters, st)) != hipSuccess) return e;
    return launch_set_u32(P.u32 + 1, 0u, st);
}

// Stage 2: the persistent launch over the work items of level litem.
hipError_t enqueue_persistent(const TracePlan& P, hipStream_t st)
{
    if (P.nsrc == 0) return hipSuccess;
    const int cur = (P.litem - P.A.level0) & 1;
    // above the first level the work items are the family records of the level before
    const int fam = P.litem > P.A.level0 ? 1 : 0;
    return launch_trace_persistent(P.A, P.precision, cur ? P.rays1 : P.rays0, P.u32 + 2 + cur, P.u32 + 1, P.spill,
                                   P.spill_cap, P.blocks, P.waves, P.refill, fam, P.stack, st);
}

// Stage 3: rates (eq:ion per absorber, section 2.8 heating) and the absorbed ledger.
hipError_t enqueue_rates(const TracePlan& P, hipStream_t st) { return launch_finalize(P.fa, st); }

// Section 2.1 iii: one source at a time, one HEALPix level per launch; the host reads
// back the number of children before launching the next level.
arc_status run_plain(arc_ctx* c, const TracePlan& P, hipStream_t st)
{
    const uint32_t npix0 = 12u << (2 * P.A.level0);
    for (int si = 0; si < P.nsrc; ++si) {
        size_t n = npix0;
        for (int i = 0; i < 2; ++i)
            if (4 * n > c->rcap[i]) HIP_TRY(c, grow_rays(c, i, 4 * n));
        HIP_TRY(c, launch_seed_roots((uint32_t)si, 1, P.A.level0, nullptr, c->rays[0], st));
        int cur = 0;
        while (n > 0) {
            const size_t need = 4 * n;
            if (need > std::min(c->rcap[0], c->rcap[1])) {
                // grow both arrays, keeping the current level's rays
                RayRec* a = nullptr;
                RayRec* bb = nullptr;
                HIP_TRY(c, hipStreamSynchronize(st));
                HIP_TRY(c, hipMalloc((void**)&a, need * sizeof(RayRec)));
                HIP_TRY(c, hipMalloc((void**)&bb, need * sizeof(RayRec)));
                HIP_TRY(c, hipMemcpyAsync(a, c->rays[cur], n * sizeof(RayRec), hipMemcpyDeviceToDevice, st));
                HIP_TRY(c, hipStreamSynchronize(st));
                HIP_TRY(c, hipFree(c->rays[0]));
                HIP_TRY(c, hipFree(c->rays[1]));
                c->rays[0] = a;
                c->rays[1] = bb;
                cur = 0;
                c->rcap[0] = c->rcap[1] = need;
            }
            HIP_TRY(c, launch_set_u32(c->u32, 0u, st));
            HIP_TRY(c, launch_trace_rays(P.A, P.precision, c->rays[cur], nullptr, (uint32_t)n, c->rays[1 - cur], c->u32,
                                         (uint32_t)std::min<size_t>(c->rcap[1 - cur], 0xFFFFFFF0u), 0, st));
            uint32_t nn = 0;
            HIP_TRY(c, hipMemcpyAsync(&nn, c->u32, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
            HIP_TRY(c, hipStreamSynchronize(st));
            n = nn;
            cur = 1 - cur;
        }
    }
    return ARC_OK;
}

// Records the four stages of the batched schedule as graphs (on the context's own
// capture stream) unless the recorded ones were made with the same arguments.
arc_status ensure_graphs(arc_ctx* c, const TracePlan& P)
{
    const unsigned char* key = reinterpret_cast<const unsigned char*>(&P);
    if (c->gexec[0] && c->graph_key.size() == sizeof P && std::memcmp(c->graph_key.data(), key, sizeof P) == 0)
        return ARC_OK;
    for (int i = 0; i < 4; ++i)
        if (c->gexec[i]) {
            HIP_TRY(c, hipGraphExecDestroy(c->gexec[i]));
            c->gexec[i] = nullptr;
        }
    c->graph_key.clear();
    if (!c->cap_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    for (int i = 0; i < 4; ++i) {
        HIP_TRY(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
        hipStream_t cs = c->cap_stream;
        const hipError_t e = i == 0   ? enqueue_common(c, P, cs)
                             : i == 1 ? enqueue_levels(P, cs)
                             : i == 2 ? enqueue_persistent(P, cs)
                                      : enqueue_rates(P, cs);
        hipGraph_t graph = nullptr;
        const hipError_t e2 = hipStreamEndCapture(c->cap_stream, &graph);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return fail(c, ARC_E_DEVICE, "graph capture of stage %d: %s", i,
                        hipGetErrorString(e != hipSuccess ? e : e2));
        }
        const hipError_t e3 = hipGraphInstantiate(&c->gexec[i], graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e3 != hipSuccess) {
            c->gexec[i] = nullptr;
            return fail(c, ARC_E_DEVICE, "graph instantiation of stage %d: %s", i, hipGetErrorString(e3));
        }
    }
    c->graph_key.assign(key, key + sizeof P);
    return ARC_OK;
}

// One whole trace with a planned shape: uploads, the stages (eagerly or as graphs),
// event timing, and the read-back of counters, ledger and error flags.
arc_status run_trace(arc_ctx* c, const TracePlan& P, const arc_sources* s, double dt, int schedule, bool graph,
                     hipStream_t st, arc_ledger* ledger)
{
    const bool batched = schedule != ARC_SCHED_PLAIN;
    std::vector<uint32_t> order;
    if (s->n > 0) {
        HIP_TRY(c, hipMemcpyAsync(c->src_pos, s->pos, s->n * 3 * sizeof(double), hipMemcpyHostToDevice, st));
        HIP_TRY(c, hipMemcpyAsync(c->src_ndot, s->ndot, s->n * sizeof(double), hipMemcpyHostToDevice, st));
        if (P.thin) {
            if (s->r_thin)
                HIP_TRY(c, hipMemcpyAsync(c->src_rthin, s->r_thin, s->n * sizeof(double), hipMemcpyHostToDevice, st));
            else
                HIP_TRY(c, launch_zero_f64(c->src_rthin, (size_t)s->n, st));
        }
        if (batched) {
            // the work queue starts with the brightest sources, whose rays travel furthest, so
            // that the longest subtrees are not the last ones taken (the field does not depend
            // on the order: integer sums)
            order.resize(s->n);
            for (int i = 0; i < s->n; ++i) order[i] = (uint32_t)i;
            std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b2) { return s->ndot[a] > s->ndot[b2]; });
            HIP_TRY(c, hipMemcpyAsync(c->src_order, order.data(), s->n * sizeof(uint32_t), hipMemcpyHostToDevice, st));
        }
    }
    c->timed_kernel = false;
    if (batched && graph) {
        arc_status rc = ensure_graphs(c, P);
        if (rc != ARC_OK) return rc;
        HIP_TRY(c, hipEventRecord(c->ev[0], st));
        HIP_TRY(c, hipGraphLaunch(c->gexec[0], st));
        HIP_TRY(c, hipEventRecord(c->ev[1], st));
        HIP_TRY(c, hipGraphLaunch(c->gexec[1], st));
        HIP_TRY(c, hipEventRecord(c->ev[4], st));
        HIP_TRY(c, hipGraphLaunch(c->gexec[2], st));
        HIP_TRY(c, hipEventRecord(c->ev[5], st));
        HIP_TRY(c, hipEventRecord(c->ev[2], st));
        HIP_TRY(c, hipGraphLaunch(c->gexec[3], st));
        HIP_TRY(c, hipEventRecord(c->ev[3], st));
        c->timed_kernel = P.nsrc > 0;
    } else {
        HIP_TRY(c, hipEventRecord(c->ev[0], st));
        HIP_TRY(c, enqueue_common(c, P, st));
        // the first levels of the batched schedule belong to the trace time
        HIP_TRY(c, hipEventRecord(c->ev[1], st));
        if (batched) {
            HIP_TRY(c, enqueue_levels(P, st));
            HIP_TRY(c, hipEventRecord(c->ev[4], st));
            HIP_TRY(c, enqueue_persistent(P, st));
            HIP_TRY(c, hipEventRecord(c->ev[5], st));
            c->timed_kernel = P.nsrc > 0;
        } else {
            arc_status rc = run_plain(c, P, st);
            if (rc != ARC_OK) return rc;
        }
        HIP_TRY(c, hipEventRecord(c->ev[2], st));
        HIP_TRY(c, enqueue_rates(P, st));
        HIP_TRY(c, hipEventRecord(c->ev[3], st));
    }

    unsigned long long cnt[kNumCounters];
    double acc[8];
    int errflag = 0;
    std::vector<uint32_t> rbits(P.thin && s->r_thin_out ? (size_t)s->n : 0);
    HIP_TRY(c, hipMemcpyAsync(cnt, c->counters, sizeof cnt, hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipMemcpyAsync(acc, c->acc, sizeof acc, hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipMemcpyAsync(&errflag, c->errflag, sizeof errflag, hipMemcpyDeviceToHost, st));
    if (!rbits.empty())
        HIP_TRY(c, hipMemcpyAsync(rbits.data(), c->r_out, rbits.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    for (size_t i = 0; i < rbits.size(); ++i) {
        float r;
        std::memcpy(&r, &rbits[i], sizeof r);
        s->r_thin_out[i] = (double)r;
    }

    c->last_nb = P.nb;
    c->last_nbp = P.nbp;
    c->last_ncell = P.ncell;
    c->last_nx = P.A.nx;
    c->last_ny = P.A.ny;
    c->last_nbx8 = P.nbx8;
    c->last_nby8 = P.nby8;
    c->last_moved = P.A.M != nullptr;
    c->have_field = true;
    if (errflag) return fail(c, ARC_E_RANGE, "grid values out of range (n_h <= 0, fraction outside [0,1] or non-finite)");
    if (cnt[kQueueOverflow]) return fail(c, ARC_E_QUEUE, "ray queue capacity exceeded (%llu rays dropped)", cnt[kQueueOverflow]);
    if (ledger) {
        std::memset(ledger, 0, sizeof *ledger);
        ledger->emitted = P.sum_ndot * dt;
        double esc = 0;
        for (int k = 0; k < P.nb; ++k) esc += acc[k] * P.uj[k];
        ledger->escaped = esc * dt;
        ledger->absorbed = acc[4] * dt;
        ledger->absorbed_thin = acc[5] * dt;
        ledger->crossings = cnt[kCrossings];
        ledger->rays = cnt[kRays];
        ledger->splits = cnt[kSplits];
        ledger->terminated = cnt[kTerminated];
        ledger->escaped_rays = cnt[kEscapedRays];
        ledger->spills = cnt[kSpills];
        ledger->deposits = cnt[kDeposits];
        if (c->timed_kernel) {
            ledger->kernel_crossings = cnt[kCrossings] - cnt[kCrossingsPre];
            ledger->kernel_deposits = cnt[kDeposits] - cnt[kDepositsPre];
        }
        ledger->tree_count = (int64_t)cnt[kTreeCount];
        for (int k = 0; k < kMaxBins; ++k) ledger->u_j[k] = k < P.nb ? P.uj[k] : 0.0;
        float ms = 0;
        HIP_TRY(c, hipEventElapsedTime(&ms, c->ev[1], c->ev[2]));
        ledger->ms_trace = ms;
        HIP_TRY(c, hipEventElapsedTime(&ms, c->ev[0], c->ev[3]));
        ledger->ms_total = ms;
        ledger->ms_kernel = 0;
        if (c->timed_kernel) {
            HIP_TRY(c, hipEventElapsedTime(&ms, c->ev[4], c->ev[5]));
            ledger->ms_kernel = ms;
        }
    }
    return ARC_OK;
}

const arc_tune_result* find_tuned(const arc_ctx* c, const arc_grid* g, const TracePlan& P)
{
    for (const auto& t : c->tuned)
        if (t.nx == g->nx && t.ny == g->ny && t.nz == g->nz && t.nb == P.nb && t.level0 == P.A.level0 &&
            t.lmax == P.lmax && t.precision == P.precision)
            return &t.shape;
    return nullptr;
}

arc_status autotune_impl(arc_ctx* c, const arc_grid* g, const arc_sources* s, const arc_freq_bins* b, double dt,
                         const arc_trace_params* p, const arc_rates* out, arc_tune_result* res);

}  // namespace

extern "C" {

arc_status arc_trace(arc_ctx* c, const arc_grid* g, const arc_sources* s, const arc_freq_bins* b, double dt,
                     const arc_trace_params* p, arc_rates* out, arc_ledger* ledger)
{
    if (!c) return ARC_E_ARG;
    c->err.clear();
    TracePlan P;
    arc_status rc = plan_trace(c, g, s, b, dt, p, out, P);
    if (rc != ARC_OK) return rc;
    hipStream_t st = (hipStream_t)p->stream;
    if (p->schedule == ARC_SCHED_BATCHED) {
        const int waves = p->tune_waves > 0 ? p->tune_waves : 4;
        const int blocks = p->tune_blocks > 0 ? p->tune_blocks : std::max(1, c->cus * (16 / std::max(1, waves)));
        const int refill = p->tune_refill > 0 ? p->tune_refill : kDefaultRefill;
        const int stack = p->tune_stack > 0 ? p->tune_stack : kDefaultStack;
        if ((rc = shape_batched(c, P, waves, blocks, refill, p->tune_item_level, stack)) != ARC_OK)
            return rc;
    } else if (p->schedule == ARC_SCHED_BATCHED_TUNED) {
        const arc_tune_result* t = find_tuned(c, g, P);
        arc_tune_result fresh;
        if (!t) {
            // tune on an evenly spaced subset of at most 256 sources
            const int step = std::max(1, (s->n + 255) / 256);
            std::vector<double> pos, nd, rt;
            for (int i = 0; i < s->n; i += step) {
                pos.insert(pos.end(), s->pos + 3 * i, s->pos + 3 * i + 3);
                nd.push_back(s->ndot[i]);
                if (s->r_thin) rt.push_back(s->r_thin[i]);
            }
            const arc_sources sub{(int32_t)nd.size(), pos.data(), nd.data(), s->r_thin ? rt.data() : nullptr,
                                  nullptr};
            if ((rc = autotune_impl(c, g, &sub, b, dt, p, out, &fresh)) != ARC_OK) return rc;
            t = &fresh;
            // the tuning runs changed the plan's buffers: plan again for all sources
            if ((rc = plan_trace(c, g, s, b, dt, p, out, P)) != ARC_OK) return rc;
        }
        const int blocks = std::max(1, c->cus * t->waves_per_cu / t->waves);
        if ((rc = shape_batched(c, P, t->waves, blocks, t->refill, P.A.level0 + t->item_delta, t->stack)) != ARC_OK)
            return rc;
    }
    return run_trace(c, P, s, dt, p->schedule, p->graph != 0, st, ledger);
}

arc_status arc_autotune(arc_ctx* c, const arc_grid* g, const arc_sources* s, const arc_freq_bins* b, double dt,
                        const arc_trace_params* p, arc_rates* out, arc_tune_result* res)
{
    if (!c) return ARC_E_ARG;
    c->err.clear();
    arc_tune_result r;
    arc_status rc = autotune_impl(c, g, s, b, dt, p, out, &r);
    if (rc == ARC_OK && res) *res = r;
    return rc;
}

}  // extern "C"

namespace {

arc_status autotune_impl(arc_ctx* c, const arc_grid* g, const arc_sources* s, const arc_freq_bins* b, double dt,
                         const arc_trace_params* p, const arc_rates* out, arc_tune_result* res)
{
    if (!p) return fail(c, ARC_E_ARG, "null params");
    arc_trace_params q = *p;
    q.schedule = ARC_SCHED_BATCHED;
    q.tree_out = nullptr;
    q.tree_cap = 0;
    TracePlan P;
    arc_status rc = plan_trace(c, g, s, b, dt, &q, out, P);
    if (rc != ARC_OK) return rc;
    if (s->n == 0) return fail(c, ARC_E_ARG, "autotuning needs at least one source");
    hipStream_t st = (hipStream_t)q.stream;
    unsigned long long ref[2] = {0, 0};
    bool have_ref = false;
    int ncand = 0;
    // time one shape twice; check its field against the first shape's
    auto time_shape = [&](const arc_tune_result& t, double* ms_out) -> arc_status {
        const int blocks = std::max(1, c->cus * t.waves_per_cu / t.waves);
        arc_status r2 = shape_batched(c, P, t.waves, blocks, t.refill, P.A.level0 + t.item_delta, t.stack);
        if (r2 != ARC_OK) return r2;
        double best = INFINITY;
        for (int rep = 0; rep < 2; ++rep) {
            arc_ledger led;
            if ((r2 = run_trace(c, P, s, dt, ARC_SCHED_BATCHED, false, st, &led)) != ARC_OK) return r2;
            best = std::min(best, led.ms_trace);
        }
        HIP_TRY(c, launch_zero_u64(c->sums, 2, st));
        const size_t words = (size_t)P.nbx8 * P.nby8 * P.nbz8 * 512 * P.nbp;
        HIP_TRY(c, launch_field_checksum(c->J, words, c->sums, st));
        if (P.A.M) HIP_TRY(c, launch_field_checksum(P.A.M, 2 * words, c->sums, st));
        unsigned long long h[2];
        HIP_TRY(c, hipMemcpyAsync(h, c->sums, sizeof h, hipMemcpyDeviceToHost, st));
        HIP_TRY(c, hipStreamSynchronize(st));
        if (!have_ref) {
            ref[0] = h[0];
            ref[1] = h[1];
            have_ref = true;
        } else if (h[0] != ref[0] || h[1] != ref[1]) {
            return fail(c, ARC_E_MISMATCH,
                        "launch shape (waves %d, waves/CU %d, refill %d, item delta %d, stack %d) changed the field",
                        t.waves, t.waves_per_cu, t.refill, t.item_delta, t.stack);
        }
        ++ncand;
        *ms_out = best;
        return ARC_OK;
    };
    arc_tune_result best{};
    best.waves = 4;
    best.waves_per_cu = 16;
    best.refill = kDefaultRefill;
    best.stack = kDefaultStack;
    best.item_delta = kDefaultItemDepth;
    double ms_best;
    if ((rc = time_shape(best, &ms_best)) != ARC_OK) return rc;
    const double ms_default = ms_best;
    auto consider = [&](arc_tune_result t) -> arc_status {
        double ms;
        arc_status r2 = time_shape(t, &ms);
        if (r2 != ARC_OK) return r2;
        if (ms < ms_best) {
            ms_best = ms;
            best = t;
        }
        return ARC_OK;
    };
    // (1) work-item level (levels below the first; the run clamps it to the memory bound). Only
    // levels at or below the default: higher ones win on a source sample, whose subtrees are few,
    // but on the full run their subtrees outgrow the LDS stacks (1024^3 x 16384 sources, four
    // levels below the first: 3.8e8 rays spilled and 760 ms against 712 ms at five).
    const arc_tune_result base1 = best;
    for (int d : {kDefaultItemDepth + 1, kDefaultItemDepth + 2}) {
        arc_tune_result t = base1;
        t.item_delta = d;
        if ((rc = consider(t)) != ARC_OK) return rc;
    }
    // (2) waves per workgroup and resident waves per CU
    const arc_tune_result base2 = best;
    for (int wv : {2, 4, 8})
        for (int wpc : {8, 12, 16}) {
            if (wv == base2.waves && wpc == base2.waves_per_cu) continue;
            arc_tune_result t = base2;
            t.waves = wv;
            t.waves_per_cu = wpc;
            if ((rc = consider(t)) != ARC_OK) return rc;
        }
    // (3) refill threshold
    const arc_tune_result base3 = best;
    for (int rf : {16, 32, 56, 64}) {
        if (rf == base3.refill) continue;
        arc_tune_result t = base3;
        t.refill = rf;
        if ((rc = consider(t)) != ARC_OK) return rc;
    }
    // (4) depth of the waves' LDS stacks
    const arc_tune_result base4 = best;
    for (int sd : {128, 256}) {
        arc_tune_result t = base4;
        t.stack = sd;
        if ((rc = consider(t)) != ARC_OK) return rc;
    }
    best.ms_best = ms_best;
    best.ms_default = ms_default;
    best.candidates = ncand;
    bool stored = false;
    for (auto& t : c->tuned)
        if (t.nx == g->nx && t.ny == g->ny && t.nz == g->nz && t.nb == P.nb && t.level0 == P.A.level0 &&
            t.lmax == P.lmax && t.precision == P.precision) {
            t.shape = best;
            stored = true;
        }
    if (!stored) c->tuned.push_back({g->nx, g->ny, g->nz, P.nb, P.A.level0, P.lmax, P.precision, best});
    *res = best;
    return ARC_OK;
}

}  // namespace

extern "C" {

arc_status arc_get_field(arc_ctx* c, int64_t* dst, int64_t count, void* stream)
{
    if (!c || !dst) return ARC_E_ARG;
    if (!c->have_field) return fail(c, ARC_E_ARG, "no field: call arc_trace first");
    const int64_t parts = c->last_moved ? 3 : 1;
    if (count < parts * (int64_t)(c->last_ncell * c->last_nb))
        return fail(c, ARC_E_ARG, "dst too small (needs %lld entries)", (long long)(parts * c->last_ncell * c->last_nb));
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, launch_get_field(c->J, c->last_moved ? c->M : nullptr, c->last_nb, c->last_nbp, c->last_nx,
                                c->last_ny, c->last_nbx8, c->last_nby8, (uint32_t)c->last_ncell, (long long*)dst, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    return ARC_OK;
}

arc_status arc_probe_requests(arc_ctx* c, int64_t items, int64_t cells, uint64_t seed, void* stream,
                              double* deposits_per_s, double* gathers_per_s)
{
    if (!c || !deposits_per_s || !gathers_per_s) return ARC_E_ARG;
    if (items <= 0) return fail(c, ARC_E_ARG, "items must be > 0");
    if (c->last_nb < 2 || !c->J || !c->kappa) return fail(c, ARC_E_ARG, "probe needs a previous trace with 2 to 4 bins");
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(c, hipSetDevice(c->device));
    const uint64_t nblocked = (uint64_t)c->last_nbx8 * (uint64_t)c->last_nby8 * 512ull *
                              (uint64_t)((c->last_ncell / ((size_t)c->last_nx * c->last_ny) + 7) / 8);
    if (cells < 0) return fail(c, ARC_E_ARG, "cells must be >= 0");
    const uint64_t ncell = cells > 0 ? std::min<uint64_t>((uint64_t)cells, nblocked) : nblocked;
    float ms = 0.0f;
    double best_d = 0.0, best_g = 0.0;
    for (int rep = 0; rep < 3; ++rep) {
        HIP_TRY(c, hipEventRecord(c->ev[0], st));
        HIP_TRY(c, launch_probe_deposits(c->J, c->last_nbp, c->last_nb, ncell, (uint64_t)items, seed + rep, c->cus, st));
        HIP_TRY(c, hipEventRecord(c->ev[1], st));
        HIP_TRY(c, launch_probe_gathers((const float4*)c->kappa, ncell, (uint64_t)items, seed + rep, (float*)c->acc,
                                        c->cus, st));
        HIP_TRY(c, hipEventRecord(c->ev[2], st));
        HIP_TRY(c, hipEventSynchronize(c->ev[2]));
        HIP_TRY(c, hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
        best_d = std::max(best_d, (double)items / (ms * 1e-3));
        HIP_TRY(c, hipEventElapsedTime(&ms, c->ev[1], c->ev[2]));
        best_g = std::max(best_g, (double)items / (ms * 1e-3));
    }
    c->have_field = false;  // the field now holds the probe's counts
    *deposits_per_s = best_d;
    *gathers_per_s = best_g;
    return ARC_OK;
}

arc_status arc_healpix_dirs(arc_ctx* c, int32_t level, float* dst, void* stream)
{
    if (!c || !dst) return ARC_E_ARG;
    if (level < 0 || level > 12) return fail(c, ARC_E_ARG, "level must be 0..12");
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(c, hipSetDevice(c->device));
    arc_status rc = ensure_dirs(c, level + 1, st);
    if (rc != ARC_OK) return rc;
    const size_t npix = (size_t)12 << (2 * level);
    // float4 table -> x, y, z triples
    std::vector<float4> h(npix);
    HIP_TRY(c, hipMemcpyAsync(h.data(), c->dirs + c->dir_off[level], npix * sizeof(float4), hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    std::vector<float> f(3 * npix);
    for (size_t i = 0; i < npix; ++i) {
        f[3 * i] = h[i].x;
        f[3 * i + 1] = h[i].y;
        f[3 * i + 2] = h[i].z;
    }
    HIP_TRY(c, hipMemcpyAsync(dst, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    return ARC_OK;
}

}  // extern "C"

namespace {

// Everything the chemistry step launches with, zero-filled (its bytes key the graphs).
struct ChemPlan {
    ChemArgs a;
    mlp::InferArgs ia;
    int mode;
    int cus;
};

// Stage 0: statistics and the work counter; stage 1 (learned modes): network and gate;
// stage 2 (plain and gated modes): the sub-cycled solver.
hipError_t chem_stage(arc_ctx* c, const ChemPlan& P, int stage, hipStream_t st)
{
    if (stage == 0) return launch_zero_u64(c->chem_stats, 5, st);
    if (stage == 1) return P.mode != ARC_CHEM_PLAIN ? mlp::launch_infer(P.ia, st) : hipSuccess;
    return P.mode != ARC_CHEM_MLP_ONLY ? launch_chem(P.a, P.cus, st) : hipSuccess;
}

arc_status ensure_chem_graphs(arc_ctx* c, const ChemPlan& P)
{
    const unsigned char* key = reinterpret_cast<const unsigned char*>(&P);
    if (c->cexec[0] && c->chem_key.size() == sizeof P && std::memcmp(c->chem_key.data(), key, sizeof P) == 0)
        return ARC_OK;
    for (int i = 0; i < 3; ++i)
        if (c->cexec[i]) {
            HIP_TRY(c, hipGraphExecDestroy(c->cexec[i]));
            c->cexec[i] = nullptr;
        }
    c->chem_key.clear();
    if (!c->cap_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    for (int i = 0; i < 3; ++i) {
        HIP_TRY(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
        const hipError_t e = chem_stage(c, P, i, c->cap_stream);
        hipGraph_t graph = nullptr;
        const hipError_t e2 = hipStreamEndCapture(c->cap_stream, &graph);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return fail(c, ARC_E_DEVICE, "graph capture of chemistry stage %d: %s", i,
                        hipGetErrorString(e != hipSuccess ? e : e2));
        }
        const hipError_t e3 = hipGraphInstantiate(&c->cexec[i], graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e3 != hipSuccess) {
            c->cexec[i] = nullptr;
            return fail(c, ARC_E_DEVICE, "graph instantiation of chemistry stage %d: %s", i, hipGetErrorString(e3));
        }
    }
    c->chem_key.assign(key, key + sizeof P);
    return ARC_OK;
}

}  // namespace

namespace {

// Checks and launch arguments of the section 2.9 time step, shared by both entry points;
// `out` receives the two minima as bit patterns of non-negative doubles.
arc_status plan_timestep(arc_ctx* c, const arc_grid* g, const arc_rates* r, const arc_freq_bins* b,
                         const arc_chem_params* p, double eps, unsigned long long* out, TimestepArgs& a)
{
    arc_status rc;
    if ((rc = check_grid(c, g)) != ARC_OK) return rc;
    if ((rc = check_bins(c, b)) != ARC_OK) return rc;
    if (!g->temp) return fail(c, ARC_E_ARG, "null temperature");
    if (!r || !r->gamma) return fail(c, ARC_E_ARG, "null rates");
    if (!p) return fail(c, ARC_E_ARG, "null params");
    if (!(eps > 0) || !std::isfinite(eps)) return fail(c, ARC_E_RANGE, "eps must be finite and > 0");
    if (p->rates != 0 && p->rates != 1) return fail(c, ARC_E_ARG, "rates must be 0 or 1");
    if (p->rates == 0 && !(p->alpha_hii >= 0)) return fail(c, ARC_E_RANGE, "alpha_hii must be >= 0");
    a = TimestepArgs{};
    a.ncell = (uint32_t)((size_t)g->nx * g->ny * g->nz);
    a.y = g->y_he;
    a.cell_cm = g->cell_cm;
    a.sigma0 = b->sigma[0];
    a.eps = eps;
    a.n_h = g->n_h;
    a.x_hi = g->x_hi;
    a.x_hei = g->x_hei;
    a.x_heii = g->x_heii;
    a.temp = g->temp;
    a.gamma_hi = r->gamma;
    a.rates = p->rates;
    a.collisional = p->collisional;
    a.alpha_hii = p->alpha_hii;
    a.out = out;
    return ARC_OK;
}

}  // namespace

extern "C" {

arc_status arc_rt_timestep(arc_ctx* c, const arc_grid* g, const arc_rates* r, const arc_freq_bins* b,
                           const arc_chem_params* p, double eps, double* dt_n, double* dt_i)
{
    if (!c) return ARC_E_ARG;
    c->err.clear();
    if (!dt_n || !dt_i) return fail(c, ARC_E_ARG, "null outputs");
    TimestepArgs a;
    arc_status rc = plan_timestep(c, g, r, b, p, eps, c->sums, a);
    if (rc != ARC_OK) return rc;
    hipStream_t st = (hipStream_t)p->stream;
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, launch_timestep_reset(c->sums, st));
    HIP_TRY(c, launch_timestep(a, c->cus, st));
    unsigned long long h[2];
    HIP_TRY(c, hipMemcpyAsync(h, c->sums, sizeof h, hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    std::memcpy(dt_n, &h[0], sizeof(double));
    std::memcpy(dt_i, &h[1], sizeof(double));
    return ARC_OK;
}

arc_status arc_rt_timestep_noalloc(arc_ctx* c, const arc_grid* g, const arc_rates* r, const arc_freq_bins* b,
                                   const arc_chem_params* p, double eps, double* dt_out)
{
    if (!c) return ARC_E_ARG;
    c->err.clear();
    if (!dt_out) return fail(c, ARC_E_ARG, "null output");
    if (!c->static_scratch) return fail(c, ARC_E_DEVICE, "static scratch of device %d not resolved", c->device);
    // the kernels use kTimestepScratchWords words of the device's static scratch, whatever the
    // grid; grids are bounded by the checks every entry point applies (below 2^31 cells)
    static_assert(kTimestepScratchWords <= kStaticScratchWords, "static scratch too small");
    TimestepArgs a;
    arc_status rc = plan_timestep(c, g, r, b, p, eps, c->static_scratch, a);
    if (rc != ARC_OK) return rc;
    hipStream_t st = (hipStream_t)p->stream;
    HIP_TRY(c, hipSetDevice(c->device));
    // the array keeps the last call's minima: reset them (a kernel, not a memset node)
    HIP_TRY(c, launch_timestep_reset(c->static_scratch, st));
    HIP_TRY(c, launch_timestep(a, c->cus, st));
    HIP_TRY(c, launch_timestep_publish(c->static_scratch, dt_out, st));
    return ARC_OK;
}

arc_status arc_chem_step(arc_ctx* c, const arc_grid* g, const arc_rates* r, double dt, const arc_chem_params* p,
                         arc_chem_stats* stats)
{
    if (!c) return ARC_E_ARG;
    c->err.clear();
    arc_status rc;
    if ((rc = check_grid(c, g)) != ARC_OK) return rc;
    if (!g->temp) return fail(c, ARC_E_ARG, "null temperature");
    if (!r || !r->gamma || !r->heat) return fail(c, ARC_E_ARG, "null rates");
    if (!p) return fail(c, ARC_E_ARG, "null params");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(c, ARC_E_RANGE, "dt must be finite and > 0");
    if (!(p->eps > 0) || !std::isfinite(p->eps)) return fail(c, ARC_E_RANGE, "eps must be > 0");
    if (p->max_sub < 1) return fail(c, ARC_E_RANGE, "max_sub must be >= 1");
    if (p->rates != 0 && p->rates != 1) return fail(c, ARC_E_ARG, "rates must be 0 or 1");
    if (p->rates == 0 && !(p->alpha_hii >= 0)) return fail(c, ARC_E_RANGE, "alpha_hii must be >= 0");
    if (!(p->t_floor > 0)) return fail(c, ARC_E_RANGE, "t_floor must be > 0");
    if (p->mode != ARC_CHEM_PLAIN && p->mode != ARC_CHEM_MLP_GATED && p->mode != ARC_CHEM_MLP_ONLY)
        return fail(c, ARC_E_ARG, "bad chemistry mode %d", p->mode);
    if (p->mode != ARC_CHEM_PLAIN && (!p->mlp || !p->mlp->trained))
        return fail(c, ARC_E_ARG, "the learned modes need a trained network");
    if (p->mode == ARC_CHEM_MLP_GATED && !(p->gate_tol >= 0)) return fail(c, ARC_E_RANGE, "gate_tol must be >= 0");
    hipStream_t st = (hipStream_t)p->stream;
    HIP_TRY(c, hipSetDevice(c->device));
    ChemPlan P;
    std::memset(&P, 0, sizeof P);
    P.mode = p->mode;
    P.cus = c->cus;
    ChemArgs& a = P.a;
    a.ncell = (uint32_t)((size_t)g->nx * g->ny * g->nz);
    a.y = g->y_he;
    a.n_h = g->n_h;
    a.x_hi = g->x_hi;
    a.x_hei = g->x_hei;
    a.x_heii = g->x_heii;
    a.temp = g->temp;
    a.gamma = r->gamma;
    a.heat = r->heat;
    a.dt = dt;
    a.isothermal = p->isothermal;
    a.rates = p->rates;
    a.collisional = p->collisional;
    a.max_sub = p->max_sub;
    a.alpha_hii = p->alpha_hii;
    a.eps = p->eps;
    a.t_floor = p->t_floor;
    a.stats = c->chem_stats;
    a.chunk_counter = (uint32_t*)(c->chem_stats + 4);
    a.mask = nullptr;
    if (p->mode != ARC_CHEM_PLAIN) {
        const size_t words = ((size_t)a.ncell + 63) / 64;
        if (words > c->reject_cap) {
            if (c->reject) HIP_TRY(c, hipFree(c->reject));
            c->reject = nullptr;
            c->reject_cap = 0;
            HIP_TRY(c, hipMalloc((void**)&c->reject, words * sizeof(unsigned long long)));
            c->reject_cap = words;
        }
        mlp::InferArgs& ia = P.ia;
        ia.model = p->mlp->model;
        ia.ncell = a.ncell;
        ia.y = a.y;
        ia.n_h = a.n_h;
        ia.x_hi = a.x_hi;
        ia.x_hei = a.x_hei;
        ia.x_heii = a.x_heii;
        ia.temp = a.temp;
        ia.gamma = a.gamma;
        ia.heat = a.heat;
        ia.dt = dt;
        ia.gated = p->mode == ARC_CHEM_MLP_GATED;
        ia.gate_tol = (float)p->gate_tol;
        ia.gate_min_count = (uint32_t)std::max(0, p->gate_min_count);
        ia.t_floor = (float)p->t_floor;
        ia.reject = c->reject;
        ia.collisional = p->rates == 1 ? p->collisional : 0;
        if (p->mode == ARC_CHEM_MLP_GATED) a.mask = c->reject;
    }
    if (p->graph) {
        if ((rc = ensure_chem_graphs(c, P)) != ARC_OK) return rc;
        HIP_TRY(c, hipGraphLaunch(c->cexec[0], st));
        HIP_TRY(c, hipEventRecord(c->ev[0], st));
        HIP_TRY(c, hipGraphLaunch(c->cexec[1], st));
        HIP_TRY(c, hipEventRecord(c->ev[2], st));
        HIP_TRY(c, hipGraphLaunch(c->cexec[2], st));
    } else {
        HIP_TRY(c, chem_stage(c, P, 0, st));
        HIP_TRY(c, hipEventRecord(c->ev[0], st));
        HIP_TRY(c, chem_stage(c, P, 1, st));
        HIP_TRY(c, hipEventRecord(c->ev[2], st));
        HIP_TRY(c, chem_stage(c, P, 2, st));
    }
    HIP_TRY(c, hipEventRecord(c->ev[1], st));
    unsigned long long cs[4];
    HIP_TRY(c, hipMemcpyAsync(cs, c->chem_stats, sizeof cs, hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    if (stats) {
        stats->cells = a.ncell;
        stats->sub_total = (int64_t)cs[0];
        stats->capped = (int64_t)cs[1];
        stats->sub_max = (int32_t)cs[2];
        float ms = 0;
        HIP_TRY(c, hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
        stats->ms = ms;
        stats->fallback = p->mode == ARC_CHEM_MLP_GATED ? (int64_t)cs[3] : 0;
        stats->ms_mlp = 0;
        if (p->mode != ARC_CHEM_PLAIN) {
            HIP_TRY(c, hipEventElapsedTime(&ms, c->ev[0], c->ev[2]));
            stats->ms_mlp = ms;
        }
    }
    return ARC_OK;
}

}  // extern "C"
