// arc_device.h -- device-side data layout and per-ray arithmetic shared by every
// tracing schedule of libarc (gfx950).
//
// The plain and the batched schedules call exactly these functions, so a ray deposits
// the same integers whichever schedule traces it; integer sums do not depend on order,
// which makes the fixed-point field bitwise identical across schedules and runs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace arc {

constexpr int kMaxBins = 4;
constexpr int kMaxLevels = 16;       // HEALPix levels 0..15 (pixel ids fit 28 bits to level 12)
constexpr int kLevelShift = 28;      // packed ray id: level << 28 | pixel
constexpr uint32_t kPixMask = (1u << kLevelShift) - 1u;
constexpr float kDtauTermMin = 0.01f;  // a terminating crossing must be this thick in every bin

enum Event : int { kContinue = 0, kSplit = 1, kTerminate = 2, kEscape = 3 };

constexpr uint32_t kNoCell = 0xFFFFFFFFu;
// Pointer qualifier of the LDS address space.
#define kLds __attribute__((address_space(3)))

// Cell layout of the opacity and the field: 8^3 blocks in x-fastest block order, Morton
// order inside a block, so that the 2x2x2 neighbourhood of a cell shares a 128-byte
// line of opacity (and two lines of field) and a block is 8 KB of opacity.
__host__ __device__ __forceinline__ uint32_t spread3(uint32_t v)
{
    // bits 0, 1, 2 -> 0, 3, 6: bit 2 moves by 4 first, then bits 1 and 2 by 2
    const uint32_t x = ((v << 4) | v) & 0x43u;
    return ((x << 2) | x) & 0x49u;
}
__host__ __device__ __forceinline__ uint32_t blocked_index(int x, int y, int z, int nbx8, int nby8)
{
    const uint32_t b = ((uint32_t)(z >> 3) * (uint32_t)nby8 + (uint32_t)(y >> 3)) * (uint32_t)nbx8 + (uint32_t)(x >> 3);
    const uint32_t m = spread3((uint32_t)x & 7u) | (spread3((uint32_t)y & 7u) << 1) | (spread3((uint32_t)z & 7u) << 2);
    return (b << 9) | m;
}

// A crossing's deposit: the cell (blocked index) and the amount of every bin in field units,
// rounded to the field's integers when the wave deposits it.
template <int NB>
struct Dep {
    uint32_t cell;        // kNoCell: nothing to deposit
    float v[NB];
};

enum Counter : int {
    kCrossings = 0, kRays, kSplits, kTerminated, kEscapedRays, kSpills, kTreeCount, kQueueOverflow,
    kDeposits,  // (cell, bins) deposit items issued as atomics after the wave-level merge
    kCrossingsPre, kDepositsPre,  // crossings and deposits before the persistent launch
    kNumCounters
};

// Per-source constants (section 2.1 keeps the source position on chip; here it is a
// 32-byte record read through L2 once per ray).
struct __align__(16) SourceRec {
    float x, y, z;        // position on the 2^-12 lattice (exact in FP32 up to 2048 cells)
    float r_thin;         // optically thin radius (section 2.6): rays start at this radius
    float scale[4];       // ndot * frac_b / (12 * u_J,b): root-ray photon rate in field units
};

// A ray waiting to be traced: its identity and the optical depth it carries. The start
// radius follows from the level (0 for roots, the parent's split radius for children).
struct __align__(16) RayRec {
    uint32_t src;
    uint32_t lp;          // level << 28 | nested pixel
    uint32_t pad0, pad1;
    float tau[4];         // optical depth per bin (high part)
    float taulo[4];       // compensation terms
};

// The same ray in the compact form kept on a wave's stack (32 bytes for three bins).
template <int NB>
struct StackRec {
    uint32_t src;
    uint32_t lp;
    float tau[NB];
    float taulo[NB];
};

struct TraceArgs {
    int nx, ny, nz, nb;
    int nbx8, nby8;            // 8^3 blocks per row and per column of the cell layout
    int level0, lmax;
    float tsplit[kMaxLevels];  // split radius of each level; +inf from lmax on
    float tau_term;            // +inf = never terminate
    const float* kappa1;       // nb == 1: optical depth per cell length, [cell] (blocked order)
    const float4* kappa4;      // nb > 1: [cell] (bins in x, y, z, w) (blocked order)
    unsigned long long* J;     // fixed-point field [cell][nbp] (blocked order)
    int nbp;                   // padded bins per cell in J (1, 2 or 4)
    const SourceRec* src;
    const float4* dirs;        // HEALPix centres of every level, concatenated
    long long dir_off[kMaxLevels];
    double* esc;               // [kMaxBins] escaped photons in field units (times u_J: photons/s)
    unsigned long long* counters;  // [kNumCounters]
    unsigned long long* tree;  // optional record of every ray traced
    long long tree_cap;
    int corr;                  // geometric correction: 0 none, 1 f_c, 2 f_c + secondary, 3 f_c^2
    // corr == 2: photons moved into a cell by the secondary correction (eq:correction2), in two
    // limbs per bin, [cell][limb][nbp]: limb 0 in units of 2^20 u_J,b, limb 1 in units of
    // 2^-12 u_J,b
    unsigned long long* M;
    // optically thin approximation (section 2.6): the bin of lowest photon energy, and per
    // source the least path length at which a ray's depth in it reaches kTauThin (FP32 bits)
    int ksoft;
    unsigned int* r_out;
};

constexpr float kTauThin = 0.1f;  // optical depth that bounds the optically thin sphere

// Per-lane ray state. Along axis i the ray meets its next cell boundary at
// t_i = a_i / e_i, where e_i = |d_i| and a_i is the (exact, lattice-valued) distance of
// that boundary from the source; crossing the boundary adds 1 to a_i. The blocked cell
// index is the sum of one term per axis, refreshed only for the axes that move.
template <int NB>
struct Ray {
    float e[3];           // |d_i|
    float ie[3];          // 1 / |d_i| (hardware reciprocal, within 1 ulp), +inf if d_i == 0
    float a[3];           // next-boundary distance along each axis (exact)
    int c[3];             // current cell
    int step[3];          // +1, -1 or 0
    uint32_t ix[3];       // per-axis terms of the blocked cell index
    float thi, tlo;       // current path length (double-float)
    float tend;           // split radius or +inf
    float tau[NB], taulo[NB];
    float w[NB];          // scale_b * 4^-level
    uint32_t src, lp;
};

struct LaneStats {
    uint32_t crossings, rays, splits, terminated, escaped;
    double esc[kMaxBins];
    __device__ void clear()
    {
        crossings = rays = splits = terminated = escaped = 0;
        for (int b = 0; b < kMaxBins; ++b) esc[b] = 0.0;
    }
};

// ---------------------------------------------------------------------------------
// Exact arithmetic helpers. All operands are non-negative FP32 values.
// ---------------------------------------------------------------------------------

// sign(a*b - c*d), exact: products are split into rounded value and FMA remainder.
__device__ __forceinline__ int cmp_prod(float a, float b, float c, float d)
{
    const float p = a * b, q = c * d;
    if (p != q) return p < q ? -1 : 1;
    const float ep = __builtin_fmaf(a, b, -p), eq = __builtin_fmaf(c, d, -q);
    return ep < eq ? -1 : (ep > eq ? 1 : 0);
}

// Cell index along one axis that the ray occupies just after path length t0:
// x = xs + t0*d. Exact: t0*d is split into a rounded part and its FMA remainder, and
// k - xs is exact on the lattice, so (xs + t0 d) vs k is decided without rounding.
// d > 0: a point on a boundary belongs to the upper cell; d < 0: to the lower cell;
// d == 0: to the upper cell.
__device__ __forceinline__ int start_index(float xs, float t0, float d)
{
    if (d == 0.0f) return (int)floorf(xs);
    const float ph = t0 * d;
    const float pl = __builtin_fmaf(t0, d, -ph);
    int k = (int)floorf(xs + ph);
    // sign((xs + t0 d) - k)
    auto side = [&](int kk) -> int {
        const float m = (float)kk - xs;
        if (ph != m) return ph > m ? 1 : -1;
        return pl > 0.0f ? 1 : (pl < 0.0f ? -1 : 0);
    };
    if (d > 0.0f) {
        while (side(k) < 0) --k;
        while (side(k + 1) >= 0) ++k;
    } else {
        while (side(k) <= 0) --k;
        while (side(k + 1) > 0) ++k;
    }
    return k;
}

// Per-axis terms of blocked_index(): index = term(x, 0) + term(y, 1) + term(z, 2).
__device__ __forceinline__ uint32_t axis_term(const TraceArgs& A, int i, int v)
{
    // grids are at most 2048 cells per axis: the block's first cell index along the axis is
    // below 2^17 and the blocks it stands for below 2^17; with those ranges stated the multiply
    // is the full-rate 24-bit one
    const uint32_t blk9 = ((uint32_t)v << 6) & 0x1FE00u;
    const uint32_t m = spread3((uint32_t)v & 7u) << i;
    if (i == 0) return blk9 + m;
    if (i == 1) return blk9 * ((uint32_t)A.nbx8 & 0x1FFFFu) + m;
    return blk9 * (((uint32_t)A.nbx8 * (uint32_t)A.nby8) & 0x1FFFFu) + m;
}

// Non-negative float to the nearest int64 (v < 2^63): two exact 32-bit halves.
__device__ __forceinline__ long long round_to_i64(float v)
{
    const float r = rintf(v);
    const float hi = floorf(r * 2.3283064365386963e-10f);   // r / 2^32, exact scaling
    const float lo = __builtin_fmaf(-hi, 4294967296.0f, r);  // exact remainder in [0, 2^32)
    return (long long)(((unsigned long long)(uint32_t)hi << 32) | (unsigned long long)(uint32_t)lo);
}

// e^-tau with the hardware exponential (relative error ~1e-6 for tau up to ~80).
__device__ __forceinline__ float transmission(float tau) { return __builtin_amdgcn_exp2f(-tau * 1.4426950408889634f); }

// ---------------------------------------------------------------------------------
// Per-ray operations.
// ---------------------------------------------------------------------------------

template <int NB>
__device__ __forceinline__ void record_tree(const TraceArgs& A, uint32_t src, uint32_t lp)
{
    if (A.tree) {
        const unsigned long long i = atomicAdd(&A.counters[kTreeCount], 1ull);
        if ((long long)i < A.tree_cap) A.tree[i] = ((unsigned long long)src << 32) | lp;
    }
}

// Load a ray: direction, source, start radius and start cell (section 2.1 iii a/c:
// roots at radius 0, children at the parent's radius with their own direction). With the
// optically thin approximation (THIN, section 2.6) a ray starts no closer than its source's
// thin radius; a ray whose split radius does not lie beyond that start splits at once (it is
// returned active with thi >= tend and crosses nothing).
// Returns false (and books the escape) when the start point lies outside the grid.
template <int NB, bool THIN, class Rec>
__device__ __forceinline__ bool ray_init(const TraceArgs& A, const Rec& r, Ray<NB>& ray, LaneStats& st)
{
    ray.src = r.src;
    ray.lp = r.lp;
    const int level = (int)(r.lp >> kLevelShift);
    const uint32_t pix = r.lp & kPixMask;
    const float4 dv = A.dirs[A.dir_off[level] + pix];
    const float d[3] = {dv.x, dv.y, dv.z};
    const SourceRec s = A.src[r.src];
    const float xs[3] = {s.x, s.y, s.z};
    float t0 = level == A.level0 ? 0.0f : A.tsplit[level - 1];
    if constexpr (THIN) t0 = fmaxf(t0, s.r_thin);
    ray.thi = t0;
    ray.tlo = 0.0f;
    ray.tend = A.tsplit[level];
    const float lw = __builtin_ldexpf(1.0f, -2 * level);  // 4^-level, exact
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        ray.tau[b] = r.tau[b];
        ray.taulo[b] = r.taulo[b];
        ray.w[b] = s.scale[b] * lw;
    }
    st.rays++;
    if constexpr (THIN) {
        if (!(t0 < ray.tend)) return true;  // splits at once
    }
    bool inside = true;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int c = start_index(xs[i], t0, d[i]);
        ray.c[i] = c;
        ray.e[i] = fabsf(d[i]);
        ray.ie[i] = d[i] != 0.0f ? __builtin_amdgcn_rcpf(ray.e[i]) : INFINITY;
        ray.step[i] = d[i] > 0.0f ? 1 : (d[i] < 0.0f ? -1 : 0);
        // d_i = 0: the distance to the upper face (no boundary is met along this axis; the
        // geometric correction reads the position from it)
        ray.a[i] = d[i] < 0.0f ? xs[i] - (float)c : (float)(c + 1) - xs[i];
        const int n = i == 0 ? A.nx : (i == 1 ? A.ny : A.nz);
        inside = inside && c >= 0 && c < n;
        ray.ix[i] = inside ? axis_term(A, i, c) : 0u;
    }
    if (!inside) {
        float ts = 0.0f;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const float tb = ray.tau[b] + ray.taulo[b];
            st.esc[b] += (double)ray.w[b] * (double)transmission(tb);
            if (b == A.ksoft) ts = tb;
        }
        // a ray that starts outside the grid while still thin bounds the thin radius by its start
        if constexpr (THIN)
            if (ts < kTauThin) atomicMin(A.r_out + ray.src, __float_as_uint(t0));
        st.escaped++;
    }
    return inside;
}

template <int NB>
__device__ __forceinline__ void kappa_at(const TraceArgs& A, uint32_t cell, float k[NB])
{
    if constexpr (NB == 1) {
        k[0] = A.kappa1[cell];
    } else {
        const float4 v = A.kappa4[cell];
        k[0] = v.x;
        k[1] = v.y;
        if constexpr (NB > 2) k[2] = v.z;
        if constexpr (NB > 3) k[3] = v.w;
    }
}

// A piece of a ray inside one cell: blocked cell index, length, and what happens at its
// end (kContinue: next cell; kSplit: the split radius; kEscape: the ray leaves the grid).
struct Seg {
    uint32_t cell;
    float ds;
    int event;
    uint32_t nb;  // geometric correction: neighbour that receives the moved share (kNoCell: none)
    float fc;     // geometric correction: share the cell keeps (1: uncorrected)
    float t1;     // path length at the segment's end (high part)
};

constexpr double kSqrtPiOver3 = 1.0233267079464885;  // width of a level-0 pixel per unit radius
// Face distances within this many cells count as tied: symmetric geometries tie exactly,
// and the last bits of a midpoint depend on how its path length was summed.
constexpr double kFaceTie = 1e-9;

// Geometric correction of the segment [t, t_next) in the ray's current cell (section 2.5,
// eq:correction): D_edge is the distance from the segment's midpoint to the nearest face of
// the cell, L_Pix the width of the ray's pixel there (r sqrt(4 pi / N_pix)); the cell keeps
// f_c = 1/2 + D_edge / L_Pix of the crossing's photons when D_edge < L_Pix / 2 (mode 3: f_c
// squared). Mode 2 also names the neighbour across that face, which receives the rest
// (eq:correction2); without one inside the grid the cell keeps everything. Distances in
// FP64 from the exact boundary numerators; faces within kFaceTie count as tied, and ties go
// to the lower axis, then the lower face.
template <int NB>
__device__ __forceinline__ void geom_correction(const TraceArgs& A, const Ray<NB>& ray, float nhi, float nlo, Seg& sg)
{
    sg.nb = kNoCell;
    sg.fc = 1.0f;
    if (A.corr == 0) return;
    const double tm = 0.5 * (((double)ray.thi + (double)ray.tlo) + ((double)nhi + (double)nlo));
    const int level = (int)(ray.lp >> kLevelShift);
    const double lpix = tm * __builtin_ldexp(kSqrtPiOver3, -level);
    double dmin = INFINITY;
    int axis = 0, side = -1;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        // distance to the face the ray heads for (the upper face when d_i = 0)
        const double ahead = (double)ray.a[i] - tm * (double)ray.e[i];
        const bool up = ray.step[i] >= 0;
        const double hi = up ? ahead : 1.0 - ahead;
        const double lo = up ? 1.0 - ahead : ahead;
        const bool upper = hi < lo - kFaceTie;
        const double di = upper ? hi : lo;
        if (di < dmin - kFaceTie) {
            dmin = di;
            axis = i;
            side = upper ? 1 : -1;
        }
    }
    if (!(dmin < 0.5 * lpix)) return;
    // the decisions above are FP64; the share itself needs FP32 only
    float fc = 0.5f + (float)dmin * __builtin_amdgcn_rcpf((float)lpix);
    if (A.corr == 3) fc *= fc;
    if (A.corr == 2) {
        // the neighbour's per-axis term replaces the cell's along `axis` (static indices only:
        // a runtime index into the ray's arrays would move them to scratch memory)
        bool inside = true;
        uint32_t nb = sg.cell;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            if (i == axis) {
                const int ca = ray.c[i] + side;
                const int na = i == 0 ? A.nx : (i == 1 ? A.ny : A.nz);
                inside = ca >= 0 && ca < na;
                if (inside) nb = nb - ray.ix[i] + axis_term(A, i, ca);
            }
        }
        if (!inside) return;  // no neighbour inside: the cell keeps everything
        sg.nb = nb;
    }
    sg.fc = fc;
}

// Geometry of the next segment (section 2.4: the step to the next x, y or z boundary, or
// to the split radius), advancing the ray's position and cell.
//
// Geometric decisions are exact: boundary times are compared through the reciprocal
// products a_i / e_i, whose relative error is below 2e-7, and any comparison closer than
// 1e-6 is settled exactly with cmp_prod (a_i e_j vs a_j e_i). The winning axis is picked
// with conditional moves (a runtime index into the per-ray arrays would move them to
// scratch memory).
template <int NB, int PREC, bool CORR = false>
__device__ __forceinline__ Seg geom_next(const TraceArgs& A, Ray<NB>& ray)
{
    constexpr float kNear = 1.000001f;
    // a_i > 0 always, and ie_i = +inf where d_i = 0, so those axes give t_i = +inf
    const float t0 = ray.a[0] * ray.ie[0];
    const float t1 = ray.a[1] * ray.ie[1];
    const float t2 = ray.a[2] * ray.ie[2];
    // the selects follow the comparisons themselves, not an axis number (a select chain on
    // w == 0, w == 1 is turned into an indexed access to the ray, which lives in scratch)
    const bool b1 = t1 < t0;
    float tw = b1 ? t1 : t0;
    float aw = b1 ? ray.a[1] : ray.a[0];
    float ew = b1 ? ray.e[1] : ray.e[0];
    float iew = b1 ? ray.ie[1] : ray.ie[0];
    const bool b2 = t2 < tw;
    tw = b2 ? t2 : tw;
    aw = b2 ? ray.a[2] : aw;
    ew = b2 ? ray.e[2] : ew;
    iew = b2 ? ray.ie[2] : iew;
    int w = b2 ? 2 : (b1 ? 1 : 0);
    int mask = b2 ? 4 : (b1 ? 2 : 1);
    bool at_end;
    if constexpr (PREC == 0) {
        const bool near = (w != 0 && t0 <= tw * kNear) || (w != 1 && t1 <= tw * kNear) || (w != 2 && t2 <= tw * kNear);
        if (near) {
            // exact argmin and ties: t_i < t_j  <=>  a_i e_j < a_j e_i
            int ww = -1;
            float ab = 0.0f, eb = 0.0f, ib = 0.0f;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                if (ray.e[i] > 0.0f && (ww < 0 || cmp_prod(ray.a[i], eb, ab, ray.e[i]) < 0)) {
                    ww = i;
                    ab = ray.a[i];
                    eb = ray.e[i];
                    ib = ray.ie[i];
                }
            }
            w = ww;
            mask = 0;
#pragma unroll
            for (int i = 0; i < 3; ++i)
                if (ray.e[i] > 0.0f && cmp_prod(ray.a[i], eb, ab, ray.e[i]) == 0) mask |= 1 << i;
            aw = ab;
            ew = eb;
            iew = ib;
            tw = aw * iew;
        }
        if (ray.tend > tw * kNear)
            at_end = false;
        else if (ray.tend * kNear < tw)
            at_end = true;
        else
            at_end = cmp_prod(ray.tend, ew, aw, 1.0f) <= 0;
    } else {
        if (w != 0 && t0 == tw) mask |= 1;
        if (w != 1 && t1 == tw) mask |= 2;
        if (w != 2 && t2 == tw) mask |= 4;
        at_end = ray.tend <= tw;
    }
    // next path length as a double-float, and the segment length ds = t_next - t_cur
    float nhi, nlo;
    if (at_end) {
        nhi = ray.tend;
        nlo = 0.0f;
    } else {
        nhi = tw;
        nlo = PREC == 0 ? __builtin_fmaf(-nhi, ew, aw) * iew : 0.0f;
    }
    Seg sg;
    if constexpr (PREC == 0) {
        const float s = nhi - ray.thi;
        const float bb = s - nhi;
        const float err = (nhi - (s - bb)) + (-ray.thi - bb);
        sg.ds = s + (err + (nlo - ray.tlo));
    } else {
        sg.ds = nhi - ray.thi;
    }
    sg.cell = ray.ix[0] + ray.ix[1] + ray.ix[2];
    sg.t1 = nhi;
    if constexpr (CORR) geom_correction(A, ray, nhi, nlo, sg);
    ray.thi = nhi;
    ray.tlo = nlo;
    if (at_end) {
        sg.event = kSplit;
        return sg;
    }
    bool inside = true;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        if (mask & (1 << i)) {
            const int c = ray.c[i] + ray.step[i];
            ray.c[i] = c;
            ray.a[i] += 1.0f;
            const int n = i == 0 ? A.nx : (i == 1 ? A.ny : A.nz);
            const bool in = c >= 0 && c < n;
            inside = inside && in;
            if (in) ray.ix[i] = axis_term(A, i, c);
        }
    }
    sg.event = inside ? kContinue : kEscape;
    return sg;
}

// Section 2.6: the least path length at which the ray's depth in the softest bin reaches
// kTauThin, within this segment (ts: depth at its start, dts: its increment, ks: its
// opacity), bounds the source's thin radius (one atomic per ray at most).
template <int NB>
__device__ __forceinline__ void thin_reach(const TraceArgs& A, const Ray<NB>& ray, const Seg& sg, float ts, float dts,
                                           float ks)
{
    if (ts < kTauThin && ts + dts >= kTauThin) {
        const float rc = (sg.t1 - sg.ds) + (kTauThin - ts) / ks;
        atomicMin(A.r_out + ray.src, __float_as_uint(rc));
    }
}

// Photons of one segment (section 2.4, eq:ion per bin): the amount v_b = S ds g(dtau) for the
// cell in field units, attenuation (compensated tau), then the termination test (a
// terminating crossing adds the rest of the photons, S / kappa, to v_b) and, with THIN, the
// thin-radius measurement. T_b carries the transmission e^-tau_b from one segment to the next
// (one exponential per bin and crossing): with S = w T_b the photons entering the cell, the
// cell absorbs S (1 - e^-dtau) = w (T_b - T'_b), so v_b = w (T_b - T'_b) / kappa_b, and below
// dtau = 0.25, where that difference would cancel, S ds g(dtau) with g's Taylor series
// (truncation < 5e-8 relative). An escaping ray leaves its remaining photons w T'_b in esc.
// Returns kTerminate, kSplit, kEscape or kContinue.
template <int NB, int PREC, bool THIN>
__device__ __forceinline__ int attenuate_seg(const TraceArgs& A, Ray<NB>& ray, const Seg& sg, const float kap[NB],
                                             LaneStats& st, float v[NB], float (&T)[NB], float (&esc)[NB])
{
    bool term = A.tau_term < INFINITY;
    float ts = 0.0f, dts = 0.0f, ks = 1.0f;
    float rk[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const float dtau = kap[b] * sg.ds;
        if constexpr (THIN) {
            if (b == A.ksoft) {
                ts = PREC == 0 ? ray.tau[b] + ray.taulo[b] : ray.tau[b];
                dts = dtau;
                ks = kap[b];
            }
        }
        if constexpr (PREC == 0) {
            const float s = ray.tau[b] + dtau;
            const float bb = s - ray.tau[b];
            ray.taulo[b] += (ray.tau[b] - (s - bb)) + (dtau - bb);
            ray.tau[b] = s;
        } else {
            ray.tau[b] += dtau;
        }
        const float taup = PREC == 0 ? ray.tau[b] + ray.taulo[b] : ray.tau[b];
        const float Tn = transmission(taup);
        // 1 / kappa (hardware reciprocal): used where dtau >= 0.25 or on termination (dtau >= 0.01)
        rk[b] = __builtin_amdgcn_rcpf(kap[b]);
        const float g = __builtin_fmaf(
            dtau, __builtin_fmaf(dtau, __builtin_fmaf(dtau, __builtin_fmaf(dtau, __builtin_fmaf(dtau, -1.0f / 720.0f, 1.0f / 120.0f), -1.0f / 24.0f), 1.0f / 6.0f), -0.5f),
            1.0f);
        const float series = ((ray.w[b] * T[b]) * sg.ds) * g;
        const float lost = (ray.w[b] * (T[b] - Tn)) * rk[b];
        v[b] = dtau < 0.25f ? series : lost;
        T[b] = Tn;
        term = term && taup >= A.tau_term && dtau >= kDtauTermMin;
    }
    st.crossings++;
    if constexpr (THIN) thin_reach<NB>(A, ray, sg, ts, dts, ks);
    if (term) {
        // absorb what is left in this cell: field += remaining photons / opacity
#pragma unroll
        for (int b = 0; b < NB; ++b) v[b] = __builtin_fmaf(ray.w[b] * T[b], rk[b], v[b]);
        st.terminated++;
        return kTerminate;
    }
    if (sg.event == kSplit) {
        st.splits++;
        return kSplit;
    }
    if (sg.event == kEscape) {
        float tsp = 0.0f;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            esc[b] = ray.w[b] * T[b];
            if (b == A.ksoft) tsp = PREC == 0 ? ray.tau[b] + ray.taulo[b] : ray.tau[b];
        }
        // a ray that leaves the grid while still thin bounds the thin radius by its exit
        if constexpr (THIN)
            if (tsp < kTauThin) atomicMin(A.r_out + ray.src, __float_as_uint(sg.t1));
        st.escaped++;
        return kEscape;
    }
    return kContinue;
}

// Transmission e^-tau of every bin of a ray at its current depth.
template <int NB, int PREC>
__device__ __forceinline__ void ray_transmission(const Ray<NB>& ray, float (&T)[NB])
{
#pragma unroll
    for (int b = 0; b < NB; ++b) T[b] = transmission(PREC == 0 ? ray.tau[b] + ray.taulo[b] : ray.tau[b]);
}

// Photons an escaping lane carried out of the grid, into the FP64 ledger (once per pass).
template <int NB>
__device__ __forceinline__ void book_escape(int ev, const float (&esc)[NB], LaneStats& st)
{
    if (ev == kEscape) {
#pragma unroll
        for (int b = 0; b < NB; ++b) st.esc[b] += (double)esc[b];
    }
}

// A segment's deposit into its own cell.
template <int NB, int PREC, bool THIN>
__device__ __forceinline__ int deposit_seg(const TraceArgs& A, Ray<NB>& ray, const Seg& sg, const float kap[NB],
                                           LaneStats& st, Dep<NB>& dep, float (&T)[NB], float (&esc)[NB])
{
    const int ev = attenuate_seg<NB, PREC, THIN>(A, ray, sg, kap, st, dep.v, T, esc);
    dep.cell = sg.cell;
    return ev;
}

// Limbs of the moved-photon field: mv = hi 2^20 + lo 2^-12 (units of u_J,b). A crossing's lo
// is below 2^32, so the limb holds 2^31 crossings; hi is bounded like the field.
constexpr float kMovedHiUnit = 1048576.0f;      // 2^20
constexpr float kMovedLoScale = 4096.0f;        // 2^12

// Integer deposit of an amount v in field units: the field's own integers (kWhole), or the
// high or low limb of the moved-photon field, hi = floor(v / 2^20) (an integer float) and the
// rest, v - hi 2^20 (exact: the bits of v below 2^20), in units of 2^-12, rounded.
enum Limb : int { kWhole = 0, kMovedHi = 1, kMovedLo = 2 };
template <int LIMB>
__device__ __forceinline__ long long to_fixed(float v)
{
    if constexpr (LIMB == kWhole) {
        return round_to_i64(v);
    } else {
        const float hi = floorf(v * (1.0f / kMovedHiUnit));
        if constexpr (LIMB == kMovedHi) return round_to_i64(hi);
        return (long long)(uint32_t)rintf(__builtin_fmaf(-hi, kMovedHiUnit, v) * kMovedLoScale);
    }
}

// Opacity ratio up to which the conserving correction's moved share enters the neighbour's
// field directly (beyond it, as photons in the two-limb field M).
constexpr float kMovedRatioJ = 16.0f;

// deposit_seg with the geometric correction (section 2.5): the cell keeps fc of the
// crossing's photons (the termination remainder included). In mode 2 the rest goes to the
// neighbour sg.nb, absorbed there at the neighbour's opacity (eq:correction2, the absorber
// ratio per bin as the opacity ratio kappa / kappa_nb), whatever that ratio. Up to a ratio of
// kMovedRatioJ it enters the neighbour's field directly, (1 - fc) v kappa / kappa_nb (dj);
// beyond it the moved photons, (1 - fc) v kappa (bounded by the ray's own), go to the
// two-limb field M (dm) and are divided by kappa_nb when the rates are formed. A neighbour
// with no absorber of the bin (kappa_nb = 0) leaves the share in the cell. Modes 1 and 3
// drop the removed share. dj and dm name the neighbour only when some bin uses them.
template <int NB, int PREC, bool THIN>
__device__ __forceinline__ int deposit_seg_corr(const TraceArgs& A, Ray<NB>& ray, const Seg& sg, const float kap[NB],
                                                const float kapn[NB], LaneStats& st, Dep<NB>& dep, Dep<NB>& dj,
                                                Dep<NB>& dm, float (&T)[NB], float (&esc)[NB])
{
    float v[NB];
    const int ev = attenuate_seg<NB, PREC, THIN>(A, ray, sg, kap, st, v, T, esc);
    bool use_j = false, use_m = false;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        float keep = v[b], mj = 0.0f, mm = 0.0f;
        if (sg.fc < 1.0f) {
            if (sg.nb == kNoCell) {
                keep = sg.fc * v[b];
            } else if (kapn[b] > 0.0f) {
                keep = sg.fc * v[b];
                const float moved = (1.0f - sg.fc) * v[b];
                if (kap[b] <= kMovedRatioJ * kapn[b]) {
                    mj = moved * (kap[b] / kapn[b]);
                    use_j = true;
                } else {
                    mm = moved * kap[b];
                    use_m = true;
                }
            }
        }
        dep.v[b] = keep;
        dj.v[b] = mj;
        dm.v[b] = mm;
    }
    dep.cell = sg.cell;
    dj.cell = use_j ? sg.nb : kNoCell;
    dm.cell = use_m ? sg.nb : kNoCell;
    return ev;
}

// Segments whose geometry is computed ahead of their deposits (opacity loads in flight
// per lane), and segments of each lane whose deposits the wave merges together: the merge
// window of four (256 crossings) fits the LDS of three waves per SIMD beside the family
// stacks, and the kernel's time follows the atomic items it leaves (1024^3 x 16384 sources:
// windows of two and ten segments ahead, 0.273 items per crossing and 715 ms; windows of four
// and eight ahead, 0.236 and 686 ms; twelve ahead, 682 ms). With thin spheres the extra state
// leaves room for eight only (twelve spill registers).
#ifndef ARC_SEG_AHEAD
#define ARC_SEG_AHEAD 12
#endif
constexpr int kSegAhead = ARC_SEG_AHEAD;
constexpr int kSegAheadThin = 8;
template <bool THIN>
constexpr int seg_ahead() { return THIN ? kSegAheadThin : kSegAhead; }
#ifndef ARC_DEP_WINDOW
#define ARC_DEP_WINDOW 4
#endif
constexpr int kDepWindow = ARC_DEP_WINDOW;

// Up to K crossings of one lane per pass: the geometry of K segments is computed first
// and their opacities are loaded together (K loads in flight per lane), then the
// segments are deposited in order; `deposit.add` is called once per kDepWindow segments by
// the whole wave. With THIN, a lane whose ray starts at or beyond its split radius (inside
// the source's thin sphere) splits at once, without a crossing.
// Returns the lane's final event of the pass (kContinue if the ray goes on).
template <int NB, int PREC, int K, bool THIN, class Depositor>
__device__ __forceinline__ int trace_pass(const TraceArgs& A, Ray<NB>& ray, bool active, LaneStats& st,
                                          Depositor& deposit)
{
    Seg sg[K];
    bool have[K];
    bool go = active;
    int ev = kContinue;
    if constexpr (THIN) {
        if (active && !(ray.thi < ray.tend)) {
            go = false;
            ev = kSplit;
            st.splits++;
        }
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
        have[j] = go;
        if (go) {
            sg[j] = geom_next<NB, PREC>(A, ray);
            go = sg[j].event == kContinue;
        }
    }
    // the gathers are issued unconditionally (cell 0 for a lane without the segment), so that
    // no branch separates them and each deposit waits for its own gather only
    float kap[K][NB];
#pragma unroll
    for (int j = 0; j < K; ++j) kappa_at<NB>(A, have[j] ? sg[j].cell : 0u, kap[j]);
    float T[NB], esc[NB];
    ray_transmission<NB, PREC>(ray, T);
    // every gather is consumed before the pass issues its first atomic (a wait for a gather
    // issued before an unknown number of atomics would wait for all of them)
    static_assert(K % kDepWindow == 0, "whole windows per pass");
    Dep<NB> dep[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        dep[j].cell = kNoCell;
        if (have[j] && ev == kContinue) ev = deposit_seg<NB, PREC, THIN>(A, ray, sg[j], kap[j], st, dep[j], T, esc);
    }
#pragma unroll
    for (int j0 = 0; j0 < K; j0 += kDepWindow) deposit.template add<kWhole>(dep + j0, A.J, A.nbp);
    book_escape<NB>(ev, esc, st);
    return ev;
}

// trace_pass with the geometric correction: up to K crossings per lane, the neighbours'
// opacities loaded with the cells'. The crossings' cells form windows, as without the
// correction; in mode 2 their neighbours' high limbs, then their low limbs, form two more.
#ifndef ARC_SEG_AHEAD_CORR
#define ARC_SEG_AHEAD_CORR 4
#endif
constexpr int kSegAheadCorr = ARC_SEG_AHEAD_CORR;
template <int NB, int PREC, int K, bool THIN, class Depositor>
__device__ __forceinline__ int trace_pass_corr(const TraceArgs& A, Ray<NB>& ray, bool active, LaneStats& st,
                                               Depositor& deposit)
{
    static_assert(K % kDepWindow == 0, "whole windows per pass");
    Seg sg[K];
    bool have[K];
    bool go = active;
    int ev = kContinue;
    if constexpr (THIN) {
        if (active && !(ray.thi < ray.tend)) {
            go = false;
            ev = kSplit;
            st.splits++;
        }
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
        have[j] = go;
        if (go) {
            sg[j] = geom_next<NB, PREC, true>(A, ray);
            go = sg[j].event == kContinue;
        }
    }
    float kap[K][NB], kapn[K][NB];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const bool hn = have[j] && sg[j].nb != kNoCell;
        kappa_at<NB>(A, have[j] ? sg[j].cell : 0u, kap[j]);
        kappa_at<NB>(A, hn ? sg[j].nb : 0u, kapn[j]);
#pragma unroll
        for (int b = 0; b < NB; ++b) kapn[j][b] = hn ? kapn[j][b] : 0.0f;
    }
    float T[NB], esc[NB];
    ray_transmission<NB, PREC>(ray, T);
    Dep<NB> dep[K], dj[K], dm[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        dep[j].cell = dj[j].cell = dm[j].cell = kNoCell;
        if (have[j] && ev == kContinue)
            ev = deposit_seg_corr<NB, PREC, THIN>(A, ray, sg[j], kap[j], kapn[j], st, dep[j], dj[j], dm[j], T, esc);
    }
#pragma unroll
    for (int j = 0; j < K; j += kDepWindow) {
        deposit.template add<kWhole>(dep + j, A.J, A.nbp);
        if (A.corr == 2) {
            deposit.template add<kWhole>(dj + j, A.J, A.nbp);
            deposit.template add<kMovedHi>(dm + j, A.M, 2 * A.nbp);
            deposit.template add<kMovedLo>(dm + j, A.M + A.nbp, 2 * A.nbp);
        }
    }
    book_escape<NB>(ev, esc, st);
    return ev;
}

// Child k of a split ray: next level, pixel 4p + k, same optical depth (section 2.1 iii c).
template <int NB>
__device__ __forceinline__ RayRec child_rec(const Ray<NB>& ray, int k)
{
    RayRec r;
    r.src = ray.src;
    const uint32_t level = (ray.lp >> kLevelShift) + 1u;
    r.lp = (level << kLevelShift) | (((ray.lp & kPixMask) << 2) + (uint32_t)k);
    r.pad0 = r.pad1 = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        r.tau[b] = b < NB ? ray.tau[b] : 0.0f;
        r.taulo[b] = b < NB ? ray.taulo[b] : 0.0f;
    }
    return r;
}

// A split ray's family record in memory (the persistent kernel's work items): the ray's id
// and optical depth, from which each of its four children is derived when it is taken.
template <int NB>
__device__ __forceinline__ RayRec family_item(const Ray<NB>& ray)
{
    RayRec r;
    r.src = ray.src;
    r.lp = ray.lp;
    r.pad0 = r.pad1 = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        r.tau[b] = b < NB ? ray.tau[b] : 0.0f;
        r.taulo[b] = b < NB ? ray.taulo[b] : 0.0f;
    }
    return r;
}

// A split ray's family record for the persistent kernel's stacks: the ray's id and optical
// depth, from which each of its four children is derived when it is taken.
template <int NB>
__device__ __forceinline__ StackRec<NB> family_rec(const Ray<NB>& ray)
{
    StackRec<NB> r;
    r.src = ray.src;
    r.lp = ray.lp;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        r.tau[b] = ray.tau[b];
        r.taulo[b] = ray.taulo[b];
    }
    return r;
}

// Child k of the split ray a family record holds (section 2.1 iii c).
template <int NB>
__device__ __forceinline__ StackRec<NB> family_child(const StackRec<NB>& f, int k)
{
    StackRec<NB> r = f;
    const uint32_t level = (f.lp >> kLevelShift) + 1u;
    r.lp = (level << kLevelShift) | (((f.lp & kPixMask) << 2) + (uint32_t)k);
    return r;
}

// Fixed-point deposition, called by all 64 lanes together, into an int64 field `base` with
// `stride` words per cell (the field J, or a limb of the moved-photon field M). Atomic adds
// cost per distinct cache line an instruction touches, so the NB bins of a cell are issued
// by NB adjacent lanes of the same instruction: instruction k, lane j adds bin (64k + j) mod
// NB of item (64k + j) / NB.
#ifndef ARC_DEDUP
#define ARC_DEDUP 1  // 0: every lane's crossing deposited on its own
#endif
constexpr int kDepSlots = 128 * kDepWindow;  // hash slots per wave
constexpr int kDepShift = kDepWindow == 1 ? 32 - 7 : (kDepWindow == 2 ? 32 - 8 : 32 - 9);
static_assert(kDepWindow == 1 || kDepWindow == 2 || kDepWindow == 4, "window of 1, 2 or 4 segments");

// Per-wave LDS space of the deduplicating deposit (item ids and ranks fit in a byte).
template <int NB>
struct DepScratch {
    uint32_t slot_cell[kDepSlots];
    uint8_t slot_id[kDepSlots];
    uint8_t slot_rank[kDepSlots];
    uint32_t cell[64 * kDepWindow];
    unsigned long long q[64 * kDepWindow][NB];
};

template <int NB, int LIMB>
__device__ __forceinline__ void deposit_wave_plain(const Dep<NB>& d, unsigned long long* base, int stride)
{
    const int lane = threadIdx.x & 63;
    long long qd[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) qd[b] = to_fixed<LIMB>(d.v[b]);
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        const int s = 64 * k + lane;
        const int item = s / NB, bin = s - item * NB;
        const uint32_t cell = (uint32_t)__shfl((int)d.cell, item, 64);
        long long q = 0;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const long long qb = __shfl(qd[b], item, 64);
            q = b == bin ? qb : q;
        }
        if (cell != kNoCell && q != 0) atomicAdd(base + (size_t)cell * (size_t)stride + (size_t)bin, (unsigned long long)q);
    }
}

// Crossings of the same cell, by several lanes and over the kDepWindow segments each lane
// brings, are first summed in LDS, so that each distinct cell costs one set of atomics
// (integer sums: the result is bitwise the same). Items hash their cell into a per-wave
// table; items whose cell owns its slot add into the slot's entry, items whose slot was
// taken by another cell go alone. LDS operations of one wave complete in issue order, and
// the racy table accesses are volatile so that each read really observes the wave's writes.
// Items whose integers are all zero are dropped. Returns the number of items issued
// (wave-uniform).
template <int NB, int LIMB>
__device__ __forceinline__ int deposit_wave_dedup(const Dep<NB>* d, DepScratch<NB>* S, unsigned long long* base,
                                                  int stride)
{
    constexpr int W = kDepWindow;
    bool v[W];
    bool anyv = false;
#pragma unroll
    for (int w = 0; w < W; ++w) anyv = anyv || d[w].cell != kNoCell;
    if (!__any(anyv)) return 0;
    long long q[W][NB];
    anyv = false;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        bool nz = false;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            q[w][b] = to_fixed<LIMB>(d[w].v[b]);
            nz = nz || q[w][b] != 0;
        }
        v[w] = d[w].cell != kNoCell && nz;
        anyv = anyv || v[w];
    }
    if (!__any(anyv)) return 0;
    // LDS-qualified views: through a generic pointer the accesses would be FLAT instructions,
    // which also wait for the wave's outstanding gathers and atomics
    volatile kLds uint32_t* slot_cell = (volatile kLds uint32_t*)S->slot_cell;
    volatile kLds uint8_t* slot_id = (volatile kLds uint8_t*)S->slot_id;
    volatile kLds uint8_t* slot_rank = (volatile kLds uint8_t*)S->slot_rank;
    volatile kLds uint32_t* st_cell = (volatile kLds uint32_t*)S->cell;
    volatile kLds unsigned long long* st_q = (volatile kLds unsigned long long*)&S->q[0][0];
    kLds unsigned long long* acc_q = (kLds unsigned long long*)&S->q[0][0];
    const int lane = threadIdx.x & 63;
    const uint64_t lt = __lanemask_lt();
    bool in[W], lead[W];
    uint32_t h[W];
#pragma unroll
    for (int w = 0; w < W; ++w) h[w] = (d[w].cell * 2654435761u) >> kDepShift;
#pragma unroll
    for (int w = 0; w < W; ++w)
        if (v[w]) slot_cell[h[w]] = d[w].cell;
#pragma unroll
    for (int w = 0; w < W; ++w) in[w] = v[w] && slot_cell[h[w]] == d[w].cell;
#pragma unroll
    for (int w = 0; w < W; ++w)
        if (in[w]) slot_id[h[w]] = (uint8_t)(64 * w + lane);
#pragma unroll
    for (int w = 0; w < W; ++w) lead[w] = in[w] && slot_id[h[w]] == (uint8_t)(64 * w + lane);
    int rank[W];
    int n = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const bool emit = lead[w] || (v[w] && !in[w]);
        const uint64_t em = __ballot(emit);
        rank[w] = emit ? n + __popcll(em & lt) : -1;
        n += __popcll(em);
    }
#pragma unroll
    for (int w = 0; w < W; ++w)
        if (lead[w]) slot_rank[h[w]] = (uint8_t)rank[w];
#pragma unroll
    for (int w = 0; w < W; ++w)
        if (rank[w] >= 0) {
            st_cell[rank[w]] = d[w].cell;
#pragma unroll
            for (int b = 0; b < NB; ++b) st_q[rank[w] * NB + b] = (unsigned long long)q[w][b];
        }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
#pragma unroll
    for (int w = 0; w < W; ++w)
        if (in[w] && !lead[w]) {
            const uint32_t r = slot_rank[h[w]];
#pragma unroll
            for (int b = 0; b < NB; ++b)
                if (q[w][b] != 0) __hip_atomic_fetch_add(acc_q + r * NB + b, (unsigned long long)q[w][b],
                                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    const int tot = n * NB;
    for (int s = lane; s < tot; s += 64) {
        const int item = s / NB, bin = s - item * NB;
        const uint32_t cell = st_cell[item];
        const unsigned long long q = st_q[item * NB + bin];
        if (q != 0) atomicAdd(base + (size_t)cell * (size_t)stride + (size_t)bin, q);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    return n;
}

// Wave-wide deposit of the crossings of a pass: add() once per window of kDepWindow
// segments, by every lane.
template <int NB>
struct Depositor {
    DepScratch<NB>* scratch;
    uint32_t items = 0;  // deposit items issued by this wave (wave-uniform)
    // the kDepWindow items d[0 .. kDepWindow) of every lane, as integers of limb LIMB
    template <int LIMB>
    __device__ void add(const Dep<NB>* d, unsigned long long* base, int stride)
    {
        if constexpr (ARC_DEDUP == 1) {
            items += (uint32_t)deposit_wave_dedup<NB, LIMB>(d, scratch, base, stride);
        } else {
#pragma unroll
            for (int w = 0; w < kDepWindow; ++w) deposit_wave_plain<NB, LIMB>(d[w], base, stride);
        }
    }
    __device__ void flush(const TraceArgs& A) const
    {
        if ((threadIdx.x & 63) == 0 && items) atomicAdd(&A.counters[kDeposits], (unsigned long long)items);
    }
};

// Wave-level reduction and flush of lane statistics into the global counters.
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ double wave_sum_f64(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int NB>
__device__ __forceinline__ void flush_stats(const TraceArgs& A, const LaneStats& st)
{
    const unsigned long long c = wave_sum_u64(st.crossings);
    const unsigned long long r = wave_sum_u64(st.rays);
    const unsigned long long s = wave_sum_u64(st.splits);
    const unsigned long long t = wave_sum_u64(st.terminated);
    const unsigned long long e = wave_sum_u64(st.escaped);
    double esc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) esc[b] = wave_sum_f64(st.esc[b]);
    if ((threadIdx.x & 63) == 0) {
        if (c) atomicAdd(&A.counters[kCrossings], c);
        if (r) atomicAdd(&A.counters[kRays], r);
        if (s) atomicAdd(&A.counters[kSplits], s);
        if (t) atomicAdd(&A.counters[kTerminated], t);
        if (e) atomicAdd(&A.counters[kEscapedRays], e);
#pragma unroll
        for (int b = 0; b < NB; ++b)
            if (esc[b] != 0.0) atomicAdd(&A.esc[b], esc[b]);
    }
}

}  // namespace arc
