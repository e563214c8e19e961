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

enum Counter : int {
    kCrossings = 0, kRays, kSplits, kTerminated, kEscapedRays, kSpills, kTreeCount, kQueueOverflow,
    kNumCounters
};

// Per-source constants (section 2.1 keeps the source position on chip; here it is a
// 32-byte record read through L2 once per ray).
struct __align__(16) SourceRec {
    float x, y, z, pad;   // position on the 2^-12 lattice (exact in FP32 up to 2048 cells)
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

struct TraceArgs {
    int nx, ny, nz, nb;
    int level0, lmax;
    float tsplit[kMaxLevels];  // split radius of each level; +inf from lmax on
    float tau_term;            // +inf = never terminate
    const float* kappa1;       // nb == 1: optical depth per cell length, [cell]
    const float4* kappa4;      // nb > 1: [cell] (bins in x, y, z, w)
    unsigned long long* J;     // fixed-point field [cell][nbp]
    int nbp;                   // padded bins per cell in J (1, 2 or 4)
    const SourceRec* src;
    const float4* dirs;        // HEALPix centres of every level, concatenated
    long long dir_off[kMaxLevels];
    double* esc;               // [kMaxBins] escaped photons in field units (times u_J: photons/s)
    unsigned long long* counters;  // [kNumCounters]
    unsigned long long* tree;  // optional record of every ray traced
    long long tree_cap;
};

// Per-lane ray state.
template <int NB>
struct Ray {
    float d[3];
    float xs[3];
    int c[3];
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
// roots at radius 0, children at the parent's radius with their own direction).
// Returns false (and books the escape) when the start point lies outside the grid.
template <int NB>
__device__ __forceinline__ bool ray_init(const TraceArgs& A, const RayRec& r, Ray<NB>& ray, LaneStats& st)
{
    ray.src = r.src;
    ray.lp = r.lp;
    const int level = (int)(r.lp >> kLevelShift);
    const uint32_t pix = r.lp & kPixMask;
    const float4 dv = A.dirs[A.dir_off[level] + pix];
    ray.d[0] = dv.x;
    ray.d[1] = dv.y;
    ray.d[2] = dv.z;
    const SourceRec s = A.src[r.src];
    ray.xs[0] = s.x;
    ray.xs[1] = s.y;
    ray.xs[2] = s.z;
    const float t0 = level == A.level0 ? 0.0f : A.tsplit[level - 1];
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
    bool inside = true;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        ray.c[i] = start_index(ray.xs[i], t0, ray.d[i]);
        const int n = i == 0 ? A.nx : (i == 1 ? A.ny : A.nz);
        inside = inside && ray.c[i] >= 0 && ray.c[i] < n;
    }
    if (!inside) {
#pragma unroll
        for (int b = 0; b < NB; ++b)
            st.esc[b] += (double)ray.w[b] * (double)expf(-(ray.tau[b] + ray.taulo[b]));
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

// One cell crossing (section 2.4): find the next x/y/z boundary (or the split radius),
// deposit S (1 - e^-dtau) into the cell as S ds g(dtau) in fixed point (eq:ion per bin),
// attenuate, then decide between continuing, splitting, terminating and escaping.
template <int NB, int PREC>
__device__ __forceinline__ int ray_step(const TraceArgs& A, Ray<NB>& ray, LaneStats& st)
{
    float a[3], e[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        if (ray.d[i] > 0.0f) {
            a[i] = (float)(ray.c[i] + 1) - ray.xs[i];
            e[i] = ray.d[i];
        } else if (ray.d[i] < 0.0f) {
            a[i] = ray.xs[i] - (float)ray.c[i];
            e[i] = -ray.d[i];
        } else {
            a[i] = 1.0f;
            e[i] = 0.0f;
        }
    }
    int w = -1;
    int mask = 0;
    bool at_end;
    float nhi, nlo;
    if constexpr (PREC == 0) {
        // exact decisions: t_i < t_j  <=>  a_i e_j < a_j e_i
#pragma unroll
        for (int i = 0; i < 3; ++i)
            if (e[i] > 0.0f && (w < 0 || cmp_prod(a[i], e[w], a[w], e[i]) < 0)) w = i;
#pragma unroll
        for (int i = 0; i < 3; ++i)
            if (e[i] > 0.0f && cmp_prod(a[i], e[w], a[w], e[i]) == 0) mask |= 1 << i;
        at_end = ray.tend < INFINITY && cmp_prod(ray.tend, e[w], a[w], 1.0f) <= 0;
        if (at_end) {
            nhi = ray.tend;
            nlo = 0.0f;
        } else {
            nhi = a[w] / e[w];
            nlo = __builtin_fmaf(-nhi, e[w], a[w]) / e[w];
        }
    } else {
        // plain FP32: compare rounded quotients
        float t[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            t[i] = e[i] > 0.0f ? a[i] / e[i] : INFINITY;
            if (e[i] > 0.0f && (w < 0 || t[i] < t[w])) w = i;
        }
#pragma unroll
        for (int i = 0; i < 3; ++i)
            if (e[i] > 0.0f && t[i] == t[w]) mask |= 1 << i;
        at_end = ray.tend <= t[w];
        nhi = at_end ? ray.tend : t[w];
        nlo = 0.0f;
    }
    // segment length ds = t_next - t_cur (double-float difference rounded to float)
    float ds;
    if constexpr (PREC == 0) {
        const float s = nhi - ray.thi;
        const float bb = s - nhi;
        const float err = (nhi - (s - bb)) + (-ray.thi - bb);
        ds = s + (err + (nlo - ray.tlo));
    } else {
        ds = nhi - ray.thi;
    }
    const uint32_t cell = (uint32_t)ray.c[0] + (uint32_t)A.nx * ((uint32_t)ray.c[1] + (uint32_t)A.ny * (uint32_t)ray.c[2]);
    float kap[NB];
    kappa_at<NB>(A, cell, kap);
    unsigned long long* Jc = A.J + (size_t)cell * (size_t)A.nbp;
    float dtau[NB];
    bool term = A.tau_term < INFINITY;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        dtau[b] = kap[b] * ds;
        const float taun = PREC == 0 ? ray.tau[b] + ray.taulo[b] : ray.tau[b];
        const float T = expf(-taun);
        const float g = dtau[b] > 0.0f ? -expm1f(-dtau[b]) / dtau[b] : 1.0f;
        const float v = ((ray.w[b] * T) * ds) * g;
        const long long q = __float2ll_rn(v);
        if (q) atomicAdd(Jc + b, (unsigned long long)q);
        if constexpr (PREC == 0) {
            const float s = ray.tau[b] + dtau[b];
            const float bb = s - ray.tau[b];
            ray.taulo[b] += (ray.tau[b] - (s - bb)) + (dtau[b] - bb);
            ray.tau[b] = s;
        } else {
            ray.tau[b] += dtau[b];
        }
        const float taup = PREC == 0 ? ray.tau[b] + ray.taulo[b] : ray.tau[b];
        term = term && taup >= A.tau_term && dtau[b] >= kDtauTermMin;
    }
    st.crossings++;
    ray.thi = nhi;
    ray.tlo = nlo;
    if (term) {
        // absorb what is left in this cell: field += remaining photons / opacity
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const float taup = PREC == 0 ? ray.tau[b] + ray.taulo[b] : ray.tau[b];
            const float v = (ray.w[b] * expf(-taup)) / kap[b];
            const long long q = __float2ll_rn(v);
            if (q) atomicAdd(Jc + b, (unsigned long long)q);
        }
        st.terminated++;
        return kTerminate;
    }
    if (at_end) {
        st.splits++;
        return kSplit;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
        if (mask & (1 << i)) ray.c[i] += ray.d[i] > 0.0f ? 1 : -1;
    const bool inside = ray.c[0] >= 0 && ray.c[0] < A.nx && ray.c[1] >= 0 && ray.c[1] < A.ny && ray.c[2] >= 0 &&
                        ray.c[2] < A.nz;
    if (!inside) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const float taup = PREC == 0 ? ray.tau[b] + ray.taulo[b] : ray.tau[b];
            st.esc[b] += (double)ray.w[b] * (double)expf(-taup);
        }
        st.escaped++;
        return kEscape;
    }
    return kContinue;
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
