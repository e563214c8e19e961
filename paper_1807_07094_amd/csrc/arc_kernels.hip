// arc_kernels.hip -- gfx950 kernels of libarc.
//
//   k_opacity          optical depth per cell length for every bin, field zeroing, input checks
//   k_healpix          FP32 HEALPix pixel centres of one level (computed in FP64)
//   k_sources          per-source table (lattice position, root-ray photon rate)
//   k_seed_roots       root rays of a range of sources (or of sources in a given order)
//   k_trace_rays       one ray per lane, rays of one HEALPix level (the per-level schedule)
//   k_trace_persistent every source in one launch: device work queue, wave-ballot refill,
//                      per-wave LDS ray stack with a private spill area in memory
//   k_thin_fill        optically thin approximation: point-source field inside each thin radius
//   k_finalize         fixed-point field -> photoionisation and photoheating rates
//   k_get_field        field copy in [bin][cell] order
#include <hip/hip_runtime.h>

#include <math.h>

#include "arc_kernels.h"

namespace arc {

namespace {

inline unsigned grid_for(size_t n, unsigned block, unsigned cap = 65536u)
{
    size_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

}  // namespace

// -------------------------------------------------------------------------------------
// Small utilities.
// -------------------------------------------------------------------------------------
__global__ void k_zero_u64(unsigned long long* p, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

__global__ void k_zero_f64(double* p, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

hipError_t launch_zero_u64(unsigned long long* p, size_t n, hipStream_t s)
{
    k_zero_u64<<<grid_for(n, 256), 256, 0, s>>>(p, n);
    return hipGetLastError();
}

// Two 64-bit sums of the fixed-point field, sum J[i] and sum J[i] (2 i + 1), modulo 2^64:
// equal fields give equal sums bit for bit (integer adds in any order).
__global__ __launch_bounds__(256) void k_field_checksum(const unsigned long long* J, size_t n, unsigned long long* out)
{
    unsigned long long s0 = 0, s1 = 0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        s0 += J[i];
        s1 += J[i] * (2ull * i + 1ull);
    }
    s0 = wave_sum_u64(s0);
    s1 = wave_sum_u64(s1);
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(out, s0);
        atomicAdd(out + 1, s1);
    }
}

hipError_t launch_field_checksum(const unsigned long long* J, size_t n, unsigned long long* out, hipStream_t s)
{
    k_field_checksum<<<grid_for(n, 256, 4096), 256, 0, s>>>(J, n, out);
    return hipGetLastError();
}

__global__ void k_set_u32(uint32_t* p, uint32_t v) { *p = v; }

// Counters of the work done before the persistent launch (its own work is the difference).
__global__ void k_snapshot_counters(unsigned long long* c)
{
    c[kCrossingsPre] = c[kCrossings];
    c[kDepositsPre] = c[kDeposits];
}

hipError_t launch_snapshot_counters(unsigned long long* counters, hipStream_t s)
{
    k_snapshot_counters<<<1, 1, 0, s>>>(counters);
    return hipGetLastError();
}

hipError_t launch_set_u32(uint32_t* p, uint32_t v, hipStream_t s)
{
    k_set_u32<<<1, 1, 0, s>>>(p, v);
    return hipGetLastError();
}

hipError_t launch_zero_f64(double* p, size_t n, hipStream_t s)
{
    k_zero_f64<<<grid_for(n, 256), 256, 0, s>>>(p, n);
    return hipGetLastError();
}

// -------------------------------------------------------------------------------------
// Opacity (section 2.2: tau per bin summed over HI, HeI, HeII) and field zeroing
// (section 2.1 step i). One pass over the grid; invalid inputs raise a flag.
// -------------------------------------------------------------------------------------
__device__ __forceinline__ uint32_t gather3(uint32_t m)
{
    return (m & 1u) | ((m >> 2) & 2u) | ((m >> 4) & 4u);
}

// The grid is handled in regions of 32 x 8 x 8 cells: four consecutive 8^3 blocks of the
// blocked layout, and 64 x-rows of 32 cells (whole 128-byte lines) of the linear arrays. One
// workgroup per region transposes between the two orders through LDS, so that both sides
// are read and written in whole lines.
constexpr int kRegionCells = 2048;

struct Region {
    uint32_t x0, y0, z0;  // first cell
    uint32_t base;        // blocked index of its first cell
    uint32_t cells;       // cells of the blocked layout it covers (512 per block)
};

__device__ __forceinline__ Region region_of(uint32_t r, int nbx8, int nby8)
{
    const uint32_t nrx = ((uint32_t)nbx8 + 3u) / 4u;
    const uint32_t rx = r % nrx, by = (r / nrx) % (uint32_t)nby8, bz = r / (nrx * (uint32_t)nby8);
    Region g;
    g.x0 = rx * 32u;
    g.y0 = by * 8u;
    g.z0 = bz * 8u;
    g.base = ((bz * (uint32_t)nby8 + by) * (uint32_t)nbx8 + 4u * rx) << 9;
    g.cells = min(4u, (uint32_t)nbx8 - 4u * rx) << 9;
    return g;
}

// Position l in [0, 2048) of the region's linear order (x fastest) <-> its offset in the
// region's blocked range.
__device__ __forceinline__ uint32_t region_blocked_offset(uint32_t l)
{
    const uint32_t xl = l & 31u, yl = (l >> 5) & 7u, zl = l >> 8;
    return ((xl >> 3) << 9) | spread3(xl & 7u) | (spread3(yl) << 1) | (spread3(zl) << 2);
}

template <int NB>
__global__ __launch_bounds__(256) void k_opacity(OpacityArgs a)
{
    __shared__ float4 st[kRegionCells];
    const uint32_t nreg = (((uint32_t)a.nbx8 + 3u) / 4u) * (uint32_t)a.nby8 * (uint32_t)a.nbz8;
    for (uint32_t r = blockIdx.x; r < nreg; r += gridDim.x) {
        const Region g = region_of(r, a.nbx8, a.nby8);
        // linear reads along x-rows, opacities into LDS at their blocked offsets
        for (uint32_t l = threadIdx.x; l < (uint32_t)kRegionCells; l += blockDim.x) {
            const uint32_t x = g.x0 + (l & 31u), y = g.y0 + ((l >> 5) & 7u), z = g.z0 + (l >> 8);
            float k[kMaxBins] = {0.0f, 0.0f, 0.0f, 0.0f};
            if (x < (uint32_t)a.nx && y < (uint32_t)a.ny && z < (uint32_t)a.nz) {
                const uint32_t c = x + (uint32_t)a.nx * (y + (uint32_t)a.ny * z);
                const float n = a.n_h[c], xh = a.x_hi[c], x1 = a.x_hei[c], x2 = a.x_heii[c];
                const bool ok = isfinite(n) && n > 0.0f && xh >= 0.0f && xh <= 1.0f && x1 >= 0.0f && x1 <= 1.0f &&
                                x2 >= 0.0f && x2 <= 1.0f;
                if (!ok) atomicOr(a.errflag, 1);
#pragma unroll
                for (int bb = 0; bb < NB; ++bb)
                    k[bb] = (float)(a.L * (double)n *
                                    (a.sigma[bb][0] * (double)xh +
                                     a.y * (a.sigma[bb][1] * (double)x1 + a.sigma[bb][2] * (double)x2)));
            }
            const uint32_t o = region_blocked_offset(l);
            if (o < g.cells) st[o] = make_float4(k[0], k[1], k[2], k[3]);
        }
        __syncthreads();
        // contiguous writes of the blocked range: opacity, and the zeroed field
        for (uint32_t o = threadIdx.x; o < g.cells; o += blockDim.x) {
            if constexpr (NB == 1)
                a.kappa1[g.base + o] = st[o].x;
            else
                a.kappa4[g.base + o] = st[o];
        }
        const uint32_t words = g.cells * (uint32_t)a.nbp;
        for (uint32_t w = threadIdx.x; w < words; w += blockDim.x) a.J[(size_t)g.base * a.nbp + w] = 0ull;
        if (a.M)
            for (uint32_t w = threadIdx.x; w < 2u * words; w += blockDim.x) a.M[2ull * g.base * a.nbp + w] = 0ull;
        __syncthreads();
    }
}

hipError_t launch_opacity(const OpacityArgs& a, hipStream_t s)
{
    const unsigned g = grid_for((size_t)((a.nbx8 + 3) / 4) * a.nby8 * a.nbz8, 1, 1u << 16);
    switch (a.nb) {
        case 1: k_opacity<1><<<g, 256, 0, s>>>(a); break;
        case 2: k_opacity<2><<<g, 256, 0, s>>>(a); break;
        case 3: k_opacity<3><<<g, 256, 0, s>>>(a); break;
        default: k_opacity<4><<<g, 256, 0, s>>>(a); break;
    }
    return hipGetLastError();
}

// -------------------------------------------------------------------------------------
// HEALPix pixel centres, nested scheme (Gorski et al. 2005). The base faces form three
// rows of four; inside a face the nested index interleaves the bits of the face
// coordinates (x even, y odd). The ring index and the position inside the ring give
// z exactly as a ratio of integers and phi as an exact multiple of pi/2.
// -------------------------------------------------------------------------------------
__device__ __forceinline__ uint64_t compact_bits(uint64_t v)
{
    v &= 0x5555555555555555ull;
    v = (v | (v >> 1)) & 0x3333333333333333ull;
    v = (v | (v >> 2)) & 0x0F0F0F0F0F0F0F0Full;
    v = (v | (v >> 4)) & 0x00FF00FF00FF00FFull;
    v = (v | (v >> 8)) & 0x0000FFFF0000FFFFull;
    v = (v | (v >> 16)) & 0x00000000FFFFFFFFull;
    return v;
}

__global__ __launch_bounds__(256) void k_healpix(int level, float4* out)
{
    const long long ns = 1ll << level;
    const long long per_face = ns * ns;
    const long long npix = 12 * per_face;
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < npix;
         p += (long long)gridDim.x * blockDim.x) {
        const int face = (int)(p / per_face);
        const uint64_t q = (uint64_t)(p - face * per_face);
        const long long fx = (long long)compact_bits(q), fy = (long long)compact_bits(q >> 1);
        const int row = face >> 2, col = face & 3;
        // the face's lowest corner sits on ring (row + 2) Nside
        const long long ring = (row + 2) * ns - fx - fy - 1;
        long long nr, num_z, den_z;
        int shift;
        if (ring < ns) {
            nr = ring;
            shift = 0;
            num_z = 3 * ns * ns - nr * nr;
            den_z = 3 * ns * ns;
        } else if (ring > 3 * ns) {
            nr = 4 * ns - ring;
            shift = 0;
            num_z = -(3 * ns * ns - nr * nr);
            den_z = 3 * ns * ns;
        } else {
            nr = ns;
            shift = (int)((ring - ns) & 1);
            num_z = 2 * (2 * ns - ring);
            den_z = 3 * ns;
        }
        const double z = (double)num_z / (double)den_z;
        // longitude index of the face corner, in units of pi/4: odd in the polar rows
        const long long lon0 = 2 * col + (row == 1 ? 0 : 1);
        long long j = (lon0 * nr + fx - fy + 1 + shift) / 2;
        if (j > 4 * nr) j -= 4 * nr;
        if (j < 1) j += 4 * nr;
        // phi / (pi/2) = (2j - 1 - shift) / (2 nr)
        const long long num = 2 * j - 1 - shift, den = 2 * nr;
        const long long quad = num / den, rem = num - quad * den;
        double sa, ca;
        sincospi(0.5 * ((double)rem / (double)den), &sa, &ca);
        double cx, cy;
        if (quad == 0) {
            cx = ca;
            cy = sa;
        } else if (quad == 1) {
            cx = -sa;
            cy = ca;
        } else if (quad == 2) {
            cx = -ca;
            cy = -sa;
        } else {
            cx = sa;
            cy = -ca;
        }
        const double st = sqrt((1.0 - z) * (1.0 + z));
        out[p] = make_float4((float)(st * cx), (float)(st * cy), (float)z, 0.0f);
    }
}

hipError_t launch_healpix(int level, float4* out, hipStream_t s)
{
    const long long npix = 12ll << (2 * level);
    k_healpix<<<grid_for((size_t)npix, 256, 1u << 20), 256, 0, s>>>(level, out);
    return hipGetLastError();
}

// -------------------------------------------------------------------------------------
// Source table and root rays (section 2.1 iii a: rays start at radius 0 with zero
// optical depth; section 2.4: each ray carries an equal share of the source's photons).
// -------------------------------------------------------------------------------------
struct ScaleArg {
    double f[kMaxBins];
};

__global__ void k_sources(int n, const double* pos, const double* ndot, const double* r_thin, ScaleArg sc, int nb,
                          SourceRec* out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    SourceRec r;
    r.x = (float)pos[3 * i];
    r.y = (float)pos[3 * i + 1];
    r.z = (float)pos[3 * i + 2];
    r.r_thin = r_thin ? (float)r_thin[i] : 0.0f;
#pragma unroll
    for (int b = 0; b < kMaxBins; ++b) r.scale[b] = b < nb ? (float)(ndot[i] * sc.f[b]) : 0.0f;
    out[i] = r;
}

hipError_t launch_sources(int n, const double* pos, const double* ndot, const double* r_thin,
                          const double* frac_over_12uj, int nb, SourceRec* out, hipStream_t s)
{
    ScaleArg sc;
    for (int b = 0; b < kMaxBins; ++b) sc.f[b] = b < nb ? frac_over_12uj[b] : 0.0;
    if (n > 0) k_sources<<<grid_for(n, 256), 256, 0, s>>>(n, pos, ndot, r_thin, sc, nb, out);
    return hipGetLastError();
}

// -------------------------------------------------------------------------------------
// Optically thin approximation (section 2.6): every cell whose centre lies within a source's
// thin radius R receives that source's point-source field S_b / (4 pi r^2), r the centre's
// distance in cells and at least half a cell (the point formula diverges in the source's own
// cell), in the field's integers. Block (i, j) covers part j of source i's bounding box.
// -------------------------------------------------------------------------------------
template <int NB>
__global__ __launch_bounds__(256) void k_thin_fill(ThinFillArgs a)
{
    const int i = blockIdx.x;
    double absorbed = 0.0;
    const double R = (double)(float)a.r_thin[i];
    if (R > 0.0) {
        const double xs[3] = {a.pos[3 * i], a.pos[3 * i + 1], a.pos[3 * i + 2]};
        const int n[3] = {a.nx, a.ny, a.nz};
        int lo[3], ext[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            lo[d] = max(0, (int)floor(xs[d] - R));
            const int hi = min(n[d] - 1, (int)ceil(xs[d] + R));
            ext[d] = max(0, hi - lo[d] + 1);
        }
        const double ndot = a.ndot[i];
        const size_t total = (size_t)ext[0] * ext[1] * ext[2];
        const size_t stride = (size_t)gridDim.y * blockDim.x;
        for (size_t l = (size_t)blockIdx.y * blockDim.x + threadIdx.x; l < total; l += stride) {
            const int cx = lo[0] + (int)(l % ext[0]);
            const int cy = lo[1] + (int)((l / ext[0]) % ext[1]);
            const int cz = lo[2] + (int)(l / ((size_t)ext[0] * ext[1]));
            const double dx = (double)cx + 0.5 - xs[0], dy = (double)cy + 0.5 - xs[1], dz = (double)cz + 0.5 - xs[2];
            const double r2 = dx * dx + dy * dy + dz * dz;  // exact: lattice positions
            if (!(r2 < R * R)) continue;
            const double inv = ndot / fmax(r2, 0.25);
            const uint32_t cell = blocked_index(cx, cy, cz, a.nbx8, a.nby8);
            float k[NB];
            if constexpr (NB == 1) {
                k[0] = a.kappa1[cell];
            } else {
                const float4 v = a.kappa4[cell];
                k[0] = v.x;
                k[1] = v.y;
                if constexpr (NB > 2) k[2] = v.z;
                if constexpr (NB > 3) k[3] = v.w;
            }
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const long long q = llrint(inv * a.coef[b]);
                if (q != 0) atomicAdd(a.J + (size_t)cell * a.nbp + b, (unsigned long long)q);
                absorbed += (double)q * a.uj[b] * (double)k[b];
            }
        }
    }
    absorbed = wave_sum_f64(absorbed);
    if ((threadIdx.x & 63) == 0 && absorbed != 0.0) atomicAdd(a.absorbed_thin, absorbed);
}

hipError_t launch_thin_fill(const ThinFillArgs& a, hipStream_t s)
{
    if (a.nsrc <= 0) return hipSuccess;
    const dim3 g((unsigned)a.nsrc, (unsigned)a.parts);
    switch (a.nb) {
        case 1: k_thin_fill<1><<<g, 256, 0, s>>>(a); break;
        case 2: k_thin_fill<2><<<g, 256, 0, s>>>(a); break;
        case 3: k_thin_fill<3><<<g, 256, 0, s>>>(a); break;
        default: k_thin_fill<4><<<g, 256, 0, s>>>(a); break;
    }
    return hipGetLastError();
}

__global__ void k_fill_u32(uint32_t* p, uint32_t n, uint32_t v)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t n, uint32_t v, hipStream_t s)
{
    if (n > 0) k_fill_u32<<<grid_for(n, 256, 1024), 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}

__global__ void k_seed_roots(uint32_t first_src, uint32_t nsrc, int level0, const uint32_t* order, RayRec* out)
{
    const uint32_t npix = 12u << (2 * level0);
    const size_t n = (size_t)nsrc * npix;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        RayRec r;
        const uint32_t k = (uint32_t)(i / npix);
        r.src = order ? order[k] : first_src + k;
        r.lp = ((uint32_t)level0 << kLevelShift) | (uint32_t)(i % npix);
        r.pad0 = r.pad1 = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) r.tau[b] = r.taulo[b] = 0.0f;
        out[i] = r;
    }
}

hipError_t launch_seed_roots(uint32_t first_src, uint32_t nsrc, int level0, const uint32_t* order, RayRec* out,
                             hipStream_t s)
{
    const size_t n = (size_t)nsrc * (12u << (2 * level0));
    k_seed_roots<<<grid_for(n, 256), 256, 0, s>>>(first_src, nsrc, level0, order, out);
    return hipGetLastError();
}

// -------------------------------------------------------------------------------------
// Per-level schedule (section 2.1 iii b/c): one ray per lane, traced until it splits,
// terminates or leaves the grid; splitting lanes write their four children into the
// next level's array, one slot reservation per wave.
// -------------------------------------------------------------------------------------
template <int NB, int PREC, bool CORR, bool THIN>
__global__ __launch_bounds__(256) void k_trace_rays(TraceArgs A, const RayRec* __restrict__ in,
                                                    const uint32_t* n_in_dev, uint32_t n_in_host,
                                                    RayRec* __restrict__ out, uint32_t* n_out, uint32_t out_cap,
                                                    int fam_out)
{
    const uint32_t n_in = n_in_dev ? *n_in_dev : n_in_host;
    __shared__ DepScratch<NB> dscr[4];
    Depositor<NB> dep{dscr + (threadIdx.x >> 6)};
    LaneStats st;
    st.clear();
    const int lane = threadIdx.x & 63;
    const uint64_t lt = __lanemask_lt();
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t base = blockIdx.x * blockDim.x; base < n_in; base += stride) {
        const uint32_t i = base + threadIdx.x;
        int ev = kEscape;
        Ray<NB> ray;
        bool act = false;
        if (i < n_in) {
            const RayRec r = in[i];
            record_tree<NB>(A, r.src, r.lp);
            act = ray_init<NB, THIN>(A, r, ray, st);
        }
        // a few crossings per lane per pass; the wave deposits each crossing together
        while (__any(act)) {
            int e;
            if constexpr (CORR)
                e = trace_pass_corr<NB, PREC, kSegAheadCorr, THIN>(A, ray, act, st, dep);
            else
                e = trace_pass<NB, PREC, seg_ahead<THIN>(), THIN>(A, ray, act, st, dep);
            if (act && e != kContinue) {
                ev = e;
                act = false;
            }
        }
        // a split ray leaves its four children, or (fam_out: the persistent launch's work
        // items) one family record from which they are derived
        const uint64_t m = __ballot(ev == kSplit);
        if (m) {
            const uint32_t per = fam_out ? 1u : 4u;
            const int leader = __ffsll((unsigned long long)m) - 1;
            uint32_t wbase = 0;
            if (lane == leader) wbase = atomicAdd(n_out, per * (uint32_t)__popcll(m));
            wbase = __shfl(wbase, leader, 64);
            if (ev == kSplit) {
                const uint32_t slot = wbase + per * (uint32_t)__popcll(m & lt);
                if (slot + per <= out_cap) {
                    if (fam_out) {
                        out[slot] = family_item<NB>(ray);
                    } else {
#pragma unroll
                        for (int k = 0; k < 4; ++k) out[slot + k] = child_rec<NB>(ray, k);
                    }
                } else {
                    atomicAdd(&A.counters[kQueueOverflow], 1ull);
                }
            }
        }
    }
    flush_stats<NB>(A, st);
    dep.flush(A);
}

template <int NB>
static hipError_t trace_rays_nb(const TraceArgs& A, int prec, const RayRec* in, const uint32_t* n_in_dev,
                                uint32_t n_in, RayRec* out, uint32_t* n_out, uint32_t out_cap, int fam_out,
                                hipStream_t s)
{
    const unsigned g = grid_for(n_in, 256, 1u << 16);
    const bool thin = A.r_out != nullptr;
    if (prec == 0 && A.corr && thin)
        k_trace_rays<NB, 0, true, true><<<g, 256, 0, s>>>(A, in, n_in_dev, n_in, out, n_out, out_cap, fam_out);
    else if (prec == 0 && A.corr)
        k_trace_rays<NB, 0, true, false><<<g, 256, 0, s>>>(A, in, n_in_dev, n_in, out, n_out, out_cap, fam_out);
    else if (prec == 0 && thin)
        k_trace_rays<NB, 0, false, true><<<g, 256, 0, s>>>(A, in, n_in_dev, n_in, out, n_out, out_cap, fam_out);
    else if (prec == 0)
        k_trace_rays<NB, 0, false, false><<<g, 256, 0, s>>>(A, in, n_in_dev, n_in, out, n_out, out_cap, fam_out);
    else
        k_trace_rays<NB, 1, false, false><<<g, 256, 0, s>>>(A, in, n_in_dev, n_in, out, n_out, out_cap, fam_out);
    return hipGetLastError();
}

hipError_t launch_trace_rays(const TraceArgs& A, int prec, const RayRec* in, const uint32_t* n_in_dev, uint32_t n_in,
                             RayRec* out, uint32_t* n_out, uint32_t out_cap, int fam_out, hipStream_t s)
{
    switch (A.nb) {
        case 1: return trace_rays_nb<1>(A, prec, in, n_in_dev, n_in, out, n_out, out_cap, fam_out, s);
        case 2: return trace_rays_nb<2>(A, prec, in, n_in_dev, n_in, out, n_out, out_cap, fam_out, s);
        case 3: return trace_rays_nb<3>(A, prec, in, n_in_dev, n_in, out, n_out, out_cap, fam_out, s);
        default: return trace_rays_nb<4>(A, prec, in, n_in_dev, n_in, out, n_out, out_cap, fam_out, s);
    }
}

// -------------------------------------------------------------------------------------
// Batched schedule: after the first levels have been traced level by level (so that there
// are enough independent subtrees), one persistent launch traces every remaining subtree.
//
// Each wave keeps 64 rays in flight, one per lane, and advances them up to seg_ahead crossings
// per iteration. A splitting lane pushes one family record (the ray, from which its four children
// are derived) and goes idle with the lanes whose ray ended; once at least `refill` lanes are
// idle they are refilled with whole families from the wave's LDS stack, then from the wave's
// private spill area, and when both are empty from the global work queue (one atomic per
// refill; its items are the family records the last level-synchronous launch left, or single
// root rays when there was none); every new ray of the iteration is started in one place. The
// stack's top holds the latest splits, so the four children of a ray, and the children of rays
// that split together, enter together and cross the same cells in the same passes: the wave's
// deposit merge then sums their crossings of a cell into one atomic item (the int64 atomics in
// L2 and the VALU issue share the limit of this kernel). The LDS stack is a ring: when it would overflow, its
// oldest entries move to the top of the spill area, so the pair behaves as one LIFO stack and
// the wave works depth first. Waves share nothing but the work-queue head, so each wave ends
// when the queue is drained and its own stacks are empty.
// -------------------------------------------------------------------------------------
// The stacks live in dynamic LDS: stack_cap family records per wave, a power of two of at
// least 64 (a split round of all lanes must fit the ring), chosen at launch (the autotuner's
// LDS stack depth).
extern __shared__ __align__(16) unsigned char arc_stack_lds[];

template <int NB, int PREC, int WPB, bool CORR, bool THIN>
__global__ __launch_bounds__(WPB * 64, NB <= 3 ? 3 : 2) void k_trace_persistent(TraceArgs A, const RayRec* __restrict__ items,
                                                               const uint32_t* n_items_dev, uint32_t* head,
                                                               RayRec* __restrict__ spill_all, uint32_t spill_cap,
                                                               int refill, int fam, int stack_cap)
{
    using SRec = StackRec<NB>;
    SRec* lds = reinterpret_cast<SRec*>(arc_stack_lds);
    const int cmask = stack_cap - 1;
    __shared__ DepScratch<NB> dscr[WPB];
    const int wid = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const uint64_t lt = __lanemask_lt();
    const uint32_t n_items = *n_items_dev;
    SRec* stk = lds + wid * stack_cap;
    Depositor<NB> dep{dscr + wid};
    // the spill area is sized in full records; compact records fit in it
    SRec* spill = reinterpret_cast<SRec*>(spill_all + (size_t)(blockIdx.x * WPB + wid) * spill_cap);
    int base = 0;          // ring start (oldest entry), wave-uniform
    int top = 0;           // entries in the ring, wave-uniform
    uint32_t nspill = 0;   // wave-uniform
    bool qdone = false;    // wave-uniform
    uint32_t spilled = 0;
    bool has = false;
    Ray<NB> ray;
    LaneStats st;
    st.clear();
    for (;;) {
        // one pass over the lanes that hold a ray
        int ev = kContinue;
        if (__any(has)) {
            if constexpr (CORR)
                ev = trace_pass_corr<NB, PREC, kSegAheadCorr, THIN>(A, ray, has, st, dep);
            else
                ev = trace_pass<NB, PREC, seg_ahead<THIN>(), THIN>(A, ray, has, st, dep);
        }
        // splits: one family record each
        const uint64_t sp = __ballot(ev == kSplit);
        if (sp) {
            const int need = __popcll(sp);
            if (top + need > stack_cap) {
                // move the oldest entries to the top of the spill area
                const int m = top + need - stack_cap;
                for (int i = lane; i < m; i += 64) {
                    const uint32_t g = nspill + (uint32_t)i;
                    if (g < spill_cap)
                        spill[g] = stk[(base + i) & cmask];
                    else
                        atomicAdd(&A.counters[kQueueOverflow], 1ull);
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                spilled += (uint32_t)m;
                nspill = min(spill_cap, nspill + (uint32_t)m);
                base = (base + m) & cmask;
                top -= m;
            }
            if (ev == kSplit) stk[(base + top + __popcll(sp & lt)) & cmask] = family_rec<NB>(ray);
            top += need;
        }
        if (ev != kContinue) has = false;
        // refill of the idle lanes: whole families from the LDS stack, then from the spill
        // area, then (both empty) single roots from the work queue; four lanes per family
        const uint64_t idle = __ballot(!has);
        const int nidle = __popcll(idle);
        const bool pending = top > 0 || nspill > 0 || !qdone;
        SRec r;
        bool got = false;
        if (nidle > 0 && pending && (nidle >= refill || nidle == 64)) {
            const int rank = __popcll(idle & lt);
            const int nfam = min(nidle >> 2, top);
            if (!has && rank < 4 * nfam) {
                r = family_child<NB>(stk[(base + top - 1 - (rank >> 2)) & cmask], rank & 3);
                got = true;
            }
            top -= nfam;
            int used = 4 * nfam;
            const int fam2 = min((nidle - used) >> 2, (int)nspill);
            if (fam2 > 0) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                if (!has && rank >= used && rank < used + 4 * fam2) {
                    r = family_child<NB>(spill[nspill - 1u - (uint32_t)((rank - used) >> 2)], (rank - used) & 3);
                    got = true;
                }
                nspill -= (uint32_t)fam2;
                used += 4 * fam2;
            }
            // work items: single rays, or (fam) family records taken whole, four lanes each
            const int rem = nidle - used;
            const uint32_t want = fam ? (uint32_t)(rem >> 2) : (uint32_t)rem;
            if (want > 0 && top == 0 && nspill == 0 && !qdone) {
                const int take = used;
                uint32_t b0 = 0;
                if (lane == 0) b0 = atomicAdd(head, want);
                b0 = __shfl(b0, 0, 64);
                if (b0 >= n_items) {
                    qdone = true;
                } else {
                    const uint32_t avail = min(want, n_items - b0);
                    const int lanes = fam ? 4 * (int)avail : (int)avail;
                    if (!has && rank >= take && rank < take + lanes) {
                        const int q = rank - take;
                        const RayRec& it = items[b0 + (uint32_t)(fam ? q >> 2 : q)];
                        r.src = it.src;
                        r.lp = it.lp;
#pragma unroll
                        for (int b = 0; b < NB; ++b) {
                            r.tau[b] = it.tau[b];
                            r.taulo[b] = it.taulo[b];
                        }
                        if (fam) r = family_child<NB>(r, q & 3);
                        got = true;
                    }
                    if (b0 + want >= n_items) qdone = true;
                }
            }
        }
        if (got) {
            record_tree<NB>(A, r.src, r.lp);
            has = ray_init<NB, THIN>(A, r, ray, st);
        }
        if (!__any(has) && top == 0 && nspill == 0 && qdone) break;
    }
    flush_stats<NB>(A, st);
    dep.flush(A);
    if (lane == 0 && spilled) atomicAdd(&A.counters[kSpills], (unsigned long long)spilled);
}

constexpr int kMaxWavesPerBlock = 8;

int persistent_max_waves() { return kMaxWavesPerBlock; }

// LDS of a persistent workgroup of `waves` waves: the stacks (dynamic) and the deposit scratch.
template <int NB>
size_t persistent_stack_bytes(int waves, int stack_cap) { return (size_t)waves * stack_cap * sizeof(StackRec<NB>); }
template <int NB>
size_t persistent_lds_bytes(int waves, int stack_cap)
{
    return persistent_stack_bytes<NB>(waves, stack_cap) + (size_t)waves * sizeof(DepScratch<NB>);
}
constexpr size_t kLdsPerCu = 163840;

template <int NB, int PREC, bool CORR, bool THIN>
static hipError_t persistent_nb(const TraceArgs& A, const RayRec* items, const uint32_t* n_items, uint32_t* head,
                                RayRec* spill, uint32_t spill_cap, int blocks, int waves, int refill, int fam,
                                int stack_cap, hipStream_t s)
{
    // eight waves only where their LDS fits a compute unit (else four, in twice the blocks)
    if (waves == 8 && persistent_lds_bytes<NB>(8, stack_cap) > kLdsPerCu) {
        waves = 4;
        blocks *= 2;
    }
    const size_t dyn = persistent_stack_bytes<NB>(waves, stack_cap);
    switch (waves) {
        case 1: k_trace_persistent<NB, PREC, 1, CORR, THIN><<<blocks, 64, dyn, s>>>(A, items, n_items, head, spill, spill_cap, refill, fam, stack_cap); break;
        case 2: k_trace_persistent<NB, PREC, 2, CORR, THIN><<<blocks, 128, dyn, s>>>(A, items, n_items, head, spill, spill_cap, refill, fam, stack_cap); break;
        case 4: k_trace_persistent<NB, PREC, 4, CORR, THIN><<<blocks, 256, dyn, s>>>(A, items, n_items, head, spill, spill_cap, refill, fam, stack_cap); break;
        default: k_trace_persistent<NB, PREC, 8, CORR, THIN><<<blocks, 512, dyn, s>>>(A, items, n_items, head, spill, spill_cap, refill, fam, stack_cap); break;
    }
    return hipGetLastError();
}

template <int NB>
static hipError_t persistent_variant(const TraceArgs& A, int prec, const RayRec* items, const uint32_t* n_items,
                                     uint32_t* head, RayRec* spill, uint32_t spill_cap, int blocks, int waves,
                                     int refill, int fam, int stack_cap, hipStream_t s)
{
    const bool thin = A.r_out != nullptr;
    if (prec != 0) return persistent_nb<NB, 1, false, false>(A, items, n_items, head, spill, spill_cap, blocks, waves, refill, fam, stack_cap, s);
    if (A.corr && thin) return persistent_nb<NB, 0, true, true>(A, items, n_items, head, spill, spill_cap, blocks, waves, refill, fam, stack_cap, s);
    if (A.corr) return persistent_nb<NB, 0, true, false>(A, items, n_items, head, spill, spill_cap, blocks, waves, refill, fam, stack_cap, s);
    if (thin) return persistent_nb<NB, 0, false, true>(A, items, n_items, head, spill, spill_cap, blocks, waves, refill, fam, stack_cap, s);
    return persistent_nb<NB, 0, false, false>(A, items, n_items, head, spill, spill_cap, blocks, waves, refill, fam, stack_cap, s);
}

hipError_t launch_trace_persistent(const TraceArgs& A, int prec, const RayRec* items, const uint32_t* n_items,
                                   uint32_t* head, RayRec* spill, uint32_t spill_cap, int blocks, int waves,
                                   int refill, int fam, int stack_cap, hipStream_t s)
{
    if (stack_cap != 64 && stack_cap != 128 && stack_cap != 256) return hipErrorInvalidValue;
    switch (A.nb) {
        case 1: return persistent_variant<1>(A, prec, items, n_items, head, spill, spill_cap, blocks, waves, refill, fam, stack_cap, s);
        case 2: return persistent_variant<2>(A, prec, items, n_items, head, spill, spill_cap, blocks, waves, refill, fam, stack_cap, s);
        case 3: return persistent_variant<3>(A, prec, items, n_items, head, spill, spill_cap, blocks, waves, refill, fam, stack_cap, s);
        default: return persistent_variant<4>(A, prec, items, n_items, head, spill, spill_cap, blocks, waves, refill, fam, stack_cap, s);
    }
}

// -------------------------------------------------------------------------------------
// Request-rate probes (measurement only): random single-sector int64 atomic deposits and
// random 16-byte gathers over the trace's own buffers, to hold the trace kernel against.
// Cells come from a counter-based hash (splitmix64 finaliser) of the item index.
// -------------------------------------------------------------------------------------
__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Item i adds 1 to the NB bins of cell hash(i) mod ncell, its bins in NB adjacent lanes of
// one instruction (as the trace's deposits are issued).
__global__ __launch_bounds__(256) void k_probe_deposits(unsigned long long* J, int nbp, int nb, uint64_t ncell,
                                                         uint64_t items, uint64_t seed)
{
    const uint64_t lanes = items * (uint64_t)nb;
    for (uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; s < lanes; s += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t item = s / (uint64_t)nb;
        const int bin = (int)(s - item * (uint64_t)nb);
        const uint64_t cell = mix64(seed + item) % ncell;
        atomicAdd(J + cell * (uint64_t)nbp + bin, 1ull);
    }
}

// Item i reads the 16-byte opacity record of cell hash(i) mod ncell; the sum of what a lane
// read is stored only if it is negative (never, opacities are >= 0), so the reads stay.
__global__ __launch_bounds__(256) void k_probe_gathers(const float4* kappa, uint64_t ncell, uint64_t items,
                                                        uint64_t seed, float* sink)
{
    float acc = 0.0f;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < items; i += (uint64_t)gridDim.x * blockDim.x) {
        const float4 v = kappa[mix64(seed + i) % ncell];
        acc += v.x + v.y + v.z;
    }
    if (acc < 0.0f) sink[0] = acc;
}

hipError_t launch_probe_deposits(unsigned long long* J, int nbp, int nb, uint64_t ncell, uint64_t items,
                                 uint64_t seed, int cus, hipStream_t s)
{
    k_probe_deposits<<<cus * 32, 256, 0, s>>>(J, nbp, nb, ncell, items, seed);
    return hipGetLastError();
}

hipError_t launch_probe_gathers(const float4* kappa, uint64_t ncell, uint64_t items, uint64_t seed, float* sink,
                                int cus, hipStream_t s)
{
    k_probe_gathers<<<cus * 32, 256, 0, s>>>(kappa, ncell, items, seed, sink);
    return hipGetLastError();
}

// -------------------------------------------------------------------------------------
// Rates from the fixed-point field (eq:ion per absorber with the in-bin species split,
// section 2.8 heating) and the absorbed-photon ledger.
// -------------------------------------------------------------------------------------
template <int NB>
__global__ __launch_bounds__(256) void k_finalize(FinalizeArgs a)
{
    // per region: contiguous reads of the field and opacity, rates into LDS in linear
    // order, then whole x-rows of the six rate arrays
    __shared__ float out[6][kRegionCells];
    double absorbed = 0.0;
    const uint32_t nreg = (((uint32_t)a.nbx8 + 3u) / 4u) * (uint32_t)a.nby8 * (uint32_t)a.nbz8;
    for (uint32_t r = blockIdx.x; r < nreg; r += gridDim.x) {
        const Region g = region_of(r, a.nbx8, a.nby8);
        for (uint32_t o = threadIdx.x; o < g.cells; o += blockDim.x) {
            const uint32_t i = g.base + o, m = o & 511u;
            const uint32_t xl = ((o >> 9) << 3) | gather3(m), yl = gather3(m >> 1), zl = gather3(m >> 2);
            const uint32_t l = (zl << 8) | (yl << 5) | xl;
            double Jb[NB];
            const unsigned long long* j = a.J + (size_t)i * a.nbp;
#pragma unroll
            for (int b = 0; b < NB; ++b) Jb[b] = (double)(long long)j[b];
            float k[NB];
            if constexpr (NB == 1) {
                k[0] = a.kappa1[i];
            } else {
                const float4 v = a.kappa4[i];
                k[0] = v.x;
                k[1] = v.y;
                if constexpr (NB > 2) k[2] = v.z;
                if constexpr (NB > 3) k[3] = v.w;
            }
            if (a.M) {
                // photons moved in by the secondary correction, absorbed at this cell's opacity
                const unsigned long long* m = a.M + (size_t)i * (2 * a.nbp);
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    const double mv = (double)(long long)m[b] * 0x1p20 + (double)(long long)m[a.nbp + b] * 0x1p-12;
                    if (k[b] > 0.0f) Jb[b] += mv / (double)k[b];
                }
            }
#pragma unroll
            for (int sp = 0; sp < 3; ++sp) {
                double gm = 0.0, h = 0.0;
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    gm += a.gam[b][sp] * Jb[b];
                    h += a.hea[b][sp] * Jb[b];
                }
                out[sp][l] = (float)gm;
                out[3 + sp][l] = (float)h;
            }
            // cells of padding blocks have a zero field
#pragma unroll
            for (int b = 0; b < NB; ++b) absorbed += a.uj[b] * Jb[b] * (double)k[b];
        }
        __syncthreads();
        for (uint32_t l = threadIdx.x; l < (uint32_t)kRegionCells; l += blockDim.x) {
            const uint32_t x = g.x0 + (l & 31u), y = g.y0 + ((l >> 5) & 7u), z = g.z0 + (l >> 8);
            if (x >= (uint32_t)a.nx || y >= (uint32_t)a.ny || z >= (uint32_t)a.nz) continue;
            const size_t c = x + (size_t)a.nx * (y + (size_t)a.ny * z);
#pragma unroll
            for (int sp = 0; sp < 3; ++sp) {
                a.gamma[(size_t)sp * a.ncell + c] = out[sp][l];
                a.heat[(size_t)sp * a.ncell + c] = out[3 + sp][l];
            }
        }
        __syncthreads();
    }
    absorbed = wave_sum_f64(absorbed);
    if ((threadIdx.x & 63) == 0 && absorbed != 0.0) atomicAdd(a.absorbed, absorbed);
}

hipError_t launch_finalize(const FinalizeArgs& a, hipStream_t s)
{
    const unsigned g = grid_for((size_t)((a.nbx8 + 3) / 4) * a.nby8 * a.nbz8, 1, 1u << 16);
    switch (a.nb) {
        case 1: k_finalize<1><<<g, 256, 0, s>>>(a); break;
        case 2: k_finalize<2><<<g, 256, 0, s>>>(a); break;
        case 3: k_finalize<3><<<g, 256, 0, s>>>(a); break;
        default: k_finalize<4><<<g, 256, 0, s>>>(a); break;
    }
    return hipGetLastError();
}

// dst [bin][cell] = J; with M, then [bin][cell] of M's low limb and [bin][cell] of its high limb.
__global__ void k_get_field(const unsigned long long* J, const unsigned long long* M, int nb, int nbp, int nx, int ny,
                            int nbx8, int nby8, uint32_t ncell, long long* dst)
{
    for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < ncell; c += gridDim.x * blockDim.x) {
        const uint32_t x = c % (uint32_t)nx, y = (c / (uint32_t)nx) % (uint32_t)ny, z = c / ((uint32_t)nx * (uint32_t)ny);
        const uint32_t i = blocked_index((int)x, (int)y, (int)z, nbx8, nby8);
        for (int b = 0; b < nb; ++b) {
            dst[(size_t)b * ncell + c] = (long long)J[(size_t)i * nbp + b];
            if (M) {
                dst[(size_t)(nb + b) * ncell + c] = (long long)M[(size_t)i * 2 * nbp + nbp + b];
                dst[(size_t)(2 * nb + b) * ncell + c] = (long long)M[(size_t)i * 2 * nbp + b];
            }
        }
    }
}

hipError_t launch_get_field(const unsigned long long* J, const unsigned long long* M, int nb, int nbp, int nx, int ny,
                            int nbx8, int nby8, uint32_t ncell, long long* dst, hipStream_t s)
{
    k_get_field<<<grid_for(ncell, 256, 1u << 16), 256, 0, s>>>(J, M, nb, nbp, nx, ny, nbx8, nby8, ncell, dst);
    return hipGetLastError();
}

}  // namespace arc
