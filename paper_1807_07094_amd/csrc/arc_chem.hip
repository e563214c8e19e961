// arc_chem.hip -- the plain chemistry step of libarc (gfx950):
//
//   k_chem             sub-cycled backward-difference chemistry and energy update, one cell
//                      per lane, lanes refilled from a chunked global cell counter
//   k_timestep         the adaptive RT time step's two grid minima (section 2.9)
#include <hip/hip_runtime.h>

#include <math.h>

#include <algorithm>

#include "arc_chem.h"
#include "arc_kernels.h"

namespace arc {

// -------------------------------------------------------------------------------------
// Chemistry (eq:diffeq in the backward-difference form of eq:anninos, sub-cycled with
// the step limit of section 2.7; heating and cooling of section 2.8). One cell per
// lane. Rate coefficients and cooling in FP32, species and energy in FP64.
// Coefficients: Hui & Gnedin (1997) fits with lambda = 2 T_i / T.
// -------------------------------------------------------------------------------------


// State of one cell during its sub-cycled update.
struct ChemCell {
    double nh, nhe, nhi, nhii, nhei, nheii, nheiii, ne, E, t;
    double ghi, ghei, gheii, hhi, hhei, hheii;
    float T;
    int n;
    bool cap;
    uint32_t c;
};

__device__ __forceinline__ void chem_load(const ChemArgs& a, uint32_t c, ChemCell& s)
{
    s.c = c;
    s.nh = a.n_h[c];
    s.nhe = a.y * s.nh;
    s.nhi = s.nh * (double)a.x_hi[c];
    s.nhii = s.nh - s.nhi;
    s.nhei = s.nhe * (double)a.x_hei[c];
    s.nheii = s.nhe * (double)a.x_heii[c];
    s.nheiii = s.nhe - s.nhei - s.nheii;
    if (s.nheiii < 0) s.nheiii = 0;
    s.T = a.temp[c];
    s.ne = s.nhii + s.nheii + 2.0 * s.nheiii;
    s.E = 1.5 * chem::kKB * (double)s.T * (s.nh + s.nhe + s.ne);
    s.ghi = a.gamma[c];
    s.ghei = a.gamma[(size_t)a.ncell + c];
    s.gheii = a.gamma[2 * (size_t)a.ncell + c];
    s.hhi = a.heat[c];
    s.hhei = a.heat[(size_t)a.ncell + c];
    s.hheii = a.heat[2 * (size_t)a.ncell + c];
    s.t = 0.0;
    s.n = 0;
    s.cap = false;
}

// 1 / b for b > 0 from the hardware reciprocal and two Newton steps (within an ulp or two
// of the rounded value; the solver's tolerances are orders of magnitude looser), far fewer
// instructions than an IEEE division.
__device__ __forceinline__ double rcp64(double b)
{
    double r = __builtin_amdgcn_rcp(b);
    r = fma(r, fma(-b, r, 1.0), r);
    return fma(r, fma(-b, r, 1.0), r);
}

// One sub-step (section 2.7: backward difference for the species, sub-step limited to a
// fraction eps of the shortest change time). Returns true once the cell has reached dt.
__device__ __forceinline__ bool chem_substep(const ChemArgs& a, ChemCell& s)
{
    chem::Coef k{};
    const chem::Lam l = chem::lambdas(s.T);
    if (a.rates == 0) {
        k.a_hii = (float)a.alpha_hii;
    } else {
        k = chem::coefficients(l);
        if (!a.collisional) k.k_hi = k.k_hei = k.k_heii = 0.0f;
    }
    const double ndot_hi = (double)k.a_hii * s.ne * s.nhii - (s.ghi + (double)k.k_hi * s.ne) * s.nhi;
    double edot = 0.0;
    if (!a.isothermal)
        edot = s.nhi * s.hhi + s.nhei * s.hhei + s.nheii * s.hheii -
               chem::cooling(s.T, l, k, s.ne, s.nhi, s.nhii, s.nhei, s.nheii, s.nheiii, a.collisional);
    double h = a.dt - s.t;
    bool last = true;
    if (s.n >= a.max_sub) {
        s.cap = true;
    } else {
        const double le = edot != 0.0 ? a.eps * s.E * rcp64(fabs(edot)) : INFINITY;
        const double in = ndot_hi != 0.0 ? rcp64(fabs(ndot_hi)) : 0.0;
        if (edot != 0.0 && le < h) {
            h = le;
            last = false;
        }
        if (s.nhi > 0.0 && ndot_hi != 0.0 && a.eps * s.nhi * in < h) {
            h = a.eps * s.nhi * in;
            last = false;
        }
        if (s.nhii > 0.0 && ndot_hi != 0.0 && a.eps * s.nhii * in < h) {
            h = a.eps * s.nhii * in;
            last = false;
        }
    }
    s.nhi = (s.nhi + (double)k.a_hii * s.ne * s.nhii * h) * rcp64(1.0 + (s.ghi + (double)k.k_hi * s.ne) * h);
    if (s.nhi > s.nh) s.nhi = s.nh;
    s.nhii = s.nh - s.nhi;
    double nhei_new = (s.nhei + (double)k.a_heii * s.ne * s.nheii * h) * rcp64(1.0 + (s.ghei + (double)k.k_hei * s.ne) * h);
    double nheiii_new =
        (s.nheiii + (s.gheii + (double)k.k_heii * s.ne) * s.nheii * h) * rcp64(1.0 + (double)k.a_heiii * s.ne * h);
    if (nhei_new > s.nhe) nhei_new = s.nhe;
    if (nheiii_new > s.nhe - nhei_new) nheiii_new = s.nhe - nhei_new;
    s.nhei = nhei_new;
    s.nheiii = nheiii_new;
    s.nheii = s.nhe - s.nhei - s.nheiii;
    if (s.nheii < 0.0) s.nheii = 0.0;
    s.ne = s.nhii + s.nheii + 2.0 * s.nheiii;
    if (!a.isothermal) {
        s.E += edot * h;
        double Td = s.E * rcp64(1.5 * chem::kKB * (s.nh + s.nhe + s.ne));
        if (Td < a.t_floor) {
            Td = a.t_floor;
            s.E = 1.5 * chem::kKB * Td * (s.nh + s.nhe + s.ne);
        }
        s.T = (float)Td;
    }
    s.t = last ? a.dt : s.t + h;
    ++s.n;
    return !(s.t < a.dt);
}

__device__ __forceinline__ void chem_store(const ChemArgs& a, const ChemCell& s)
{
    a.x_hi[s.c] = (float)(s.nhi / s.nh);
    if (s.nhe > 0.0) {
        a.x_hei[s.c] = (float)(s.nhei / s.nhe);
        a.x_heii[s.c] = (float)(s.nheii / s.nhe);
    }
    a.temp[s.c] = s.T;
}

// Per-cell chemistry (section 2.7). Cells need from one to many sub-steps, so a wave does
// not take 64 cells and wait for the slowest: each lane advances its cell one sub-step per
// iteration and takes the next cell of the wave's chunk when done (refilled once kChemRefill
// lanes are idle); chunks of kChemChunk cells come from a global counter.
constexpr uint32_t kChemChunk = 2048;
constexpr int kChemRefill = 16;

__global__ __launch_bounds__(256) void k_chem(ChemArgs a)
{
    unsigned long long sub_total = 0, capped = 0, cells = 0;
    unsigned int sub_max = 0;
    const int lane = threadIdx.x & 63;
    const uint64_t lt = __lanemask_lt();
    uint32_t lo = 0, hi = 0;  // the wave's remaining chunk [lo, hi), wave-uniform
    bool drained = false;     // wave-uniform
    bool have = false;
    ChemCell s;
    for (;;) {
        const uint64_t idle = __ballot(!have);
        const int nidle = __popcll(idle);
        if (!drained && (nidle >= kChemRefill || nidle == 64)) {
            // hand the next cells to the idle lanes, in lane order
            int given = 0;
            while (given < nidle && !drained) {
                if (lo >= hi) {
                    uint32_t b0 = 0;
                    if (lane == 0) b0 = atomicAdd(a.chunk_counter, kChemChunk);
                    b0 = (uint32_t)__shfl((int)b0, 0, 64);
                    if (b0 >= a.ncell) {
                        drained = true;
                        break;
                    }
                    lo = b0;
                    hi = min(a.ncell, b0 + kChemChunk);
                }
                const int take = min(nidle - given, (int)(hi - lo));
                const int rank = __popcll(idle & lt) - given;
                if (!have && rank >= 0 && rank < take) {
                    const uint32_t c = lo + (uint32_t)rank;
                    if (!a.mask || ((a.mask[c >> 6] >> (c & 63)) & 1ull)) {
                        chem_load(a, c, s);
                        have = true;
                        ++cells;
                    }
                }
                lo += (uint32_t)take;
                given += take;
            }
        }
        if (!__any(have)) {
            if (drained) break;
            continue;
        }
        if (have && chem_substep(a, s)) {
            chem_store(a, s);
            sub_total += (unsigned long long)s.n;
            capped += s.cap ? 1ull : 0ull;
            sub_max = max(sub_max, (unsigned)s.n);
            have = false;
        }
    }
    sub_total = wave_sum_u64(sub_total);
    capped = wave_sum_u64(capped);
    cells = wave_sum_u64(cells);
    for (int off = 32; off > 0; off >>= 1) sub_max = max(sub_max, (unsigned)__shfl_xor((int)sub_max, off, 64));
    if ((threadIdx.x & 63) == 0) {
        if (sub_total) atomicAdd(&a.stats[0], sub_total);
        if (capped) atomicAdd(&a.stats[1], capped);
        atomicMax(&a.stats[2], (unsigned long long)sub_max);
        if (cells) atomicAdd(&a.stats[3], cells);
    }
}

hipError_t launch_chem(const ChemArgs& a, int cus, hipStream_t s)
{
    // resident waves only: every wave loops until the chunk counter passes ncell
    const size_t want = ((size_t)a.ncell + 255) / 256;
    const unsigned blocks = (unsigned)std::max<size_t>(1, std::min<size_t>(want, (size_t)std::max(1, cus) * 8));
    k_chem<<<blocks, 256, 0, s>>>(a);
    return hipGetLastError();
}

// -------------------------------------------------------------------------------------
// Adaptive RT time step (section 2.9). Per cell, from the current state and rates, the
// source term of the HI equation ndot = alpha_HII n_e n_HII - (Gamma_HI + k_HI n_e) n_HI
// (FP32 coefficients, FP64 densities, as in the solver); then the neutral-fraction limit
// eps n_HI / |ndot| over cells with tau = n_HI sigma0 L > 0.5 and the intensity limit
// eps / (sigma0 L |ndot|) over all cells. Minima over the grid: per wave, then one atomic
// min per wave on the bit patterns of the non-negative doubles (the order of the updates
// cannot change the result).
// -------------------------------------------------------------------------------------
__global__ void k_timestep_reset(unsigned long long* out)
{
    if (threadIdx.x < 2) out[threadIdx.x] = 0x7FF0000000000000ull;  // +inf
}

hipError_t launch_timestep_reset(unsigned long long* out, hipStream_t s)
{
    k_timestep_reset<<<1, 64, 0, s>>>(out);
    return hipGetLastError();
}

__device__ __forceinline__ double wave_min_f64(double v)
{
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}

__global__ __launch_bounds__(256) void k_timestep(TimestepArgs a)
{
    double mn = INFINITY, mi = INFINITY;
    const double sl = a.sigma0 * a.cell_cm;
    for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < a.ncell; c += gridDim.x * blockDim.x) {
        const double nh = a.n_h[c], nhe = a.y * nh;
        const double nhi = nh * (double)a.x_hi[c], nhii = nh - nhi;
        const double nhei = nhe * (double)a.x_hei[c], nheii = nhe * (double)a.x_heii[c];
        double nheiii = nhe - nhei - nheii;
        if (nheiii < 0) nheiii = 0;
        const double ne = nhii + nheii + 2.0 * nheiii;
        double a_hii, k_hi = 0.0;
        if (a.rates == 0) {
            a_hii = a.alpha_hii;
        } else {
            const chem::Coef k = chem::coefficients(a.temp[c]);
            a_hii = (double)k.a_hii;
            if (a.collisional) k_hi = (double)k.k_hi;
        }
        const double ndot = fabs(a_hii * ne * nhii - ((double)a.gamma_hi[c] + k_hi * ne) * nhi);
        if (!(ndot > 0.0)) continue;
        if (nhi * sl > 0.5) mn = fmin(mn, a.eps * nhi / ndot);
        mi = fmin(mi, a.eps / (sl * ndot));
    }
    mn = wave_min_f64(mn);
    mi = wave_min_f64(mi);
    if ((threadIdx.x & 63) == 0) {
        if (mn < INFINITY) atomicMin(&a.out[0], (unsigned long long)__double_as_longlong(mn));
        if (mi < INFINITY) atomicMin(&a.out[1], (unsigned long long)__double_as_longlong(mi));
    }
}

// The two minima as doubles into caller memory (device pointer out[2]).
__global__ void k_timestep_publish(const unsigned long long* bits, double* out)
{
    if (threadIdx.x < 2) out[threadIdx.x] = __longlong_as_double((long long)bits[threadIdx.x]);
}

hipError_t launch_timestep_publish(const unsigned long long* bits, double* out, hipStream_t s)
{
    k_timestep_publish<<<1, 64, 0, s>>>(bits, out);
    return hipGetLastError();
}

hipError_t launch_timestep(const TimestepArgs& a, int cus, hipStream_t s)
{
    const size_t want = ((size_t)a.ncell + 255) / 256;
    const unsigned blocks = (unsigned)std::max<size_t>(1, std::min<size_t>(want, (size_t)std::max(1, cus) * 8));
    k_timestep<<<blocks, 256, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace arc
