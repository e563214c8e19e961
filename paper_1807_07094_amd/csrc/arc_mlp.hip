// arc_mlp.hip -- learned chemistry step on gfx950 MFMA.
//
// Network: 8 -> 64 -> 64 -> 2, ReLU hidden units, BF16 weights and activations, FP32
// accumulation (v_mfma_f32_16x16x32_bf16). Inputs: log10 n_H, x_HI, log10 T, log10 Gamma_HI,
// log10 dt, log10 h (photoheating per H atom), x_HeII, x_HeI, standardised. Outputs: the
// standardised corrections x_HI' - x_base and log10 (T'/T), where x_base relaxes x_HI
// exponentially towards photoionisation equilibrium with the rates of the start of the step.
// Helium is not an output: the gate accepts a cell only when its helium is close to steady.
//
//   k_infer       per cell: features, forward pass with the activations kept in registers
//                 (each layer's MFMA output is the next layer's operand), gate; accepted
//                 cells are written, rejected cells are appended to a list for the plain solver
//   k_predict     the same forward pass without the gate (validation, evaluation)
//   k_train_grad  quantisation-aware forward and backward of a minibatch (MFMA through LDS),
//                 one gradient partial per wave (summed in fixed order: deterministic)
//   k_adam        Adam update of the FP32 master parameters
//   k_publish     BF16 weight images for the MFMA operands
#include <hip/hip_runtime.h>

#include <math.h>

#include "arc_chem.h"
#include "arc_mlp.h"

namespace arc {
namespace mlp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------------
// MFMA building block. v_mfma_f32_16x16x32_bf16: D[16x16] += A[16x32] B[32x16]; lane l
// supplies A[l % 16][8 (l / 16) + i] and B[8 (l / 16) + i][l % 16] for i = 0..7 and
// receives D[4 (l / 16) + r][l % 16] for r = 0..3.
// ---------------------------------------------------------------------------------
__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// 8 elements (row, k0 .. k0+7) of a bf16 matrix with element strides sr (row) and sk (k).
__device__ __forceinline__ bf16x8 frag(const __bf16* m, int row, int k0, int sr, int sk)
{
    bf16x8 v;
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = m[row * sr + (k0 + i) * sk];
    return v;
}

// One 16x16 tile of D = A B over depth K (multiple of 32); A(m, k) = A[m sar + k sak],
// B(k, n) = B[k sbk + n sbn]. Lane l receives D[m0 + 4 (l/16) + r][n0 + l % 16].
__device__ __forceinline__ f32x4 tile_mm(const __bf16* A, int sar, int sak, const __bf16* B, int sbk, int sbn, int m0,
                                         int n0, int K)
{
    const int lane = threadIdx.x & 63, r16 = lane & 15, q = lane >> 4;
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = 0; k0 < K; k0 += 32) {
        const bf16x8 a = frag(A, m0 + r16, k0 + 8 * q, sar, sak);
        const bf16x8 b = frag(B, n0 + r16, k0 + 8 * q, sbn, sbk);
        acc = mfma(a, b, acc);
    }
    return acc;
}

__device__ __forceinline__ float act(float x) { return fmaxf(x, 0.0f); }  // ReLU

// Orders one wave's LDS writes before its later reads by other lanes: LDS operations of
// a wave complete in issue order; the fence keeps the compiler from moving accesses.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Forward pass of 64 rows held in LDS: X [64][kK1] -> H (in place, [64][kHid]) -> O [64][2].
// W1t [kHid][kK1], W2t [kHid][kHid], W3t [kOutP][kHid] and the biases are in LDS.
// Every lane of the wave must call it. H1 (if given) keeps the first hidden layer.
__device__ __forceinline__ void forward64(const __bf16* X, __bf16* H, __bf16* H1keep, float* O, const __bf16* w1t,
                                          const __bf16* w2t, const __bf16* w3t, const float* b1, const float* b2,
                                          const float* b3)
{
    const int lane = threadIdx.x & 63, r16 = lane & 15, q = lane >> 4;
    // layer 1: [64 x 32] x [32 x 64]
    for (int t = 0; t < 4; ++t) {
        f32x4 d[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) d[nt] = tile_mm(X, kK1, 1, w1t, 1, kK1, 16 * t, 16 * nt, kK1);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * t + 4 * q + r, col = 16 * nt + r16;
                const __bf16 h = (__bf16)act(d[nt][r] + b1[col]);
                H[row * kHid + col] = h;
                if (H1keep) H1keep[row * kHid + col] = h;
            }
    }
    wave_sync();
    // layer 2: [64 x 64] x [64 x 64], written back over the rows it reads
    for (int t = 0; t < 4; ++t) {
        f32x4 d[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) d[nt] = tile_mm(H, kHid, 1, w2t, 1, kHid, 16 * t, 16 * nt, kHid);
        wave_sync();
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * t + 4 * q + r, col = 16 * nt + r16;
                H[row * kHid + col] = (__bf16)act(d[nt][r] + b2[col]);
            }
        wave_sync();
    }
    // layer 3: [64 x 64] x [64 x 16]
    for (int t = 0; t < 4; ++t) {
        const f32x4 d = tile_mm(H, kHid, 1, w3t, 1, kHid, 16 * t, 0, kHid);
        if (r16 < kOut)
#pragma unroll
            for (int r = 0; r < 4; ++r) O[(16 * t + 4 * q + r) * kOut + r16] = d[r] + b3[r16];
    }
    wave_sync();
}

// Model weights into LDS (called by the whole block).
struct SharedModel {
    __bf16 w1t[kHid * kK1];
    __bf16 w2t[kHid * kHid];
    __bf16 w3t[kOutP * kHid];
    float b1[kHid], b2[kHid], b3[kOut];
};

__device__ __forceinline__ void load_model(const Model* m, SharedModel& s)
{
    for (int i = threadIdx.x; i < kHid * kK1; i += blockDim.x) s.w1t[i] = (&m->w1t[0][0])[i];
    for (int i = threadIdx.x; i < kHid * kHid; i += blockDim.x) s.w2t[i] = (&m->w2t[0][0])[i];
    for (int i = threadIdx.x; i < kOutP * kHid; i += blockDim.x) s.w3t[i] = (&m->w3t[0][0])[i];
    for (int i = threadIdx.x; i < kHid; i += blockDim.x) {
        s.b1[i] = m->b1[i];
        s.b2[i] = m->b2[i];
    }
    if (threadIdx.x < kOut) s.b3[threadIdx.x] = m->b3[threadIdx.x];
}


// ---------------------------------------------------------------------------------
// Forward pass with the activations in registers.
//
// Each layer computes out^T = W in^T as 16x16 tiles: rows (the MFMA M dimension) are output
// units, columns (N) are 16 cells, the depth (K) runs over the layer's inputs. Lane l = 16q + n
// receives rows 4q..4q+3 of column n, which are exactly 4 of the 8 depth values that lane must
// supply as the B operand of the next layer, provided that layer's depth slots are taken in
// the order perm_k: slot 8q + i of k-step s stands for input unit 32s + 4q + i (i < 4) or
// 32s + 16 + 4q + i - 4 (i >= 4). The A operands (weights) are laid out in LDS in that same
// order, so no activation leaves the registers.
// ---------------------------------------------------------------------------------
__device__ __forceinline__ int perm_k(int s, int q, int i) { return 32 * s + (i < 4 ? 4 * q + i : 12 + 4 * q + i); }

// The weights as the operand fragments each lane supplies, in LDS (shared by the block):
// frag[f][lane] for f = 0..3 layer 1 (M-tile t = f), 4..11 layer 2 (t = (f - 4) / 2,
// k-step s = (f - 4) % 2), 12..13 layer 3 (k-step s = f - 12); biases as float4 per four rows.
constexpr int kFrags = 14;
struct LdsWeights {
    bf16x8 frag[kFrags][64];
    float4 b1[kHid / 4], b2[kHid / 4];
    float b3[kOut];
};

// Called by the whole block, followed by a barrier.
__device__ __forceinline__ void load_lds_weights(const Model* M, LdsWeights& L)
{
    for (int idx = threadIdx.x; idx < kFrags * 64; idx += blockDim.x) {
        const int f = idx >> 6, l = idx & 63, m = l & 15, q = l >> 4;
        bf16x8 v;
        if (f < 4) {
#pragma unroll
            for (int i = 0; i < 8; ++i) v[i] = M->w1t[16 * f + m][8 * q + i];
        } else if (f < 12) {
            const int t = (f - 4) >> 1, s2 = (f - 4) & 1;
#pragma unroll
            for (int i = 0; i < 8; ++i) v[i] = M->w2t[16 * t + m][perm_k(s2, q, i)];
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) v[i] = M->w3t[m][perm_k(f - 12, q, i)];
        }
        L.frag[f][l] = v;
    }
    for (int i = threadIdx.x; i < kHid / 4; i += blockDim.x) {
        L.b1[i] = make_float4(M->b1[4 * i], M->b1[4 * i + 1], M->b1[4 * i + 2], M->b1[4 * i + 3]);
        L.b2[i] = make_float4(M->b2[4 * i], M->b2[4 * i + 1], M->b2[4 * i + 2], M->b2[4 * i + 3]);
    }
    if (threadIdx.x < kOut) L.b3[threadIdx.x] = M->b3[threadIdx.x];
}

// ReLU of a pair after its BF16 rounding (rounding keeps the sign, so this equals rounding
// after the ReLU): as 16-bit integers the negative BF16 values, -0 included, are exactly
// the negative numbers, and one packed integer max clears both halves.
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef short i16x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t relu_bf16x2(float a, float b)
{
    const f32x2 p = {a, b};
    const bf16x2 v = __builtin_convertvector(p, bf16x2);  // one packed round-to-nearest-even
    const i16x2 z = {0, 0};
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(i16x2, v), z));
}

// Hidden layer: ReLU and BF16 rounding of four M-tiles (biases already in the
// accumulators), packed as the two k-steps of the next layer's B operand (elements 2j and
// 2j + 1 of an operand are the low and high halves of its word j).
__device__ __forceinline__ void hidden_to_operand(const f32x4 d[4], bf16x8 h[2])
{
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2) {
        const f32x4 a = d[2 * s2], b = d[2 * s2 + 1];
        const u32x4 w = {relu_bf16x2(a[0], a[1]), relu_bf16x2(a[2], a[3]), relu_bf16x2(b[0], b[1]),
                         relu_bf16x2(b[2], b[3])};
        h[s2] = __builtin_bit_cast(bf16x8, w);
    }
}

// Accumulator start of M-tile t: rows 4q..4q+3 of every column carry the biases of hidden
// units 16t + 4q .. 16t + 4q + 3, so the MFMA adds them.
__device__ __forceinline__ f32x4 bias_acc(const float4* bias, int t)
{
    const float4 b = bias[4 * t + ((threadIdx.x & 63) >> 4)];
    const f32x4 v = {b.x, b.y, b.z, b.w};
    return v;
}

// One tile of 16 cells: x = the layer-1 B operand (lanes with q = 0 hold the 8 standardised
// features of cell n, other lanes zeros). Returns rows 4q..4q+3 of the output tile; lanes
// with q = 0 hold the two outputs of cell n in elements 0 and 1 (biases included).
__device__ __forceinline__ f32x4 forward_tile(const LdsWeights& w, bf16x8 x)
{
    const int lane = threadIdx.x & 63;
    f32x4 d[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) d[t] = mfma(w.frag[t][lane], x, bias_acc(w.b1, t));
    bf16x8 h[2];
    hidden_to_operand(d, h);
#pragma unroll
    for (int t = 0; t < 4; ++t)
        d[t] = mfma(w.frag[5 + 2 * t][lane], h[1], mfma(w.frag[4 + 2 * t][lane], h[0], bias_acc(w.b2, t)));
    hidden_to_operand(d, h);
    const bool q0 = lane < 16;
    const f32x4 b3 = {q0 ? w.b3[0] : 0.0f, q0 ? w.b3[1] : 0.0f, 0.0f, 0.0f};
    return mfma(w.frag[13][lane], h[1], mfma(w.frag[12][lane], h[0], b3));
}

// Forward pass of the 64 cells of a wave, one per lane: f = the lane's standardised
// features; returns the lane's two outputs. Tiles of 16 cells with no bit in `need`
// (wave-uniform) are skipped and their outputs left at zero.
__device__ __forceinline__ void forward_wave(const LdsWeights& w, const float f[kIn], float& o0, float& o1,
                                             uint64_t need = ~0ull)
{
    const int lane = threadIdx.x & 63, n = lane & 15, q = lane >> 4;
    // the eight features as four packed BF16 pairs
    uint32_t pk[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const __bf16 lo = (__bf16)f[2 * j];
        const __bf16 hi = (__bf16)f[2 * j + 1];
        pk[j] = (uint32_t)__builtin_bit_cast(uint16_t, lo) | ((uint32_t)__builtin_bit_cast(uint16_t, hi) << 16);
    }
    o0 = o1 = 0.0f;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        if (((need >> (16 * c)) & 0xFFFFull) == 0) continue;  // no lane of these 16 cells needs it
        bf16x8 x;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t v = (uint32_t)__shfl((int)pk[j], 16 * c + n, 64);
            x[2 * j] = __builtin_bit_cast(__bf16, (uint16_t)(q == 0 ? v & 0xFFFFu : 0u));
            x[2 * j + 1] = __builtin_bit_cast(__bf16, (uint16_t)(q == 0 ? v >> 16 : 0u));
        }
        const f32x4 o = forward_tile(w, x);
        const float v0 = __shfl(o[0], n, 64), v1 = __shfl(o[1], n, 64);
        if (q == c) {
            o0 = v0;
            o1 = v1;
        }
    }
}

// Decimal logarithm and power from the hardware base-2 functions (the features and the
// targets of training go through the same two functions as inference).
__device__ __forceinline__ float flog10(float v) { return __builtin_amdgcn_logf(v) * 0.30102999566398120f; }
__device__ __forceinline__ float fexp10(float v) { return __builtin_amdgcn_exp2f(v * 3.3219280948873623f); }
__device__ __forceinline__ float safe_log10(float v, float floor_) { return flog10(fmaxf(v, floor_)); }

// Features of a cell: n_H, x_HI, T, Gamma_HI, dt [s], h = photoheating per H atom, x_HeII, x_HeI.
__device__ __forceinline__ void cell_features(float nh, float x, float T, float gam, float ldt, float h, float xheii,
                                              float xhei, float f[kIn])
{
    static_assert(kIn == 8, "eight features fill the first MFMA depth group");
    f[0] = flog10(nh);
    f[1] = x;
    f[2] = flog10(T);
    f[3] = safe_log10(gam, kGammaFloor);
    f[4] = ldt;
    f[5] = safe_log10(h, kHeatFloor);
    f[6] = xheii;
    f[7] = xhei;
}

// Baseline of x_HI': dx/dt = a (1 - x) - b x with a = alpha_HII(T) n_e and b = Gamma_HI +
// k_HI(T) n_e held at their start-of-step values (section 2.7 rates), solved exactly:
// x_base = x_eq + (x - x_eq) exp(-(a + b) dt), x_eq = a / (a + b).
__device__ __forceinline__ float x_baseline(const chem::Coef& k, float nh, float x, float gam, float xheii, float xhei,
                                            float dt, float y, int collisional)
{
    const float xheiii = fmaxf(0.0f, 1.0f - xhei - xheii);
    const float ne = nh * ((1.0f - x) + y * (xheii + 2.0f * xheiii));
    const float a = k.a_hii * ne;
    const float b = gam + (collisional ? k.k_hi * ne : 0.0f);
    const float lam = a + b;
    if (!(lam > 0.0f)) return x;
    const float xeq = a / lam;
    return xeq + (x - xeq) * expf(-lam * dt);
}

// Reciprocals of the standardisation scales and of the gate ranges, taken once per thread
// (correctly rounded, as on the host, so that both sides bin and scale identically).
struct Scales {
    float isd[kIn];
    float igate[kGateDims];
};

__device__ __forceinline__ Scales scales_of(const Model* M)
{
    Scales z;
#pragma unroll
    for (int k = 0; k < kIn; ++k) z.isd[k] = 1.0f / M->in_sd[k];
#pragma unroll
    for (int k = 0; k < kGateDims; ++k) z.igate[k] = 1.0f / (M->hi[k] - M->lo[k]);
    return z;
}

__device__ __forceinline__ void standardise(const Model* M, const Scales& z, bool valid, float f[kIn])
{
#pragma unroll
    for (int k = 0; k < kIn; ++k) f[k] = valid ? (f[k] - M->in_mu[k]) * z.isd[k] : 0.0f;
}

// ---------------------------------------------------------------------------------
// Inference with the gate.
// ---------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_infer(InferArgs a)
{
    const Model* M = a.model;
    __shared__ LdsWeights w;
    // the gate's verdict per bin (enough samples, small held-out error) as one bit each, so that
    // a cell's gate test reads LDS instead of two scattered loads from the model's tables
    __shared__ uint32_t gate_ok[kGateBins / 32];
    load_lds_weights(M, w);
    if (a.gated) {
        static_assert(kGateBins % 256 == 0, "whole rounds of the workgroup over the bins");
        for (uint32_t bin = threadIdx.x; bin < (uint32_t)kGateBins; bin += blockDim.x) {
            const bool ok = M->gate_count[bin] >= a.gate_min_count && M->gate_err[bin] <= a.gate_tol;
            const uint64_t bits = __ballot(ok);
            // lane 0 of each wave holds the 64 bins (two words) starting at its own bin
            if ((threadIdx.x & 63) == 0) {
                gate_ok[bin >> 5] = (uint32_t)bits;
                gate_ok[(bin >> 5) + 1] = (uint32_t)(bits >> 32);
            }
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const Scales z = scales_of(M);
    const float dtf = (float)a.dt, ldt = flog10(dtf);
    const float yf = (float)a.y;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t base = blockIdx.x * blockDim.x + (threadIdx.x & ~63u); base < a.ncell; base += stride) {
        const uint32_t c = base + lane;
        const bool valid = c < a.ncell;
        float nh = 1.0f, T = 1.0f, x0 = 0.0f, xhei = 0.0f, xheii = 0.0f, gam = 0.0f, h = 0.0f, xb = 0.0f;
        if (valid) {
            nh = a.n_h[c];
            T = a.temp[c];
            x0 = a.x_hi[c];
            xhei = a.x_hei[c];
            xheii = a.x_heii[c];
            gam = a.gamma[c];
            h = a.heat[c] * x0 + yf * (a.heat[(size_t)a.ncell + c] * xhei + a.heat[2 * (size_t)a.ncell + c] * xheii);
        }
        float f[kIn];
        cell_features(nh, x0, T, gam, ldt, h, xheii, xhei, f);
        // (1) gate bins: inside the training range, in a bin with enough samples and a small
        //     held-out error
        bool accept = valid;
        if (valid && a.gated) {
            uint32_t bin = 0;
#pragma unroll
            for (int k = kGateDims - 1; k >= 0; --k) {
                const float u = (f[k] - M->lo[k]) * z.igate[k];
                accept = accept && u >= 0.0f && u <= 1.0f;
                const int b = min(kGate - 1, max(0, (int)(u * kGate)));
                bin = bin * kGate + (uint32_t)b;
            }
            accept = accept && ((gate_ok[bin >> 5] >> (bin & 31u)) & 1u) != 0u;
        }
        float xn = 0.0f, Tn = 0.0f;
        chem::Coef k{};
        // the network runs only for waves with a cell past the gate bins (wave-uniform branch)
        const uint64_t cand = __ballot(accept);
        if (cand) {
            standardise(M, z, valid, f);
            float o0, o1;
            forward_wave(w, f, o0, o1, cand);
            // the outputs (the baseline only where they can still be used)
            if (accept) {
                k = chem::coefficients(T);
                xb = x_baseline(k, nh, x0, gam, xheii, xhei, dtf, M->base_y, M->base_collisional);
                xn = fminf(fmaxf(xb + (o0 * M->out_sd[0] + M->out_mu[0]), 0.0f), 1.0f);
                Tn = T * fexp10(o1 * M->out_sd[1] + M->out_mu[1]);
            }
        }
        if (accept) {
            if (a.gated) {
                // (2) physical output temperature
                accept = accept && Tn >= a.t_floor && Tn < 1e9f;
                // (3) helium close to steady over dt (the network does not predict helium)
                //     (a screening test: FP32 is ample for a 1e-3 threshold)
                if (accept && a.y > 0.0) {
                    const float nhe = yf * nh;
                    const float nhei = nhe * xhei, nheii = nhe * xheii;
                    const float nheiii = fmaxf(0.0f, nhe - nhei - nheii);
                    const float ne = nh * (1.0f - x0) + nheii + 2.0f * nheiii;
                    const float kc = a.collisional ? 1.0f : 0.0f;
                    const float dhei = k.a_heii * ne * nheii - (a.gamma[(size_t)a.ncell + c] + kc * k.k_hei * ne) * nhei;
                    const float dheiii =
                        (a.gamma[2 * (size_t)a.ncell + c] + kc * k.k_heii * ne) * nheii - k.a_heiii * ne * nheiii;
                    accept = fabsf(dhei) * dtf <= 1e-3f * nhe && fabsf(dheiii) * dtf <= 1e-3f * nhe;
                }
            }
        }
        if (accept) {
            a.x_hi[c] = xn;
            a.temp[c] = Tn;
        }
        // the cells for the plain solver, one bit per cell of the tile
        const uint64_t rej = __ballot(valid && !accept);
        if (lane == 0) a.reject[base >> 6] = (unsigned long long)rej;
    }
}

hipError_t launch_infer(const InferArgs& a, hipStream_t s)
{
    size_t blocks = (a.ncell + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    k_infer<<<(unsigned)blocks, 256, 0, s>>>(a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Forward only (validation, gate calibration, evaluation): raw samples to (x_HI', T').
// ---------------------------------------------------------------------------------
__device__ __forceinline__ void raw_features(const float* x, float f[kIn])
{
    cell_features(x[0], x[1], x[2], x[3], flog10(x[4]), x[5], x[6], x[7], f);
}

__device__ __forceinline__ float raw_baseline(const float* x, float y, int collisional)
{
    return x_baseline(chem::coefficients(x[2]), x[0], x[1], x[3], x[6], x[7], x[4], y, collisional);
}

__global__ __launch_bounds__(256) void k_predict(const Model* M, const float* X, const uint32_t* idx, uint32_t m,
                                                 float* P)
{
    __shared__ LdsWeights w;
    load_lds_weights(M, w);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const Scales z = scales_of(M);
    for (uint32_t base = blockIdx.x * blockDim.x + (threadIdx.x & ~63u); base < m; base += gridDim.x * blockDim.x) {
        const uint32_t i = base + lane;
        const bool valid = i < m;
        const float* x = X + (size_t)(valid ? (idx ? idx[i] : i) : 0u) * kIn;
        float f[kIn] = {1.0f, 0.0f, 1.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        float xb = 0.0f;
        if (valid) {
            raw_features(x, f);
            xb = raw_baseline(x, M->base_y, M->base_collisional);
        }
        standardise(M, z, valid, f);
        float o0, o1;
        forward_wave(w, f, o0, o1);
        if (valid) {
            P[(size_t)i * 2] = fminf(fmaxf(xb + (o0 * M->out_sd[0] + M->out_mu[0]), 0.0f), 1.0f);
            P[(size_t)i * 2 + 1] = x[2] * fexp10(o1 * M->out_sd[1] + M->out_mu[1]);
        }
    }
}

hipError_t launch_predict(const Model* model, const float* X, const uint32_t* idx, uint32_t m, float* P,
                          hipStream_t s)
{
    size_t blocks = (m + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    k_predict<<<(unsigned)blocks, 256, 0, s>>>(model, X, idx, m, P);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Features and targets of raw samples X [m][kIn] and (x_HI', T').
// ---------------------------------------------------------------------------------
__global__ void k_features(const float* X, const float* Y, uint32_t m, float y, int collisional, float* F, float* Yt)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
        const float* x = X + (size_t)i * kIn;
        raw_features(x, F + (size_t)i * kIn);
        Yt[(size_t)i * 2] = Y[(size_t)i * 2] - raw_baseline(x, y, collisional);
        Yt[(size_t)i * 2 + 1] = flog10(Y[(size_t)i * 2 + 1]) - flog10(x[2]);
    }
}

hipError_t launch_features(const float* X, const float* Y, uint32_t m, float y, int collisional, float* F, float* Yt,
                           hipStream_t s)
{
    size_t blocks = (m + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    k_features<<<(unsigned)blocks, 256, 0, s>>>(X, Y, m, y, collisional, F, Yt);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Training: gradient of the minibatch loss
//   L = sum_s (o0 - y0)^2 + (o1 - y1)^2     (standardised targets; divided by the batch
//                                            size in Adam)
// through the same BF16 forward as inference. One wave per block, 64 samples per wave.
// ---------------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_train_grad(TrainArgs a)
{
    __shared__ SharedModel sm;
    __shared__ __bf16 w3pad[32 * kHid];  // W3t with zero rows to depth 32
    __shared__ __bf16 X[64 * kK1];
    __shared__ __bf16 H[64 * kHid];      // second hidden layer after the forward pass
    __shared__ __bf16 H1[64 * kHid];
    __shared__ __bf16 D2[64 * kHid];     // dL/dz2
    __shared__ __bf16 D1[64 * kHid];     // dL/dz1
    __shared__ __bf16 DO[64 * 32];       // dL/do, zero-padded to depth 32
    __shared__ float O[64 * kOut];
    load_model(a.model, sm);
    for (int i = threadIdx.x; i < 32 * kHid; i += blockDim.x) w3pad[i] = i < kOutP * kHid ? sm.w3t[i] : (__bf16)0.0f;
    __syncthreads();
    const int lane = threadIdx.x, r16 = lane & 15, q = lane >> 4;
    const uint32_t s_local = blockIdx.x * 64u + (uint32_t)lane;
    const bool valid = s_local < a.count;
    float y0 = 0.0f, y1 = 0.0f;
    {
        const uint32_t i = valid ? a.idx[a.first + s_local] : 0u;
#pragma unroll
        for (int k = 0; k < kK1; ++k) X[lane * kK1 + k] = (__bf16)(k < kIn && valid ? a.F[(size_t)i * kIn + k] : 0.0f);
        if (valid) {
            y0 = a.Y[(size_t)i * 2];
            y1 = a.Y[(size_t)i * 2 + 1];
        }
    }
    wave_sync();
    forward64(X, H, H1, O, sm.w1t, sm.w2t, sm.w3t, sm.b1, sm.b2, sm.b3);
    // output gradient
    {
        const float g0 = valid ? 2.0f * (O[lane * kOut] - y0) : 0.0f;
        const float g1 = valid ? 2.0f * (O[lane * kOut + 1] - y1) : 0.0f;
#pragma unroll
        for (int k = 0; k < 32; ++k) DO[lane * 32 + k] = (__bf16)(k == 0 ? g0 : (k == 1 ? g1 : 0.0f));
    }
    wave_sync();
    float* P = a.partial + (size_t)blockIdx.x * kNParams;
    // dW3[k][n] = sum_s H2[s][k] dO[s][n]   (M = 64 k, N = 16 n, K = 64 s)
    for (int t = 0; t < 4; ++t) {
        const f32x4 d = tile_mm(H, 1, kHid, DO, 32, 1, 16 * t, 0, 64);
        if (r16 < kOut)
#pragma unroll
            for (int r = 0; r < 4; ++r) P[kW3 + (16 * t + 4 * q + r) * kOut + r16] = d[r];
    }
    // dz2 = (dO W3^T) * [H2 > 0]               (M = 64 s, N = 64 k, K = 32 n)
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const f32x4 d = tile_mm(DO, 32, 1, w3pad, kHid, 1, 16 * t, 16 * nt, 32);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * t + 4 * q + r, col = 16 * nt + r16;
                const float h = (float)H[row * kHid + col];
                D2[row * kHid + col] = (__bf16)(h > 0.0f ? d[r] : 0.0f);
            }
        }
    wave_sync();
    // dW2[k][n] = sum_s H1[s][k] dz2[s][n]     (M = 64, N = 64, K = 64)
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const f32x4 d = tile_mm(H1, 1, kHid, D2, kHid, 1, 16 * t, 16 * nt, 64);
#pragma unroll
            for (int r = 0; r < 4; ++r) P[kW2 + (16 * t + 4 * q + r) * kHid + 16 * nt + r16] = d[r];
        }
    // dz1 = (dz2 W2^T) * [H1 > 0]              (M = 64 s, N = 64 k, K = 64 n)
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const f32x4 d = tile_mm(D2, kHid, 1, sm.w2t, kHid, 1, 16 * t, 16 * nt, 64);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * t + 4 * q + r, col = 16 * nt + r16;
                const float h = (float)H1[row * kHid + col];
                D1[row * kHid + col] = (__bf16)(h > 0.0f ? d[r] : 0.0f);
            }
        }
    wave_sync();
    // dW1[k][n] = sum_s X[s][k] dz1[s][n]      (M = 16 k (5 used), N = 64, K = 64)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const f32x4 d = tile_mm(X, 1, kK1, D1, kHid, 1, 0, 16 * nt, 64);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int k = 4 * q + r;
            if (k < kIn) P[kW1 + k * kHid + 16 * nt + r16] = d[r];
        }
    }
    // bias gradients: column sums
    {
        float s1 = 0.0f, s2 = 0.0f;
        for (int s = 0; s < 64; ++s) {
            s1 += (float)D1[s * kHid + lane];
            s2 += (float)D2[s * kHid + lane];
        }
        P[kB1 + lane] = s1;
        P[kB2 + lane] = s2;
        if (lane < kOut) {
            float s3 = 0.0f;
            for (int s = 0; s < 64; ++s) s3 += (float)DO[s * 32 + lane];
            P[kB3 + lane] = s3;
        }
    }
}

hipError_t launch_train_grad(const TrainArgs& a, hipStream_t s)
{
    const unsigned waves = (a.count + 63) / 64;
    k_train_grad<<<waves, 64, 0, s>>>(a);
    return hipGetLastError();
}

__global__ void k_adam(AdamArgs a)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kNParams) return;
    float g = 0.0f;
    for (int w = 0; w < a.nwaves; ++w) g += a.partial[(size_t)w * kNParams + p];
    g *= a.inv_batch;
    const float m = a.beta1 * a.m[p] + (1.0f - a.beta1) * g;
    const float v = a.beta2 * a.v[p] + (1.0f - a.beta2) * g * g;
    a.m[p] = m;
    a.v[p] = v;
    const float mh = m / (1.0f - powf(a.beta1, (float)a.step));
    const float vh = v / (1.0f - powf(a.beta2, (float)a.step));
    a.params[p] -= a.lr * mh / (sqrtf(vh) + a.eps);
}

__global__ void k_publish(const float* P, Model* M)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kHid * kHid; i += gridDim.x * blockDim.x) {
        const int n = i / kHid, k = i % kHid;  // w2t[n][k] = w2[k][n]
        M->w2t[n][k] = (__bf16)P[kW2 + k * kHid + n];
    }
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kHid * kK1; i += gridDim.x * blockDim.x) {
        const int n = i / kK1, k = i % kK1;
        M->w1t[n][k] = (__bf16)(k < kIn ? P[kW1 + k * kHid + n] : 0.0f);
    }
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kOutP * kHid; i += gridDim.x * blockDim.x) {
        const int n = i / kHid, k = i % kHid;
        M->w3t[n][k] = (__bf16)(n < kOut ? P[kW3 + k * kOut + n] : 0.0f);
    }
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kHid; i += gridDim.x * blockDim.x) {
        M->b1[i] = P[kB1 + i];
        M->b2[i] = P[kB2 + i];
    }
    if (blockIdx.x == 0 && threadIdx.x < kOut) M->b3[threadIdx.x] = P[kB3 + threadIdx.x];
}

hipError_t launch_adam(const AdamArgs& a, hipStream_t s)
{
    k_adam<<<(kNParams + 255) / 256, 256, 0, s>>>(a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_publish(a.params, a.model, s);
}

hipError_t launch_publish(const float* params, Model* model, hipStream_t s)
{
    k_publish<<<16, 256, 0, s>>>(params, model);
    return hipGetLastError();
}

}  // namespace mlp
}  // namespace arc
