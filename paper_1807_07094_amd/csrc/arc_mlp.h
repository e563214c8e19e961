// arc_mlp.h -- learned chemistry step: an 8 -> 64 -> 64 -> 2 BF16 network on MFMA with FP32
// accumulation that stands in for the per-cell sub-cycled update, with a per-cell gate and
// the plain solver as fallback.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace arc {
namespace mlp {

// Features: log10 n_H, x_HI, log10 T, log10 Gamma_HI, log10 dt, log10 h, x_HeII, x_HeI, where
// h = H_HI x_HI + y (H_HeI x_HeI + H_HeII x_HeII) is the photoheating per hydrogen atom [erg/s].
constexpr int kIn = 8;
constexpr int kGateDims = 5; // the gate bins the first five features
constexpr int kHid = 64;
constexpr int kOut = 2;      // standardised x_HI' - x_base and log10 (T'/T)
constexpr int kK1 = 32;      // layer-1 depth padded to one MFMA step
constexpr int kOutP = 16;    // layer-3 width padded to one MFMA tile
constexpr int kGate = 8;     // gate bins per input feature
constexpr int kGateBins = kGate * kGate * kGate * kGate * kGate;
static_assert(kGateDims == 5, "kGateBins spans five features");
constexpr float kGammaFloor = 1e-30f;
constexpr float kHeatFloor = 1e-35f;  // a normal float: the hardware log flushes denormals

// Offsets of the FP32 master parameters in one flat array.
constexpr int kW1 = 0;                      // [kIn][kHid]
constexpr int kB1 = kW1 + kIn * kHid;       // [kHid]
constexpr int kW2 = kB1 + kHid;             // [kHid][kHid]
constexpr int kB2 = kW2 + kHid * kHid;      // [kHid]
constexpr int kW3 = kB2 + kHid;             // [kHid][kOut]
constexpr int kB3 = kW3 + kHid * kOut;      // [kOut]
constexpr int kNParams = kB3 + kOut;

// Everything inference needs, in device memory.
struct Model {
    float in_mu[kIn], in_sd[kIn];   // feature standardisation
    float lo[kIn], hi[kIn];         // training range of each feature (gate)
    float out_mu[kOut], out_sd[kOut];  // standardisation of the outputs (x_HI' - x_base, log10 T'/T)
    float base_y;                   // He/H and collisional flag of the baseline x_base (those of
    int32_t base_collisional;       // the training samples)
    float b1[kHid], b2[kHid], b3[kOut];
    __bf16 w1t[kHid][kK1];          // W1 transposed, rows padded with zeros
    __bf16 w2t[kHid][kHid];         // W2 transposed
    __bf16 w3t[kOutP][kHid];        // W3 transposed, rows >= kOut zero
    uint32_t gate_count[kGateBins]; // training samples per bin
    float gate_err[kGateBins];      // twice the largest held-out error per bin (max of |dx| and |dT|/(10 T))
};

struct InferArgs {
    const Model* model;
    uint32_t ncell;
    double y;
    const float* n_h;
    float *x_hi, *x_hei, *x_heii, *temp;
    const float *gamma, *heat;      // [3][ncell]
    double dt;
    int gated;                      // 0: accept every cell (evaluation)
    float gate_tol;
    uint32_t gate_min_count;
    float t_floor;
    unsigned long long* reject;     // per 64-cell tile, bit set = the plain solver updates the cell
    int collisional;
};

hipError_t launch_infer(const InferArgs& a, hipStream_t s);

// Training on standardised features F [m][kIn] and standardised targets Y [m][2]
// (x_HI' - x_base, log10 (T'/T)), minibatch rows given by idx.
struct TrainArgs {
    const Model* model;       // bf16 weights used by the forward pass
    const float* F;
    const float* Y;
    const uint32_t* idx;      // sample order
    uint32_t first, count;    // the minibatch: idx[first .. first + count)
    float* partial;           // [waves][kNParams] gradient partial sums
};
hipError_t launch_train_grad(const TrainArgs& a, hipStream_t s);

struct AdamArgs {
    float* params;            // [kNParams] FP32 master
    float* m;
    float* v;
    const float* partial;
    int nwaves;
    float lr, beta1, beta2, eps, inv_batch;
    int step;
    Model* model;             // refreshed bf16 images and biases
};
hipError_t launch_adam(const AdamArgs& a, hipStream_t s);
hipError_t launch_publish(const float* params, Model* model, hipStream_t s);

// Forward pass only: predictions P [m][2] = (x_HI', T') for raw samples X [m][8] =
// (n_H, x_HI, T, Gamma_HI, dt, h, x_HeII, x_HeI); rows idx[i] of X if idx is given, else row i.
hipError_t launch_predict(const Model* model, const float* X, const uint32_t* idx, uint32_t m, float* P,
                          hipStream_t s);

// Raw samples X [m][8] and targets (x_HI', T') to unstandardised features and training
// targets (x_HI' - x_base, log10 (T'/T)); y and collisional define x_base.
hipError_t launch_features(const float* X, const float* Y, uint32_t m, float y, int collisional, float* F, float* Yt,
                           hipStream_t s);

}  // namespace mlp
}  // namespace arc
