// arc_mlp_api.hip -- host side of the learned chemistry step: training, gate calibration,
// serialisation and prediction through the C ABI of include/arc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <random>
#include <vector>

#include "arc.h"
#include "arc_mlp.h"
#include "arc_mlp_host.h"

using namespace arc;
using namespace arc::mlp;

namespace {

constexpr uint32_t kMagic = 0x41524d31u;  // "ARM1"
constexpr uint32_t kVersion = 4;           // eight features, ReLU, corrections of an x_HI baseline
// Gate calibration: a bin's error is kGateSafety times the largest held-out error in it
// (the held-out maximum of a few dozen samples underestimates the bin's true maximum), with
// the relative temperature error counted against kTempTol times the fraction tolerance.
constexpr float kGateSafety = 2.0f;
constexpr double kTempTol = 10.0;

struct Blob {
    uint32_t magic, version, nparams, pad;
    Model model;
    float params[kNParams];
};

hipError_t ensure_bytes(void** p, size_t* cap, size_t need)
{
    if (*p && *cap >= need) return hipSuccess;
    if (*p) {
        hipError_t e = hipFree(*p);
        if (e != hipSuccess) return e;
        *p = nullptr;
        *cap = 0;
    }
    hipError_t e = hipMalloc(p, need);
    if (e == hipSuccess) *cap = need;
    return e;
}

int gate_bin(const float* f, const float* lo, const float* hi)
{
    int bin = 0;
    for (int k = kGateDims - 1; k >= 0; --k) {
        const float u = (f[k] - lo[k]) * (1.0f / (hi[k] - lo[k]));  // as the inference kernel bins
        const int b = std::min(kGate - 1, std::max(0, (int)(u * kGate)));
        bin = bin * kGate + b;
    }
    return bin;
}

}  // namespace

extern "C" {

arc_status arc_mlp_create(arc_ctx* ctx, arc_mlp** out)
{
    if (!ctx || !out) return ARC_E_ARG;
    *out = nullptr;
    arc_mlp* m = new (std::nothrow) arc_mlp();
    if (!m) return ARC_E_NOMEM;
    m->device = arc::ctx_device(ctx);
    if (hipSetDevice(m->device) != hipSuccess) {
        delete m;
        return ARC_E_DEVICE;
    }
    if (hipMalloc((void**)&m->model, sizeof(Model)) != hipSuccess ||
        hipMalloc((void**)&m->params, 3 * kNParams * sizeof(float)) != hipSuccess) {
        arc_mlp_destroy(m);
        return ARC_E_NOMEM;
    }
    if (hipMemset(m->model, 0, sizeof(Model)) != hipSuccess ||
        hipMemset(m->params, 0, 3 * kNParams * sizeof(float)) != hipSuccess) {
        arc_mlp_destroy(m);
        return ARC_E_DEVICE;
    }
    *out = m;
    return ARC_OK;
}

void arc_mlp_destroy(arc_mlp* m)
{
    if (!m) return;
    (void)hipSetDevice(m->device);
    if (m->model) (void)hipFree(m->model);
    if (m->params) (void)hipFree(m->params);
    delete m;
}

arc_status arc_mlp_train(arc_ctx* ctx, arc_mlp* mlp, const float* X, const float* Y, int64_t m,
                         const arc_train_params* p, arc_train_report* rep)
{
    if (!ctx || !mlp || !X || !Y || !p) return ARC_E_ARG;
    if (m < 1024 || m > (int64_t)1 << 28) return arc::ctx_fail(ctx, ARC_E_ARG, "sample count must be in [1024, 2^28]");
    if (p->epochs < 1 || p->batch < 64 || !(p->lr > 0) || !(p->val_frac > 0 && p->val_frac < 1))
        return arc::ctx_fail(ctx, ARC_E_ARG, "bad training parameters");
    const auto t_start = std::chrono::steady_clock::now();
    hipStream_t st = (hipStream_t)p->stream;
    if (hipSetDevice(mlp->device) != hipSuccess) return ARC_E_DEVICE;
#define TRY(expr)                                                                                      \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) return arc::ctx_fail(ctx, ARC_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

    // features and targets on the device, then the standardisation on the host
    float* F = nullptr;
    float* Yt = nullptr;
    float* P = nullptr;
    uint32_t* idx = nullptr;
    float* partial = nullptr;
    struct Guard {
        std::vector<void*> ptrs;
        ~Guard()
        {
            for (void* q : ptrs)
                if (q) (void)hipFree(q);
        }
    } guard;
    TRY(hipMalloc((void**)&F, (size_t)m * kIn * sizeof(float)));
    guard.ptrs.push_back(F);
    TRY(hipMalloc((void**)&Yt, (size_t)m * 2 * sizeof(float)));
    guard.ptrs.push_back(Yt);
    if (!(p->y_he >= 0) || !std::isfinite(p->y_he)) return arc::ctx_fail(ctx, ARC_E_RANGE, "y_he must be >= 0");
    TRY(launch_features(X, Y, (uint32_t)m, (float)p->y_he, p->collisional ? 1 : 0, F, Yt, st));
    std::vector<float> hF((size_t)m * kIn), hY((size_t)m * 2);
    TRY(hipMemcpyAsync(hF.data(), F, hF.size() * sizeof(float), hipMemcpyDeviceToHost, st));
    TRY(hipMemcpyAsync(hY.data(), Yt, hY.size() * sizeof(float), hipMemcpyDeviceToHost, st));
    TRY(hipStreamSynchronize(st));
    for (size_t i = 0; i < hF.size(); ++i)
        if (!std::isfinite(hF[i])) return arc::ctx_fail(ctx, ARC_E_RANGE, "non-finite training input (sample %zu)", i / kIn);
    for (size_t i = 0; i < hY.size(); ++i)
        if (!std::isfinite(hY[i])) return arc::ctx_fail(ctx, ARC_E_RANGE, "non-finite training target (sample %zu)", i / 2);

    // deterministic split: a seeded permutation, the first val_frac of it held out
    std::vector<uint32_t> order((size_t)m);
    std::iota(order.begin(), order.end(), 0u);
    std::mt19937_64 rng(p->seed);
    std::shuffle(order.begin(), order.end(), rng);
    const size_t n_val = std::max<size_t>(64, (size_t)(p->val_frac * (double)m));
    const size_t n_train = (size_t)m - n_val;
    std::vector<uint32_t> val(order.begin(), order.begin() + n_val), train(order.begin() + n_val, order.end());

    Model hm;
    std::memset(&hm, 0, sizeof hm);
    hm.base_y = (float)p->y_he;
    hm.base_collisional = p->collisional ? 1 : 0;
    for (int k = 0; k < kIn; ++k) {
        double s = 0, s2 = 0;
        float lo = INFINITY, hi = -INFINITY;
        for (uint32_t i : train) {
            const double v = hF[(size_t)i * kIn + k];
            s += v;
            s2 += v * v;
            lo = std::min(lo, (float)v);
            hi = std::max(hi, (float)v);
        }
        const double mu = s / n_train, sd = std::sqrt(std::max(1e-12, s2 / n_train - mu * mu));
        hm.in_mu[k] = (float)mu;
        hm.in_sd[k] = (float)sd;
        hm.lo[k] = lo;
        hm.hi[k] = hi > lo ? hi : lo + 1e-6f;
    }
    for (int k = 0; k < kOut; ++k) {
        double s = 0, s2 = 0;
        for (uint32_t i : train) {
            const double v = hY[(size_t)i * 2 + k];
            s += v;
            s2 += v * v;
        }
        const double mu = s / n_train, sd = std::sqrt(std::max(1e-12, s2 / n_train - mu * mu));
        hm.out_mu[k] = (float)mu;
        hm.out_sd[k] = (float)sd;
    }
    // gate counts from the training samples (raw features)
    for (uint32_t i : train) hm.gate_count[gate_bin(&hF[(size_t)i * kIn], hm.lo, hm.hi)]++;
    // standardised copies for training
    std::vector<float> sF(hF), sY(hY);
    for (size_t i = 0; i < (size_t)m; ++i) {
        for (int k = 0; k < kIn; ++k) sF[i * kIn + k] = (hF[i * kIn + k] - hm.in_mu[k]) * (1.0f / hm.in_sd[k]);
        for (int k = 0; k < kOut; ++k) sY[i * 2 + k] = (hY[i * 2 + k] - hm.out_mu[k]) / hm.out_sd[k];
    }
    TRY(hipMemcpyAsync(F, sF.data(), sF.size() * sizeof(float), hipMemcpyHostToDevice, st));
    TRY(hipMemcpyAsync(Yt, sY.data(), sY.size() * sizeof(float), hipMemcpyHostToDevice, st));

    // initial parameters: uniform(-a, a) with a = sqrt(6 / (fan_in + fan_out)), biases 0
    std::vector<float> params(kNParams, 0.0f);
    auto init = [&](int off, int fin, int fout) {
        std::uniform_real_distribution<float> u(-std::sqrt(6.0f / (fin + fout)), std::sqrt(6.0f / (fin + fout)));
        for (int i = 0; i < fin * fout; ++i) params[off + i] = u(rng);
    };
    init(kW1, kIn, kHid);
    init(kW2, kHid, kHid);
    init(kW3, kHid, kOut);
    TRY(hipMemcpyAsync(mlp->params, params.data(), kNParams * sizeof(float), hipMemcpyHostToDevice, st));
    TRY(hipMemsetAsync(mlp->params + kNParams, 0, 2 * kNParams * sizeof(float), st));
    TRY(hipMemcpyAsync(mlp->model, &hm, sizeof hm, hipMemcpyHostToDevice, st));
    TRY(launch_publish(mlp->params, mlp->model, st));

    // minibatch Adam
    const int batch = p->batch;
    const int max_waves = (batch + 63) / 64;
    TRY(hipMalloc((void**)&idx, n_train * sizeof(uint32_t)));
    guard.ptrs.push_back(idx);
    TRY(hipMalloc((void**)&partial, (size_t)max_waves * kNParams * sizeof(float)));
    guard.ptrs.push_back(partial);
    int step = 0;
    const double total_steps = (double)p->epochs * (double)((n_train + batch - 1) / batch);
    for (int ep = 0; ep < p->epochs; ++ep) {
        std::shuffle(train.begin(), train.end(), rng);
        TRY(hipMemcpyAsync(idx, train.data(), n_train * sizeof(uint32_t), hipMemcpyHostToDevice, st));
        TRY(hipStreamSynchronize(st));  // train is reshuffled next epoch
        for (size_t first = 0; first < n_train; first += batch) {
            const uint32_t count = (uint32_t)std::min<size_t>(batch, n_train - first);
            TrainArgs ta{mlp->model, F, Yt, idx, (uint32_t)first, count, partial};
            TRY(launch_train_grad(ta, st));
            AdamArgs aa{};
            aa.params = mlp->params;
            aa.m = mlp->params + kNParams;
            aa.v = mlp->params + 2 * kNParams;
            aa.partial = partial;
            aa.nwaves = (int)((count + 63) / 64);
            // cosine decay from lr to lr/20 over the run: the late small steps settle the
            // minibatch noise that a constant rate leaves in the weights
            const double frac = (double)step / total_steps;
            aa.lr = (float)(p->lr * (0.05 + 0.95 * 0.5 * (1.0 + std::cos(M_PI * frac))));
            aa.beta1 = 0.9f;
            aa.beta2 = 0.999f;
            aa.eps = 1e-8f;
            aa.inv_batch = 1.0f / (float)count;
            aa.step = ++step;
            aa.model = mlp->model;
            TRY(launch_adam(aa, st));
        }
    }

    // held-out predictions (the inference arithmetic, from the raw samples), errors and
    // the gate calibration
    std::vector<float> rY((size_t)m * 2);
    TRY(hipMemcpyAsync(rY.data(), Y, rY.size() * sizeof(float), hipMemcpyDeviceToHost, st));
    uint32_t* dval = nullptr;
    TRY(hipMalloc((void**)&dval, n_val * sizeof(uint32_t)));
    guard.ptrs.push_back(dval);
    TRY(hipMalloc((void**)&P, n_val * 2 * sizeof(float)));
    guard.ptrs.push_back(P);
    TRY(hipMemcpyAsync(dval, val.data(), n_val * sizeof(uint32_t), hipMemcpyHostToDevice, st));
    TRY(launch_predict(mlp->model, X, dval, (uint32_t)n_val, P, st));
    std::vector<float> hP(n_val * 2);
    TRY(hipMemcpyAsync(hP.data(), P, hP.size() * sizeof(float), hipMemcpyDeviceToHost, st));
    TRY(hipStreamSynchronize(st));
    double se_x = 0, se_t = 0, emax = 0;
    for (size_t j = 0; j < n_val; ++j) {
        const uint32_t i = val[j];
        const double ex = std::fabs((double)hP[2 * j] - (double)rY[(size_t)i * 2]);
        const double et = std::fabs((double)hP[2 * j + 1] / (double)rY[(size_t)i * 2 + 1] - 1.0);
        const double dl = std::log10((double)hP[2 * j + 1] / (double)rY[(size_t)i * 2 + 1]);
        se_x += ex * ex;
        se_t += dl * dl;
        // one error per sample: the x_HI' error, or the relative T' error over kTempTol
        const float e = (float)std::max(ex, et / kTempTol);
        emax = std::max(emax, (double)e);
        const int b = gate_bin(&hF[(size_t)i * kIn], hm.lo, hm.hi);
        hm.gate_err[b] = std::max(hm.gate_err[b], kGateSafety * e);
    }
    // bins without held-out samples stay closed
    {
        std::vector<uint8_t> seen(kGateBins, 0);
        for (size_t j = 0; j < n_val; ++j) seen[gate_bin(&hF[(size_t)val[j] * kIn], hm.lo, hm.hi)] = 1;
        for (int b = 0; b < kGateBins; ++b)
            if (!seen[b]) hm.gate_err[b] = INFINITY;
    }
    // publish the gate into the device model (the weights already live there)
    TRY(hipMemcpyAsync((char*)mlp->model + offsetof(Model, gate_count), hm.gate_count, sizeof hm.gate_count,
                       hipMemcpyHostToDevice, st));
    TRY(hipMemcpyAsync((char*)mlp->model + offsetof(Model, gate_err), hm.gate_err, sizeof hm.gate_err,
                       hipMemcpyHostToDevice, st));
    TRY(hipStreamSynchronize(st));
    mlp->trained = true;
    if (rep) {
        rep->val_rmse_x = std::sqrt(se_x / n_val);
        rep->val_rmse_logt = std::sqrt(se_t / n_val);
        rep->val_max_err = emax;
        rep->n_train = (int64_t)n_train;
        rep->n_val = (int64_t)n_val;
        int64_t used = 0;
        for (int b = 0; b < kGateBins; ++b) used += hm.gate_count[b] > 0;
        rep->bins_used = used;
        rep->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    }
#undef TRY
    return ARC_OK;
}

arc_status arc_mlp_save(const arc_mlp* mlp, void* buf, size_t* size)
{
    if (!mlp || !size) return ARC_E_ARG;
    if (!buf) {
        *size = sizeof(Blob);
        return ARC_OK;
    }
    if (*size < sizeof(Blob)) return ARC_E_ARG;
    if (!mlp->trained) return ARC_E_ARG;
    if (hipSetDevice(mlp->device) != hipSuccess) return ARC_E_DEVICE;
    Blob* b = new (std::nothrow) Blob();
    if (!b) return ARC_E_NOMEM;
    b->magic = kMagic;
    b->version = kVersion;
    b->nparams = kNParams;
    b->pad = 0;
    bool ok = hipMemcpy(&b->model, mlp->model, sizeof(Model), hipMemcpyDeviceToHost) == hipSuccess &&
              hipMemcpy(b->params, mlp->params, sizeof b->params, hipMemcpyDeviceToHost) == hipSuccess;
    if (ok) std::memcpy(buf, b, sizeof(Blob));
    delete b;
    *size = sizeof(Blob);
    return ok ? ARC_OK : ARC_E_DEVICE;
}

arc_status arc_mlp_load(arc_mlp* mlp, const void* buf, size_t size)
{
    if (!mlp || !buf || size < sizeof(Blob)) return ARC_E_ARG;
    Blob* b = new (std::nothrow) Blob();
    if (!b) return ARC_E_NOMEM;
    std::memcpy(b, buf, sizeof(Blob));
    if (b->magic != kMagic || b->version != kVersion || b->nparams != (uint32_t)kNParams) {
        delete b;
        return ARC_E_ARG;
    }
    if (hipSetDevice(mlp->device) != hipSuccess) {
        delete b;
        return ARC_E_DEVICE;
    }
    bool ok = hipMemcpy(mlp->model, &b->model, sizeof(Model), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(mlp->params, b->params, sizeof b->params, hipMemcpyHostToDevice) == hipSuccess;
    delete b;
    if (!ok) return ARC_E_DEVICE;
    mlp->trained = true;
    return ARC_OK;
}

arc_status arc_mlp_predict(arc_ctx* ctx, const arc_mlp* mlp, const float* X, int64_t m, float* P, void* stream)
{
    if (!ctx || !mlp || !X || !P || m < 0) return ARC_E_ARG;
    if (!mlp->trained) return arc::ctx_fail(ctx, ARC_E_ARG, "network not trained");
    if (m == 0) return ARC_OK;
    hipStream_t st = (hipStream_t)stream;
    if (hipSetDevice(mlp->device) != hipSuccess) return ARC_E_DEVICE;
    if (m > (int64_t)UINT32_MAX) return arc::ctx_fail(ctx, ARC_E_ARG, "too many samples");
    const hipError_t e = launch_predict(mlp->model, X, nullptr, (uint32_t)m, P, st);
    return e == hipSuccess ? ARC_OK : arc::ctx_fail(ctx, ARC_E_DEVICE, "prediction failed: %s", hipGetErrorString(e));
}

}  // extern "C"
