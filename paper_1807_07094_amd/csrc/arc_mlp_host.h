// arc_mlp_host.h -- host-side state of a learned chemistry network, shared by the
// C ABI translation units.
#pragma once

#include "arc.h"
#include "arc_mlp.h"

struct arc_mlp {
    int device = 0;
    arc::mlp::Model* model = nullptr;  // device: weights, standardisation, gate
    float* params = nullptr;           // device: FP32 master parameters, Adam m and v
    bool trained = false;
};

namespace arc {
int ctx_device(const arc_ctx* c);
arc_status ctx_fail(arc_ctx* c, arc_status s, const char* fmt, ...);
}  // namespace arc
