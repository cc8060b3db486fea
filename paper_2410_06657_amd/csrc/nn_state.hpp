// Internal state of a network handle (shared by the network entry points and the warm-start
// entry points of the solver).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>


// hidden activation buffers: one per layer but the last (six layers)
constexpr int NN_HIDDEN = 5;

struct lbm_nn {
    int64_t cap = 0;           // pixel capacity of the activation buffers
    hipStream_t stream = nullptr;
    float* p = nullptr;        // FP32 master parameters: weights (layer by layer) then biases
    float* mo = nullptr;       // Adam first moments
    float* ve = nullptr;       // Adam second moments
    float* g = nullptr;        // gradient
    _Float16* wh = nullptr;    // FP16 weights
    _Float16* wflip = nullptr; // flipped weights of the layer being propagated
    _Float16* xh = nullptr;    // packed input (8 channels)
    _Float16* act[NN_HIDDEN] = {};  // hidden activations
    _Float16* dz[2] = {};      // gradients w.r.t. pre-activations (ping-pong)
    float* x = nullptr;        // FP32 input maps (3 channels), for callers without their own
    float* y = nullptr;        // FP32 output
    double* lpart = nullptr;   // loss partials
    double* lsum = nullptr;    // loss (device)
    float* dwpart = nullptr;   // weight-gradient partials
    double* hloss = nullptr;   // pinned host copy of the loss
    long long t = 0;           // Adam step
    std::string err;
};

namespace nnapi {
constexpr int DW_PARTS = 120;  // workgroups of the weight-gradient kernel
// Forward pass of n images of h x w from x (FP32 NHWC, 3 maps) to y (FP32), on `stream`.
int forward(lbm_nn* nn, const float* x, float* y, int n, int h, int w, hipStream_t stream);
}  // namespace nnapi
