// The learned pruner's handle, shared by the pruner kernels and the
// checkpoint files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mhr.h"

struct mhr_pruner {
    uint32_t d = 0, H = 0;
    size_t np = 0;                      // parameter count
    float *theta = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;   // FP32 master weights, gradient, Adam moments
    uint16_t *W1b = nullptr, *W2b = nullptr, *w3b = nullptr;                 // bfloat16 copies for the products
    uint32_t step = 0;                  // Adam step count
    bool owns = true;                   // false: the arrays live in the caller's buffer
};

namespace mhr {
// Rewrites the bfloat16 copies of W1, W2 and w3 from the FP32 masters.
hipError_t pruner_refresh_bf16(mhr_pruner *p, hipStream_t st);
}  // namespace mhr
