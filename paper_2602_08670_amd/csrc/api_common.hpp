// Shared pieces of the C-ABI host code (solver, training, serving).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "../../include/fv.h"
#include "cnn_internal.hpp"

namespace fvapi {

// Record a thread-local error message (fv_last_error) and return code.
fv_status fail(fv_status code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
fv_status hip_fail(hipError_t e, const char *what);
const char *last_error();

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace fvapi

struct fv_model {
    fv_model_desc desc;
    const float *params;  // FP32 master vector (caller-owned)
    void *packed;         // packed BF16 weights (caller-owned workspace)
    hipStream_t stream;
    cnn::Norm nrm;
    cnn::Proj pr;
};
