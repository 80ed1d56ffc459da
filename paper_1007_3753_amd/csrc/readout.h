// Read-outs that run after a batched solve (csrc/classify.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace l1 {

// Per-subject residuals ||b - e - A delta_i(x)||_2 and their argmin, one
// workgroup per instance; `res` (C x N) may be null, `e` may be null.
void class_residuals(hipStream_t s, const float* A, int m, int n_dict, int lda, const float* x, int ldx,
                     const float* e, int lde, const float* b, int ldb, int N, const int* ptr, int C,
                     float* res, int* label);

}  // namespace l1
