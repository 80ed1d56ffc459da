// The recognition criterion of the face experiments (Sec. VI-B): per
// instance, the l1 mass of every subject's coefficients, the subject with the
// largest mass and its sparsity concentration index.  One workgroup per
// instance; masses and the norm are summed in FP64 in a fixed order, so the
// label is decided in the same precision as the FP64 definition.
#include "internal.h"

namespace l1 {

constexpr int CLS_THREADS = 256;

__global__ __launch_bounds__(CLS_THREADS) void classify_kernel(const float* x, int ldx, int n_dict,
                                                               const int* ptr, int C, float* mass_out,
                                                               int* label_out, float* score_out) {
  extern __shared__ double s_mass[];                 // C masses
  __shared__ double s_sum[CLS_THREADS];
  __shared__ int s_arg[CLS_THREADS];
  const int j = blockIdx.x, tid = threadIdx.x;
  const float* xj = x + (long)j * ldx;
  for (int c = tid; c < C; c += CLS_THREADS) {
    // ranges are clamped to the columns, a decreasing one is empty
    const int lo = min(max(ptr[c], 0), n_dict), hi = min(max(ptr[c + 1], lo), n_dict);
    double m = 0.0;
    for (int k = lo; k < hi; ++k) m += fabs((double)xj[k]);
    s_mass[c] = m;
    if (mass_out) mass_out[(long)j * C + c] = (float)m;
  }
  __syncthreads();
  // per thread: its subjects' sum and first maximum, in subject order
  double sum = 0.0, best = -1.0;
  int arg = -1;
  for (int c = tid; c < C; c += CLS_THREADS) {
    const double m = s_mass[c];
    sum += m;
    if (m > best) {
      best = m;
      arg = c;
    }
  }
  s_sum[tid] = sum;
  s_arg[tid] = arg;
  __syncthreads();
  // fixed-shape tree over the threads: the norm, and the largest mass with
  // the lowest subject index among equals
  for (int h = CLS_THREADS / 2; h > 0; h >>= 1) {
    if (tid < h) {
      s_sum[tid] += s_sum[tid + h];
      const int a = s_arg[tid], b = s_arg[tid + h];
      if (b >= 0 && (a < 0 || s_mass[b] > s_mass[a] || (s_mass[b] == s_mass[a] && b < a))) s_arg[tid] = b;
    }
    __syncthreads();
  }
  if (tid == 0) {
    const double total = s_sum[0];
    const int a = s_arg[0];
    if (total > 0.0 && a >= 0) {
      label_out[j] = a;
      score_out[j] = (float)(((double)C * s_mass[a] / total - 1.0) / (double)(C - 1));
    } else {
      label_out[j] = -1;
      score_out[j] = 0.0f;
    }
  }
}

void classify(hipStream_t s, const float* x, int ldx, int n_dict, int N, const int* ptr, int C,
              float* mass, int* label, float* score) {
  if (N <= 0) return;
  const size_t lds = sizeof(double) * (size_t)C;
  classify_kernel<<<N, CLS_THREADS, lds, s>>>(x, ldx, n_dict, ptr, C, mass, label, score);
  L1_HIP(hipGetLastError());
}

}  // namespace l1
