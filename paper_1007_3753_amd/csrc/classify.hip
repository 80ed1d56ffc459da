// The recognition criterion of the face experiments (Sec. VI-B): per
// instance, the l1 mass of every subject's coefficients, the subject with the
// largest mass and its sparsity concentration index.  One workgroup per
// instance; masses and the norm are summed in FP64 in a fixed order, so the
// label is decided in the same precision as the FP64 definition.
#include "internal.h"
#include "readout.h"

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

// The residual rule of the sparse-representation classifier the paper builds
// on (Sec. I, Sec. II-A): res_i = ||b - e - A delta_i(x)||_2 for every subject
// i, label = argmin_i res_i (the lowest i among equal residuals).  One
// workgroup per instance.  The subjects are taken 16 at a time: every thread
// walks its rows (tid + 256 r) and, per row, forms A delta_i(x) for the 16
// subjects and adds the squared residuals into 16 FP64 registers (all
// arithmetic in FP64 from the FP32 inputs, so the label is decided in the
// precision of the definition); the 16 sums are reduced over the workgroup
// in a fixed order (DPP row sums, then 16 row partials through LDS).
constexpr int RES_CHUNK = 16;

namespace {

template <int N>
__device__ inline double res_row_ror(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x120 + N, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x120 + N, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// sum over the 16 lanes of this lane's row (read it from one lane); every
// lane of the wave must be active
__device__ inline double res_row_sum(double v) {
  v += res_row_ror<8>(v);
  v += res_row_ror<4>(v);
  v += res_row_ror<2>(v);
  v += res_row_ror<1>(v);
  return v;
}

}  // namespace

__global__ __launch_bounds__(CLS_THREADS) void class_residual_kernel(const float* A, int m, int n_dict, int lda,
                                                                     const float* x, int ldx, const float* e,
                                                                     int lde, const float* b, int ldb,
                                                                     const int* ptr, int C, float* res_out,
                                                                     int* label_out) {
  extern __shared__ double s_res2[];                  // C squared residuals
  __shared__ double s_part[2][16][RES_CHUNK];         // 16 row partials per subject, two chunks
  __shared__ double s_val[CLS_THREADS];
  __shared__ int s_arg[CLS_THREADS];
  const int j = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
  const int slot = (tid >> 6) * 4 + (lane >> 4);
  const float* xj = x + (long)j * ldx;
  const float* bj = b + (long)j * ldb;
  const float* ej = e ? e + (long)j * lde : nullptr;
  const int nchunk = (C + RES_CHUNK - 1) / RES_CHUNK;
  for (int ch = 0; ch < nchunk; ++ch) {
    int lo[RES_CHUNK], hi[RES_CHUNK];
#pragma unroll
    for (int q = 0; q < RES_CHUNK; ++q) {
      const int c = ch * RES_CHUNK + q;
      // ranges are clamped to the columns, a decreasing one is empty
      lo[q] = c < C ? min(max(ptr[c], 0), n_dict) : 0;
      hi[q] = c < C ? min(max(ptr[c + 1], lo[q]), n_dict) : 0;
    }
    double acc[RES_CHUNK];
#pragma unroll
    for (int q = 0; q < RES_CHUNK; ++q) acc[q] = 0.0;
    for (int i = tid; i < m; i += CLS_THREADS) {
      const double t = (double)bj[i] - (ej ? (double)ej[i] : 0.0);
#pragma unroll
      for (int q = 0; q < RES_CHUNK; ++q) {
        double y = 0.0;
        for (int k = lo[q]; k < hi[q]; ++k) y += (double)A[i + (long)lda * k] * (double)xj[k];
        const double r = t - y;
        acc[q] += r * r;
      }
    }
#pragma unroll
    for (int q = 0; q < RES_CHUNK; ++q) {
      const double v = res_row_sum(acc[q]);
      if ((lane & 15) == 0) s_part[ch & 1][slot][q] = v;
    }
    __syncthreads();
    if (tid < RES_CHUNK && ch * RES_CHUNK + tid < C) {
      double r2 = 0.0;
#pragma unroll
      for (int p = 0; p < 16; ++p) r2 += s_part[ch & 1][p][tid];
      s_res2[ch * RES_CHUNK + tid] = r2;
    }
  }
  __syncthreads();
  // the residuals, and per thread the first smallest of its subjects
  double best = 0.0;
  int arg = -1;
  for (int c = tid; c < C; c += CLS_THREADS) {
    const double r = sqrt(s_res2[c]);
    if (res_out) res_out[(long)j * C + c] = (float)r;
    if (arg < 0 || r < best) {
      best = r;
      arg = c;
    }
  }
  s_val[tid] = best;
  s_arg[tid] = arg;
  __syncthreads();
  // fixed-shape tree: the smallest residual, the lowest subject among equals
  for (int h = CLS_THREADS / 2; h > 0; h >>= 1) {
    if (tid < h) {
      const int a0 = s_arg[tid], a1 = s_arg[tid + h];
      const double v0 = s_val[tid], v1 = s_val[tid + h];
      if (a1 >= 0 && (a0 < 0 || v1 < v0 || (v1 == v0 && a1 < a0))) {
        s_arg[tid] = a1;
        s_val[tid] = v1;
      }
    }
    __syncthreads();
  }
  if (tid == 0) label_out[j] = s_arg[0];
}

void class_residuals(hipStream_t s, const float* A, int m, int n_dict, int lda, const float* x, int ldx,
                     const float* e, int lde, const float* b, int ldb, int N, const int* ptr, int C,
                     float* res, int* label) {
  if (N <= 0) return;
  const size_t lds = sizeof(double) * (size_t)C;
  class_residual_kernel<<<N, CLS_THREADS, lds, s>>>(A, m, n_dict, lda, x, ldx, e, lde, b, ldb, ptr, C, res,
                                                    label);
  L1_HIP(hipGetLastError());
}

void classify(hipStream_t s, const float* x, int ldx, int n_dict, int N, const int* ptr, int C,
              float* mass, int* label, float* score) {
  if (N <= 0) return;
  const size_t lds = sizeof(double) * (size_t)C;
  classify_kernel<<<N, CLS_THREADS, lds, s>>>(x, ldx, n_dict, ptr, C, mass, label, score);
  L1_HIP(hipGetLastError());
}

}  // namespace l1
