// The l1 problem of the alignment step (Sec. II-B, eq. (align-simple)),
//     min ||e||_1  s.t.  b = B_j w + e,   B_j m x k, k = n_i + q_i small,
// solved for a batch of instances, each with its own dictionary, by the
// primal ALM as the alignment experiment runs it (Sec. V-A / Algorithm 1
// with the unpenalised block, Sec. VI-C):
//     e     <- shrink(b - B w + theta/xi, 1/xi)
//     w     <- (B^T B)^{-1} B^T (b - e + theta/xi)      (the exact minimiser)
//     theta <- theta + xi (b - B w - e)
// from w = 0, theta = 0, xi = 2m/||b||_1, until ||w_new - w|| < tol ||w||.
//
// One workgroup per instance runs all of its iterations in one launch: its
// dictionary stays in LDS, b, e and theta in registers (rows tid + 256 r).
// Per iteration the dictionary is read twice from LDS (B w and B^T s); the
// k x k inverse of B^T B is formed once in FP64, and B^T s is summed and
// multiplied by it in FP64, so the normal equations do not square the
// dictionary's condition number in FP32.
#include "internal.h"

namespace l1 {

namespace {

constexpr int AL_THREADS = 256;

__device__ inline float softa(float x, float a) {
  const float m = fabsf(x) - a;
  return m > 0.0f ? copysignf(m, x) : 0.0f;
}

// sum of v over the workgroup (all threads call; result in every thread)
__device__ inline double wg_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

}  // namespace

__global__ __launch_bounds__(AL_THREADS) void align_kernel(const float* Bg, int m, int k, const float* bg,
                                                           int ldb, float tol, int cap, int fixed,
                                                           float* wg, float* eg, int lde, int* iters,
                                                           int* status) {
  extern __shared__ __attribute__((aligned(16))) float sB[];   // m x k, column-major
  __shared__ double s_ginv[ALIGN_KMAX][ALIGN_KMAX];
  __shared__ double s_g[ALIGN_KMAX];
  __shared__ double s_red[4];
  __shared__ double s_part[4][ALIGN_KMAX];
  __shared__ double s_aug[ALIGN_KMAX][2 * ALIGN_KMAX];
  __shared__ double s_fac[ALIGN_KMAX];
  __shared__ float s_w[ALIGN_KMAX];
  __shared__ int s_flag;
  const int j = blockIdx.x, tid = threadIdx.x;
  const float* B = Bg + (long)j * m * k;
  for (int i = tid; i < m * k; i += AL_THREADS) sB[i] = B[i];
  float bv[ALIGN_R], ev[ALIGN_R], th[ALIGN_R], tv[ALIGN_R];
  double n1 = 0.0;
#pragma unroll
  for (int r = 0; r < ALIGN_R; ++r) {
    const int i = tid + AL_THREADS * r;
    bv[r] = i < m ? bg[(long)j * ldb + i] : 0.0f;
    ev[r] = bv[r];
    th[r] = 0.0f;
    tv[r] = 0.0f;   // B w with w = 0
    n1 += fabs((double)bv[r]);
  }
  n1 = wg_sum(n1, s_red);
  const float xi = n1 > 0.0 ? (float)(2.0 * m / n1) : 1.0f;
  const float ixi = 1.0f / xi;

  // Gram matrix G = B^T B (FP64), one column of it per pass
  for (int c = 0; c < k; ++c) {
    double p[ALIGN_KMAX];
#pragma unroll
    for (int d = 0; d < ALIGN_KMAX; ++d) p[d] = 0.0;
    for (int i = tid; i < m; i += AL_THREADS) {
      const double bc = sB[i + (long)m * c];
#pragma unroll
      for (int d = 0; d < ALIGN_KMAX; ++d)
        if (d < k) p[d] += bc * (double)sB[i + (long)m * d];
    }
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int d = 0; d < ALIGN_KMAX; ++d) {
      double v = p[d];
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
      if (lane == 0 && d < k) s_part[wave][d] = v;
    }
    __syncthreads();
    if (tid < k) s_ginv[c][tid] = (s_part[0][tid] + s_part[1][tid]) + (s_part[2][tid] + s_part[3][tid]);
    __syncthreads();
  }
  // its inverse (Gauss-Jordan on [G | I] in LDS, the row operations of a
  // pivot spread over the threads)
  {
    const int w2 = 2 * k;
    for (int t = tid; t < k * w2; t += AL_THREADS) {
      const int r = t / w2, c = t % w2;
      s_aug[r][c] = c < k ? s_ginv[r][c] : (c - k == r ? 1.0 : 0.0);
    }
    if (tid == 0) s_flag = 1;
    __syncthreads();
    for (int pv = 0; pv < k; ++pv) {
      // s_ginv still holds G here: a pivot below 1e-12 of its diagonal
      // entry marks a rank-deficient dictionary
      const double piv = s_aug[pv][pv];
      if (!(piv > 1e-12 * s_ginv[pv][pv])) {
        if (tid == 0) s_flag = 0;
        break;   // uniform: every thread read the same pivot
      }
      if (tid < k) s_fac[tid] = s_aug[tid][pv];
      __syncthreads();
      if (tid < w2) s_aug[pv][tid] /= piv;
      __syncthreads();
      for (int t = tid; t < k * w2; t += AL_THREADS) {
        const int r = t / w2, c = t % w2;
        if (r != pv) s_aug[r][c] -= s_fac[r] * s_aug[pv][c];
      }
      __syncthreads();
    }
    __syncthreads();
    for (int t = tid; t < k * k; t += AL_THREADS) {
      const int r = t / k, c = t % k;
      s_ginv[r][c] = s_flag ? s_aug[r][k + c] : 0.0;
    }
  }
  if (tid < ALIGN_KMAX) s_w[tid] = 0.0f;
  __syncthreads();
  if (!s_flag) {
    if (tid < k) wg[(long)j * k + tid] = 0.0f;
    for (int i = tid; i < m; i += AL_THREADS) eg[(long)j * lde + i] = bg[(long)j * ldb + i];
    if (tid == 0) {
      iters[j] = 0;
      status[j] = L1_NONFINITE;
    }
    return;
  }

  int it = 0, st = L1_MAXITER;
  for (it = 1; it <= cap; ++it) {
    // e-step and s = b - e + theta/xi; partial B^T s in FP64
    double p[ALIGN_KMAX];
#pragma unroll
    for (int d = 0; d < ALIGN_KMAX; ++d) p[d] = 0.0;
#pragma unroll
    for (int r = 0; r < ALIGN_R; ++r) {
      const int i = tid + AL_THREADS * r;
      if (i < m) {
        ev[r] = softa(bv[r] - tv[r] + th[r] * ixi, ixi);
        const double s = (double)(bv[r] - ev[r] + th[r] * ixi);
#pragma unroll
        for (int d = 0; d < ALIGN_KMAX; ++d)
          if (d < k) p[d] += (double)sB[i + (long)m * d] * s;
      }
    }
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int d = 0; d < ALIGN_KMAX; ++d) {
      double v = p[d];
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
      if (lane == 0 && d < k) s_part[wave][d] = v;
    }
    __syncthreads();
    if (tid < k) s_g[tid] = (s_part[0][tid] + s_part[1][tid]) + (s_part[2][tid] + s_part[3][tid]);
    __syncthreads();
    // w = G^{-1} g (FP64), the relative change of w, and its FP32 copy
    double wn = 0.0;
    if (tid < k) {
      for (int d = 0; d < k; ++d) wn += s_ginv[tid][d] * s_g[d];
    }
    double dw2 = 0.0, w2 = 0.0;
    if (tid < k) {
      const double wo = s_w[tid];
      dw2 = (wn - wo) * (wn - wo);
      w2 = wo * wo;
    }
    // reduce over the first wave (k <= 16 < 64)
    for (int o = 32; o > 0; o >>= 1) {
      dw2 += __shfl_xor(dw2, o);
      w2 += __shfl_xor(w2, o);
    }
    __syncthreads();   // every thread has read s_w (the old w)
    if (tid < k) s_w[tid] = (float)wn;
    if (tid == 0) {
      int f = 0;
      if (!(isfinite(dw2) && isfinite(w2))) f = 2;
      else if (!fixed && sqrt(dw2) < (double)tol * sqrt(w2)) f = 1;
      s_flag = f;
    }
    __syncthreads();
    // theta-step with t = B w (kept for the next e-step)
#pragma unroll
    for (int r = 0; r < ALIGN_R; ++r) {
      const int i = tid + AL_THREADS * r;
      if (i < m) {
        float t = 0.0f;
#pragma unroll
        for (int d = 0; d < ALIGN_KMAX; ++d)
          if (d < k) t += sB[i + (long)m * d] * s_w[d];
        tv[r] = t;
        th[r] += xi * (bv[r] - t - ev[r]);
      }
    }
    if (s_flag == 1) {
      st = L1_CONVERGED;
      break;
    }
    if (s_flag == 2) {
      st = L1_NONFINITE;
      break;
    }
  }
  if (it > cap) it = cap;
  if (tid < k) wg[(long)j * k + tid] = s_w[tid];
#pragma unroll
  for (int r = 0; r < ALIGN_R; ++r) {
    const int i = tid + AL_THREADS * r;
    if (i < m) eg[(long)j * lde + i] = ev[r];
  }
  if (tid == 0) {
    iters[j] = it;
    status[j] = st;
  }
}

void align_solve(hipStream_t s, const float* B, int m, int k, int N, const float* b, int ldb, float tol,
                 int max_iter, float* w, float* e, int lde, int* iters, int* status) {
  if (N <= 0) return;
  const size_t lds = sizeof(float) * (size_t)m * k;
  static const bool attr_ok =
      hipFuncSetAttribute(reinterpret_cast<const void*>(align_kernel),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)(sizeof(float) * ALIGN_MK_MAX)) ==
      hipSuccess;
  L1_REQUIRE(attr_ok, "cannot give the alignment kernel its LDS");
  const int fixed = max_iter < 0;
  const int cap = fixed ? -max_iter : max_iter;
  align_kernel<<<N, AL_THREADS, lds, s>>>(B, m, k, b, ldb, tol, cap, fixed, w, e, lde, iters, status);
  L1_HIP(hipGetLastError());
}

}  // namespace l1
