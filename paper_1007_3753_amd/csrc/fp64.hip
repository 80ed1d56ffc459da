// FP64 kernels: the one-time factorisation of a plan (Gram matrix, blocked
// Cholesky, triangular inverse, operator assembly, power iteration for the
// FISTA step) and the FP64 optimality report.  The GEMM runs on the FP64
// matrix cores; the rest is LDS-tiled vector code.
#include "internal.h"

#include <cmath>

namespace l1 {

// ---------------------------------------------------------------------------
// GEMM: C = alpha op(A) op(B) + beta C (column-major), on the FP64 matrix
// cores.  64x64 tile per workgroup, K staged through LDS 32 at a time (the
// next slice's global loads in flight during the current one's MFMAs); wave w
// computes the 32x32 quarter (w / 2, w % 2) as 2x2 blocks of
// v_mfma_f64_16x16x4f64.  Operand lane layout: lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16] of a 16x4 / 4x16 step; accumulator register v of lane
// l holds D[l / 16 + 4 v][l % 16].
typedef double v4d64 __attribute__((ext_vector_type(4)));
constexpr int G64_KS = 32;   // K slice staged through LDS

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void gemm64_kernel(int M, int N, int K, double alpha,
                                                     const double* __restrict__ A, int lda,
                                                     const double* __restrict__ B, int ldb,
                                                     double beta, double* __restrict__ C,
                                                     int ldc) {
  __shared__ double As[G64_KS][68];   // As[k][i]
  __shared__ double Bs[G64_KS][68];   // Bs[k][j]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int fi = lane & 15, fk = lane >> 4;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
  v4d64 acc[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = v4d64{0.0, 0.0, 0.0, 0.0};
  // the next slice's elements of this thread, loaded while the current one
  // is multiplied (8 of A and 8 of B; the index along the contiguous
  // dimension of each operand runs over consecutive threads)
  double pa[8], pb[8];
  auto load = [&](int k0) {
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int e = tid + t * 256;
      int ii, kk;
      if (!TA) { ii = e & 63; kk = e >> 6; } else { kk = e & 31; ii = e >> 5; }
      const int gi = i0 + ii, gk = k0 + kk;
      pa[t] = (gi < M && gk < K) ? (TA ? A[gk + (long)gi * lda] : A[gi + (long)gk * lda]) : 0.0;
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int e = tid + t * 256;
      int jj, kk;
      if (!TB) { kk = e & 31; jj = e >> 5; } else { jj = e & 63; kk = e >> 6; }
      const int gj = j0 + jj, gk = k0 + kk;
      pb[t] = (gj < N && gk < K) ? (TB ? B[gj + (long)gk * ldb] : B[gk + (long)gj * ldb]) : 0.0;
    }
  };
  load(0);
  for (int k0 = 0; k0 < K; k0 += G64_KS) {
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int e = tid + t * 256;
      if (!TA) As[e >> 6][e & 63] = pa[t];
      else As[e & 31][e >> 5] = pa[t];
      if (!TB) Bs[e & 31][e >> 5] = pb[t];
      else Bs[e >> 6][e & 63] = pb[t];
    }
    __syncthreads();
    if (k0 + G64_KS < K) load(k0 + G64_KS);
#pragma unroll
    for (int ks = 0; ks < G64_KS / 4; ++ks) {
      const int kr = 4 * ks + fk;
      const double a0 = As[kr][wr + fi], a1 = As[kr][wr + 16 + fi];
      const double b0 = Bs[kr][wc + fi], b1 = Bs[kr][wc + 16 + fi];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gi = i0 + wr + 16 * bi + fk + 4 * v;
        const int gj = j0 + wc + 16 * bj + fi;
        if (gi < M && gj < N) {
          double* p = C + gi + (long)gj * ldc;
          const double r = alpha * acc[bi][bj][v];
          *p = (beta == 0.0) ? r : r + beta * (*p);
        }
      }
}

void gemm64(hipStream_t s, char ta, char tb, int M, int N, int K, double alpha,
            const double* A, int lda, const double* B, int ldb, double beta, double* C,
            int ldc) {
  if (M <= 0 || N <= 0) return;
  dim3 grid((M + 63) / 64, (N + 63) / 64);
  const bool TA = (ta == 'T'), TB = (tb == 'T');
  if (!TA && !TB) gemm64_kernel<false, false><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
  else if (!TA && TB) gemm64_kernel<false, true><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
  else if (TA && !TB) gemm64_kernel<true, false><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
  else gemm64_kernel<true, true><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
  L1_HIP(hipGetLastError());
}

__global__ void add_diag64_kernel(int n, double* A, int lda, double c) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) A[i + (long)i * lda] += c;
}
void add_diag64(hipStream_t s, int n, double* A, int lda, double c) {
  if (n <= 0) return;
  add_diag64_kernel<<<(n + 255) / 256, 256, 0, s>>>(n, A, lda, c);
  L1_HIP(hipGetLastError());
}

__global__ void f32_to_f64_kernel(int rows, int cols, const float* src, int lds, double* dst,
                                  int ldd) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)rows * cols) return;
  const int i = (int)(e % rows), k = (int)(e / rows);
  dst[i + (long)k * ldd] = (double)src[i + (long)k * lds];
}
void f32_to_f64(hipStream_t s, int rows, int cols, const float* src, int lds, double* dst,
                int ldd) {
  const long n = (long)rows * cols;
  if (n <= 0) return;
  f32_to_f64_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(rows, cols, src, lds, dst, ldd);
  L1_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Cholesky of one diagonal block (kb <= 64) in LDS, then the in-place inverse
// of the lower-triangular factor.  One workgroup.
__global__ __launch_bounds__(256) void potf2_kernel(double* A, int lda, int kb, int k0,
                                                    int* info, double* dinv) {
  __shared__ double a[64][65];
  __shared__ double tmp[64];
  const int tid = threadIdx.x;
  for (int e = tid; e < kb * kb; e += 256) {
    const int i = e % kb, k = e / kb;
    a[i][k] = A[i + (long)k * lda];
  }
  __syncthreads();
  for (int j = 0; j < kb; ++j) {
    if (tid == 0) {
      double d = a[j][j];
      if (!(d > 0.0)) {
        atomicCAS(info, 0, k0 + j + 1);
        d = 1.0;
      }
      a[j][j] = sqrt(d);
    }
    __syncthreads();
    const double ljj = a[j][j];
    for (int i = j + 1 + tid; i < kb; i += 256) a[i][j] /= ljj;
    __syncthreads();
    const int r = kb - j - 1;
    for (int e = tid; e < r * r; e += 256) {
      const int ii = j + 1 + e % r, kk = j + 1 + e / r;
      if (kk <= ii) a[ii][kk] -= a[ii][j] * a[kk][j];
    }
    __syncthreads();
  }
  for (int e = tid; e < kb * kb; e += 256) {
    const int i = e % kb, k = e / kb;
    A[i + (long)k * lda] = (k <= i) ? a[i][k] : 0.0;
  }
  __syncthreads();
  // in-place inverse of the lower-triangular factor, last column first
  for (int j = kb - 1; j >= 0; --j) {
    if (tid == 0) a[j][j] = 1.0 / a[j][j];
    __syncthreads();
    const double ajj = -a[j][j];
    double acc = 0.0;
    const int i = j + 1 + tid;
    if (tid < 64 && i < kb) {
      for (int p = j + 1; p <= i; ++p) acc += a[i][p] * a[p][j];
      tmp[tid] = acc;
    }
    __syncthreads();
    if (tid < 64 && i < kb) a[i][j] = ajj * tmp[tid];
    __syncthreads();
  }
  for (int e = tid; e < 64 * 64; e += 256) {
    const int i = e % 64, k = e / 64;
    dinv[i + k * 64] = (i < kb && k < kb && k <= i) ? a[i][k] : 0.0;
  }
}

__global__ void zero_upper64_kernel(int n, double* A, int lda) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * n) return;
  const int i = (int)(e % n), k = (int)(e / n);
  if (k > i) A[i + (long)k * lda] = 0.0;
}

void potrf64(hipStream_t s, int n, double* A, int lda, double* diaginv, int* info_dev,
             double* work) {
  L1_HIP(hipMemsetAsync(info_dev, 0, sizeof(int), s));
  for (int k0 = 0; k0 < n; k0 += 64) {
    const int kb = (n - k0 < 64) ? n - k0 : 64;
    double* dblk = diaginv + (long)(k0 / 64) * 64 * 64;
    potf2_kernel<<<1, 256, 0, s>>>(A + k0 + (long)k0 * lda, lda, kb, k0, info_dev, dblk);
    L1_HIP(hipGetLastError());
    const int n2 = n - k0 - kb;
    if (n2 > 0) {
      double* A21 = A + (k0 + kb) + (long)k0 * lda;
      double* A22 = A + (k0 + kb) + (long)(k0 + kb) * lda;
      L1_HIP(hipMemcpy2DAsync(work, sizeof(double) * n2, A21, sizeof(double) * lda,
                              sizeof(double) * n2, kb, hipMemcpyDeviceToDevice, s));
      gemm64(s, 'N', 'T', n2, kb, kb, 1.0, work, n2, dblk, 64, 0.0, A21, lda);
      gemm64(s, 'N', 'T', n2, n2, kb, -1.0, A21, lda, A21, lda, 1.0, A22, lda);
    }
  }
  const long nn = (long)n * n;
  zero_upper64_kernel<<<(unsigned)((nn + 255) / 256), 256, 0, s>>>(n, A, lda);
  L1_HIP(hipGetLastError());
}

void lower_inverse64(hipStream_t s, int n, const double* L, int lda, const double* diaginv,
                     double* X, int ldx, double* work) {
  L1_HIP(hipMemset2DAsync(X, sizeof(double) * ldx, 0, sizeof(double) * n, n, s));
  for (int i0 = 0; i0 < n; i0 += 64) {
    const int ib = (n - i0 < 64) ? n - i0 : 64;
    const double* dblk = diaginv + (long)(i0 / 64) * 64 * 64;
    L1_HIP(hipMemcpy2DAsync(X + i0 + (long)i0 * ldx, sizeof(double) * ldx, dblk,
                            sizeof(double) * 64, sizeof(double) * ib, ib,
                            hipMemcpyDeviceToDevice, s));
    if (i0 > 0) {
      gemm64(s, 'N', 'N', ib, i0, i0, 1.0, L + i0, lda, X, ldx, 0.0, work, 64);
      gemm64(s, 'N', 'N', ib, i0, ib, -1.0, dblk, 64, work, 64, 0.0, X + i0, ldx);
    }
  }
}

// ---------------------------------------------------------------------------
// power iteration for the largest eigenvalue of a symmetric PSD matrix
__global__ void gemv64_kernel(int n, const double* M, int ldm, const double* v, double* w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int k = 0; k < n; ++k) acc = fma(M[i + (long)k * ldm], v[k], acc);
  w[i] = acc;
}
// scal[0] = v.w, scal[1] = ||w||^2 ; then v = w / ||w||
__global__ __launch_bounds__(1024) void rayleigh64_kernel(int n, double* v, const double* w,
                                                          double* scal) {
  __shared__ double s1[1024], s2[1024];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) {
    a += v[i] * w[i];
    b += w[i] * w[i];
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  __syncthreads();
  for (int st = 512; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      s1[threadIdx.x] += s1[threadIdx.x + st];
      s2[threadIdx.x] += s2[threadIdx.x + st];
    }
    __syncthreads();
  }
  const double nrm = sqrt(s2[0]);
  for (int i = threadIdx.x; i < n; i += 1024) v[i] = (nrm > 0.0) ? w[i] / nrm : 0.0;
  if (threadIdx.x == 0) {
    scal[0] = s1[0];
    scal[1] = s2[0];
  }
}
__global__ void init_power_kernel(int n, double* v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = (1.0 + 0.25 * sin(0.7 * i + 0.3)) / sqrt((double)n);
}

double power_lambda_max64(hipStream_t s, int n, const double* M, int ldm, double* work,
                          int max_iter, double rtol) {
  if (n <= 0) return 0.0;
  double* v = work;
  double* w = work + n;
  double* scal = work + 2 * n;
  init_power_kernel<<<(n + 255) / 256, 256, 0, s>>>(n, v);
  L1_HIP(hipGetLastError());
  double prev = 0.0, lam = 0.0;
  for (int it = 0; it < max_iter; it += 25) {
    for (int t = 0; t < 25; ++t) {
      gemv64_kernel<<<(n + 255) / 256, 256, 0, s>>>(n, M, ldm, v, w);
      rayleigh64_kernel<<<1, 1024, 0, s>>>(n, v, w, scal);
    }
    L1_HIP(hipGetLastError());
    double h[2];
    L1_HIP(hipMemcpyAsync(h, scal, sizeof(h), hipMemcpyDeviceToHost, s));
    L1_HIP(hipStreamSynchronize(s));
    lam = h[0];  // Rayleigh quotient v^T M v with ||v|| = 1
    if (it > 0 && fabs(lam - prev) <= rtol * fabs(lam)) break;
    prev = lam;
  }
  return lam;
}

// ---------------------------------------------------------------------------
// operator layout: dst[i*ldd + k] = src[i + k*lds], through a 32x32 LDS tile
__device__ inline uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf16_to_f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

__global__ void to_rowmajor_kernel(int rows, int cols, const double* src, int lds, float* dst,
                                   int ldd, uint16_t* hi, uint16_t* lo) {
  __shared__ double t[32][33];
  const int bi = blockIdx.y * 32, bk = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: 8 rows at a time
  for (int r = ty; r < 32; r += 8) {
    const int i = bi + tx, k = bk + r;
    t[r][tx] = (i < rows && k < cols) ? src[i + (long)k * lds] : 0.0;  // t[k][i]
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int i = bi + r, k = bk + tx;
    if (i < rows && k < cols) {
      const double x = t[tx][r];
      const long o = (long)i * ldd + k;
      if (dst) dst[o] = (float)x;
      if (hi) {
        const uint16_t h = bf16_rne((float)x);
        hi[o] = h;
        lo[o] = bf16_rne((float)(x - (double)bf16_to_f(h)));
      }
    }
  }
}
void to_rowmajor_f32(hipStream_t s, int rows, int cols, const double* src, int lds, float* dst,
                     int ldd, uint16_t* hi, uint16_t* lo) {
  if (rows <= 0 || cols <= 0) return;
  dim3 grid((cols + 31) / 32, (rows + 31) / 32);
  to_rowmajor_kernel<<<grid, 256, 0, s>>>(rows, cols, src, lds, dst, ldd, hi, lo);
  L1_HIP(hipGetLastError());
}
__global__ void copy_rows_f64_to_f32_kernel(int rows, int cols, const double* src, int lds,
                                            float* dst, int ldd, uint16_t* hi, uint16_t* lo) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)rows * cols) return;
  const int k = (int)(e % cols), i = (int)(e / cols);
  const double x = src[k + (long)i * lds];
  const long o = (long)i * ldd + k;
  dst[o] = (float)x;
  if (hi) {
    const uint16_t h = bf16_rne((float)x);
    hi[o] = h;
    lo[o] = bf16_rne((float)(x - (double)bf16_to_f(h)));
  }
}
void transpose_f64_to_f32(hipStream_t s, int rows, int cols, const double* src, int lds,
                          float* dst, int ldd, uint16_t* hi, uint16_t* lo) {
  // dst row i is column i of src: dst[i*ldd + k] = src[k + i*lds]
  const long n = (long)rows * cols;
  if (n <= 0) return;
  copy_rows_f64_to_f32_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(rows, cols, src, lds,
                                                                        dst, ldd, hi, lo);
  L1_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// FP64 optimality report: one workgroup per instance.
__device__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}
__device__ double block_max(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + st]);
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// problem: 0 P1, 1 P12, 2 QP.  split: the full matrix is [A, I] and e holds
// the identity block (CAB).  For P12 the certificate uses x only.
__global__ __launch_bounds__(256) void kkt64_kernel(int problem, int m, int nd, int split,
                                                    const float* A, int lda, const float* b,
                                                    int ldb, const float* x, int ldx,
                                                    const float* e, int lde, const float* y,
                                                    int ldy, const float* eps, double lambda,
                                                    double* rbuf, double* report) {
  __shared__ double sh[256];
  const int j = blockIdx.x;
  const float* bj = b + (long)j * ldb;
  const float* xj = x + (long)j * ldx;
  const float* ej = (split && e) ? e + (long)j * lde : nullptr;
  const float* yj = y ? y + (long)j * ldy : nullptr;
  double* r = rbuf + (long)j * m;
  // residual r = b - A x (- e)
  double rr = 0.0, bb = 0.0, by = 0.0, yy = 0.0;
  for (int i = threadIdx.x; i < m; i += 256) {
    double acc = (double)bj[i];
    for (int k = 0; k < nd; ++k) acc -= (double)A[i + (long)k * lda] * (double)xj[k];
    if (ej) acc -= (double)ej[i];
    r[i] = acc;
    rr += acc * acc;
    bb += (double)bj[i] * (double)bj[i];
    if (yj) {
      by += (double)bj[i] * (double)yj[i];
      yy += (double)yj[i] * (double)yj[i];
    }
  }
  rr = block_sum(rr, sh);
  bb = block_sum(bb, sh);
  by = block_sum(by, sh);
  yy = block_sum(yy, sh);
  __syncthreads();
  // l1 norm and max of the l1-penalised block
  double l1 = 0.0, wmax = 0.0;
  for (int k = threadIdx.x; k < nd; k += 256) {
    l1 += fabs((double)xj[k]);
    wmax = fmax(wmax, fabs((double)xj[k]));
  }
  if (ej && problem == 0)
    for (int i = threadIdx.x; i < m; i += 256) {
      l1 += fabs((double)ej[i]);
      wmax = fmax(wmax, fabs((double)ej[i]));
    }
  l1 = block_sum(l1, sh);
  wmax = block_max(wmax, sh);
  // g = A_full^T u with u = y (P1, P12) or r / lambda (QP)
  double gmax = 0.0, serr = 0.0;
  const double thr = 1e-6 * wmax;
  for (int k = threadIdx.x; k < nd; k += 256) {
    double g = 0.0;
    for (int i = 0; i < m; ++i) {
      const double u = (problem == 2) ? r[i] / lambda : (yj ? (double)yj[i] : 0.0);
      g += (double)A[i + (long)k * lda] * u;
    }
    gmax = fmax(gmax, fabs(g));
    const double wk = (double)xj[k];
    if (fabs(wk) > thr && wmax > 0.0) serr = fmax(serr, fabs(g - (wk > 0 ? 1.0 : -1.0)));
  }
  if (ej && problem == 0 && yj)
    for (int i = threadIdx.x; i < m; i += 256) {
      const double g = (double)yj[i];
      gmax = fmax(gmax, fabs(g));
      const double wk = (double)ej[i];
      if (fabs(wk) > thr && wmax > 0.0) serr = fmax(serr, fabs(g - (wk > 0 ? 1.0 : -1.0)));
    }
  gmax = block_max(gmax, sh);
  serr = block_max(serr, sh);
  if (threadIdx.x == 0) {
    double* out = report + 4 * (long)j;
    const double nb = fmax(sqrt(bb), 1e-300);
    if (problem == 0) {
      out[0] = sqrt(rr) / nb;
      out[1] = fmax(gmax - 1.0, 0.0);
      out[2] = serr;
      out[3] = fabs(l1 - by) / fmax(l1, 1e-300);
    } else if (problem == 2) {
      out[0] = 0.0;
      out[1] = fmax(gmax - 1.0, 0.0);
      out[2] = serr;
    } else {
      const double ep = (double)eps[j];
      out[0] = fmax(sqrt(rr) - ep, 0.0) / nb;
      out[1] = fmax(gmax - 1.0, 0.0);
      out[2] = serr;
      out[3] = fabs(l1 - (by - ep * sqrt(yy))) / fmax(l1, 1e-300);
    }
  }
  if (problem == 2) {
    // gap: primal 1/2||r||^2 + lambda||x||_1, dual b^T th - 1/2||th||^2, th = r / max(gmax,1)
    double br = 0.0;
    for (int i = threadIdx.x; i < m; i += 256) br += (double)bj[i] * r[i];
    br = block_sum(br, sh);
    if (threadIdx.x == 0) {
      const double sc = fmax(gmax, 1.0);
      const double pobj = 0.5 * rr + lambda * l1;
      const double dobj = br / sc - 0.5 * rr / (sc * sc);
      report[4 * (long)j + 3] = fabs(pobj - dobj) / fmax(fabs(pobj), 1e-300);
    }
  }
}

void kkt64(hipStream_t s, int problem, int m, int nd, int split, const float* A, int lda,
           const float* b, int ldb, const float* x, int ldx, const float* e, int lde,
           const float* y, int ldy, const float* eps, double lambda, int N, double* rbuf,
           double* report) {
  if (N <= 0) return;
  kkt64_kernel<<<N, 256, 0, s>>>(problem, m, nd, split, A, lda, b, ldb, x, ldx, e, lde, y, ldy,
                                 eps, lambda, rbuf, report);
  L1_HIP(hipGetLastError());
}

__global__ void to_f64_kernel(long n, const float* src, double* dst) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    dst[i] = (double)src[i];
}
void to_f64(hipStream_t s, long n, const float* src, double* dst) {
  if (n <= 0) return;
  to_f64_kernel<<<(unsigned)std::min<long>((n + 255) / 256, 8192), 256, 0, s>>>(n, src, dst);
  L1_HIP(hipGetLastError());
}

// operands of the batched report: R = b - e (the product is subtracted
// next), X = x and U = y in FP64
__global__ void kkt_prep_kernel(int m, int nd, int N, const float* b, int ldb, const float* e,
                                int lde, const float* x, int ldx, const float* y, int ldy,
                                double* R, double* X, double* U) {
  const int j = blockIdx.y;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < max(m, nd); i += gridDim.x * blockDim.x) {
    if (i < m) {
      R[i + (long)j * m] = (double)b[i + (long)j * ldb] - (e ? (double)e[i + (long)j * lde] : 0.0);
      if (y) U[i + (long)j * m] = (double)y[i + (long)j * ldy];
    }
    if (i < nd) X[i + (long)j * nd] = (double)x[i + (long)j * ldx];
  }
}
__global__ void kkt_scale_kernel(long n, const double* R, double c, double* U) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    U[i] = R[i] * c;
}

// the report of instance j from R (its residual) and G (A^T u); the same
// quantities and formulas as kkt64_kernel
__global__ __launch_bounds__(256) void kkt_report_kernel(int problem, int m, int nd, int split,
                                                         const float* b, int ldb, const float* x,
                                                         int ldx, const float* e, int lde,
                                                         const float* y, int ldy, const float* eps,
                                                         double lambda, const double* R,
                                                         const double* G, double* report) {
  __shared__ double sh[256];
  const int j = blockIdx.x;
  const float* bj = b + (long)j * ldb;
  const float* xj = x + (long)j * ldx;
  const float* ej = (split && e) ? e + (long)j * lde : nullptr;
  const float* yj = y ? y + (long)j * ldy : nullptr;
  const double* r = R + (long)j * m;
  const double* g = G + (long)j * nd;
  double rr = 0.0, bb = 0.0, by = 0.0, yy = 0.0, br = 0.0;
  for (int i = threadIdx.x; i < m; i += 256) {
    const double bi = (double)bj[i];
    rr += r[i] * r[i];
    bb += bi * bi;
    br += bi * r[i];
    if (yj) {
      by += bi * (double)yj[i];
      yy += (double)yj[i] * (double)yj[i];
    }
  }
  rr = block_sum(rr, sh);
  bb = block_sum(bb, sh);
  by = block_sum(by, sh);
  yy = block_sum(yy, sh);
  br = block_sum(br, sh);
  double l1 = 0.0, wmax = 0.0;
  for (int k = threadIdx.x; k < nd; k += 256) {
    l1 += fabs((double)xj[k]);
    wmax = fmax(wmax, fabs((double)xj[k]));
  }
  if (ej && problem == 0)
    for (int i = threadIdx.x; i < m; i += 256) {
      l1 += fabs((double)ej[i]);
      wmax = fmax(wmax, fabs((double)ej[i]));
    }
  l1 = block_sum(l1, sh);
  wmax = block_max(wmax, sh);
  double gmax = 0.0, serr = 0.0;
  const double thr = 1e-6 * wmax;
  for (int k = threadIdx.x; k < nd; k += 256) {
    gmax = fmax(gmax, fabs(g[k]));
    const double wk = (double)xj[k];
    if (fabs(wk) > thr && wmax > 0.0) serr = fmax(serr, fabs(g[k] - (wk > 0 ? 1.0 : -1.0)));
  }
  if (ej && problem == 0 && yj)
    for (int i = threadIdx.x; i < m; i += 256) {
      const double gi = (double)yj[i];
      gmax = fmax(gmax, fabs(gi));
      const double wk = (double)ej[i];
      if (fabs(wk) > thr && wmax > 0.0) serr = fmax(serr, fabs(gi - (wk > 0 ? 1.0 : -1.0)));
    }
  gmax = block_max(gmax, sh);
  serr = block_max(serr, sh);
  if (threadIdx.x == 0) {
    double* out = report + 4 * (long)j;
    const double nb = fmax(sqrt(bb), 1e-300);
    if (problem == 0) {
      out[0] = sqrt(rr) / nb;
      out[1] = fmax(gmax - 1.0, 0.0);
      out[2] = serr;
      out[3] = fabs(l1 - by) / fmax(l1, 1e-300);
    } else if (problem == 2) {
      // gap: primal 1/2||r||^2 + lambda||x||_1, dual b^T th - 1/2||th||^2, th = r / max(gmax,1)
      const double sc = fmax(gmax, 1.0);
      const double pobj = 0.5 * rr + lambda * l1;
      const double dobj = br / sc - 0.5 * rr / (sc * sc);
      out[0] = 0.0;
      out[1] = fmax(gmax - 1.0, 0.0);
      out[2] = serr;
      out[3] = fabs(pobj - dobj) / fmax(fabs(pobj), 1e-300);
    } else {
      const double ep = (double)eps[j];
      out[0] = fmax(sqrt(rr) - ep, 0.0) / nb;
      out[1] = fmax(gmax - 1.0, 0.0);
      out[2] = serr;
      out[3] = fabs(l1 - (by - ep * sqrt(yy))) / fmax(l1, 1e-300);
    }
  }
}

void kkt64_batched(hipStream_t s, int problem, int m, int nd, int split, const double* A64,
                   const float* b, int ldb, const float* x, int ldx, const float* e, int lde,
                   const float* y, int ldy, const float* eps, double lambda, int N, double* R,
                   double* X, double* U, double* G, double* report) {
  if (N <= 0) return;
  const float* ef = split ? e : nullptr;
  const float* yu = (problem == 2) ? nullptr : y;
  dim3 grid((unsigned)std::min((std::max(m, nd) + 255) / 256, 64), (unsigned)N);
  kkt_prep_kernel<<<grid, 256, 0, s>>>(m, nd, N, b, ldb, ef, lde, x, ldx, yu, ldy, R, X, U);
  L1_HIP(hipGetLastError());
  if (nd > 0) gemm64(s, 'N', 'N', m, N, nd, -1.0, A64, m, X, nd, 1.0, R, m);
  if (problem == 2) {
    const long n = (long)m * N;
    kkt_scale_kernel<<<(unsigned)std::min<long>((n + 255) / 256, 8192), 256, 0, s>>>(n, R, 1.0 / lambda, U);
    L1_HIP(hipGetLastError());
  } else if (!y) {
    L1_HIP(hipMemsetAsync(U, 0, sizeof(double) * (size_t)m * N, s));
  }
  if (nd > 0) gemm64(s, 'T', 'N', nd, N, m, 1.0, A64, m, U, m, 0.0, G, nd);
  kkt_report_kernel<<<N, 256, 0, s>>>(problem, m, nd, split, b, ldb, x, ldx, e, lde, y, ldy, eps,
                                      lambda, R, G, report);
  L1_HIP(hipGetLastError());
}

}  // namespace l1
