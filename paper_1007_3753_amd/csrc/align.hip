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
// One workgroup of 256 threads per instance runs all of its iterations in
// one launch.  Thread tid owns rows tid + 256 r (r < R) and keeps those rows
// of B (k padded to KP columns with zeros), of b, e, theta and B w in
// registers, so B is read from HBM once and the workgroup needs a few KB of
// LDS.  Per iteration:
//   rows     e, s = b - e + theta/xi, and the thread's partial B^T s (FP32
//            over its R rows)
//   reduce   the partials through LDS: the 16 lanes of a row of the wave
//            take one column, add 16 partials each in FP64 and then sum
//            over the row with DPP rotations
//   w-step   thread (t, d) = (tid / 16, tid % 16) holds (B^T B)^{-1}[t][d]
//            (FP64, formed once) and forms w_t = sum_d Ginv[t][d] g_d with
//            the same row sum; the row also leaves (w_t - w_t_old)^2 and
//            w_t_old^2
//   test     every thread reads the new w and those squares from LDS and
//            takes the same stopping decision (FP64, a fixed order)
//   rows     B w (FP32) and the theta-step.
// Three workgroup barriers per iteration.  B^T B is formed once on the FP64
// matrix cores from the FP32 dictionary (exact products) and B^T s is
// combined in FP64, so the normal equations do not square the dictionary's
// condition number in FP32.
#include "internal.h"

namespace l1 {

namespace {

constexpr int AL_THREADS = 256;
typedef double v4d __attribute__((ext_vector_type(4)));

__device__ inline float softa(float x, float a) {
  const float m = fabsf(x) - a;
  return m > 0.0f ? copysignf(m, x) : 0.0f;
}

// v of the lane N places along in this lane's row of 16 (DPP row_ror:N)
template <int N>
__device__ inline double row_ror(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x120 + N, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x120 + N, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// the sum over the 16 lanes of this lane's row, in every lane of the row
// (the order of the additions differs between lanes: use one lane's value).
// Called with every lane of the wave active.
__device__ inline double row_sum(double v) {
  v += row_ror<8>(v);
  v += row_ror<4>(v);
  v += row_ror<2>(v);
  v += row_ror<1>(v);
  return v;
}

}  // namespace

template <int R, int KP>
__global__ __launch_bounds__(AL_THREADS) void align_kernel(const float* Bg, int m, int k, const float* bg,
                                                           int ldb, float tol, int cap, int fixed,
                                                           float* wg, float* eg, int lde, int* iters,
                                                           int* status) {
  __shared__ double s_red[16];
  // rows of B on their way to the matrix cores and the waves' partial Gram
  // matrices (set-up), then the threads' partial B^T s (iterations; rows
  // padded by 16 floats so that the segment sums read without bank conflicts)
  __shared__ union {
    float chunk[AL_THREADS][16];
    double gw[4][16][16];
    float p[KP][AL_THREADS + 16];
  } s_u;
  __shared__ double s_g[16];
  __shared__ double s_aug[ALIGN_KMAX][2 * ALIGN_KMAX];
  __shared__ double s_fac[ALIGN_KMAX], s_diag[ALIGN_KMAX];
  __shared__ double s_w[16], s_dw[16], s_wo[16];
  __shared__ int s_flag;
  const int j = blockIdx.x, tid = threadIdx.x;
  const int lane = tid & 63;
  const int slot = (tid >> 6) * 4 + (lane >> 4);   // which row of 16 lanes
  const bool row_lead = (lane & 15) == 0;
  const int tt = tid >> 4, dd = tid & 15;            // the (t, d) pair of the w-step
  const float* B = Bg + (long)j * m * k;
  const float* bj = bg + (long)j * ldb;

  // this thread's rows of B and b (zero past m and past k)
  float Br[R][KP], bv[R], ev[R], th[R], tv[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = tid + AL_THREADS * r;
#pragma unroll
    for (int d = 0; d < KP; ++d) Br[r][d] = (i < m && d < k) ? B[i + (long)m * d] : 0.0f;
    bv[r] = i < m ? bj[i] : 0.0f;
  }
  double n1 = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    ev[r] = bv[r];
    th[r] = 0.0f;
    tv[r] = 0.0f;   // B w with w = 0
    n1 += fabs((double)bv[r]);
  }
  n1 = row_sum(n1);
  if (row_lead) s_red[slot] = n1;
  if (tid < 16) s_w[tid] = 0.0;
  __syncthreads();
  n1 = 0.0;
#pragma unroll
  for (int q = 0; q < 16; ++q) n1 += s_red[q];
  const float xi = n1 > 0.0 ? (float)(2.0 * m / n1) : 1.0f;
  const float ixi = 1.0f / xi;

  // Gram matrix G = B^T B on the FP64 matrix cores (the FP32 entries and
  // their products are exact in FP64).  The rows pass through LDS 256 at a
  // time; each wave takes 64 of them as 16 steps of
  // v_mfma_f64_16x16x4f64 (A = the 4 rows transposed, B = the 4 rows: lane
  // (q, d) = (lane / 16, lane % 16) supplies entry (row 4 s + q, column d)
  // to both), accumulating its 16 x 16 partial Gram matrix; lane (q, d)
  // ends with entries (q + 4 v, d), v < 4 (G is symmetric, so the
  // orientation of that layout does not matter).  The four partials are
  // added through LDS.
  {
    const int wave = tid >> 6, q = lane >> 4, dl = lane & 15;
    v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
      for (int d = 0; d < 16; ++d) s_u.chunk[tid][d] = d < KP ? Br[r][d] : 0.0f;
      __syncthreads();
#pragma unroll
      for (int st = 0; st < 16; ++st) {
        const double x = (double)s_u.chunk[64 * wave + 4 * st + q][dl];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x, x, acc, 0, 0, 0);
      }
      __syncthreads();
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) s_u.gw[wave][q + 4 * v][dl] = acc[v];
    __syncthreads();
    for (int t = tid; t < k * k; t += AL_THREADS) {
      const int i = t / k, c = t % k;
      const double g = (s_u.gw[0][i][c] + s_u.gw[1][i][c]) + (s_u.gw[2][i][c] + s_u.gw[3][i][c]);
      s_aug[i][c] = g;
      s_aug[i][k + c] = i == c ? 1.0 : 0.0;
      if (i == c) s_diag[i] = g;
    }
  }

  // its inverse: Gauss-Jordan on [G | I] in LDS, the row operations of a
  // pivot spread over the threads; a pivot below 1e-12 of its diagonal entry
  // marks a rank-deficient dictionary
  if (tid == 0) s_flag = 1;
  __syncthreads();
  for (int pv = 0; pv < k; ++pv) {
    const double piv = s_aug[pv][pv];
    if (!(piv > 1e-12 * s_diag[pv])) {
      if (tid == 0) s_flag = 0;
      break;   // uniform: every thread read the same pivot
    }
    if (tid < k) s_fac[tid] = s_aug[tid][pv];
    __syncthreads();
    if (tid < 2 * k) s_aug[pv][tid] /= piv;
    __syncthreads();
    for (int t = tid; t < 2 * k * k; t += AL_THREADS) {
      const int r = t / (2 * k), c = t % (2 * k);
      if (r != pv) s_aug[r][c] -= s_fac[r] * s_aug[pv][c];
    }
    __syncthreads();
  }
  __syncthreads();
  if (!s_flag) {
    if (tid < k) wg[(long)j * k + tid] = 0.0f;
    for (int i = tid; i < m; i += AL_THREADS) eg[(long)j * lde + i] = bj[i];
    if (tid == 0) {
      iters[j] = 0;
      status[j] = L1_NONFINITE;
    }
    return;
  }
  const double ginv = (tt < k && dd < k) ? s_aug[tt][k + dd] : 0.0;

  int it = 0, st = L1_MAXITER;
  for (it = 1; it <= cap; ++it) {
    // e-step, s = b - e + theta/xi and this thread's partial B^T s
    float p[KP];
#pragma unroll
    for (int d = 0; d < KP; ++d) p[d] = 0.0f;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const float u = th[r] * ixi;
      ev[r] = softa(bv[r] - tv[r] + u, ixi);
      const float s = bv[r] - ev[r] + u;
#pragma unroll
      for (int d = 0; d < KP; ++d) p[d] = fmaf(Br[r][d], s, p[d]);
    }
#pragma unroll
    for (int d = 0; d < KP; ++d) s_u.p[d][tid] = p[d];
    __syncthreads();
    // g_c = (B^T s)_c for c = tid / 16: lane q = tid % 16 adds 16 of the
    // threads' partials in FP64, then the row sum over q
    {
      const int c = tid >> 4, q = tid & 15;
      double g = 0.0;
      if (c < KP) {
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) g += (double)s_u.p[c][q + 16 * jj];
      }
      g = row_sum(g);
      if (q == 0 && c < KP) s_g[c] = g;
    }
    __syncthreads();
    // w-step: w_t = sum_d Ginv[t][d] g_d in the row of 16 lanes of t
    {
      const double wt = row_sum(ginv * (dd < k ? s_g[dd] : 0.0));
      const double wo = s_w[tt & 15];
      if (tt < k) {
        if (dd == 0) s_w[tt] = wt;
        if (dd == 1) s_dw[tt] = (wt - wo) * (wt - wo);
        if (dd == 2) s_wo[tt] = wo * wo;
      }
    }
    __syncthreads();
    double dw2 = 0.0, w2 = 0.0;
    float wf[KP];
#pragma unroll
    for (int d = 0; d < KP; ++d) {
      wf[d] = 0.0f;
      if (d < k) {
        dw2 += s_dw[d];
        w2 += s_wo[d];
        wf[d] = (float)s_w[d];
      }
    }
    // theta-step with t = B w (kept for the next e-step)
#pragma unroll
    for (int r = 0; r < R; ++r) {
      float t = 0.0f;
#pragma unroll
      for (int d = 0; d < KP; ++d) t = fmaf(Br[r][d], wf[d], t);
      tv[r] = t;
      th[r] += xi * (bv[r] - t - ev[r]);
    }
    if (!(isfinite(dw2) && isfinite(w2))) {
      st = L1_NONFINITE;
      break;
    }
    if (!fixed && dw2 < (double)tol * (double)tol * w2) {
      st = L1_CONVERGED;
      break;
    }
  }
  if (it > cap) it = cap;
  if (tid < k) wg[(long)j * k + tid] = (float)s_w[tid];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = tid + AL_THREADS * r;
    if (i < m) eg[(long)j * lde + i] = ev[r];
  }
  if (tid == 0) {
    iters[j] = it;
    status[j] = st;
  }
}

namespace {

template <int R, int KP>
void launch_align(hipStream_t s, const float* B, int m, int k, int N, const float* b, int ldb, float tol,
                  int cap, int fixed, float* w, float* e, int lde, int* iters, int* status) {
  align_kernel<R, KP><<<N, AL_THREADS, 0, s>>>(B, m, k, b, ldb, tol, cap, fixed, w, e, lde, iters, status);
}

template <int R>
void launch_kp(hipStream_t s, const float* B, int m, int k, int N, const float* b, int ldb, float tol,
               int cap, int fixed, float* w, float* e, int lde, int* iters, int* status) {
  if (k <= 4)
    launch_align<R, 4>(s, B, m, k, N, b, ldb, tol, cap, fixed, w, e, lde, iters, status);
  else if (k <= 8)
    launch_align<R, 8>(s, B, m, k, N, b, ldb, tol, cap, fixed, w, e, lde, iters, status);
  else if (k <= 12)
    launch_align<R, 12>(s, B, m, k, N, b, ldb, tol, cap, fixed, w, e, lde, iters, status);
  else
    launch_align<R, 16>(s, B, m, k, N, b, ldb, tol, cap, fixed, w, e, lde, iters, status);
}

}  // namespace

void align_solve(hipStream_t s, const float* B, int m, int k, int N, const float* b, int ldb, float tol,
                 int max_iter, float* w, float* e, int lde, int* iters, int* status) {
  if (N <= 0) return;
  L1_REQUIRE(k >= 1 && k <= ALIGN_KMAX && m >= 1 && m <= AL_THREADS * ALIGN_R, "alignment sizes");
  const int fixed = max_iter < 0;
  const int cap = fixed ? -max_iter : max_iter;
  const int rows = (m + AL_THREADS - 1) / AL_THREADS;   // rows per thread
  switch (rows) {
    case 1: launch_kp<1>(s, B, m, k, N, b, ldb, tol, cap, fixed, w, e, lde, iters, status); break;
    case 2: launch_kp<2>(s, B, m, k, N, b, ldb, tol, cap, fixed, w, e, lde, iters, status); break;
    case 3: launch_kp<3>(s, B, m, k, N, b, ldb, tol, cap, fixed, w, e, lde, iters, status); break;
    case 4: launch_kp<4>(s, B, m, k, N, b, ldb, tol, cap, fixed, w, e, lde, iters, status); break;
    case 5: launch_kp<5>(s, B, m, k, N, b, ldb, tol, cap, fixed, w, e, lde, iters, status); break;
    case 6: launch_kp<6>(s, B, m, k, N, b, ldb, tol, cap, fixed, w, e, lde, iters, status); break;
    default: launch_kp<8>(s, B, m, k, N, b, ldb, tol, cap, fixed, w, e, lde, iters, status); break;
  }
  L1_HIP(hipGetLastError());
}

}  // namespace l1
