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
//   w-step   every wave forms all of w = Ginv g: lane (t, d) = (lane / 16
//            + 4 pass, lane % 16) holds (B^T B)^{-1}[t][d] (FP64, formed
//            once), the row sum gives w_t, read into scalar registers
//   test     so every wave holds the same w (FP64) and takes the same
//            stopping decision, with no barrier
//   rows     B w (FP32) and the theta-step.
// Two workgroup barriers per iteration.  B^T B is formed once on the FP64
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
  // rows of B on their way to the matrix cores (a row per thread, padded to
  // 17 floats so that the threads' row writes fall in different banks) and
  // the waves' partial Gram matrices (set-up), then the threads' partial
  // B^T s (iterations; rows padded by 16 floats so that the segment sums
  // read without bank conflicts)
  __shared__ union {
    float chunk[AL_THREADS][17];
    double gw[4][16][16];
    float p[KP][AL_THREADS + 16];
  } s_u;
  __shared__ double s_g[16];
  __shared__ double s_aug[2][ALIGN_KMAX][2 * ALIGN_KMAX];
  __shared__ double s_diag[ALIGN_KMAX];
  __shared__ int s_flag;
  const int j = blockIdx.x, tid = threadIdx.x;
  const int lane = tid & 63;
  const int slot = (tid >> 6) * 4 + (lane >> 4);   // which row of 16 lanes
  const bool row_lead = (lane & 15) == 0;
  const int dd = tid & 15;                           // the column d of the w-step
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
      s_aug[0][i][c] = g;
      s_aug[0][i][k + c] = i == c ? 1.0 : 0.0;
      if (i == c) s_diag[i] = g;
    }
  }

  // its inverse: Gauss-Jordan on [G | I], each pivot one step from one LDS
  // copy of the augmented matrix into the other (every entry of the new one
  // depends only on the old one), one barrier a step; a pivot below 1e-12 of
  // its diagonal entry marks a rank-deficient dictionary
  if (tid == 0) s_flag = 1;
  __syncthreads();
  int cur = 0;
  {
    const int w2 = 2 * k;
    const int r0 = tid / w2, c0 = tid % w2;                                 // entry tid
    const int r1 = (tid + AL_THREADS) / w2, c1 = (tid + AL_THREADS) % w2;   // entry tid + 256
    const bool has0 = tid < k * w2, has1 = tid + AL_THREADS < k * w2;
    for (int pv = 0; pv < k; ++pv) {
      const double piv = s_aug[cur][pv][pv];
      if (!(piv > 1e-12 * s_diag[pv])) {
        if (tid == 0) s_flag = 0;
        break;   // uniform: every thread read the same pivot
      }
      const double ip = 1.0 / piv;
      if (has0) {
        const double pr = s_aug[cur][pv][c0] * ip;
        s_aug[cur ^ 1][r0][c0] = r0 == pv ? pr : s_aug[cur][r0][c0] - s_aug[cur][r0][pv] * pr;
      }
      if (has1) {
        const double pr = s_aug[cur][pv][c1] * ip;
        s_aug[cur ^ 1][r1][c1] = r1 == pv ? pr : s_aug[cur][r1][c1] - s_aug[cur][r1][pv] * pr;
      }
      __syncthreads();
      cur ^= 1;
    }
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
  // Ginv[t][d] for t = lane / 16 + 4 pass, d = lane % 16 (zero past k)
  constexpr int NP = KP / 4;   // passes of the w-step
  double ginv[NP];
#pragma unroll
  for (int ps = 0; ps < NP; ++ps) {
    const int t = (lane >> 4) + 4 * ps;
    ginv[ps] = (t < k && dd < k) ? s_aug[cur][t][k + dd] : 0.0;
  }
  double w[KP];   // the current w, the same in every lane of every wave
#pragma unroll
  for (int d = 0; d < KP; ++d) w[d] = 0.0;

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
    // w-step, in every wave: w_t = sum_d Ginv[t][d] g_d as the row sum of
    // row t % 4 in pass t / 4, taken from the row's first lane
    const double gd = dd < k ? s_g[dd] : 0.0;
    double dw2 = 0.0, w2 = 0.0;
    float wf[KP];
#pragma unroll
    for (int ps = 0; ps < NP; ++ps) {
      const double v = row_sum(ginv[ps] * gd);
#pragma unroll
      for (int t4 = 0; t4 < 4; ++t4) {
        const int t = 4 * ps + t4;
        const double wt = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 16 * t4),
                                           __builtin_amdgcn_readlane(__double2loint(v), 16 * t4));
        dw2 += (wt - w[t]) * (wt - w[t]);
        w2 += w[t] * w[t];
        w[t] = wt;
        wf[t] = (float)wt;
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
  if (tid < k) {
    float wv = 0.0f;
#pragma unroll
    for (int d = 0; d < KP; ++d)
      if (d == tid) wv = (float)w[d];
    wg[(long)j * k + tid] = wv;
  }
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
