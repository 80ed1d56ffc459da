// DALM with the y-step replaced by one conjugate-gradient step (the cheaper
// heuristic mentioned in Sec. V-B), for (P1), dense or cross-and-bouquet.
// With v = A^T y, one iteration from (w, y, v) is
//     z  = clamp(v + w/beta)                                   (z-step)
//     g  = A (v - z + w/beta) - b/beta                         (gradient of the
//          y-subproblem  q(y) = y^T A A^T y / 2 - (A (z - w/beta) + b/beta)^T y)
//     alpha = ||g||^2 / ||A^T g||^2                            (exact step length:
//          the first CG step from y is steepest descent)
//     y <- y - alpha g,   v <- v - alpha A^T g                 (no third product)
//     w <- w - beta (z - v)                                    (w-step)
// Per iteration: an elementwise launch (z and u = v - z + w/beta), the FP32
// product A u (A = B for the cross-and-bouquet form, whose identity block is
// added in the next launch), a launch forming g and ||g||^2, the product
// A^T g, and one launch per instance that forms ||A^T g||^2, updates y, v, w
// and runs the stopping test of Algorithm 2 (relative change of w and the
// complementarity gap, FP64 sums in a fixed order).  Finished instances stay
// in the batch and are skipped by the elementwise launches.
#include <chrono>
#include <cmath>

#include "internal.h"
#include "plan.h"
#include "steps.h"

namespace l1 {

namespace {

constexpr int CG_THREADS = 256;

// sum over the workgroup in a fixed order (every thread calls; the result is
// returned to every thread)
__device__ inline double cg_sum(double v, double* red) {
  const int tid = threadIdx.x;
  __syncthreads();
  red[tid] = v;
  __syncthreads();
  for (int h = CG_THREADS / 2; h > 0; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  return red[0];
}

// z and u = v - z + w/beta for rows < n; u = 0 on rows [n, n_zero)
__global__ __launch_bounds__(CG_THREADS) void cg1_pre_kernel(int n, int n_zero, int lds, const int* state,
                                                             const float* W, const float* V,
                                                             const float* ipen, float* Z, float* U) {
  const int j = blockIdx.x;
  if (state[j] != 0) return;
  const float ib = ipen[j];
  const long o = (long)j * lds;
  for (int i = threadIdx.x; i < n_zero; i += CG_THREADS) {
    if (i < n) {
      const float wb = W[o + i] * ib;
      const float z = fminf(fmaxf(V[o + i] + wb, -1.0f), 1.0f);
      Z[o + i] = z;
      U[o + i] = V[o + i] - z + wb;
    } else {
      U[o + i] = 0.0f;
    }
  }
}

// g = A u - b/beta (the product of B plus, for the cross-and-bouquet form,
// the identity block's u_e) and ||g||^2; g is zero on the padding rows
__global__ __launch_bounds__(CG_THREADS) void cg1_grad_kernel(int m, int m_pad, int nd, int cab, int lds,
                                                              const int* state, const float* AU,
                                                              const float* U, const float* bb,
                                                              const float* ipen, float* G, double* gg) {
  __shared__ double red[CG_THREADS];
  const int j = blockIdx.x;
  if (state[j] != 0) return;
  const float ib = ipen[j];
  const long om = (long)j * m_pad, ou = (long)j * lds;
  double acc = 0.0;
  for (int i = threadIdx.x; i < m_pad; i += CG_THREADS) {
    float g = 0.0f;
    if (i < m) {
      g = AU[om + i] + (cab ? U[ou + nd + i] : 0.0f) - bb[om + i] * ib;
      acc += (double)g * (double)g;
    }
    G[om + i] = g;
  }
  acc = cg_sum(acc, red);
  if (threadIdx.x == 0) gg[j] = acc;
}

// step length, y, v and w updates, and the stopping test
__global__ __launch_bounds__(CG_THREADS) void cg1_update_kernel(int m, int m_pad, int nd, int n, int cab,
                                                                int lds, float tol, int fixed, int* state,
                                                                int* iters, int* status, const float* H,
                                                                const float* G, const double* gg,
                                                                const float* Z, const float* pen,
                                                                const float* wcap2, float* W,
                                                                float* V, float* Y) {
  __shared__ double red[CG_THREADS];
  const int j = blockIdx.x, tid = threadIdx.x;
  if (state[j] != 0) return;
  const long om = (long)j * m_pad, o = (long)j * lds;
  double d = 0.0;
  for (int i = tid; i < nd; i += CG_THREADS) d += (double)H[o + i] * (double)H[o + i];
  d = cg_sum(d, red);
  const double g2 = gg[j];
  if (cab) d += g2;   // the identity block of A^T g is g itself
  const float alpha = d > 0.0 ? (float)(g2 / d) : 0.0f;
  const float beta = pen[j];
  for (int i = tid; i < m; i += CG_THREADS) Y[om + i] -= alpha * G[om + i];
  double dw2 = 0.0, nw2 = 0.0, wl1 = 0.0, wv = 0.0;
  for (int i = tid; i < n; i += CG_THREADS) {
    const float atg = i < nd ? H[o + i] : G[om + (i - nd)];
    const float vn = V[o + i] - alpha * atg;
    const float wo = W[o + i];
    const float wn = wo - beta * (Z[o + i] - vn);
    const double dw = (double)wn - (double)wo;
    dw2 += dw * dw;
    nw2 += (double)wn * (double)wn;
    wl1 += fabs((double)wn);
    wv += (double)wn * (double)vn;
    W[o + i] = wn;
    V[o + i] = vn;
  }
  dw2 = cg_sum(dw2, red);
  nw2 = cg_sum(nw2, red);
  wl1 = cg_sum(wl1, red);
  wv = cg_sum(wv, red);
  if (tid == 0) {
    iters[j] += 1;
    const double gap = fabs(wl1 - wv);
    if (!(isfinite(nw2) && isfinite(gap))) {
      status[j] = L1_NONFINITE;
      state[j] = 2;
    } else if (!fixed && nw2 > (double)wcap2[j]) {
      status[j] = L1_DIVERGED;
      state[j] = 2;
    } else if (!fixed && sqrt(dw2) <= (double)tol * sqrt(nw2) && gap <= (double)tol * wl1) {
      status[j] = L1_CONVERGED;
      state[j] = 1;
    }
  }
}

__global__ void cg1_count_kernel(int N, const int* state, int* out) {
  __shared__ int c;
  if (threadIdx.x == 0) c = 0;
  __syncthreads();
  int k = 0;
  for (int j = threadIdx.x; j < N; j += blockDim.x) k += state[j] == 0;
  atomicAdd(&c, k);
  __syncthreads();
  if (threadIdx.x == 0) *out = c;
}

__global__ void cg1_copy_kernel(int rows, int N, const float* src, int lds, int r0, float* dst, int ldd) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)rows * N) return;
  const int j = (int)(t / rows), i = (int)(t % rows);
  dst[(long)j * ldd + i] = src[(long)j * lds + r0 + i];
}

void copy_rows(hipStream_t s, int rows, int N, const float* src, int lds, int r0, float* dst, int ldd) {
  const long t = (long)rows * N;
  if (t <= 0 || dst == nullptr) return;
  cg1_copy_kernel<<<(unsigned)((t + 255) / 256), 256, 0, s>>>(rows, N, src, lds, r0, dst, ldd);
  L1_HIP(hipGetLastError());
}

}  // namespace

void solve_dalm_cg1(Plan* p, const SolveArgs& sa) {
  L1_REQUIRE(sa.N >= 0 && sa.N <= p->d.max_batch, "N must be in [0, max_batch]");
  if (sa.N == 0) return;
  L1_REQUIRE(sa.b != nullptr && sa.x != nullptr, "b and x must be non-NULL");
  L1_REQUIRE(sa.ldb >= p->m && sa.ldx >= std::max(p->nd, 1), "bad leading dimension");
  L1_REQUIRE(sa.e == nullptr || sa.lde >= p->m, "lde < m");
  L1_REQUIRE(sa.y == nullptr || sa.ldy >= p->m, "ldy < m");
  L1_REQUIRE(sa.max_iter != 0, "max_iter must be nonzero");
  L1_REQUIRE(std::isfinite(sa.tol) && sa.tol >= 0.0f, "tol must be finite and >= 0");
  L1_REQUIRE(sa.w0 == nullptr && sa.y0 == nullptr, "warm start is supported for DALM only");
  const auto t_start = std::chrono::steady_clock::now();
  hipStream_t us = sa.s;
  hipStream_t s;
  hipEvent_t ev;
  L1_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  L1_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  L1_HIP(hipEventRecord(ev, us));
  L1_HIP(hipStreamWaitEvent(s, ev, 0));
  struct Done {
    hipStream_t us, s;
    hipEvent_t ev;
    ~Done() {
      (void)hipEventRecord(ev, s);
      (void)hipStreamWaitEvent(us, ev, 0);
      (void)hipStreamSynchronize(s);
      (void)hipEventDestroy(ev);
      (void)hipStreamDestroy(s);
    }
  } guard{us, s, ev};

  const int N = sa.N, m = p->m, nd = p->nd, n = p->n, lds = p->lds, Np = p->N_pad, ldm = p->m_pad;
  const int cab = p->split ? 1 : 0;
  const bool fixed = sa.max_iter < 0;
  const int cap = fixed ? -sa.max_iter : sa.max_iter;
  // the FP32 floor of the stopping test (as for the DALM path)
  const float t_eff = fixed ? 0.0f : std::max(sa.tol, 2e-6f);
  float* Y = p->aux;
  float* AU = p->aux + (size_t)ldm * Np;
  float* G = p->aux + (size_t)2 * ldm * Np;
  float* U = p->Uf[0];
  float* H = p->Uf[1];
  double* gg = p->kkt_rbuf;
  int* state = p->ints;
  int* iters = p->ints + Np;
  int* status = p->ints + 2 * Np;
  int* count = p->ints + 3 * Np;

  L1_HIP(hipMemsetAsync(p->bb, 0, sizeof(float) * ldm * N, s));
  L1_HIP(hipMemcpy2DAsync(p->bb, sizeof(float) * ldm, sa.b, sizeof(float) * sa.ldb, sizeof(float) * m, N,
                          hipMemcpyDeviceToDevice, s));
  penalties(s, N, m, p->bb, ldm, sa.pen, p->d.beta > 0 ? (float)p->d.beta : 0.0f, 0, 1.0f, 0.0f, div_factor(p),
            p->pen, p->ipen, p->wcap2, nullptr);
  L1_HIP(hipMemsetAsync(p->W, 0, sizeof(float) * (size_t)lds * N, s));
  L1_HIP(hipMemsetAsync(p->V, 0, sizeof(float) * (size_t)lds * N, s));
  L1_HIP(hipMemsetAsync(U, 0, sizeof(float) * (size_t)lds * N, s));
  L1_HIP(hipMemsetAsync(H, 0, sizeof(float) * (size_t)lds * N, s));
  L1_HIP(hipMemsetAsync(p->aux, 0, sizeof(float) * (size_t)3 * ldm * Np, s));
  L1_HIP(hipMemsetAsync(state, 0, sizeof(int) * 3 * Np, s));
  L1_HIP(hipMemsetAsync(status, 0xFF, sizeof(int) * Np, s));   // -1 until decided
  L1_HIP(hipMemsetAsync(p->stat, 0, sizeof(long long) * 8, s));

  GemmArgs g1{};   // A u: the dictionary block of A (B for the cross-and-bouquet form)
  g1.A32 = p->Arow;
  g1.lda = p->nd_pad;
  g1.B = U;
  g1.ldb = lds;
  g1.M = ldm;
  g1.K = p->nd_pad;
  g1.n_cols = N;
  g1.prec = PREC_F32;
  g1.m_true = ldm;
  g1.out = AU;
  g1.ldo = ldm;
  GemmArgs g2{};   // the dictionary block of A^T g
  g2.A32 = p->Acol;
  g2.lda = ldm;
  g2.B = G;
  g2.ldb = ldm;
  g2.M = p->nd_pad;
  g2.K = ldm;
  g2.n_cols = N;
  g2.prec = PREC_F32;
  g2.m_true = p->nd_pad;
  g2.out = H;
  g2.ldo = lds;
  const int ntc = (N + TILE - 1) / TILE;
  constexpr int kPoll = 16;   // iterations between host checks of the batch

  int it = 0;
  while (it < cap) {
    cg1_pre_kernel<<<N, CG_THREADS, 0, s>>>(n, std::max(n, p->nd_pad), lds, state, p->W, p->V, p->ipen,
                                            p->Z[0], U);
    L1_HIP(hipGetLastError());
    if (nd > 0) launch_gemm(s, EPI_STORE, g1, ntc);
    cg1_grad_kernel<<<N, CG_THREADS, 0, s>>>(m, ldm, nd, cab, lds, state, AU, U, p->bb, p->ipen, G, gg);
    L1_HIP(hipGetLastError());
    if (nd > 0) launch_gemm(s, EPI_STORE, g2, ntc);
    cg1_update_kernel<<<N, CG_THREADS, 0, s>>>(m, ldm, nd, n, cab, lds, t_eff, fixed ? 1 : 0, state, iters,
                                               status, H, G, gg, p->Z[0], p->pen, p->wcap2, p->W, p->V, Y);
    L1_HIP(hipGetLastError());
    ++it;
    if (!fixed && (it % kPoll == 0 || it == cap)) {
      cg1_count_kernel<<<1, 256, 0, s>>>(N, state, count);
      L1_HIP(hipGetLastError());
      L1_HIP(hipMemcpyAsync(p->h_total, count, sizeof(int), hipMemcpyDeviceToHost, s));
      L1_HIP(hipStreamSynchronize(s));
      if (*p->h_total == 0) break;
    }
  }
  // instances still running reached the cap
  {
    std::vector<int> st(N);
    L1_HIP(hipMemcpyAsync(st.data(), status, sizeof(int) * N, hipMemcpyDeviceToHost, s));
    L1_HIP(hipStreamSynchronize(s));
    for (int j = 0; j < N; ++j)
      if (st[j] < 0) st[j] = L1_MAXITER;
    L1_HIP(hipMemcpyAsync(status, st.data(), sizeof(int) * N, hipMemcpyHostToDevice, s));
  }
  copy_rows(s, nd, N, p->W, lds, 0, sa.x, sa.ldx);
  if (cab) copy_rows(s, m, N, p->W, lds, nd, sa.e, sa.lde);
  copy_rows(s, m, N, Y, ldm, 0, sa.y, sa.ldy);
  finish_status(s, N, fixed ? cap : 0, iters, status, sa.iters, sa.status);
  L1_HIP(hipStreamSynchronize(s));
  for (int i = 0; i < 14; ++i) p->last_stats[i] = 0.0;
  p->last_stats[8] = (double)it;
  p->last_stats[9] =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
}

}  // namespace l1
