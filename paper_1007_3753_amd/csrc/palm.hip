// Primal ALM (Sec. V-A): the method of multipliers on the augmented
// Lagrangian, with FISTA (Sec. IV-A) for the x-subproblem; for the
// cross-and-bouquet problem the e-subproblem has the closed form of
// Algorithm 1 (steps 3 and 10).  Per outer step k, for every unfinished
// instance:
//   e-step   e = prox(b - A x + theta/xi), c = b - e + theta/xi     (palm_estep)
//   h = A^T c                                                        (FP32 GEMM)
//   FISTA    w <- shrink(z + (h - M z)/L, 1/(xi L)), z <- w + gamma (w - w_prev),
//            M = A^T A, from z = w = x, until the relative change of w is
//            <= tol_inner or max_inner steps                      (GEMM, EPI_FISTA)
//   q = A w                                                          (FP32 GEMM)
//   update   theta += xi (b - q - e), outer test, x = w, xi *= growth (palm_update)
// The e-step prox: shrink(., 1/xi) for the cross-and-bouquet (P1); for
// (QP_lambda) the scaling xi lam/(1 + xi lam); for (P_{1,2}) the projection
// onto the eps-ball; none for the dense (P1).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>

#include "plan.h"
#include "steps.h"

namespace l1 {

namespace {

__device__ inline uint16_t f2bf_p(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf2f_p(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

__device__ float blk_sum(float v, float* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  const float r = sh[0];
  __syncthreads();
  return r;
}

enum EProx { EP_NONE = 0, EP_SHRINK = 1, EP_SCALE = 2, EP_BALL = 3 };

struct PalmArgs {
  int m, nd, lds, ldm, ldb, N;   // lds: ld of the n_dict-row buffers, ldm: of the m-row ones
  int eprox;
  float lambda;
  const float* b;       // m_pad x N, ld ldb
  const float* q;       // A x (m rows)
  float* E;             // e (m rows)
  float* Eprev;         // e of the previous outer step
  float* Th;            // theta (m rows)
  float* Cv;            // c = b - e + theta/xi (m_pad rows; the K operand of h = A^T c)
  float* X;             // x (nd rows)
  float* Wv;            // FISTA shrink output (nd rows)
  float* Z;             // FISTA point, buffer 0 (nd rows)
  uint16_t* Zhi;        // its BF16 split (or null)
  uint16_t* Zlo;
  float* xi;            // penalty per instance
  const float* eps;     // P_{1,2} radii
  const float* wcap2;   // squared L1_DIVERGED thresholds
  int* state;           // 0 active, NPHASE finished (outer loop)
  int* inner_state[2];  // inner-loop phase buffers: reset to `phase` for active instances
  int phase;            // phase index of the inner products
  int* iters;
  int* status;
  const int* slot_col;
  const int* phase_off;
  float tol, growth;
};

// e-step and the start of the FISTA loop (one workgroup per listed instance)
__global__ __launch_bounds__(256) void palm_estep_kernel(PalmArgs a) {
  __shared__ float sh[256];
  const int slot = blockIdx.x;
  if (slot >= a.phase_off[NPHASE]) return;
  const int c = a.slot_col[slot];
  if (c < 0 || a.state[c] >= NPHASE) return;
  const float xi = a.xi[c], ixi = 1.0f / xi;
  const float* b = a.b + (long)c * a.ldb;
  const long o = (long)c * a.ldm, on = (long)c * a.lds;
  float scale = 1.0f;
  if (a.eprox == EP_BALL) {
    float s2 = 0.0f;
    for (int i = threadIdx.x; i < a.m; i += 256) {
      const float v = b[i] - a.q[o + i] + a.Th[o + i] * ixi;
      s2 += v * v;
    }
    s2 = blk_sum(s2, sh);
    const float nv = sqrtf(s2);
    scale = (nv > a.eps[c]) ? a.eps[c] / nv : 1.0f;
  }
  for (int i = threadIdx.x; i < a.m; i += 256) {
    const float v = b[i] - a.q[o + i] + a.Th[o + i] * ixi;
    float e;
    if (a.eprox == EP_SHRINK) {
      const float mm = fabsf(v) - ixi;
      e = mm > 0.0f ? copysignf(mm, v) : 0.0f;
    } else if (a.eprox == EP_SCALE) {
      e = (xi * a.lambda / (1.0f + xi * a.lambda)) * v;
    } else if (a.eprox == EP_BALL) {
      e = v * scale;
    } else {
      e = 0.0f;
    }
    a.Eprev[o + i] = a.E[o + i];
    a.E[o + i] = e;
    a.Cv[o + i] = b[i] - e + a.Th[o + i] * ixi;
  }
  // FISTA starts from z = w = x
  for (int i = threadIdx.x; i < a.nd; i += 256) {
    const float x = a.X[on + i];
    a.Wv[on + i] = x;
    a.Z[on + i] = x;
    if (a.Zhi) {
      const uint16_t h = f2bf_p(x);
      a.Zhi[on + i] = h;
      a.Zlo[on + i] = f2bf_p(x - bf2f_p(h));
    }
  }
  if (threadIdx.x == 0) {
    a.inner_state[0][c] = a.phase;
    a.inner_state[1][c] = a.phase;
  }
}

// multiplier update, outer test, x <- w (one workgroup per listed instance)
__global__ __launch_bounds__(256) void palm_update_kernel(PalmArgs a) {
  __shared__ float sh[256];
  const int slot = blockIdx.x;
  if (slot >= a.phase_off[NPHASE]) return;
  const int c = a.slot_col[slot];
  if (c < 0 || a.state[c] >= NPHASE) return;
  const float xi = a.xi[c];
  const float* b = a.b + (long)c * a.ldb;
  const long o = (long)c * a.ldm, on = (long)c * a.lds;
  float rr = 0.0f, bb = 0.0f, de = 0.0f, ee = 0.0f, dx = 0.0f, xx = 0.0f;
  for (int i = threadIdx.x; i < a.m; i += 256) {
    const float r = b[i] - a.q[o + i] - a.E[o + i];
    a.Th[o + i] += xi * r;
    rr += r * r;
    bb += b[i] * b[i];
    const float d = a.E[o + i] - a.Eprev[o + i];
    de += d * d;
    ee += a.E[o + i] * a.E[o + i];
  }
  for (int i = threadIdx.x; i < a.nd; i += 256) {
    const float w = a.Wv[on + i];
    const float d = w - a.X[on + i];
    dx += d * d;
    xx += w * w;
    a.X[on + i] = w;
  }
  rr = blk_sum(rr, sh);
  bb = blk_sum(bb, sh);
  de = blk_sum(de, sh);
  ee = blk_sum(ee, sh);
  dx = blk_sum(dx, sh);
  xx = blk_sum(xx, sh);
  if (threadIdx.x == 0) {
    a.iters[c] += 1;
    const float dw = dx + de, nw = xx + ee;
    if (!(isfinite(dw) && isfinite(nw) && isfinite(rr))) {
      a.state[c] = NPHASE;
      a.status[c] = L1_NONFINITE;
    } else if (a.tol >= 0.0f && nw > a.wcap2[c]) {
      a.state[c] = NPHASE;
      a.status[c] = L1_DIVERGED;
    } else if (a.tol >= 0.0f && dw <= a.tol * a.tol * nw && rr <= a.tol * a.tol * bb) {
      a.state[c] = NPHASE;
      a.status[c] = L1_CONVERGED;
    } else {
      a.xi[c] = xi * a.growth;
    }
  }
}

// initial state: x = w = z = 0, e = b (Algorithm 1 input) or 0, theta = 0
__global__ void palm_init_kernel(PalmArgs a, int has_e) {
  const int c = blockIdx.y;
  const long o = (long)c * a.ldm, on = (long)c * a.lds;
  const float* b = a.b + (long)c * a.ldb;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < a.lds; i += gridDim.x * blockDim.x) {
    a.X[on + i] = 0.0f;
    a.Wv[on + i] = 0.0f;
    a.Z[on + i] = 0.0f;
  }
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < a.ldm; i += gridDim.x * blockDim.x) {
    a.Th[o + i] = 0.0f;
    a.Cv[o + i] = 0.0f;
    const float e = (has_e && i < a.m) ? b[i] : 0.0f;
    a.E[o + i] = e;
    a.Eprev[o + i] = e;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.state[c] = 0;
    a.iters[c] = 0;
    a.status[c] = L1_MAXITER;
  }
}

// active-instance list of the outer loop; two phase layouts are written:
// off32 (every slot FP32) for the A x / A^T c products and offp (every slot
// in the inner products' phase) for the FISTA products
__global__ __launch_bounds__(1024) void palm_compact_kernel(int N, const int* state, int* slot_col,
                                                            int* off32, int* offp, int phase,
                                                            int* n_total) {
  __shared__ int wt[16];
  int base = 0;
  for (int c0 = 0; c0 < N; c0 += 1024) {
    const int c = c0 + threadIdx.x;
    const bool f = c < N && state[c] < NPHASE;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const unsigned long long mk = __ballot(f);
    if (lane == 0) wt[wave] = __popcll(mk);
    __syncthreads();
    int off = 0, tot = 0;
    for (int w = 0; w < 16; ++w) {
      if (w < wave) off += wt[w];
      tot += wt[w];
    }
    if (f) slot_col[base + off + __popcll(mk & ((1ull << lane) - 1ull))] = c;
    base += tot;
    __syncthreads();
  }
  const int npad = (base + TILE - 1) / TILE * TILE;
  for (int s = base + threadIdx.x; s < npad; s += 1024) slot_col[s] = -1;
  if (threadIdx.x == 0) {
    for (int p = 0; p <= NPHASE; ++p) {
      off32[p] = (p <= PREC_F32) ? 0 : npad;
      offp[p] = (p <= phase) ? 0 : npad;
    }
    *n_total = base;
  }
}

// number of listed instances still inside the FISTA loop
__global__ __launch_bounds__(1024) void palm_inner_live_kernel(const int* slot_col,
                                                               const int* phase_off,
                                                               const int* inner_state, int* out) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  int k = 0;
  for (int sl = threadIdx.x; sl < phase_off[NPHASE]; sl += 1024) {
    const int c = slot_col[sl];
    if (c >= 0 && inner_state[c] < NPHASE) ++k;
  }
  if (k) atomicAdd(&cnt, k);
  __syncthreads();
  if (threadIdx.x == 0) *out = cnt;
}

__global__ void copy_out_kernel(int rows, int N, const float* src, int lds, float* dst, int ldd) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)rows * N) return;
  const int i = (int)(e % rows), c = (int)(e / rows);
  dst[(long)c * ldd + i] = src[(long)c * lds + i];
}

}  // namespace

void solve_palm(Plan* p, const SolveArgs& sa) {
  L1_REQUIRE(sa.N >= 0 && sa.N <= p->d.max_batch, "N must be in [0, max_batch]");
  if (sa.N == 0) return;
  L1_REQUIRE(sa.b != nullptr && sa.x != nullptr, "b and x must be non-NULL");
  L1_REQUIRE(sa.ldb >= p->m && sa.ldx >= std::max(p->nd, 1), "bad leading dimension");
  L1_REQUIRE(sa.e == nullptr || sa.lde >= p->m, "lde < m");
  L1_REQUIRE(p->d.problem != L1_P12 || sa.eps != nullptr, "P_{1,2} needs eps (N radii)");
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

  const int N = sa.N, m = p->m, nd = p->nd, lds = p->lds, Np = p->N_pad;
  const bool fixed = sa.max_iter < 0;
  const int cap = fixed ? -sa.max_iter : sa.max_iter;
  const int max_inner = p->d.max_inner > 0 ? p->d.max_inner : 100;
  const float tol_in = fixed ? -1.0f : (p->d.tol_inner > 0 ? (float)p->d.tol_inner : sa.tol);
  const float growth = p->d.xi_growth > 0 ? (float)p->d.xi_growth : 1.0f;
  const int phase = (p->d.precision == L1_FP32) ? PREC_F32 : PREC_BF16X3;
  const bool low = phase != PREC_F32;
  const bool has_e = p->split || p->d.problem == L1_QPLAMBDA;

  // buffers: the n_dict-row vectors are column-major with leading dimension
  // lds, the m-row vectors with leading dimension m_pad (N_pad columns)
  const int ldm = p->m_pad;
  float* Q = p->aux;
  float* Th = p->aux + (size_t)ldm * Np;
  float* Cv = p->aux + (size_t)2 * ldm * Np;
  float* Eprev = p->aux + (size_t)3 * ldm * Np;
  float* E = p->V;
  float* X = p->W;
  float* Wv = p->C;
  float* Zb[2] = {p->Z[0], p->Z[1]};
  float* H = p->Uf[0];
  int* q = p->ints;
  int* state = q;
  int* iters = q + Np;
  int* status = q + 2 * Np;
  int* slot_col = q + 3 * Np;                    // Np + NPHASE*TILE
  int* off32 = q + 4 * Np + NPHASE * TILE;       // NPHASE + 1
  int* offp = off32 + NPHASE + 1;                // NPHASE + 1
  int* n_total = offp + NPHASE + 1;
  int* n_inner = n_total + 1;
  int* inner_st[2] = {q + 5 * Np + 256, q + 6 * Np + 256};
  int* inner_it = q + 7 * Np + 256;
  float* part[2] = {p->partial, p->partial + (size_t)p->ntiles * NPART * Np};

  L1_HIP(hipMemsetAsync(p->bb, 0, sizeof(float) * ldm * N, s));
  L1_HIP(hipMemcpy2DAsync(p->bb, sizeof(float) * ldm, sa.b, sizeof(float) * sa.ldb,
                          sizeof(float) * m, N, hipMemcpyDeviceToDevice, s));
  penalties(s, N, m, p->bb, ldm, sa.pen, p->d.xi > 0 ? (float)p->d.xi : 0.0f, 1, 1.0f, 0.0f, div_factor(p),
            p->pen, p->ipen, p->wcap2, nullptr);
  float* eps = nullptr;
  if (p->d.problem == L1_P12) {
    eps = p->tscal;
    L1_HIP(hipMemcpyAsync(eps, sa.eps, sizeof(float) * N, hipMemcpyDeviceToDevice, s));
  }
  // zero padding rows of every product operand
  L1_HIP(hipMemsetAsync(Q, 0, sizeof(float) * (size_t)ldm * N, s));
  L1_HIP(hipMemsetAsync(Zb[1], 0, sizeof(float) * (size_t)lds * N, s));
  L1_HIP(hipMemsetAsync(H, 0, sizeof(float) * (size_t)lds * N, s));
  L1_HIP(hipMemsetAsync(inner_it, 0, sizeof(int) * N, s));
  L1_HIP(hipMemsetAsync(p->stat, 0, sizeof(long long) * 8, s));

  PalmArgs pa{};
  pa.m = m;
  pa.nd = nd;
  pa.lds = lds;
  pa.ldm = ldm;
  pa.ldb = ldm;
  pa.N = N;
  pa.eprox = (p->d.structure == L1_CAB) ? EP_SHRINK
             : (p->d.problem == L1_QPLAMBDA) ? EP_SCALE
             : (p->d.problem == L1_P12) ? EP_BALL : EP_NONE;
  pa.lambda = (float)p->d.lambda;
  pa.b = p->bb;
  pa.q = Q;
  pa.E = E;
  pa.Eprev = Eprev;
  pa.Th = Th;
  pa.Cv = Cv;
  pa.X = X;
  pa.Wv = Wv;
  pa.Z = Zb[0];
  pa.Zhi = low ? p->Uh[0] : nullptr;
  pa.Zlo = low ? p->Ul[0] : nullptr;
  pa.xi = p->pen;
  pa.eps = eps;
  pa.wcap2 = p->wcap2;
  pa.state = state;
  pa.inner_state[0] = inner_st[0];
  pa.inner_state[1] = inner_st[1];
  pa.phase = phase;
  pa.iters = iters;
  pa.status = status;
  pa.slot_col = slot_col;
  pa.phase_off = off32;
  pa.tol = fixed ? -1.0f : sa.tol;
  pa.growth = growth;
  palm_init_kernel<<<dim3((lds + 255) / 256, N), 256, 0, s>>>(pa, has_e ? 1 : 0);
  L1_HIP(hipGetLastError());
  palm_compact_kernel<<<1, 1024, 0, s>>>(N, state, slot_col, off32, offp, phase, n_total);
  L1_HIP(hipGetLastError());

  // products
  GemmArgs gq{};          // q = A w
  gq.A32 = p->Arow;
  gq.lda = p->nd_pad;
  gq.B = Wv;
  gq.ldb = lds;
  gq.M = p->m_pad;
  gq.K = p->nd_pad;
  gq.slot_col = slot_col;
  gq.phase_off = off32;
  gq.n_cols = N;
  gq.m_true = p->m_pad;
  gq.out = Q;
  gq.ldo = ldm;
  GemmArgs gh = gq;       // h = A^T c
  gh.A32 = p->Acol;
  gh.lda = p->m_pad;
  gh.B = Cv;
  gh.ldb = ldm;
  gh.M = p->nd_pad;
  gh.K = p->m_pad;
  gh.m_true = p->nd_pad;
  gh.out = H;
  gh.ldo = lds;
  GemmArgs gf{};          // FISTA step with M = A^T A
  gf.A32 = p->M32;
  gf.Ahi = p->Mhi;
  gf.Alo = p->Mlo;
  gf.lda = p->nd_pad;
  gf.ldb = lds;
  gf.M = p->nd_pad;
  gf.K = p->nd_pad;
  gf.slot_col = slot_col;
  gf.phase_off = offp;
  gf.n_cols = N;
  gf.m_true = p->nd_pad;
  gf.lds = lds;
  gf.W = Wv;
  gf.C = H;
  gf.beta = p->pen;
  gf.ldp = Np;
  gf.inv_L = (float)(1.0 / p->Lf);
  gf.iters = inner_it;
  gf.tp_tol = tol_in;
  gf.test_kind = 1;
  gf.stat = p->stat;
  const int ctiles = col_tiles_for(N);
  const int blocks = ctiles * TILE;
  constexpr int kInnerPoll = 8;   // FISTA steps between host checks of the inner loop
  constexpr int kOuterPoll = 4;   // outer steps between host checks of the batch

  int outer = 0;
  long long inner_total = 0;
  while (outer < cap) {
    // e-step from q = A x of the current x; FISTA starts from z = w = x
    palm_estep_kernel<<<blocks, 256, 0, s>>>(pa);
    L1_HIP(hipGetLastError());
    launch_gemm(s, EPI_STORE, gh, ctiles);
    // FISTA loop over the listed instances, t_1 = 1.  Launch l tests the
    // shrink output of launch l - 1 in its prologue; a finished instance
    // keeps its last shrink output in Wv.
    double t = 1.0;
    for (int l = 0; l < max_inner; ++l) {
      const double tn = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * t * t));
      const int cur = l & 1;
      gf.B = Zb[cur];
      gf.Bhi = low ? p->Uh[cur] : nullptr;
      gf.Blo = low ? p->Ul[cur] : nullptr;
      gf.V = Zb[cur];
      gf.out = Zb[1 - cur];
      gf.Uhi = low ? p->Uh[1 - cur] : nullptr;
      gf.Ulo = low ? p->Ul[1 - cur] : nullptr;
      gf.gamma = (float)((t - 1.0) / tn);
      gf.state_in = inner_st[cur];
      gf.state_out = inner_st[1 - cur];
      gf.prev_partial = (l == 0) ? nullptr : part[1 - cur];
      gf.partial = part[cur];
      launch_gemm(s, EPI_FISTA, gf, ctiles);
      t = tn;
      ++inner_total;
      if (!fixed && (l + 1) % kInnerPoll == 0 && l + 1 < max_inner) {
        // instances whose test (up to launch l - 1) has not yet passed
        palm_inner_live_kernel<<<1, 1024, 0, s>>>(slot_col, offp, inner_st[1 - cur], n_inner);
        L1_HIP(hipGetLastError());
        L1_HIP(hipMemcpyAsync(p->h_total + 1, n_inner, sizeof(int), hipMemcpyDeviceToHost, s));
        L1_HIP(hipStreamSynchronize(s));
        if (p->h_total[1] == 0) break;
      }
    }
    // q = A w, multiplier update and outer test; x <- w
    launch_gemm(s, EPI_STORE, gq, ctiles);
    palm_update_kernel<<<blocks, 256, 0, s>>>(pa);
    L1_HIP(hipGetLastError());
    palm_compact_kernel<<<1, 1024, 0, s>>>(N, state, slot_col, off32, offp, phase, n_total);
    L1_HIP(hipGetLastError());
    ++outer;
    if (!fixed && (outer % kOuterPoll == 0 || outer == cap)) {
      L1_HIP(hipMemcpyAsync(p->h_total, n_total, sizeof(int), hipMemcpyDeviceToHost, s));
      L1_HIP(hipStreamSynchronize(s));
      if (*p->h_total == 0) break;
    }
  }
  // outputs
  {
    const long nx = (long)nd * N;
    if (nx > 0)
      copy_out_kernel<<<(unsigned)((nx + 255) / 256), 256, 0, s>>>(nd, N, X, lds, sa.x, sa.ldx);
    if (sa.e && has_e) {
      const long ne = (long)m * N;
      copy_out_kernel<<<(unsigned)((ne + 255) / 256), 256, 0, s>>>(m, N, E, ldm, sa.e, sa.lde);
    }
    L1_HIP(hipGetLastError());
  }
  finish_status(s, N, fixed ? cap : 0, iters, status, sa.iters, sa.status);
  long long hstat[8];
  L1_HIP(hipMemcpyAsync(hstat, p->stat, sizeof(hstat), hipMemcpyDeviceToHost, s));
  L1_HIP(hipStreamSynchronize(s));
  const int map[3] = {PREC_F32, PREC_BF16, PREC_BF16X3};
  for (int i = 0; i < 14; ++i) p->last_stats[i] = 0.0;
  for (int i = 0; i < 3; ++i) {
    p->last_stats[i] = (double)hstat[map[i]];
    p->last_stats[3 + i] = (double)hstat[3 + map[i]];
  }
  p->last_stats[8] = (double)outer;
  p->last_stats[11] = (double)inner_total;
  p->last_stats[9] =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
}

}  // namespace l1
