// Small per-solve and per-iteration kernels: penalty per instance, initial
// z/u, the convergence test with active-list compaction, the P_{1,2} block
// prox fix-up, PALM's outer-step elementwise work, and output extraction.
#include "steps.h"
#include "dalm_test.h"

namespace l1 {

__device__ inline uint16_t f2bf_s(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf2f_s(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
// the iterate as FP32 and, when requested, as a BF16 hi / lo split
__device__ inline void put_u(float* U, uint16_t* Uhi, uint16_t* Ulo, long idx, float u) {
  U[idx] = u;
  if (Uhi) {
    const uint16_t h = f2bf_s(u);
    Uhi[idx] = h;
    Ulo[idx] = f2bf_s(u - bf2f_s(h));
  }
}

__device__ float wg_sum(float v, float* sh) {
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

// ---- penalties ------------------------------------------------------------
// mode 0 (DALM):     pen = beta > 0 ? beta : dflt ||b||_1 / m
// mode 1 (PALM):     pen = xi > 0 ? xi : 2m/||b||_1
// (1 in place of ||b||_1 / m when b = 0); a positive finite pen_in[c]
// replaces the plan's value and the default
__global__ __launch_bounds__(256) void penalty_kernel(int m, const float* b, int ldb,
                                                      const float* pen_in, float fixed, int mode,
                                                      float dflt, float gfl, float div, float* pen,
                                                      float* ipen, float* wcap2, float* dscale2) {
  __shared__ float sh[256];
  const int c = blockIdx.x;
  float s = 0.0f, s2 = 0.0f;
  for (int i = threadIdx.x; i < m; i += 256) {
    const float v = b[(long)c * ldb + i];
    s += fabsf(v);
    s2 += v * v;
  }
  s = wg_sum(s, sh);
  s2 = wg_sum(s2, sh);
  if (threadIdx.x == 0) {
    const float beta0 = (s > 0.0f) ? s / (float)m : 1.0f;
    float p;
    const float given = pen_in ? pen_in[c] : 0.0f;
    if (given > 0.0f && isfinite(given)) p = given;
    else if (fixed > 0.0f) p = fixed;
    else if (mode == 0) p = dflt * beta0;
    else p = (s > 0.0f) ? 2.0f * (float)m / s : 1.0f;
    pen[c] = p;
    ipen[c] = 1.0f / p;
    if (wcap2) wcap2[c] = div * div * (float)m * s2;
    if (dscale2) {
      // pair per instance: the stopping test's (beta0 / beta)^2, and the
      // floor of its gap scale (||b||_1 / 4 for the cross-and-bouquet form)
      dscale2[2 * c] = (beta0 / p) * (beta0 / p);
      dscale2[2 * c + 1] = gfl * s;
    }
  }
}
void penalties(hipStream_t s, int N, int m, const float* b, int ldb, const float* pen_in,
               float fixed, int mode, float dflt, float gfl, float div, float* pen, float* ipen,
               float* wcap2, float* dscale2) {
  if (N <= 0) return;
  penalty_kernel<<<N, 256, 0, s>>>(m, b, ldb, pen_in, fixed, mode, dflt, gfl, div, pen, ipen, wcap2,
                                   dscale2);
  L1_HIP(hipGetLastError());
}

// ---- DALM initial operand: u = z_1 - w_0/beta, z_1 = prox(v_0 + w_0/beta) ----
__global__ __launch_bounds__(256) void dalm_init_u_kernel(DalmInit a) {
  __shared__ float sh[256];
  const int c = blockIdx.x;
  const float bt = a.beta[c], ib = 1.0f / bt;
  const float* V = a.V + (long)c * a.lds;
  const float* W = a.W + (long)c * a.lds;
  float zs = 1.0f;
  if (a.e0 < a.n) {
    float se = 0.0f;
    for (int i = a.e0 + threadIdx.x; i < a.n; i += 256) {
      const float s = V[i] + W[i] * ib;
      se += s * s;
    }
    se = wg_sum(se, sh);
    const float tau = a.eps[c] * ib;
    zs = (se > 0.0f) ? fmaxf(0.0f, 1.0f - tau / sqrtf(se)) : 0.0f;
    if (threadIdx.x == 0) a.zscale[c] = zs;
  }
  for (int i = threadIdx.x; i < a.n_pad; i += 256) {
    const float s = V[i] + W[i] * ib;
    const float z = (i >= a.e0) ? s * zs : fminf(fmaxf(s, -1.0f), 1.0f);
    put_u(a.U, a.Uhi, a.Ulo, (long)c * a.lds + i, z - W[i] * ib);
  }
}
void dalm_init_u(hipStream_t s, int N, const DalmInit& a) {
  if (N <= 0) return;
  dalm_init_u_kernel<<<N, 256, 0, s>>>(a);
  L1_HIP(hipGetLastError());
}

// ---- lists -------------------------------------------------------------------
__global__ void init_lists_kernel(int N, int phase0, Lists L, int* state_other, long long* stat) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < N) {
    L.state[c] = phase0;
    state_other[c] = phase0;
    L.iters[c] = 0;
    L.status[c] = L1_MAXITER;
  }
  const int npad = (N + TILE - 1) / TILE * TILE;
  if (c < npad) L.slot_col[c] = (c < N) ? c : -1;
  if (c == 0) {
    for (int p = 0; p <= NPHASE; ++p) L.phase_off[p] = (p <= phase0) ? 0 : npad;
    for (int p = 0; p < NPHASE; ++p) L.cnt[p] = (p == phase0) ? N : 0;
    *L.n_total = N;
    for (int i = 0; i < 8; ++i) stat[i] = 0;
  }
}
void init_lists(hipStream_t s, int N, int phase0, const Lists& L, int* state_other,
                long long* stat) {
  const int npad = (N + TILE - 1) / TILE * TILE;
  init_lists_kernel<<<(npad + 255) / 256, 256, 0, s>>>(N, phase0, L, state_other, stat);
  L1_HIP(hipGetLastError());
}

// Block-wide stable compaction of per-thread flags (1024 threads = 16 waves).
__device__ int compact_pos(bool flag, int* wave_tot, int* total_out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long m = __ballot(flag);
  const int before = __popcll(m & ((1ull << lane) - 1ull));
  if (lane == 0) wave_tot[wave] = __popcll(m);
  __syncthreads();
  int off = 0, total = 0;
  for (int w = 0; w < 16; ++w) {
    if (w < wave) off += wave_tot[w];
    total += wave_tot[w];
  }
  __syncthreads();
  *total_out = total;
  return off + before;
}

__global__ __launch_bounds__(1024) void dalm_compact_kernel(DalmCheck a) {
  __shared__ int wt[16];
  __shared__ int cnt[NPHASE], mx;
  if (threadIdx.x < NPHASE) cnt[threadIdx.x] = 0;
  if (threadIdx.x == 0) mx = 0;
  __syncthreads();
  int my[NPHASE] = {0, 0, 0}, mymax = 0;
  for (int c = threadIdx.x; c < a.N; c += 1024) {
    int st = a.L.state[c];
    // an instance whose low-precision iteration stalls above the switch
    // threshold would never leave its phase: after low_cap iterations it
    // moves on (its next test then sees sums of the old arithmetic and
    // decides nothing)
    if (st < NPHASE && st != a.final_phase && a.low_cap > 0 && a.L.iters[c] >= a.low_cap) {
      st += 1;
      a.L.state[c] = st;
    }
    a.state_other[c] = st;
    if (st < NPHASE) my[st] += 1;
    mymax = max(mymax, a.L.iters[c]);
  }
  for (int p = 0; p < NPHASE; ++p)
    if (my[p]) atomicAdd(&cnt[p], my[p]);
  atomicMax(&mx, mymax);
  __syncthreads();
  int off[NPHASE + 1];
  off[0] = 0;
  for (int p = 0; p < NPHASE; ++p) off[p + 1] = off[p] + (cnt[p] + TILE - 1) / TILE * TILE;
  int base[NPHASE] = {0, 0, 0};
  for (int c0 = 0; c0 < a.N; c0 += 1024) {
    const int c = c0 + threadIdx.x;
    const int st = (c < a.N) ? a.L.state[c] : NPHASE;
    for (int p = 0; p < NPHASE; ++p) {
      int tot;
      const int pos = compact_pos(st == p, wt, &tot);
      if (st == p) a.L.slot_col[off[p] + base[p] + pos] = c;
      base[p] += tot;
    }
  }
  for (int p = 0; p < NPHASE; ++p)
    for (int s = off[p] + cnt[p] + threadIdx.x; s < off[p + 1]; s += 1024) a.L.slot_col[s] = -1;
  if (threadIdx.x == 0) {
    for (int p = 0; p <= NPHASE; ++p) a.L.phase_off[p] = off[p];
    for (int p = 0; p < NPHASE; ++p) a.L.cnt[p] = cnt[p];
    *a.L.n_total = cnt[0] + cnt[1] + cnt[2];
    if (a.stat) a.stat[7] = mx;
  }
}
void dalm_compact(hipStream_t s, const DalmCheck& a) {
  dalm_compact_kernel<<<1, 1024, 0, s>>>(a);
  L1_HIP(hipGetLastError());
}

// the test of the last iteration: 4 lanes per instance, no iteration counted
__global__ __launch_bounds__(256) void dalm_final_test_kernel(DalmCheck a) {
  const int c = blockIdx.x * 64 + (threadIdx.x >> 2), part = threadIdx.x & 3;
  const int st0 = (c < a.N) ? a.L.state[c] : NPHASE;
  float sm[NPART];
  column_sums(a.partial, a.ldp, a.ntiles, c, st0 < NPHASE, part, sm);
  if (part != 0 || st0 >= NPHASE) return;
  TestParams tp;
  tp.tol = a.tol;
  tp.sw = a.sw;
  tp.final_phase = a.final_phase;
  for (int q = 0; q < NPHASE; ++q) tp.floor[q] = a.floor[q];
  tp.wcap2 = a.wcap2 ? a.wcap2[c] : INFINITY;
  tp.dscale2 = a.dscale2 ? a.dscale2[2 * c] : 1.0f;
  tp.gfloor = a.dscale2 ? a.dscale2[2 * c + 1] : 0.0f;
  int status = L1_MAXITER;
  const int st = decide_in(tp, st0, a.arith ? a.arith[c] : NPHASE, sm, &status);
  if (st != st0) a.L.state[c] = st;
  if (st >= NPHASE) a.L.status[c] = status;
}
void dalm_final_test(hipStream_t s, const DalmCheck& a) {
  dalm_final_test_kernel<<<(a.N + 63) / 64, 256, 0, s>>>(a);
  L1_HIP(hipGetLastError());
}

// ---- P_{1,2}: next operand on the eps-ball rows once the column norm is known --
__global__ __launch_bounds__(256) void p12_fix_kernel(P12Fix a) {
  const int slot = blockIdx.x;
  if (slot >= a.phase_off[NPHASE]) return;
  const int c = a.slot_col[slot];
  if (c < 0 || a.state[c] >= NPHASE) return;
  __shared__ float sh_scale;
  if (threadIdx.x < 64) {
    // the same sums, in the same order, as the next launch's prologue
    float sm[NPART];
    column_sums(a.partial, a.ldp, a.ntiles, c, true, threadIdx.x & 3, sm);
    if (threadIdx.x == 0) sh_scale = ball_scale(sm[4], a.eps[c], a.beta[c]);
  }
  __syncthreads();
  const float ib = 1.0f / a.beta[c];
  const float zs = sh_scale;
  for (int i = a.e0 + threadIdx.x; i < a.n; i += 256) {
    const long idx = (long)c * a.lds + i;
    const float w = a.W[idx];
    const float s2 = a.V[idx] + w * ib;
    put_u(a.U, a.Uhi, a.Ulo, idx, s2 * zs - w * ib);
  }
}
void p12_fix(hipStream_t s, int n_blocks, const P12Fix& a) {
  if (n_blocks <= 0) return;
  p12_fix_kernel<<<n_blocks, 256, 0, s>>>(a);
  L1_HIP(hipGetLastError());
}

// ---- outputs -------------------------------------------------------------------
__global__ void copy_block_kernel(int rows, int N, const float* src, int lds, int r0, float* dst,
                                  int ldd) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)rows * N) return;
  const int i = (int)(e % rows), c = (int)(e / rows);
  dst[(long)c * ldd + i] = src[(long)c * lds + r0 + i];
}
void copy_block(hipStream_t s, int rows, int N, const float* src, int lds, int r0, float* dst,
                int ldd) {
  const long n = (long)rows * N;
  if (n <= 0 || !dst) return;
  copy_block_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(rows, N, src, lds, r0, dst, ldd);
  L1_HIP(hipGetLastError());
}
__global__ void copy_in_kernel(int rows, int N, const float* src, int lds, float* dst, int ldd,
                               int r0) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)rows * N) return;
  const int i = (int)(e % rows), c = (int)(e / rows);
  dst[(long)c * ldd + r0 + i] = src[(long)c * lds + i];
}
void copy_in(hipStream_t s, int rows, int N, const float* src, int lds, float* dst, int ldd,
             int r0) {
  const long n = (long)rows * N;
  if (n <= 0) return;
  copy_in_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(rows, N, src, lds, dst, ldd, r0);
  L1_HIP(hipGetLastError());
}
__global__ void finish_status_kernel(int N, int fixed, const int* iters, const int* status,
                                     int* it_out, int* st_out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  if (it_out) it_out[c] = (fixed > 0) ? fixed : iters[c];
  if (st_out) st_out[c] = (fixed > 0) ? (status[c] == L1_NONFINITE ? L1_NONFINITE : L1_CONVERGED)
                                      : status[c];
}
void finish_status(hipStream_t s, int N, int fixed, const int* iters, const int* status,
                   int* it_out, int* st_out) {
  if (N <= 0 || (!it_out && !st_out)) return;
  finish_status_kernel<<<(N + 255) / 256, 256, 0, s>>>(N, fixed, iters, status, it_out, st_out);
  L1_HIP(hipGetLastError());
}

}  // namespace l1
