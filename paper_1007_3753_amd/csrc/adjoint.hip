// Reverse mode of a fixed number of dual ALM iterations (Sec. V-B,
// Algorithm 2) with respect to the right-hand sides b and the dictionary.
//
// The iteration runs in the form of the forward solve: with v = A^T y,
//   s_k = v_k + w_k/beta,  z_k = clamp(s_k),  u_k = z_k - w_k/beta
//   v_{k+1} = P u_k + c,   P = A^T M A,  c = A^T M b/beta,  M = (A A^T + shift I)^{-1}
//   w_{k+1} = w_k - beta z_k + beta v_{k+1}
// (the y-step composed with A^T; A = [B, I] for the cross-and-bouquet form).
// Given the adjoints of w_K (gx, ge), one reverse step is
//   vt   = vbar_{k+1} + beta wbar_{k+1}          (total adjoint of v_{k+1})
//   ubar = P vt                                  (P is symmetric)
//   sbar = 1{|s_k| < 1} (ubar - beta wbar_{k+1})
//   vbar_k = sbar,  wbar_k = wbar_{k+1} - ubar/beta + sbar/beta
// and the products accumulate Pbar = sum_k vt_k u_k^T and cbar = sum_k vt_k.
// From those, with Y = M A and bt = b/beta (per column),
//   bbar  = Y cbar / beta
//   Abar  = Y (Pbar + Pbar^T) + M bt cbar^T + (Gbar + Gbar^T) A,
//   Gbar  = -M (A Pbar A^T + A cbar bt^T) M
// and the dictionary gradient is the B block of Abar (the identity block is
// constant).  beta is held constant (it is not differentiated).
//
// The forward states are recomputed segment by segment from the checkpoints
// the recording solve kept, with the same product launches, so each segment
// reproduces the recorded iterates exactly.  The FP32 reverse steps use the
// iteration GEMM; Pbar, cbar and the dictionary terms are accumulated in FP64.
#include <algorithm>
#include <vector>

#include "plan.h"
#include "steps.h"

namespace l1 {

namespace {

struct Bufs {
  std::vector<void*> v;
  ~Bufs() {
    for (void* q : v) (void)hipFree(q);
  }
  template <class T>
  T* get(size_t n) {
    void* q = nullptr;
    if (hipMalloc(&q, sizeof(T) * std::max<size_t>(n, 1)) != hipSuccess) {
      (void)hipGetLastError();
      set_error("out of device memory in l1_alm_backward");
      throw Fail{L1_ENOMEM};
    }
    v.push_back(q);
    return reinterpret_cast<T*>(q);
  }
};

// Workspaces of the backward that the plan keeps: the k-th request of a call
// gets the k-th kept buffer when it is large enough (the requests come in the
// same order in every call), else a new one replaces it.  The previous
// backward ended with a stream synchronisation, so no kernel still uses a
// buffer that is replaced.
struct Arena {
  Plan* p;
  size_t i = 0;
  template <class T>
  T* get(size_t n) {
    const size_t bytes = sizeof(T) * std::max<size_t>(n, 1);
    auto& v = p->adj_ws;
    if (i < v.size() && v[i].first >= bytes) return reinterpret_cast<T*>(v[i++].second);
    if (i < v.size()) {
      (void)hipFree(v[i].second);
      v[i] = {0, nullptr};
    }
    void* q = nullptr;
    if (hipMalloc(&q, bytes) != hipSuccess) {
      (void)hipGetLastError();
      set_error("out of device memory in l1_alm_backward");
      throw Fail{L1_ENOMEM};
    }
    if (i < v.size()) v[i] = {bytes, q};
    else v.push_back({bytes, q});
    return reinterpret_cast<T*>(v[i++].second);
  }
};

// wbar = [gx; ge] (the adjoints of the outputs), vt = beta wbar (vbar_K = 0)
__global__ void adj_init_kernel(int nd, int m, int split, int n, int lds, int N, const float* gx,
                                const float* ge, const float* beta, float* Wb, float* Vt) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)lds * N) return;
  const int i = (int)(e % lds), c = (int)(e / lds);
  float g = 0.0f;
  if (i < nd) g = gx[(long)c * nd + i];
  else if (split && i < n && ge) g = ge[(long)c * m + (i - nd)];
  Wb[e] = g;
  Vt[e] = beta[c] * g;
}

// one reverse step through iteration k (state v_k, w_k; Ub = P vt_k)
__global__ void adj_step_kernel(int n, int lds, int N, const float* v, const float* w,
                                const float* beta, const float* ibeta, const float* Ub, float* Wb,
                                float* Vt, float* seg_vt, float* seg_u, double* cbar) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * N) return;
  const int i = (int)(e % n), c = (int)(e / n);
  const long o = (long)c * lds + i;
  const float bt = beta[c], ib = ibeta[c];
  const float s = v[o] + w[o] * ib;
  const float z = fminf(fmaxf(s, -1.0f), 1.0f);
  const float vt = Vt[o], ub = Ub[o], wb = Wb[o];
  seg_vt[o] = vt;
  seg_u[o] = z - w[o] * ib;
  cbar[(long)c * n + i] += (double)vt;
  const float sb = (fabsf(s) < 1.0f) ? ub - bt * wb : 0.0f;
  const float wn = wb - ub * ib + sb * ib;
  Wb[o] = wn;
  Vt[o] = sb + bt * wn;
}

// A = [B, I] (split) or A = B, FP64, ld m
__global__ void full_matrix64_kernel(int m, int nd, int n, const float* B, double* A) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)m * n) return;
  const int i = (int)(e % m), j = (int)(e / m);
  A[e] = (j < nd) ? (double)B[(long)j * m + i] : ((j - nd == i) ? 1.0 : 0.0);
}

// dst(i, c) = src(i, c) * scale[c], FP32 -> FP64 (scale may be null)
__global__ void scale_cols64_kernel(int rows, int N, const float* src, int lds, const float* scale,
                                    double* dst, int ldd) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)rows * N) return;
  const int i = (int)(e % rows), c = (int)(e / rows);
  dst[(long)c * ldd + i] = (double)src[(long)c * lds + i] * (scale ? (double)scale[c] : 1.0);
}

// out(i, c) = src(i, c) * scale[c] (FP64 -> FP32), overwrite
// dst (rows_pad x ldd, row-major) = src^T for src (rows x cols, column-major,
// ld lds), zero in the padding: the K-contiguous operand layout of the
// iteration GEMM.  32 x 32 tiles through LDS, both sides coalesced.
__global__ __launch_bounds__(256) void transpose_pad_kernel(int rows, int cols, const float* src,
                                                            int lds, float* dst, int ldd) {
  __shared__ float t[32][33];
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  for (int k = ty; k < 32; k += 8) {
    const int c = c0 + k, r = r0 + tx;
    t[k][tx] = (c < cols && r < rows) ? src[(long)c * lds + r] : 0.0f;
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int r = r0 + k, c = c0 + tx;
    if (c < ldd) dst[(long)r * ldd + c] = t[tx][k];
  }
}
// D (FP64, n x n, ld ldd) += S (FP32, n x n, ld lds)
__global__ void add_f32_to_f64_kernel(int n, const float* S, int lds, double* D, int ldd) {
  const long total = (long)n * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), j = (int)(e / n);
    D[i + (long)j * ldd] += (double)S[i + (long)j * lds];
  }
}

__global__ void store_cols_kernel(int rows, int N, const double* src, int lds, const float* scale,
                                  float* out, int ldo) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)rows * N) return;
  const int i = (int)(e % rows), c = (int)(e / rows);
  out[(long)c * ldo + i] = (float)(src[(long)c * lds + i] * (double)scale[c]);
}

// out(i, j) += src(i, j) (FP64 -> FP32)
__global__ void add_block_kernel(int rows, int cols, const double* src, int lds, float* out,
                                 int ldo) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)rows * cols) return;
  const int i = (int)(e % rows), j = (int)(e / rows);
  out[(long)j * ldo + i] += (float)src[(long)j * lds + i];
}

inline unsigned blocks_for(long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

void backward_dalm(Plan* p, const float* gx, const float* ge, float* gb, float* gA,
                   hipStream_t us) {
  if (p->tape.empty() || p->tape_N <= 0) {
    set_error("no recorded tape: solve with max_iter < 0 and desc.record_tape = 1 first");
    throw Fail{L1_ENOTAPE};
  }
  L1_REQUIRE(gx != nullptr || p->nd == 0, "gx must be non-NULL");
  L1_REQUIRE(gb != nullptr || gA != nullptr, "nothing to compute: gb and gA are both NULL");
  const int N = p->tape_N, K = p->tape_K, every = p->tape_every;
  const int m = p->m, nd = p->nd, n = p->n, lds = p->lds, n_pad = p->n_pad;
  const int nseg = (K + every - 1) / every;
  const int ntc = (N + TILE - 1) / TILE;
  const int ks = dalm_ksplit(p, N, 1);

  hipStream_t s;
  hipEvent_t ev;
  L1_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  L1_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
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
  L1_HIP(hipEventRecord(ev, us));
  L1_HIP(hipStreamWaitEvent(s, ev, 0));

  Arena bf{p};
  Bufs once;   // buffers of the one-time factorisation
  const size_t st = (size_t)lds * N;
  float* Wb = bf.get<float>(st);
  float* Vt = bf.get<float>(st);
  float* Ub = bf.get<float>(st);
  float* seg_v = bf.get<float>(st * every);
  float* seg_w = bf.get<float>(st * every);
  float* seg_vt = bf.get<float>(st * every);
  float* seg_u = bf.get<float>(st * every);
  double* cbar = bf.get<double>((size_t)n * N);
  double* Pbar = bf.get<double>((size_t)n * n);
  // the segment's operands of P-bar, K-contiguous FP32 (K = len N padded to
  // 64), and its FP32 product
  const int cpad = (N * every + 63) / 64 * 64;
  float* VtT = bf.get<float>((size_t)n_pad * cpad);
  float* UT = bf.get<float>((size_t)n_pad * cpad);
  float* Pseg = bf.get<float>((size_t)n_pad * n);
  L1_HIP(hipMemsetAsync(Vt, 0, sizeof(float) * st, s));
  L1_HIP(hipMemsetAsync(Ub, 0, sizeof(float) * st, s));
  L1_HIP(hipMemsetAsync(cbar, 0, sizeof(double) * n * N, s));
  L1_HIP(hipMemsetAsync(Pbar, 0, sizeof(double) * n * n, s));

  // the recorded instance data: b, beta, c = A^T M b / beta
  const float* beta = p->tape_pen;
  const float* ibeta = p->tape_pen + N;
  L1_HIP(hipMemcpyAsync(p->pen, beta, sizeof(float) * N, hipMemcpyDeviceToDevice, s));
  L1_HIP(hipMemcpyAsync(p->ipen, ibeta, sizeof(float) * N, hipMemcpyDeviceToDevice, s));
  {
    GemmArgs g{};
    g.A32 = p->Cop;
    g.lda = p->m_pad;
    g.B = p->tape_b;
    g.ldb = p->m_pad;
    g.M = n_pad;
    g.K = p->m_pad;
    g.n_cols = N;
    g.prec = PREC_F32;
    g.m_true = n_pad;
    g.out = p->C;
    g.ldo = lds;
    g.col_scale = p->ipen;
    launch_gemm(s, EPI_STORE, g, ntc);
  }
  adj_init_kernel<<<blocks_for((long)st), 256, 0, s>>>(nd, m, p->split, n, lds, N, gx, ge, beta,
                                                       Wb, Vt);
  L1_HIP(hipGetLastError());

  // forward product of the recomputation (the launch shape of the recording solve)
  GemmArgs it{};
  it.A32 = p->P32;
  it.lda = n_pad;
  it.ldb = lds;
  it.M = n_pad;
  it.K = n_pad;
  it.n_cols = N;
  it.prec = PREC_F32;
  it.lds = lds;
  it.V = p->V;
  it.W = p->W;
  it.C = p->C;
  it.beta = p->pen;
  it.partial = p->partial;
  it.ldp = p->N_pad;
  it.n_l1 = p->n_l1;
  it.e0 = 1 << 30;
  it.ws = p->ws;
  // reverse product ubar = P vt
  GemmArgs rb{};
  rb.A32 = p->P32;
  rb.lda = n_pad;
  rb.B = Vt;
  rb.ldb = lds;
  rb.M = n_pad;
  rb.K = n_pad;
  rb.n_cols = N;
  rb.prec = PREC_F32;
  rb.m_true = n_pad;
  rb.out = Ub;
  rb.ldo = lds;

  for (int sg = nseg - 1; sg >= 0; --sg) {
    const int k0 = sg * every, k1 = std::min(K, k0 + every), len = k1 - k0;
    // restore the checkpoint of iteration k0 and recompute the segment
    L1_HIP(hipMemcpyAsync(p->W, p->tape[2 * sg], sizeof(float) * st, hipMemcpyDeviceToDevice, s));
    L1_HIP(hipMemcpyAsync(p->V, p->tape[2 * sg + 1], sizeof(float) * st, hipMemcpyDeviceToDevice,
                          s));
    {
      DalmInit di{};
      di.n = n;
      di.n_pad = n_pad;
      di.lds = lds;
      di.e0 = 1 << 30;
      di.V = p->V;
      di.W = p->W;
      di.beta = p->pen;
      di.U = p->Uf[k0 & 1];
      dalm_init_u(s, N, di);
    }
    for (int k = k0; k < k1; ++k) {
      L1_HIP(hipMemcpyAsync(seg_v + st * (k - k0), p->V, sizeof(float) * st,
                            hipMemcpyDeviceToDevice, s));
      L1_HIP(hipMemcpyAsync(seg_w + st * (k - k0), p->W, sizeof(float) * st,
                            hipMemcpyDeviceToDevice, s));
      if (k == k1 - 1) break;  // the state after the segment's last step is not needed
      const int cur = k & 1;
      it.B = p->Uf[cur];
      it.U = p->Uf[1 - cur];
      launch_product(s, EPI_DALM, it, ntc, ks);
    }
    // reverse steps k1-1 .. k0
    for (int k = k1 - 1; k >= k0; --k) {
      launch_gemm(s, EPI_STORE, rb, ntc);
      const size_t off = st * (k - k0);
      adj_step_kernel<<<blocks_for((long)n * N), 256, 0, s>>>(
          n, lds, N, seg_v + off, seg_w + off, beta, ibeta, Ub, Wb, Vt, seg_vt + off, seg_u + off,
          cbar);
      L1_HIP(hipGetLastError());
    }
    // Pbar += [vt_k0 .. vt_{k1-1}] [u_k0 .. u_{k1-1}]^T: the segment's sum
    // of len N outer products on the FP32 matrix cores (relative rounding
    // ~1e-7 sqrt(len N), well inside the gradient's 1e-3), accumulated over
    // the segments in FP64, where the assembly below cancels its terms
    const int cols = len * N, kp = (cols + 63) / 64 * 64;
    const dim3 tg((unsigned)(kp / 32), (unsigned)(n_pad / 32));
    transpose_pad_kernel<<<tg, 256, 0, s>>>(n, cols, seg_vt, lds, VtT, kp);
    transpose_pad_kernel<<<tg, 256, 0, s>>>(n, cols, seg_u, lds, UT, kp);
    L1_HIP(hipGetLastError());
    {
      GemmArgs pg{};
      pg.A32 = VtT;
      pg.lda = kp;
      pg.B = UT;
      pg.ldb = kp;
      pg.M = n_pad;
      pg.K = kp;
      pg.n_cols = n;
      pg.prec = PREC_F32;
      pg.m_true = n;
      pg.out = Pseg;
      pg.ldo = n_pad;
      launch_gemm(s, EPI_STORE, pg, (n + TILE - 1) / TILE);
    }
    add_f32_to_f64_kernel<<<blocks_for((long)n * n), 256, 0, s>>>(n, Pseg, n_pad, Pbar, n);
    L1_HIP(hipGetLastError());
  }

  // ---- FP64 assembly -------------------------------------------------------
  double* A64 = bf.get<double>((size_t)m * n);
  full_matrix64_kernel<<<blocks_for((long)m * n), 256, 0, s>>>(m, nd, n, p->A, A64);
  L1_HIP(hipGetLastError());
  double* G = bf.get<double>((size_t)m * m);
  if (!p->adj_M) {
    // M = (A A^T + shift I)^{-1} and Y = M A depend only on the dictionary:
    // formed once per plan
    double* Mk = nullptr;
    double* Yk = nullptr;
    // owned by the plan from here on (freed with it), valid once formed
    if (hipMalloc((void**)&Mk, sizeof(double) * (size_t)m * m) == hipSuccess) p->owned.push_back(Mk);
    else Mk = nullptr;
    if (Mk && hipMalloc((void**)&Yk, sizeof(double) * (size_t)m * n) == hipSuccess) p->owned.push_back(Yk);
    else Yk = nullptr;
    if (!Mk || !Yk) {
      (void)hipGetLastError();
      set_error("out of device memory in l1_alm_backward");
      throw Fail{L1_ENOMEM};
    }
    double* X = once.get<double>((size_t)m * m);
    double* dinv = once.get<double>((size_t)((m + 63) / 64) * 64 * 64);
    double* work = once.get<double>((size_t)128 * m);
    int* info = once.get<int>(1);
    gemm64(s, 'N', 'T', m, m, n, 1.0, A64, m, A64, m, 0.0, G, m);
    if (p->shift != 0.0) add_diag64(s, m, G, m, p->shift);
    potrf64(s, m, G, m, dinv, info, work);
    lower_inverse64(s, m, G, m, dinv, X, m, work);
    gemm64(s, 'T', 'N', m, m, m, 1.0, X, m, X, m, 0.0, Mk, m);   // M = L^{-T} L^{-1}
    gemm64(s, 'N', 'N', m, n, m, 1.0, Mk, m, A64, m, 0.0, Yk, m);  // Y = M A
    L1_HIP(hipStreamSynchronize(s));
    p->adj_M = Mk;
    p->adj_Y = Yk;
  }
  const double* M = p->adj_M;
  const double* Y = p->adj_Y;
  double* bt = bf.get<double>((size_t)m * N);
  scale_cols64_kernel<<<blocks_for((long)m * N), 256, 0, s>>>(m, N, p->tape_b, p->m_pad, ibeta,
                                                              bt, m);
  L1_HIP(hipGetLastError());
  double* Yc = bf.get<double>((size_t)m * N);
  gemm64(s, 'N', 'N', m, N, n, 1.0, Y, m, cbar, n, 0.0, Yc, m);  // M A cbar
  if (gb) {
    store_cols_kernel<<<blocks_for((long)m * N), 256, 0, s>>>(m, N, Yc, m, ibeta, gb, m);
    L1_HIP(hipGetLastError());
  }
  if (gA && nd > 0) {
    double* Ab = bf.get<double>((size_t)m * n);
    gemm64(s, 'N', 'N', m, n, n, 1.0, Y, m, Pbar, n, 0.0, Ab, m);
    gemm64(s, 'N', 'T', m, n, n, 1.0, Y, m, Pbar, n, 1.0, Ab, m);
    double* Mbt = bf.get<double>((size_t)m * N);
    gemm64(s, 'N', 'N', m, N, m, 1.0, M, m, bt, m, 0.0, Mbt, m);
    gemm64(s, 'N', 'T', m, n, N, 1.0, Mbt, m, cbar, n, 1.0, Ab, m);  // M bt cbar^T
    // Mbar = A Pbar A^T + A cbar bt^T
    double* T = bf.get<double>((size_t)m * n);
    double* Mb = bf.get<double>((size_t)m * m);
    double* Ac = bf.get<double>((size_t)m * N);
    gemm64(s, 'N', 'N', m, n, n, 1.0, A64, m, Pbar, n, 0.0, T, m);
    gemm64(s, 'N', 'T', m, m, n, 1.0, T, m, A64, m, 0.0, Mb, m);
    gemm64(s, 'N', 'N', m, N, n, 1.0, A64, m, cbar, n, 0.0, Ac, m);
    gemm64(s, 'N', 'T', m, m, N, 1.0, Ac, m, bt, m, 1.0, Mb, m);
    // Gbar = -M Mbar M;  Abar += (Gbar + Gbar^T) A
    double* W1 = bf.get<double>((size_t)m * m);
    gemm64(s, 'N', 'N', m, m, m, 1.0, M, m, Mb, m, 0.0, W1, m);
    gemm64(s, 'N', 'N', m, m, m, -1.0, W1, m, M, m, 0.0, G, m);
    gemm64(s, 'N', 'N', m, nd, m, 1.0, G, m, A64, m, 1.0, Ab, m);
    gemm64(s, 'T', 'N', m, nd, m, 1.0, G, m, A64, m, 1.0, Ab, m);
    add_block_kernel<<<blocks_for((long)m * nd), 256, 0, s>>>(m, nd, Ab, m, gA, m);
    L1_HIP(hipGetLastError());
  }
  L1_HIP(hipStreamSynchronize(s));
}

}  // namespace l1
