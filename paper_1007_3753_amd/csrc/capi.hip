// C ABI of libl1alm: plan construction, the solve drivers, the FP64
// certificate and error reporting.  See include/l1_alm.h for the contract.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>

#include "internal.h"
#include "plan.h"
#include "readout.h"
#include "tail.h"
#include "steps.h"

namespace l1 {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

template <class T>
static T* dalloc(size_t count, std::vector<void*>& owned) {
  void* p = nullptr;
  if (count == 0) count = 1;
  const hipError_t e = hipMalloc(&p, count * sizeof(T));
  if (e != hipSuccess) {
    set_error("hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed: " +
              hipGetErrorString(e));
    throw Fail{L1_ENOMEM};
  }
  owned.push_back(p);
  return reinterpret_cast<T*>(p);
}

// FP64 scratch that lives only during plan construction
struct Scratch {
  std::vector<void*> v;
  ~Scratch() {
    for (void* p : v) (void)hipFree(p);
  }
  double* d(size_t n) { return dalloc<double>(n, v); }
};

static void check_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) {
    set_error("no HIP device");
    throw Fail{L1_ENODEVICE};
  }
  hipDeviceProp_t prop;
  L1_HIP(hipGetDeviceProperties(&prop, dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    set_error(std::string("device is ") + prop.gcnArchName + ", libl1alm is built for gfx950");
    throw Fail{L1_ENODEVICE};
  }
}

// Spectral factor X = L^{-1} of S = L L^T (n x n, SPD), FP64, in `X` (ld n).
static void inverse_factor(hipStream_t s, int n, double* S, double* X, Scratch& sc, int* info) {
  double* dinv = sc.d((size_t)((n + 63) / 64) * 64 * 64);
  double* work = sc.d((size_t)64 * n + (size_t)n * 64);
  potrf64(s, n, S, n, dinv, info, work);
  int h_info = 0;
  L1_HIP(hipMemcpyAsync(&h_info, info, sizeof(int), hipMemcpyDeviceToHost, s));
  L1_HIP(hipStreamSynchronize(s));
  if (h_info != 0) {
    set_error("Gram matrix is not positive definite (Cholesky pivot " + std::to_string(h_info) +
              " <= 0); the rows of the dictionary are linearly dependent");
    throw Fail{L1_ENOTSPD};
  }
  lower_inverse64(s, n, S, n, dinv, X, n, work);
}

static void build_dalm(Plan* p, hipStream_t s, const double* A64, Scratch& sc, int* info) {
  const int m = p->m, nd = p->nd, n = p->n;
  double* P64 = sc.d((size_t)n * n);
  if (p->split) {
    if (nd <= m) {
      // Woodbury: K = I + B^T B (nd x nd), H = K^{-1} = X^T X, T1 = B X^T
      // P = [[I - X^T X, X^T T1^T], [T1 X, I - T1 T1^T]]
      double* K = sc.d((size_t)nd * nd);
      double* X = sc.d((size_t)nd * nd);
      double* T1 = sc.d((size_t)m * nd);
      gemm64(s, 'T', 'N', nd, nd, m, 1.0, A64, m, A64, m, 0.0, K, nd);
      add_diag64(s, nd, K, nd, 1.0);
      inverse_factor(s, nd, K, X, sc, info);
      gemm64(s, 'N', 'T', m, nd, nd, 1.0, A64, m, X, nd, 0.0, T1, m);
      gemm64(s, 'T', 'N', nd, nd, nd, -1.0, X, nd, X, nd, 0.0, P64, n);
      add_diag64(s, nd, P64, n, 1.0);
      gemm64(s, 'N', 'N', m, nd, nd, 1.0, T1, m, X, nd, 0.0, P64 + nd, n);
      gemm64(s, 'T', 'T', nd, m, nd, 1.0, X, nd, T1, m, 0.0, P64 + (size_t)nd * n, n);
      gemm64(s, 'N', 'T', m, m, nd, -1.0, T1, m, T1, m, 0.0, P64 + nd + (size_t)nd * n, n);
      add_diag64(s, m, P64 + nd + (size_t)nd * n, n, 1.0);
    } else {
      // G = B B^T + I (m x m), G^{-1} = X^T X, T2 = X B
      double* G = sc.d((size_t)m * m);
      double* X = sc.d((size_t)m * m);
      double* T2 = sc.d((size_t)m * nd);
      gemm64(s, 'N', 'T', m, m, nd, 1.0, A64, m, A64, m, 0.0, G, m);
      add_diag64(s, m, G, m, 1.0);
      inverse_factor(s, m, G, X, sc, info);
      gemm64(s, 'N', 'N', m, nd, m, 1.0, X, m, A64, m, 0.0, T2, m);
      gemm64(s, 'T', 'N', nd, nd, m, 1.0, T2, m, T2, m, 0.0, P64, n);
      gemm64(s, 'T', 'N', nd, m, m, 1.0, T2, m, X, m, 0.0, P64 + (size_t)nd * n, n);
      gemm64(s, 'T', 'N', m, nd, m, 1.0, X, m, T2, m, 0.0, P64 + nd, n);
      gemm64(s, 'T', 'N', m, m, m, 1.0, X, m, X, m, 0.0, P64 + nd + (size_t)nd * n, n);
    }
    // c = A^T G^{-1} b / beta is the block of P that multiplies the identity part
    to_rowmajor_f32(s, n, m, P64 + (size_t)nd * n, n, p->Cop, p->m_pad, nullptr, nullptr);
    // structured form: B row-major for the second product
    if (p->st_ok == 1) to_rowmajor_f32(s, m, nd, A64, m, p->Bq32, p->nd_pad, p->Bqhi, p->Bqlo);
  } else {
    // dense: G = A A^T + shift I = L L^T, X = L^{-1}, T2 = X A,
    // P = T2^T T2, c-operator A^T G^{-1} = T2^T X, y-operator (A A^T)^{-1} A
    double* G = sc.d((size_t)m * m);
    double* X = sc.d((size_t)m * m);
    double* T2 = sc.d((size_t)m * nd);
    double* C64 = sc.d((size_t)nd * m);
    gemm64(s, 'N', 'T', m, m, nd, 1.0, A64, m, A64, m, 0.0, G, m);
    if (p->shift != 0.0) add_diag64(s, m, G, m, p->shift);
    inverse_factor(s, m, G, X, sc, info);
    gemm64(s, 'N', 'N', m, nd, m, 1.0, X, m, A64, m, 0.0, T2, m);
    gemm64(s, 'T', 'N', nd, nd, m, 1.0, T2, m, T2, m, 0.0, P64, n);
    gemm64(s, 'T', 'N', nd, m, m, 1.0, T2, m, X, m, 0.0, C64, nd);
    to_rowmajor_f32(s, nd, m, C64, nd, p->Cop, p->m_pad, nullptr, nullptr);
    double* Y64 = sc.d((size_t)m * nd);
    if (p->shift == 0.0) {
      gemm64(s, 'T', 'N', m, nd, m, 1.0, X, m, T2, m, 0.0, Y64, m);
    } else {
      double* G0 = sc.d((size_t)m * m);
      double* X0 = sc.d((size_t)m * m);
      double* T0 = sc.d((size_t)m * nd);
      gemm64(s, 'N', 'T', m, m, nd, 1.0, A64, m, A64, m, 0.0, G0, m);
      inverse_factor(s, m, G0, X0, sc, info);
      gemm64(s, 'N', 'N', m, nd, m, 1.0, X0, m, A64, m, 0.0, T0, m);
      gemm64(s, 'T', 'N', m, nd, m, 1.0, X0, m, T0, m, 0.0, Y64, m);
    }
    to_rowmajor_f32(s, m, nd, Y64, m, p->Yop, p->n_pad, nullptr, nullptr);
    if (p->st_ok == 2) {
      // structured form: t = G^{-1} A u (G with the shift), then v = A^T t + c
      double* R64 = sc.d((size_t)m * nd);
      gemm64(s, 'T', 'N', m, nd, m, 1.0, X, m, T2, m, 0.0, R64, m);
      to_rowmajor_f32(s, m, nd, R64, m, p->R32, p->n_pad, p->Rhi, p->Rlo);
      transpose_f64_to_f32(s, nd, m, A64, m, p->Bq32, p->m_pad, p->Bqhi, p->Bqlo);
    }
  }
  to_rowmajor_f32(s, n, n, P64, n, p->P32, p->n_pad, p->Phi, p->Plo);
}

static void build_palm(Plan* p, hipStream_t s, const double* A64, Scratch& sc) {
  const int m = p->m, nd = p->nd;
  double* M64 = sc.d((size_t)nd * nd);
  gemm64(s, 'T', 'N', nd, nd, m, 1.0, A64, m, A64, m, 0.0, M64, nd);
  to_rowmajor_f32(s, nd, nd, M64, nd, p->M32, p->nd_pad, p->Mhi, p->Mlo);
  double* work = sc.d((size_t)2 * nd + 8);
  p->Lf = power_lambda_max64(s, nd, M64, nd, work, 20000, 1e-13);
}

Plan* create_plan(const l1_alm_desc* d, const float* A_dev, hipStream_t s) {
  L1_REQUIRE(d != nullptr && A_dev != nullptr, "desc and A must be non-NULL");
  L1_REQUIRE(d->m >= 1 && d->n_dict >= 0 && d->lda >= d->m, "bad sizes: need m >= 1, n_dict >= 0, lda >= m");
  L1_REQUIRE(d->max_batch >= 1, "max_batch must be >= 1");
  L1_REQUIRE(d->problem >= 0 && d->problem <= 2, "unknown problem");
  L1_REQUIRE(d->structure == L1_DENSE || d->structure == L1_CAB, "unknown structure");
  L1_REQUIRE(d->method == L1_DALM || d->method == L1_PALM || d->method == L1_DALM_CG1, "unknown method");
  L1_REQUIRE(d->method != L1_DALM_CG1 || (d->problem == L1_P1 && d->precision == L1_FP32),
             "L1_DALM_CG1 runs (P1) with L1_FP32 products");
  L1_REQUIRE(d->precision >= 0 && d->precision <= 2, "unknown precision");
  L1_REQUIRE(d->iteration_form >= 0 && d->iteration_form <= 2, "unknown iteration form");
  L1_REQUIRE(!(d->structure == L1_CAB && d->problem != L1_P1),
             "QP_lambda and P_{1,2} are defined on a dense dictionary (structure L1_DENSE)");
  L1_REQUIRE(d->problem != L1_QPLAMBDA || d->lambda > 0, "QP_lambda needs lambda > 0");
  L1_REQUIRE(!(d->method == L1_DALM && d->problem == L1_QPLAMBDA && !(d->beta > 0)),
             "DALM on QP_lambda needs beta > 0 (it enters the factor A A^T + lambda/beta I)");
  L1_REQUIRE(d->structure == L1_CAB || d->n_dict >= 1, "a dense dictionary needs n_dict >= 1");
  L1_REQUIRE((long)d->m * d->n_dict < (1L << 31) && d->m + d->n_dict < (1 << 20), "dictionary too large");
  check_device();

  std::unique_ptr<Plan> p(new Plan());
  p->d = *d;
  L1_HIP(hipGetDevice(&p->dev));
  const int m = d->m, nd = d->n_dict;
  p->m = m;
  p->nd = nd;
  p->split = (d->structure == L1_CAB || d->problem == L1_P12) ? 1 : 0;
  p->n = p->split ? nd + m : nd;
  p->m_pad = round_up(m, KPAD);
  p->nd_pad = round_up(nd > 0 ? nd : 1, KPAD);
  p->n_pad = round_up(p->n, KPAD);
  p->N_pad = round_up(d->max_batch, TILE);
  p->e0 = (d->problem == L1_P12) ? nd : (1 << 30);
  p->n_l1 = (d->problem == L1_P12) ? nd : p->n;
  p->shift = (d->problem == L1_QPLAMBDA && d->method == L1_DALM) ? d->lambda / d->beta : 0.0;
  const bool low = d->precision != L1_FP32;
  auto& o = p->owned;

  // dictionary copies (FP32)
  p->A = dalloc<float>((size_t)m * (nd > 0 ? nd : 1), o);
  if (nd > 0)
    L1_HIP(hipMemcpy2DAsync(p->A, sizeof(float) * m, A_dev, sizeof(float) * d->lda,
                            sizeof(float) * m, nd, hipMemcpyDeviceToDevice, s));
  p->Acol = dalloc<float>((size_t)p->nd_pad * p->m_pad, o);
  p->Arow = dalloc<float>((size_t)p->m_pad * p->nd_pad, o);
  L1_HIP(hipMemsetAsync(p->Acol, 0, sizeof(float) * p->nd_pad * p->m_pad, s));
  L1_HIP(hipMemsetAsync(p->Arow, 0, sizeof(float) * p->m_pad * p->nd_pad, s));
  // Acol[i*m_pad + k] = A[k + i*m]: row i is column i of A
  if (nd > 0)
    L1_HIP(hipMemcpy2DAsync(p->Acol, sizeof(float) * p->m_pad, p->A, sizeof(float) * m,
                            sizeof(float) * m, nd, hipMemcpyDeviceToDevice, s));

  Scratch sc;
  double* A64 = sc.d((size_t)m * (nd > 0 ? nd : 1));
  f32_to_f64(s, m, nd, p->A, m, A64, m);
  // Arow[r*nd_pad + k] = A[r + k*m]
  to_rowmajor_f32(s, m, nd, A64, m, p->Arow, p->nd_pad, nullptr, nullptr);
  int* info = reinterpret_cast<int*>(sc.d(1));

  if (d->method == L1_DALM) {
    const size_t nn = (size_t)p->n_pad * p->n_pad;
    p->P32 = dalloc<float>(nn, o);
    L1_HIP(hipMemsetAsync(p->P32, 0, sizeof(float) * nn, s));
    if (low) {
      p->Phi = dalloc<uint16_t>(nn, o);
      p->Plo = dalloc<uint16_t>(nn, o);
      L1_HIP(hipMemsetAsync(p->Phi, 0, sizeof(uint16_t) * nn, s));
      L1_HIP(hipMemsetAsync(p->Plo, 0, sizeof(uint16_t) * nn, s));
    }
    p->Cop = dalloc<float>((size_t)p->n_pad * p->m_pad, o);
    L1_HIP(hipMemsetAsync(p->Cop, 0, sizeof(float) * p->n_pad * p->m_pad, s));
    if (!p->split) {
      p->Yop = dalloc<float>((size_t)p->m_pad * p->n_pad, o);
      L1_HIP(hipMemsetAsync(p->Yop, 0, sizeof(float) * p->m_pad * p->n_pad, s));
    }
    // structured iteration forms (include/l1_alm.h): cross-and-bouquet (P1)
    // with n_dict < m, or a dense dictionary with m < n_dict, when its two
    // products cost at most 0.8 of the dense operator's
    const double f_dense = 2.0 * p->n_pad * (double)p->n_pad;
    const int R1 = round_up(nd > 0 ? nd : 1, TILE);
    size_t nt_rows = 0;
    if (d->iteration_form != 1 && p->split && d->problem == L1_P1 && nd >= 1 && nd < m &&
        2.0 * R1 * p->n_pad + 2.0 * (p->n_pad - R1) * (double)p->nd_pad <= 0.8 * f_dense) {
      // B with TILE spare zero rows: the second launch starts at state row R1,
      // i.e. at B row R1 - n_dict
      p->st_ok = 1;
      p->R1 = R1;
      p->ldt = p->nd_pad;
      nt_rows = p->nd_pad;
      const size_t nb = (size_t)(p->m_pad + TILE) * p->nd_pad;
      p->Bq32 = dalloc<float>(nb, o);
      L1_HIP(hipMemsetAsync(p->Bq32, 0, sizeof(float) * nb, s));
      if (low) {
        p->Bqhi = dalloc<uint16_t>(nb, o);
        p->Bqlo = dalloc<uint16_t>(nb, o);
        L1_HIP(hipMemsetAsync(p->Bqhi, 0, sizeof(uint16_t) * nb, s));
        L1_HIP(hipMemsetAsync(p->Bqlo, 0, sizeof(uint16_t) * nb, s));
      }
    } else if (d->iteration_form != 1 && !p->split && nd >= 1 && m < nd &&
               4.0 * p->m_pad * (double)p->n_pad <= 0.8 * f_dense) {
      p->st_ok = 2;
      p->ldt = p->m_pad;
      nt_rows = p->m_pad;
      const size_t nb = (size_t)p->n_pad * p->m_pad;
      p->Bq32 = dalloc<float>(nb, o);
      p->R32 = dalloc<float>(nb, o);
      L1_HIP(hipMemsetAsync(p->Bq32, 0, sizeof(float) * nb, s));
      L1_HIP(hipMemsetAsync(p->R32, 0, sizeof(float) * nb, s));
      if (low) {
        for (uint16_t** q : {&p->Bqhi, &p->Bqlo, &p->Rhi, &p->Rlo}) {
          *q = dalloc<uint16_t>(nb, o);
          L1_HIP(hipMemsetAsync(*q, 0, sizeof(uint16_t) * nb, s));
        }
      }
    }
    if (p->st_ok) {
      const size_t nt = nt_rows * round_up(d->max_batch, TILE);
      p->Tf = dalloc<float>(nt, o);
      L1_HIP(hipMemsetAsync(p->Tf, 0, sizeof(float) * nt, s));
      if (low) {
        p->Th = dalloc<uint16_t>(nt, o);
        p->Tl = dalloc<uint16_t>(nt, o);
        L1_HIP(hipMemsetAsync(p->Th, 0, sizeof(uint16_t) * nt, s));
        L1_HIP(hipMemsetAsync(p->Tl, 0, sizeof(uint16_t) * nt, s));
      }
    }
    build_dalm(p.get(), s, A64, sc, info);
  } else if (d->method == L1_PALM) {
    const size_t nn = (size_t)p->nd_pad * p->nd_pad;
    p->M32 = dalloc<float>(nn, o);
    L1_HIP(hipMemsetAsync(p->M32, 0, sizeof(float) * nn, s));
    if (low) {
      p->Mhi = dalloc<uint16_t>(nn, o);
      p->Mlo = dalloc<uint16_t>(nn, o);
      L1_HIP(hipMemsetAsync(p->Mhi, 0, sizeof(uint16_t) * nn, s));
      L1_HIP(hipMemsetAsync(p->Mlo, 0, sizeof(uint16_t) * nn, s));
    }
    if (nd > 0) build_palm(p.get(), s, A64, sc);
  }

  // per-solve workspace
  const size_t Np = p->N_pad;
  const int rows = (d->method != L1_PALM) ? p->n_pad : std::max(p->nd_pad, p->m_pad);
  p->lds = rows;
  const size_t st = (size_t)rows * Np;
  p->W = dalloc<float>(st, o);
  p->V = dalloc<float>(st, o);
  p->C = dalloc<float>(st, o);
  p->C0 = dalloc<float>(st, o);
  p->Wref = dalloc<float>(st, o);
  p->Z[0] = dalloc<float>(st, o);
  p->Z[1] = dalloc<float>(st, o);
  for (int b = 0; b < 2; ++b) {
    p->Uf[b] = dalloc<float>(st, o);
    L1_HIP(hipMemsetAsync(p->Uf[b], 0, sizeof(float) * st, s));
    if (low) {
      p->Uh[b] = dalloc<uint16_t>(st, o);
      p->Ul[b] = dalloc<uint16_t>(st, o);
      L1_HIP(hipMemsetAsync(p->Uh[b], 0, sizeof(uint16_t) * st, s));
      L1_HIP(hipMemsetAsync(p->Ul[b], 0, sizeof(uint16_t) * st, s));
    }
  }
  p->bb = dalloc<float>((size_t)p->m_pad * Np, o);
  p->aux = dalloc<float>((size_t)p->m_pad * Np * 4, o);
  p->pen = dalloc<float>(Np, o);
  p->ipen = dalloc<float>(Np, o);
  p->zscale = dalloc<float>(Np, o);
  p->tscal = dalloc<float>(Np * 4, o);
  p->wcap2 = dalloc<float>(Np, o);
  p->dscale2 = dalloc<float>(2 * Np, o);
  const int ntiles = rows / TILE;
  p->ntiles = ntiles;
  p->partial = dalloc<float>((size_t)2 * ntiles * NPART * Np, o);  // two buffers
  // split-K workspace and policy (L1ALM_KSPLIT_TARGET: workgroups aimed for;
  // L1ALM_KSPLIT_MAX: largest split)
  p->ws_tiles = 48;
  p->ws = dalloc<float>((size_t)p->ws_tiles * TILE * rows, o);
  if (const char* e = std::getenv("L1ALM_KSPLIT_TARGET")) p->ks_target = std::max(1, std::atoi(e));
  if (const char* e = std::getenv("L1ALM_KSPLIT_MAX")) p->ks_max = std::max(1, std::min(8, std::atoi(e)));
  p->ints = dalloc<int>(Np * 8 + 512, o);
  p->stat = dalloc<long long>(8, o);
  p->kkt_rbuf = dalloc<double>((size_t)m * Np, o);
  L1_HIP(hipHostMalloc((void**)&p->h_total, sizeof(int) * 8, 0));
  L1_HIP(hipStreamSynchronize(s));
  return p.release();
}

void destroy_plan(Plan* p) {
  if (!p) return;
  int cur = -1;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(p->dev);
  (void)hipDeviceSynchronize();
  for (void* q : p->owned) (void)hipFree(q);
  for (auto& w : p->adj_ws)
    if (w.second) (void)hipFree(w.second);
  for (void* q : p->tape) (void)hipFree(q);
  if (p->h_total) (void)hipHostFree(p->h_total);
  tail_region_put(p->dev, p->tail_mem, p->tail_bytes);
  if (cur >= 0) (void)hipSetDevice(cur);
  delete p;
}

}  // namespace l1

using namespace l1;

extern "C" {

const char* l1_alm_last_error(void) { return g_err.c_str(); }

int l1_alm_plan(const l1_alm_desc* desc, const float* A_dev, void* stream, l1_alm_plan_t* out) {
  try {
    L1_REQUIRE(out != nullptr, "out must be non-NULL");
    *out = nullptr;
    const auto t0 = std::chrono::steady_clock::now();
    Plan* p = create_plan(desc, A_dev, reinterpret_cast<hipStream_t>(stream));
    p->plan_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = reinterpret_cast<l1_alm_plan_t>(p);
    return L1_OK;
  } catch (const Fail& f) {
    return f.code;
  } catch (const std::exception& e) {
    set_error(e.what());
    return L1_EHIP;
  }
}

int l1_alm_destroy(l1_alm_plan_t plan) {
  destroy_plan(reinterpret_cast<Plan*>(plan));
  return L1_OK;
}

int l1_alm_solve(l1_alm_plan_t plan, const float* b_dev, int ldb, int N, const float* eps_dev,
                 const float* pen_dev, float tol, int max_iter, const float* w0_dev,
                 const float* y0_dev, float* x_dev, int ldx, float* e_dev, int lde, float* y_dev,
                 int ldy, int* iters_dev, int* status_dev, void* stream) {
  try {
    Plan* p = reinterpret_cast<Plan*>(plan);
    L1_REQUIRE(p != nullptr, "plan is NULL");
    SolveArgs a{b_dev, ldb, N, eps_dev, pen_dev, tol, max_iter, w0_dev, y0_dev, x_dev, ldx, e_dev,
                lde, y_dev, ldy, iters_dev, status_dev, reinterpret_cast<hipStream_t>(stream)};
    if (p->d.method == L1_DALM) solve_dalm(p, a);
    else if (p->d.method == L1_PALM) solve_palm(p, a);
    else solve_dalm_cg1(p, a);
    return L1_OK;
  } catch (const Fail& f) {
    return f.code;
  } catch (const std::exception& e) {
    set_error(e.what());
    return L1_EHIP;
  }
}

int l1_alm_kkt(l1_alm_plan_t plan, const float* b_dev, int ldb, int N, const float* eps_dev,
               const float* x_dev, int ldx, const float* e_dev, int lde, const float* y_dev,
               int ldy, double* report_dev, void* stream) {
  try {
    Plan* p = reinterpret_cast<Plan*>(plan);
    L1_REQUIRE(p != nullptr, "plan is NULL");
    L1_REQUIRE(N >= 0 && N <= p->N_pad, "N out of range (max_batch)");
    if (N == 0) return L1_OK;
    L1_REQUIRE(b_dev && x_dev && report_dev, "b, x and report must be non-NULL");
    L1_REQUIRE(ldb >= p->m && ldx >= std::max(p->nd, 1), "bad leading dimension");
    const int prob = p->d.problem;
    L1_REQUIRE(prob == L1_QPLAMBDA || y_dev != nullptr, "y is needed for P1 and P_{1,2}");
    L1_REQUIRE(prob != L1_P12 || eps_dev != nullptr, "P_{1,2} needs eps");
    L1_REQUIRE(p->d.structure != L1_CAB || e_dev != nullptr, "CAB needs e");
    if (y_dev) L1_REQUIRE(ldy >= p->m, "bad ldy");
    if (e_dev) L1_REQUIRE(lde >= p->m, "bad lde");
    const int split = (p->d.structure == L1_CAB) ? 1 : 0;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (!p->kkt_A64) {
      const size_t Np = (size_t)p->N_pad;
      double* A64 = dalloc<double>((size_t)p->m * std::max(p->nd, 1), p->owned);
      p->kkt_X = dalloc<double>((size_t)std::max(p->nd, 1) * Np, p->owned);
      p->kkt_U = dalloc<double>((size_t)p->m * Np, p->owned);
      p->kkt_G = dalloc<double>((size_t)std::max(p->nd, 1) * Np, p->owned);
      to_f64(s, (long)p->m * p->nd, p->A, A64);
      p->kkt_A64 = A64;
    }
    kkt64_batched(s, prob, p->m, p->nd, split, p->kkt_A64, b_dev, ldb, x_dev, ldx, e_dev, lde,
                  y_dev, ldy, eps_dev, p->d.lambda, N, p->kkt_rbuf, p->kkt_X, p->kkt_U, p->kkt_G,
                  report_dev);
    return L1_OK;
  } catch (const Fail& f) {
    return f.code;
  } catch (const std::exception& e) {
    set_error(e.what());
    return L1_EHIP;
  }
}

int l1_alm_classify(const float* x_dev, int ldx, int n_dict, int N, const int* class_ptr_dev,
                    int C, float* mass_dev, int* label_dev, float* score_dev, void* stream) {
  try {
    L1_REQUIRE(N >= 0 && n_dict >= 1 && ldx >= n_dict, "bad n_dict, ldx or N");
    L1_REQUIRE(C >= 2 && C <= L1_CLASSIFY_MAX_SUBJECTS, "C must be in [2, 4096]");
    if (N == 0) return L1_OK;
    L1_REQUIRE(x_dev && class_ptr_dev && label_dev && score_dev,
               "x, class_ptr, label and score must be non-NULL");
    classify(reinterpret_cast<hipStream_t>(stream), x_dev, ldx, n_dict, N, class_ptr_dev, C,
             mass_dev, label_dev, score_dev);
    return L1_OK;
  } catch (const Fail& f) {
    return f.code;
  } catch (const std::exception& e) {
    set_error(e.what());
    return L1_EHIP;
  }
}

int l1_alm_class_residuals(const float* A_dev, int m, int n_dict, int lda, const float* x_dev, int ldx,
                           const float* e_dev, int lde, const float* b_dev, int ldb, int N,
                           const int* class_ptr_dev, int C, float* res_dev, int* label_dev, void* stream) {
  try {
    L1_REQUIRE(N >= 0 && m >= 1 && n_dict >= 1, "bad m, n_dict or N");
    L1_REQUIRE(lda >= m && ldx >= n_dict && ldb >= m && (!e_dev || lde >= m), "bad leading dimension");
    L1_REQUIRE(C >= 2 && C <= L1_CLASSIFY_MAX_SUBJECTS, "C must be in [2, 4096]");
    if (N == 0) return L1_OK;
    L1_REQUIRE(A_dev && x_dev && b_dev && class_ptr_dev && label_dev,
               "A, x, b, class_ptr and label must be non-NULL");
    class_residuals(reinterpret_cast<hipStream_t>(stream), A_dev, m, n_dict, lda, x_dev, ldx, e_dev, lde, b_dev,
                    ldb, N, class_ptr_dev, C, res_dev, label_dev);
    return L1_OK;
  } catch (const Fail& f) {
    return f.code;
  } catch (const std::exception& e) {
    set_error(e.what());
    return L1_EHIP;
  }
}

int l1_alm_align(const float* B_dev, int m, int k, int N, const float* b_dev, int ldb, float tol,
                 int max_iter, float* w_dev, float* e_dev, int lde, int* iters_dev, int* status_dev,
                 void* stream) {
  static_assert(L1_ALIGN_MAX_K == ALIGN_KMAX && L1_ALIGN_MAX_M == 256 * ALIGN_R, "alignment limits");
  try {
    L1_REQUIRE(N >= 0, "N must be >= 0");
    L1_REQUIRE(k >= 1 && k <= L1_ALIGN_MAX_K, "k must be in [1, 16]");
    L1_REQUIRE(m >= 1 && m <= L1_ALIGN_MAX_M, "m must be in [1, 2048]");
    L1_REQUIRE(ldb >= m && lde >= m, "ldb and lde must be >= m");
    L1_REQUIRE(max_iter != 0, "max_iter must be non-zero");
    L1_REQUIRE(max_iter < 0 || (std::isfinite(tol) && tol > 0.0f), "tol must be positive and finite");
    if (N == 0) return L1_OK;
    L1_REQUIRE(B_dev && b_dev && w_dev && e_dev && iters_dev && status_dev, "NULL buffer");
    align_solve(reinterpret_cast<hipStream_t>(stream), B_dev, m, k, N, b_dev, ldb, tol, max_iter, w_dev,
                e_dev, lde, iters_dev, status_dev);
    return L1_OK;
  } catch (const Fail& f) {
    return f.code;
  } catch (const std::exception& e) {
    set_error(e.what());
    return L1_EHIP;
  }
}

int l1_alm_set_ksplit(l1_alm_plan_t plan, const int* ks_by_tiles, int n) {
  try {
    Plan* p = reinterpret_cast<Plan*>(plan);
    L1_REQUIRE(p != nullptr, "plan is NULL");
    L1_REQUIRE(n >= 0 && n <= L1_KSPLIT_TILES && (n == 0 || ks_by_tiles != nullptr), "bad table");
    for (int i = 0; i < n; ++i)
      L1_REQUIRE(ks_by_tiles[i] >= 0 && ks_by_tiles[i] <= L1_KSPLIT_MAX, "split-K parts must be in [0, 4]");
    for (int t = 1; t <= L1_KSPLIT_TILES; ++t) p->ks_table[t] = t <= n ? ks_by_tiles[t - 1] : 0;
    return L1_OK;
  } catch (const Fail& f) {
    return f.code;
  } catch (const std::exception& e) {
    set_error(e.what());
    return L1_EHIP;
  }
}

int l1_alm_tune_ksplit(l1_alm_plan_t plan, int iters, int* ks_out, int n, void* stream) {
  float* b = nullptr;
  float* x = nullptr;
  int* it = nullptr;
  int* st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  // the tuner's solves must neither replace the plan's recorded tape nor
  // leave a trial split in the table when they fail
  Plan* pp = reinterpret_cast<Plan*>(plan);
  int saved_tape = 0, saved_ks[9] = {0};
  bool saved = false;
  auto release = [&]() {
    if (saved) {
      pp->d.record_tape = saved_tape;
      std::memcpy(pp->ks_table, saved_ks, sizeof(saved_ks));
    }
    if (b) (void)hipFree(b);
    if (x) (void)hipFree(x);
    if (it) (void)hipFree(it);
    if (st) (void)hipFree(st);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  try {
    Plan* p = reinterpret_cast<Plan*>(plan);
    L1_REQUIRE(p != nullptr, "plan is NULL");
    L1_REQUIRE(p->d.method == L1_DALM, "the split-K table belongs to the DALM iteration");
    L1_REQUIRE(iters >= 16 && iters <= 4096, "iters must be in [16, 4096]");
    L1_REQUIRE(n >= 0 && n <= L1_KSPLIT_TILES && (n == 0 || ks_out != nullptr), "bad table");
    L1_REQUIRE(p->d.problem != L1_P12, "tuning runs (P1) and (QP_lambda) plans");
    saved_tape = p->d.record_tape;
    std::memcpy(saved_ks, p->ks_table, sizeof(saved_ks));
    saved = true;
    p->d.record_tape = 0;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int m = p->m, nd = std::max(p->nd, 1);
    const int tmax = std::min(L1_KSPLIT_TILES, p->d.max_batch / TILE);
    const int Nmax = std::max(tmax, 1) * TILE;
    // synthetic right-hand sides: U[0, 1) entries (the timing of a fixed
    // count of iterations does not depend on the values)
    std::vector<float> hb((size_t)m * Nmax);
    unsigned long long r = 0x9E3779B97F4A7C15ull;
    for (auto& v : hb) {
      r ^= r << 13;
      r ^= r >> 7;
      r ^= r << 17;
      v = (float)((r >> 40) & 0xFFFFFF) / 16777216.0f;
    }
    L1_HIP(hipMalloc((void**)&b, sizeof(float) * hb.size()));
    L1_HIP(hipMalloc((void**)&x, sizeof(float) * (size_t)nd * Nmax));
    L1_HIP(hipMalloc((void**)&it, sizeof(int) * Nmax));
    L1_HIP(hipMalloc((void**)&st, sizeof(int) * Nmax));
    L1_HIP(hipMemcpyAsync(b, hb.data(), sizeof(float) * hb.size(), hipMemcpyHostToDevice, s));
    L1_HIP(hipEventCreate(&e0));
    L1_HIP(hipEventCreate(&e1));
    // one active column tile stays with the heuristic when the tail kernel
    // can take over there (it runs the parts the heuristic gives it); when
    // its workgroups could not hold the operator rows it never runs, and the
    // one-tile shape is tuned too
    const int phases_used = p->d.precision == L1_BF16_REFINE ? 2 : 1;
    const bool tail_possible = tail_fits(p->n_pad, p->ntiles, std::min(dalm_ksplit(p, 1, phases_used), 8));
    for (int t = tail_possible ? 2 : 1; t <= tmax; ++t) {
      const int N = t * TILE;
      SolveArgs a{b, m, N, nullptr, nullptr, 0.0f, -iters, nullptr, nullptr, x, nd, nullptr, 0,
                  nullptr, 0, it, st, s};
      float best = 0.0f;
      int best_ks = 0;
      for (int ks = 1; ks <= L1_KSPLIT_MAX; ++ks) {
        p->ks_table[t] = ks;
        solve_dalm(p, a);   // warm-up (graphs, code objects)
        float ms[3];
        for (int rep = 0; rep < 3; ++rep) {
          L1_HIP(hipEventRecord(e0, s));
          solve_dalm(p, a);
          L1_HIP(hipEventRecord(e1, s));
          L1_HIP(hipEventSynchronize(e1));
          L1_HIP(hipEventElapsedTime(&ms[rep], e0, e1));
        }
        std::sort(ms, ms + 3);
        if (best_ks == 0 || ms[1] < best) {
          best = ms[1];
          best_ks = ks;
        }
      }
      p->ks_table[t] = best_ks;
    }
    for (int t = 1; t <= n; ++t) ks_out[t - 1] = p->ks_table[t];
    // keep the tuned table; restore only the tape flag
    std::memcpy(saved_ks, p->ks_table, sizeof(saved_ks));
    release();
    return L1_OK;
  } catch (const Fail& f) {
    release();
    return f.code;
  } catch (const std::exception& e) {
    release();
    set_error(e.what());
    return L1_EHIP;
  }
}

int l1_alm_last_stats(l1_alm_plan_t plan, double* out, int n) {
  try {
    Plan* p = reinterpret_cast<Plan*>(plan);
    L1_REQUIRE(p != nullptr && out != nullptr, "plan and out must be non-NULL");
    p->last_stats[10] = p->plan_ms;
    for (int i = 0; i < n && i < 14; ++i) out[i] = p->last_stats[i];
    return L1_OK;
  } catch (const Fail& f) {
    return f.code;
  }
}

int l1_alm_backward(l1_alm_plan_t plan, const float* gx_dev, const float* ge_dev, float* gb_dev,
                    float* gA_dev, void* stream) {
  try {
    Plan* p = reinterpret_cast<Plan*>(plan);
    L1_REQUIRE(p != nullptr, "plan is NULL");
    backward_dalm(p, gx_dev, ge_dev, gb_dev, gA_dev, reinterpret_cast<hipStream_t>(stream));
    return L1_OK;
  } catch (const Fail& f) {
    return f.code;
  } catch (const std::exception& e) {
    set_error(e.what());
    return L1_EHIP;
  }
}

}  // extern "C"
