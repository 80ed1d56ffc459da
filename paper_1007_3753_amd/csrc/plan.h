// The plan object and the solver drivers.
#pragma once
#include "internal.h"

namespace l1 {

struct Plan {
  l1_alm_desc d{};
  int dev = 0;
  int m = 0, nd = 0, n = 0, split = 0;
  int m_pad = 0, nd_pad = 0, n_pad = 0, N_pad = 0;
  int e0 = 0, n_l1 = 0;
  int lds = 0, ntiles = 0;
  double shift = 0.0;   // lambda / beta in the DALM factor for QP_lambda
  double Lf = 0.0;      // PALM: ||A^T A||_2
  std::vector<void*> owned;
  // dictionary (FP32)
  float* A = nullptr;     // m x nd, ld m
  float* Acol = nullptr;  // nd_pad x m_pad, row i = column i of A
  float* Arow = nullptr;  // m_pad x nd_pad, row r = row r of A
  // DALM operators (rows K-contiguous, zero padded)
  float* P32 = nullptr;   // n_pad x n_pad
  uint16_t* Phi = nullptr;
  uint16_t* Plo = nullptr;
  float* Cop = nullptr;   // n_pad x m_pad
  float* Yop = nullptr;   // m_pad x n_pad (dense only)
  // structured iteration forms (st_ok: 0 none, 1 cross-and-bouquet, 2 dense)
  //  1: Bq = B row-major (rows K-contiguous, m_pad + TILE rows, zero padded),
  //     T holds q = K^{-1} (u_x - B^T u_e) per column (ldt = nd_pad); R1 =
  //     rows of the first launch
  //  2: Rop = (A A^T + shift I)^{-1} A (m_pad x n_pad) and Bq = A^T (n_pad x
  //     m_pad), both rows K-contiguous; T holds t = Rop u (ldt = m_pad)
  int st_ok = 0, R1 = 0, ldt = 0;
  float* Bq32 = nullptr;
  uint16_t* Bqhi = nullptr;
  uint16_t* Bqlo = nullptr;
  float* R32 = nullptr;
  uint16_t* Rhi = nullptr;
  uint16_t* Rlo = nullptr;
  float* Tf = nullptr;
  uint16_t* Th = nullptr;
  uint16_t* Tl = nullptr;
  // PALM operators
  float* M32 = nullptr;   // nd_pad x nd_pad
  uint16_t* Mhi = nullptr;
  uint16_t* Mlo = nullptr;
  // workspace, column-major with leading dimension lds, N_pad columns
  float* W = nullptr;
  float* V = nullptr;
  float* C = nullptr;      // c, then c_ref = (C0 - P w_ref) / beta after each refresh
  float* C0 = nullptr;     // A^T G^{-1} b (unscaled)
  float* Wref = nullptr;   // reference point of the DALM operand (see EPI_REFRESH)
  float* Z[2] = {nullptr, nullptr};
  float* Uf[2] = {nullptr, nullptr};       // ping-pong B-operand of the iteration (FP32)
  uint16_t* Uh[2] = {nullptr, nullptr};    // its BF16 hi / lo split (BF16 precisions)
  uint16_t* Ul[2] = {nullptr, nullptr};
  float* bb = nullptr;    // m_pad x N_pad copy of b
  float* aux = nullptr;   // 4 x (m_pad x N_pad) scratch
  float* pen = nullptr;   // beta (DALM) or xi (PALM) per column
  float* ipen = nullptr;  // its reciprocal
  float* zscale = nullptr;
  float* tscal = nullptr;
  float* wcap2 = nullptr; // per instance: squared L1_DIVERGED threshold on ||w||_2
  float* dscale2 = nullptr; // per instance: (beta0 / beta)^2 of the DALM stopping test
  float* partial = nullptr;
  float* ws = nullptr;    // split-K workspace: ws_tiles x TILE x lds floats
  int ws_tiles = 0, ks_target = 192, ks_max = 4;
  // split-K parts of the DALM iteration product by the number of active
  // 64-instance column tiles (index 1..8); 0 = the heuristic (dalm_ksplit)
  int ks_table[9] = {0};
  int* ints = nullptr;    // lists and counters
  long long* stat = nullptr;
  double* kkt_rbuf = nullptr;
  // the batched FP64 report's dictionary and workspaces (allocated by its
  // first call, held with the plan)
  double* kkt_A64 = nullptr;
  double* kkt_X = nullptr;
  double* kkt_U = nullptr;
  double* kkt_G = nullptr;
  int* h_total = nullptr; // pinned
  // the tail kernel's uncached exchange region (barrier, flags, u and
  // partial sums), owned by this plan and given back to the device's free
  // list when it is destroyed
  void* tail_mem = nullptr;
  size_t tail_bytes = 0;
  double last_stats[14] = {0};
  double plan_ms = 0.0;
  // tape of the last recorded fixed-count solve
  std::vector<void*> tape;
  int tape_N = 0, tape_K = 0, tape_every = 0;   // tape_N = 0: no complete tape
  float* tape_b = nullptr;    // b of the recorded solve (m_pad x N)
  // the backward's FP64 (A A^T + shift I)^{-1} (m x m) and its product with
  // the full matrix A (m x n): depend only on the dictionary, formed by the
  // first l1_alm_backward and kept (owned)
  double* adj_M = nullptr;
  double* adj_Y = nullptr;
  // the backward's workspaces (bytes, pointer), taken in the order the
  // backward asks for them and kept for the next call (freed with the plan)
  std::vector<std::pair<size_t, void*>> adj_ws;
  float* tape_pen = nullptr;  // its beta (N) and 1/beta (N)
};

struct SolveArgs {
  const float* b;
  int ldb;
  int N;
  const float* eps;
  const float* pen;   // per-instance penalties or null
  float tol;
  int max_iter;
  const float* w0;
  const float* y0;
  float* x;
  int ldx;
  float* e;
  int lde;
  float* y;
  int ldy;
  int* iters;
  int* status;
  hipStream_t s;
};

// Default DALM penalty as a multiple of beta0 = ||b||_1 / m, for the
// cross-and-bouquet form: 1/16 for batches of more than 64 instances, 1/8
// (FP32) or 1 (BF16) for smaller ones; 1 for dense dictionaries.  On
// face-shaped problems a smaller penalty reaches a given error in several
// times fewer iterations on the slowest instances (as many on the others;
// swept 1/32 to 1/4 on the 1200 x 700 and 4800 x 2100 batches: 1/16 within
// 2 % of the best on both, in every arithmetic); on Gaussian dictionaries
// beta0 is the faster one.  The smaller penalty enlarges the operand
// u = z - (w - w_ref)/beta until its reference is refreshed, which happens
// only while two or more column tiles are active: a batch that fits one
// tile stalls its stopping test at 1/16 in FP32 (measured at 4800 x 2100)
// and at 1/8 in split BF16.
inline float default_beta_scale(const Plan* p, int N) {
  if (p->d.structure != L1_CAB) return 1.0f;
  if (N <= TILE) return p->d.precision != L1_FP32 ? 1.0f : 0.125f;
  return 0.0625f;
}

// L1_DIVERGED threshold factor of the plan (desc.div_factor, default 1e6)
inline float div_factor(const Plan* p) {
  return p->d.div_factor > 0 ? (float)p->d.div_factor : 1e6f;
}

Plan* create_plan(const l1_alm_desc* d, const float* A_dev, hipStream_t s);
void destroy_plan(Plan* p);
void solve_dalm(Plan* p, const SolveArgs& a);
// K-range split of the DALM iteration product for `active` instances spread
// over `phases_used` precision phases (1 = no split)
int dalm_ksplit(const Plan* p, int active, int phases_used);
void solve_palm(Plan* p, const SolveArgs& a);
// DALM with one conjugate-gradient step for the y-step (csrc/cg1.hip)
void solve_dalm_cg1(Plan* p, const SolveArgs& a);
void backward_dalm(Plan* p, const float* gx, const float* ge, float* gb, float* gA,
                   hipStream_t s);

}  // namespace l1
