// Internal declarations shared by the translation units of libl1alm.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/l1_alm.h"

namespace l1 {

constexpr int TILE = 64;          // output tile edge of the iteration GEMMs
constexpr int KPAD = 64;          // reduction dimension padding
// per-column partial sums written by the DALM epilogue: ||dw||^2, ||w||^2,
// ||w||_1, sum |w|(1 - sign(w) v) (the l1/duality gap), ||s_ball||^2
constexpr int NPART = 5;

inline int round_up(int x, int r) { return (x + r - 1) / r * r; }

// ---- error plumbing ------------------------------------------------------
void set_error(const std::string& msg);
struct Fail {
  int code;
};
#define L1_HIP(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess) {                                                       \
      ::l1::set_error(std::string(#call) + ": " + hipGetErrorString(e_));         \
      throw ::l1::Fail{L1_EHIP};                                                  \
    }                                                                             \
  } while (0)
#define L1_REQUIRE(cond, msg)                                                     \
  do {                                                                            \
    if (!(cond)) {                                                                \
      ::l1::set_error(msg);                                                       \
      throw ::l1::Fail{L1_EINVAL};                                                \
    }                                                                             \
  } while (0)

// ---- FP64 dense kernels (plan set-up and certificates) -------------------
// C = alpha op(A) op(B) + beta C; column-major; ta/tb 'N' or 'T'.
void gemm64(hipStream_t s, char ta, char tb, int M, int N, int K, double alpha,
            const double* A, int lda, const double* B, int ldb, double beta,
            double* C, int ldc);
void add_diag64(hipStream_t s, int n, double* A, int lda, double c);
void f32_to_f64(hipStream_t s, int rows, int cols, const float* src, int lds,
                double* dst, int ldd);
// In-place lower Cholesky of the SPD matrix A (n x n); the strictly upper part
// is zeroed.  Diagonal-block inverses go to diaginv (64*64 per block).
// *info_dev receives 0, or 1 + the index of the first non-positive pivot.
void potrf64(hipStream_t s, int n, double* A, int lda, double* diaginv, int* info_dev,
             double* work);
// X = L^{-1} for the factor produced by potrf64.
void lower_inverse64(hipStream_t s, int n, const double* L, int lda,
                     const double* diaginv, double* X, int ldx, double* work);
// Largest eigenvalue of the symmetric PSD matrix M (n x n) by power iteration.
double power_lambda_max64(hipStream_t s, int n, const double* M, int ldm, double* work,
                          int max_iter, double rtol);

// Operator layout helpers: dst[i*ldd + k] = src[i + k*lds]  (i < rows, k < cols)
// written as FP32, and optionally as a BF16 hi/lo split.
void to_rowmajor_f32(hipStream_t s, int rows, int cols, const double* src, int lds,
                     float* dst, int ldd, uint16_t* hi, uint16_t* lo);
// dst[i*ldd + k] = src[k + i*lds]: the transpose in FP32, and optionally as
// a BF16 hi/lo split.
void transpose_f64_to_f32(hipStream_t s, int rows, int cols, const double* src, int lds,
                          float* dst, int ldd, uint16_t* hi = nullptr, uint16_t* lo = nullptr);

// FP64 optimality report, one workgroup per instance.
void kkt64(hipStream_t s, int problem, int m, int nd, int split, const float* A, int lda,
           const float* b, int ldb, const float* x, int ldx, const float* e, int lde,
           const float* y, int ldy, const float* eps, double lambda, int N, double* rbuf,
           double* report);
// The same report with its two products over the whole batch on the FP64
// matrix cores: R = b - A x (- e) and G = A^T u (u = y, or R / lambda for
// QP_lambda).  A64 is the dictionary (m x nd, ld m) in FP64; R (m x N),
// X (nd x N), U (m x N) and G (nd x N) are workspaces.
void kkt64_batched(hipStream_t s, int problem, int m, int nd, int split, const double* A64,
                   const float* b, int ldb, const float* x, int ldx, const float* e, int lde,
                   const float* y, int ldy, const float* eps, double lambda, int N, double* R,
                   double* X, double* U, double* G, double* report);
void to_f64(hipStream_t s, long n, const float* src, double* dst);

// ---- iteration kernels ---------------------------------------------------
// Arithmetic of a product.  Phase p of an instance selects PHASE_PREC[p].
enum Prec { PREC_BF16 = 0, PREC_BF16X3 = 1, PREC_F32 = 2 };
enum Epi { EPI_STORE = 0, EPI_DALM = 1, EPI_FISTA = 2, EPI_PARTIAL = 3, EPI_REFRESH = 4 };
constexpr int NPHASE = 3;   // phase index == Prec

struct GemmArgs {
  // A-operand: M x K, element (i, k) at A[i*lda + k] (rows padded to TILE,
  // K padded to KPAD with zeros).  FP32 copy (A32) and BF16 hi/lo split
  // (Ahi, Alo; may be null when no BF16 phase runs).
  const float* A32;
  const uint16_t* Ahi;
  const uint16_t* Alo;
  int lda;
  // B-operand: K x ncols, element (k, col) at B[col*ldb + k]: FP32 (B) and,
  // for BF16 tiles, its BF16 hi / lo split (Bhi, Blo).
  const float* B;
  const uint16_t* Bhi;
  const uint16_t* Blo;
  int ldb;
  int M;   // padded rows (multiple of TILE)
  int K;   // padded reduction length (multiple of KPAD)
  // Columns: tile slot s holds column slot_col[s] (-1 = idle).  Slots are
  // grouped by phase: phase p owns [phase_off[p], phase_off[p+1]), each range
  // a multiple of TILE.  With slot_col == null, slot s < n_cols is column s
  // and every tile uses `prec`.
  const int* slot_col;
  const int* phase_off;
  int n_cols;
  int prec;
  // ---- epilogue -----------------------------------------------------------
  int m_true;              // rows < m_true are written (EPI_STORE)
  float* out;              // EPI_STORE: out[col*ldo + i]; EPI_FISTA: next point z
  int ldo;
  const float* col_scale;  // EPI_STORE: multiply by col_scale[col] (or 1)
  // EPI_DALM / EPI_FISTA state, all column-major with leading dimension lds
  int lds;
  float* V;             // DALM: v = A^T y              | FISTA: current point z (read)
  float* W;             // DALM: w = [x; e]             | FISTA: w (last shrink output)
  const float* C;       // DALM: c_ref = c - P w_ref / beta (c = A^T G^{-1} b/beta) | FISTA: h
  // DALM re-centred operand: u = z - (w - w_ref)/beta (w_ref null: 0), so
  // that v = P u + c_ref = P (z - w/beta) + c exactly while the operand stays
  // O(1) in the low-precision products; EPI_REFRESH sets w_ref = w and
  // c_ref = (C0 - P w) / beta with an FP32 product (C0 = A^T G^{-1} b)
  float* Wref;
  const float* C0;
  int force_f32;        // EPI_REFRESH: FP32 product whatever the tile's phase
  const float* beta;    // DALM: beta per column        | FISTA: xi per column
  float* U;             // DALM: next B-operand u (FP32) ...
  uint16_t* Uhi;        // ... and its BF16 hi / lo split (may be null when
  uint16_t* Ulo;        //     no BF16 phase runs)
  float* partial;       // partial[(tile*NPART + q)*ldp + col]
  int ldp;
  int n_l1;             // DALM: rows < n_l1 carry the l1 norm (gap sums)
  int e0;               // DALM P_{1,2}: rows >= e0 are the eps-ball block (block prox)
  const float* zscale;  // DALM P_{1,2}: block-prox scale of the previous z-step per column
  float inv_L;          // FISTA: 1/L
  float gamma;          // FISTA: (t_l - 1)/t_{l+1}
  // ---- split-K: EPI_PARTIAL launches split the K range in ksplit parts and
  // write raw products ws[(s*ws_slots + slot)*M + row]; the following
  // EPI_DALM / EPI_FISTA launch with the same ws sums the parts in order
  // s = 0..ksplit-1 instead of running a main loop.
  int ksplit;           // >= 1
  float* ws;            // null: no split-K
  int ws_slots;         // slot stride of ws (= n_col_tiles * TILE of the launch)
  int n_ctiles;         // column tiles covered by the launch grid
  // ---- per-instance state (DALM iteration launches; null otherwise).  A
  // launch multiplies every listed column of its tile in the arithmetic of
  // the tile's phase group (slot_col / phase_off, regrouped by compaction),
  // tests the previous iteration of its columns from prev_partial while the
  // product runs, and updates only the columns that go on; row tile 0
  // records the new state.
  const int* state_in;   // phases before this launch (read by every workgroup)
  int* state_out;        // phases after its test (written by row tile 0)
  // arithmetic (phase) of each column's product in the previous launch and
  // in this one (written by row tile 0); null: not tracked.  Sums made in a
  // lower arithmetic than the instance's phase decide nothing.
  const int* arith_in;
  int* arith_out;
  int* iters;
  int* status;
  const float* prev_partial;   // null: no test (first iteration of a solve)
  float tp_tol, tp_sw, tp_floor[3];
  int tp_final;
  int test_kind;               // 0: DALM test (decide()), 1: FISTA inner test (relative change)
  const float* eps;            // P_{1,2} radii (the ball scale comes from prev_partial)
  const float* wcap2;          // squared L1_DIVERGED thresholds per column (null: none)
  const float* dscale2;        // (beta0 / beta)^2 per column (null: 1)
  long long* stat;             // [3 + prec] += live columns, [prec] += column tiles,
                               // [6] += live columns of structured-form launches
  // ---- structured DALM form (cross-and-bouquet): the iteration is two
  // launches.  The first multiplies u by the first rows of P and also writes
  // q = u - (P u) for its rows below q_rows (0 at and beyond them); the
  // second multiplies q by B and adds the current operand u (add_u).
  int row_off;            // state row of the launch's output row 0 (a multiple of TILE)
  int ptiles;             // row tiles of partial sums the test adds (0: M / TILE)
  int test_passive;       // 1: decide like the first launch, record nothing
  int add_u;              // DALM epilogue: v = acc + u + c (u from Ucur*, the current operand)
  const float* Ucur;
  const uint16_t* Ucur_hi;
  const uint16_t* Ucur_lo;
  float* Tq;              // q out (column-major, leading dimension ldt), FP32 ...
  uint16_t* Tq_hi;        // ... and its BF16 hi / lo split
  uint16_t* Tq_lo;
  int q_rows;             // rows < q_rows carry q (0: no q output)
  int ldt;                // leading dimension of T; > 0 marks a structured-form launch
  int prec_mask;          // bit p set: the launch runs the tiles of arithmetic p (0: all)
  int fam;                // 1: every tile is BF16 or split BF16 (the lighter kernel instance)
};

// The alignment l1 problem of Sec. II-B (csrc/align.hip): per instance its
// own m x k dictionary, k <= ALIGN_KMAX, m <= 256 * ALIGN_R.
constexpr int ALIGN_KMAX = 16;
constexpr int ALIGN_R = 8;
void align_solve(hipStream_t s, const float* B, int m, int k, int N, const float* b, int ldb, float tol,
                 int max_iter, float* w, float* e, int lde, int* iters, int* status);

// The recognition criterion of Sec. VI-B (csrc/classify.hip).
void classify(hipStream_t s, const float* x, int ldx, int n_dict, int N, const int* ptr, int C,
              float* mass, int* label, float* score);

// Number of column tiles a launch must cover for up to n columns split over
// the phases (each phase range is padded to a multiple of TILE).
inline int col_tiles_for(int n) { return (n + TILE - 1) / TILE + NPHASE - 1; }
void launch_gemm(hipStream_t s, int epi, const GemmArgs& a, int n_col_tiles);
// One iteration product with epilogue `epi`, split over ksplit K ranges when
// ksplit > 1 (two launches, workspace a.ws), else fused in one launch.
void launch_product(hipStream_t s, int epi, GemmArgs a, int n_col_tiles, int ksplit);

// ---- small per-iteration kernels ---------------------------------------
void fill_iota(hipStream_t s, int* p, int n);
void fill_f32(hipStream_t s, float* p, long n, float v);

}  // namespace l1
