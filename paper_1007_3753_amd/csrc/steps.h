// Declarations of the small per-solve / per-iteration kernels (steps.hip).
#pragma once
#include "internal.h"

namespace l1 {

// Per-instance state of a solve: 0 = BF16 products, 1 = split-BF16 products,
// 2 = FP32 products (the phase index equals the Prec of its products),
// 3 = finished.  The active instances of the next iteration are listed in
// slot_col, grouped by phase: phase p owns slots [phase_off[p],
// phase_off[p+1]), each range padded with -1 to a multiple of TILE.
struct Lists {
  int* state;
  int* iters;
  int* status;
  int* slot_col;    // N_pad + NPHASE*TILE entries
  int* phase_off;   // NPHASE + 1 entries
  int* n_total;     // number of unfinished instances (read by the host)
  int* cnt;         // NPHASE entries: instances per phase in the current lists
};

struct DalmInit {
  int n, n_pad, lds, e0;
  const float* V;
  const float* W;
  const float* beta;
  const float* eps;
  float* zscale;
  float* U;
  uint16_t* Uhi;   // optional BF16 split of U
  uint16_t* Ulo;
};

struct DalmCheck {
  int N;
  const float* partial;  // partial sums of the iteration to test (final test)
  const int* arith;      // arithmetic of that iteration's products (null: not tracked)
  int ldp, ntiles;
  float tol;             // < 0: never converge (fixed iteration count)
  float floor[NPHASE];   // the final test uses max(tol, floor[phase])
  float sw;              // exit threshold of a non-final phase
  int final_phase;
  int low_cap;           // > 0: compaction moves an instance out of a non-final
                         // phase once it has run this many iterations
  Lists L;               // L.state: the current phase buffer
  int* state_other;      // the other phase buffer (compaction copies into it)
  const float* eps;      // P_{1,2} radii
  const float* beta;
  const float* wcap2;    // squared L1_DIVERGED thresholds (null: no test)
  const float* dscale2;  // per instance {(beta0 / beta)^2, gap-scale floor} (null: {1, 0})
  long long* stat;       // [7] = largest per-instance iteration count
};

struct P12Fix {
  int n, e0, lds, ldp, ntiles;
  const int* slot_col;
  const int* phase_off;
  const int* state;       // phases after the launch
  const float* partial;   // partial sums of the launch (ball block norm)
  const float* V;
  const float* W;
  const float* beta;
  const float* eps;
  float* U;
  uint16_t* Uhi;          // optional BF16 split of U
  uint16_t* Ulo;
};

// Per-instance penalty from pen_in[c] when it is positive and finite, else
// `fixed` when > 0, else the default of the instance: mode 0 (DALM) beta =
// dflt ||b||_1 / m, mode 1 (PALM) xi = 2 m / ||b||_1; the squared
// L1_DIVERGED threshold (div sqrt(m) ||b||_2)^2; and per instance the pair
// dscale2[2c] = (beta0 / beta)^2 with beta0 = ||b||_1 / m, the unit of the
// DALM stopping test, and dscale2[2c + 1] = gfl ||b||_1, the floor of its gap
// scale (may be null).
void penalties(hipStream_t s, int N, int m, const float* b, int ldb, const float* pen_in,
               float fixed, int mode, float dflt, float gfl, float div, float* pen, float* ipen,
               float* wcap2, float* dscale2);
void dalm_init_u(hipStream_t s, int N, const DalmInit& a);
void init_lists(hipStream_t s, int N, int phase0, const Lists& L, int* state_other,
                long long* stat);
// Compaction of the unfinished instances into the phase segments of the
// slot list (one workgroup); also copies the phases into state_other.
void dalm_compact(hipStream_t s, const DalmCheck& a);
// Convergence test of the last iteration (the iteration launches test the
// previous one in their prologue).
void dalm_final_test(hipStream_t s, const DalmCheck& a);
void p12_fix(hipStream_t s, int n_blocks, const P12Fix& a);
void copy_block(hipStream_t s, int rows, int N, const float* src, int lds, int r0, float* dst,
                int ldd);
void copy_in(hipStream_t s, int rows, int N, const float* src, int lds, float* dst, int ldd,
             int r0);
void finish_status(hipStream_t s, int N, int fixed, const int* iters, const int* status,
                   int* it_out, int* st_out);

}  // namespace l1
