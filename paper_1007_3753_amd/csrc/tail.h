// The DALM tail kernel: the last few unfinished instances, many iterations
// in one cooperative launch.
#pragma once
#include "dalm_test.h"

namespace l1 {

constexpr int TAIL_NC = 16;     // instances one tail launch can carry
constexpr int TAIL_ROWS = 16;   // operator rows per workgroup
constexpr int TAIL_MAXU = 8;    // 64-element K units one wave keeps in registers
constexpr int TAIL_UV = 12;     // 16-byte vectors of u one thread stages per iteration
constexpr int TAIL_TG = 8;      // partial-sum groups one thread adds per iteration

struct TailArgs {
  // operator P (row-major, ld n_pad): FP32 and its BF16 hi / lo split
  const float* P32;
  const uint16_t* Phi;
  const uint16_t* Plo;
  int n_pad, n_l1, lds;
  int f32;                      // 1: FP32 products, 0: split-BF16 products
  int ncap;                     // columns the LDS stage holds (<= TAIL_NC)
  // per-instance state (ordinary device memory; rows of V, W are touched only
  // by the workgroup that owns them)
  float* V;
  float* W;
  const float* C;
  const float* beta;
  int* st[2];                   // phase buffers; st[k0 & 1] holds the phases on entry
  int* iters;
  int* status;
  const int* slot_col;
  const int* phase_off;
  // the iteration before the tail: its partial sums (tile layout) and the
  // B operand it produced
  const float* reg_partial;
  const int* reg_arith;         // arithmetic of that iteration's products
  int ldp, ntiles;
  const float* U32;
  const uint16_t* Uhi;
  const uint16_t* Ulo;
  TestParams tp;
  // exchange buffers in uncached device memory: the next B operand of the
  // listed instances ([TAIL_NC][n_pad] each: FP32, or the BF16 hi and lo
  // halves packed into one 32-bit word, hi in the low half) and the
  // per-workgroup partial sums ([G][NPART][TAIL_NC]), both double-buffered by
  // iteration parity
  float* xu32[2];
  uint32_t* xpk[2];
  float* xpart[2];
  unsigned* bar;                // barrier counter (uncached, zero at launch)
  int* flag;                    // [0] barrier gave up, [1] iterations done
  int k0, k_end;
  int ks;                       // K split of the product (1..8), as the iteration GEMM's
  long long* stat;
};

// Launches the tail kernel (grid n_pad / TAIL_ROWS workgroups); returns false
// without launching when the grid cannot be co-resident or the LDS stage does
// not fit.  The kernel declines (flag[1] = k0, nothing changed) unless every
// listed instance is in the final phase.
bool launch_dalm_tail(hipStream_t s, const TailArgs& t);
// Columns of B operand the tail kernel can stage for an operator of n_pad rows.
int tail_capacity(int n_pad, int f32);

// Uncached exchange memory for the tail kernel on the current device (never
// freed: memory of this kind must not be released while the process runs).
// Returns null when it cannot be allocated or is too small.
void* tail_pool(size_t bytes);

}  // namespace l1
