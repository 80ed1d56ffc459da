// The DALM tail kernel: the last few unfinished instances, many iterations
// in one cooperative launch.
#pragma once
#include "dalm_test.h"

namespace l1 {

constexpr int TAIL_NC = 16;     // instances one tail launch can carry
constexpr int TAIL_ROWS = 16;   // operator rows per workgroup
constexpr int TAIL_MAXU = 8;    // 64-element K units one wave keeps in registers
constexpr int TAIL_UV = 24;     // 16-byte vectors of u one thread stages per iteration
constexpr int TAIL_UR = 12;     // ... of them in registers at once (one round)
constexpr int TAIL_PR = 16;     // tagged partial sums one thread loads per iteration
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
  const float* Wref;            // reference point of the operand (null: 0)
  const float* beta;
  const float* wcap2;           // squared L1_DIVERGED thresholds (null: none)
  const float* dscale2;         // (beta0 / beta)^2 of the stopping test (null: 1)
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
  // exchange buffers in uncached device memory, cleared before the launch:
  // 64-bit words (value in the low half, tag in the high half) holding the
  // next B operand of the listed instances ([TAIL_NC][n_pad]: FP32 bits, or
  // the BF16 hi and lo halves packed hi | lo << 16) and the per-workgroup
  // partial sums ([G][NPART][TAIL_NC] FP32 bits), both by iteration parity
  unsigned long long* xu[2];
  unsigned long long* xpart[2];
  int* flag;                    // [0] a wait gave up, [1] iterations done
  int k0, k_end;
  int ks;                       // K split of the product (1..8), as the iteration GEMM's
  long long* stat;
};

// Launches the tail kernel (grid n_pad / TAIL_ROWS workgroups); returns false
// without launching when the grid cannot be co-resident or the LDS stage does
// not fit.  The kernel declines (flag[1] = k0, nothing changed) unless every
// listed instance is in the final phase.
bool launch_dalm_tail(hipStream_t s, const TailArgs& t);
// Whether the tail kernel can run an operator of n_pad rows (ntiles row tiles
// of partial sums before it) with its product split in ks K parts.
bool tail_fits(int n_pad, int ntiles, int ks);
// Columns of B operand the tail kernel can stage for an operator of n_pad rows.
int tail_capacity(int n_pad, int f32);

// Uncached exchange memory for the tail kernel on the current device, one
// region per plan: tail_region_get returns a region of at least `bytes`
// (reusing one a destroyed plan gave back) and its size in *got, or null;
// tail_region_put gives a plan's region back.  Regions are never freed:
// memory of this kind must not be released while the process runs.
void* tail_region_get(size_t bytes, size_t* got);
void tail_region_put(int dev, void* p, size_t bytes);

}  // namespace l1
