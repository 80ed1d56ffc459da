// The per-instance convergence test of the dual ALM iteration, shared by the
// GEMM prologue (which tests the previous iteration of its own columns) and
// the final test after the last iteration.
#pragma once
#include "internal.h"

namespace l1 {

struct TestParams {
  float tol;             // < 0: never converge (fixed iteration count)
  float floor[NPHASE];   // the final test uses max(tol, floor[phase])
  float sw;              // exit threshold of a non-final phase
  int final_phase;
  float wcap2;           // ||w||^2 above this: L1_DIVERGED (with tol >= 0 only)
  float dscale2;         // (beta0 / beta)^2: ||dw||^2 = beta^2 ||z - v||^2 is tested
                         // as beta0^2 ||z - v||^2 (beta0 = ||b||_1 / m)
  float gfloor;          // the gap is tested against tol * max(||w||_1, gfloor)
};

// Sums of the per-row-tile partials of column c, taken by 4 cooperating lanes
// (part = lane & 3) in a fixed order; every lane of the group returns the same
// sums.  All 64 lanes of the wave must call this (it shuffles).
__device__ inline void column_sums(const float* partial, int ldp, int ntiles, int c, bool live,
                                   int part, float (&sm)[NPART]) {
#pragma unroll
  for (int q = 0; q < NPART; ++q) sm[q] = 0.0f;
  if (live) {
#pragma unroll 4
    for (int t = part; t < ntiles; t += 4) {
      const float* p = partial + (long)t * NPART * ldp + c;
#pragma unroll
      for (int q = 0; q < NPART; ++q) sm[q] += p[(long)q * ldp];
    }
  }
#pragma unroll
  for (int q = 0; q < NPART; ++q) {
    sm[q] += __shfl_xor(sm[q], 1);
    sm[q] += __shfl_xor(sm[q], 2);
  }
}

// New phase of an instance in phase st (< NPHASE) from its sums: NPHASE
// means finished, with *status set to L1_CONVERGED or L1_NONFINITE.
//   sums: ||dw||^2, ||w||^2, ||w||_1, sum |w|(1 - sign(w) v), ||s_ball||^2
__device__ inline int decide(const TestParams& tp, int st, const float (&sm)[NPART], int* status) {
  const float d2 = sm[0] * tp.dscale2, w2 = sm[1], l1 = fmaxf(sm[2], tp.gfloor), gap = fabsf(sm[3]);
  if (!(isfinite(d2) && isfinite(w2) && isfinite(gap))) {
    *status = L1_NONFINITE;
    return NPHASE;
  }
  if (tp.tol >= 0.0f && w2 > tp.wcap2) {
    *status = L1_DIVERGED;
    return NPHASE;
  }
  if (st != tp.final_phase) {
    if (d2 <= tp.sw * tp.sw * w2 && gap <= tp.sw * l1) return st + 1;
    return st;
  }
  if (tp.tol >= 0.0f) {
    const float t = fmaxf(tp.tol, tp.floor[st]);
    if (d2 <= t * t * w2 && gap <= t * l1) {
      *status = L1_CONVERGED;
      return NPHASE;
    }
  }
  return st;
}

// decide() for sums that come from a product made in arithmetic `arith`:
// when that is below the phase st the instance has reached since (it was
// switched while its tile still ran the lower arithmetic), the sums measure
// the lower arithmetic's stall and decide nothing but a non-finite value.
__device__ inline int decide_in(const TestParams& tp, int st, int arith, const float (&sm)[NPART],
                                int* status) {
  if (arith >= st) return decide(tp, st, sm, status);
  if (!(isfinite(sm[0]) && isfinite(sm[1]) && isfinite(fabsf(sm[3])))) {
    *status = L1_NONFINITE;
    return NPHASE;
  }
  return st;
}

// Block soft-threshold scale of the eps-ball block of P_{1,2}:
// prox of (eps/beta)||.||_2 applied to s is s * max(0, 1 - (eps/beta)/||s||).
__device__ inline float ball_scale(float se, float eps, float beta) {
  const float tau = eps / beta;
  return (se > 0.0f) ? fmaxf(0.0f, 1.0f - tau / sqrtf(se)) : 0.0f;
}

}  // namespace l1
