// Per-iteration kernels of the batched ALM solvers.
//
// The hot kernel is one MFMA GEMM  out = Op * U  over the batch, where every
// column of U is one instance, with the method's elementwise step fused into
// the epilogue:
//   EPI_DALM   the z-, y- and w-steps of the dual ALM (Sec. V-B, Algorithm 2)
//              in operator form: v = A^T y = P u + c with P = A^T G^{-1} A,
//              c = A^T G^{-1} b / beta, u = z - w/beta; then
//              w <- w - beta (z - v), next z = P_Binf(v + w/beta), next u.
//   EPI_FISTA  one FISTA step of the primal ALM inner loop (Sec. V-A,
//              Algorithm 1 steps 5-8) in Gram form: with M = A^T A and
//              h = A^T (b - e + theta/xi), w <- shrink(z + (h - M z)/L,
//              1/(xi L)), z <- w + gamma (w - w_prev).
//   EPI_STORE  out = scale[col] * (Op U) for the one-time products.
// Columns are addressed through an active list, so converged instances cost
// nothing and the launch geometry stays fixed.
//
// Tile: 64 x 64 outputs per workgroup, 4 waves of 32 x 32 (2 x 2 blocks of
// 16 x 16 MFMA), 128-byte K slices of both operands staged through LDS with a
// register prefetch of the next slice.  Both operands are K-contiguous, so
// every lane moves 16-byte vectors.
#include "internal.h"

namespace l1 {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));
typedef unsigned short us4 __attribute__((ext_vector_type(4)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

__device__ inline uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

constexpr int ROWB = 128;        // bytes of one K slice per row
constexpr int LDSROW = ROWB + 16;  // padded LDS row (bank spread for 16-byte reads)

__device__ inline float clamp1(float x) { return fminf(fmaxf(x, -1.0f), 1.0f); }
__device__ inline float softf(float x, float a) {
  const float m = fabsf(x) - a;
  return m > 0.0f ? copysignf(m, x) : 0.0f;
}
__device__ inline u4 ld16(const void* p) { return *reinterpret_cast<const u4*>(p); }
__device__ inline void st16(void* p, u4 v) { *reinterpret_cast<u4*>(p) = v; }

// LDS tiles: 0 = A (hi), 1 = B (hi), 2 = A lo, 3 = B lo; rows of LDSROW bytes
constexpr int LDSTILE = 64 * LDSROW;

// ---- FP32 main loop: 32-element K slices, v_mfma_f32_16x16x4_f32 ----------
__device__ inline void mainloop_f32(const GemmArgs& a, int i0, const int* colidx,
                                    unsigned char* lds, f4 (&acc)[2][2]) {
  const int tid = threadIdx.x;
  const int ch = tid & 7, rr = tid >> 3;
  const char* A = reinterpret_cast<const char*>(a.A32);
  const char* B = reinterpret_cast<const char*>(a.B);
  const long arow0 = (long)(i0 + rr) * a.lda * 4, arow1 = (long)(i0 + rr + 32) * a.lda * 4;
  const int bc0 = colidx[rr], bc1 = colidx[rr + 32];
  const long brow0 = (long)(bc0 < 0 ? 0 : bc0) * a.ldb * 4;
  const long brow1 = (long)(bc1 < 0 ? 0 : bc1) * a.ldb * 4;
  const u4 z4 = {0u, 0u, 0u, 0u};
  u4 ra0, ra1, rb0, rb1;
  auto fetch = [&](long kb) {
    const long off = kb + ch * 16;
    ra0 = ld16(A + arow0 + off);
    ra1 = ld16(A + arow1 + off);
    rb0 = bc0 >= 0 ? ld16(B + brow0 + off) : z4;
    rb1 = bc1 >= 0 ? ld16(B + brow1 + off) : z4;
  };
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1, li = lane & 15, q = lane >> 4;
  const int nk = a.K / 32;
  fetch(0);
  for (int kt = 0; kt < nk; ++kt) {
    st16(&lds[rr * LDSROW + ch * 16], ra0);
    st16(&lds[(rr + 32) * LDSROW + ch * 16], ra1);
    st16(&lds[LDSTILE + rr * LDSROW + ch * 16], rb0);
    st16(&lds[LDSTILE + (rr + 32) * LDSROW + ch * 16], rb1);
    __syncthreads();
    if (kt + 1 < nk) fetch((long)(kt + 1) * 128);
#pragma unroll
    for (int kc = 0; kc < 2; ++kc) {
      const int boff = kc * 64 + q * 16;
      u4 fa[2], fb[2];
#pragma unroll
      for (int bi = 0; bi < 2; ++bi) fa[bi] = ld16(&lds[(wm * 32 + bi * 16 + li) * LDSROW + boff]);
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
        fb[bj] = ld16(&lds[LDSTILE + (wn * 32 + bj * 16 + li) * LDSROW + boff]);
      // lane (li, q) holds k = 4q..4q+3 of this 16-wide chunk; MFMA step s
      // takes element s from every lane, so the four steps cover the chunk
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj)
            acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                __uint_as_float(fa[bi][s]), __uint_as_float(fb[bj][s]), acc[bi][bj], 0, 0, 0);
    }
    __syncthreads();
  }
}

// ---- BF16 main loops: 64-element K slices, v_mfma_f32_16x16x32_bf16 -------
// The FP32 B-operand is split into BF16 hi (+ lo) while it is staged to LDS.
template <bool SPLIT>
__device__ inline void mainloop_bf16(const GemmArgs& a, int i0, const int* colidx,
                                     unsigned char* lds, f4 (&acc)[2][2]) {
  const int tid = threadIdx.x;
  const int ch = tid & 7, rr = tid >> 3;    // A: 16-byte chunk, rows rr, rr + 32
  const int bq = tid & 3, bcs = tid >> 2;   // B: quarter of the 256-byte FP32 slice, column slot
  const char* Ah = reinterpret_cast<const char*>(a.Ahi);
  const char* Al = reinterpret_cast<const char*>(a.Alo);
  const char* B = reinterpret_cast<const char*>(a.B);
  const long arow0 = (long)(i0 + rr) * a.lda * 2, arow1 = (long)(i0 + rr + 32) * a.lda * 2;
  const int bc = colidx[bcs];
  const long brow = (long)(bc < 0 ? 0 : bc) * a.ldb * 4;
  const u4 z4 = {0u, 0u, 0u, 0u};
  u4 rah0, rah1, ral0, ral1, rb[4];
  auto fetch = [&](int kt) {
    const long offa = (long)kt * 128 + ch * 16;
    rah0 = ld16(Ah + arow0 + offa);
    rah1 = ld16(Ah + arow1 + offa);
    if (SPLIT) {
      ral0 = ld16(Al + arow0 + offa);
      ral1 = ld16(Al + arow1 + offa);
    }
    const long offb = (long)kt * 256 + bq * 64;
#pragma unroll
    for (int t = 0; t < 4; ++t) rb[t] = bc >= 0 ? ld16(B + brow + offb + 16 * t) : z4;
  };
  auto stash = [&]() {
    st16(&lds[rr * LDSROW + ch * 16], rah0);
    st16(&lds[(rr + 32) * LDSROW + ch * 16], rah1);
    if (SPLIT) {
      st16(&lds[2 * LDSTILE + rr * LDSROW + ch * 16], ral0);
      st16(&lds[2 * LDSTILE + (rr + 32) * LDSROW + ch * 16], ral1);
    }
    // 16 FP32 values -> 16 BF16 hi (+ 16 lo): two 16-byte vectors each
    u4 h[2], l[2];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int e = 0; e < 4; e += 2) {
        const float x0 = __uint_as_float(rb[t][e]), x1 = __uint_as_float(rb[t][e + 1]);
        const uint32_t h0 = f2bf(x0), h1 = f2bf(x1);
        h[t >> 1][(t & 1) * 2 + (e >> 1)] = h0 | (h1 << 16);
        if (SPLIT) {
          const uint32_t l0 = f2bf(x0 - bf2f((uint16_t)h0)), l1 = f2bf(x1 - bf2f((uint16_t)h1));
          l[t >> 1][(t & 1) * 2 + (e >> 1)] = l0 | (l1 << 16);
        }
      }
    st16(&lds[LDSTILE + bcs * LDSROW + bq * 32], h[0]);
    st16(&lds[LDSTILE + bcs * LDSROW + bq * 32 + 16], h[1]);
    if (SPLIT) {
      st16(&lds[3 * LDSTILE + bcs * LDSROW + bq * 32], l[0]);
      st16(&lds[3 * LDSTILE + bcs * LDSROW + bq * 32 + 16], l[1]);
    }
  };
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1, li = lane & 15, q = lane >> 4;
  const int nk = a.K / 64;
  fetch(0);
  for (int kt = 0; kt < nk; ++kt) {
    stash();
    __syncthreads();
    if (kt + 1 < nk) fetch(kt + 1);
#pragma unroll
    for (int kc = 0; kc < 2; ++kc) {
      const int boff = kc * 64 + q * 16;
#pragma unroll
      for (int bi = 0; bi < 2; ++bi) {
        const int ar = (wm * 32 + bi * 16 + li) * LDSROW + boff;
        const bf8 ah = __builtin_bit_cast(bf8, ld16(&lds[ar]));
        bf8 al;
        if (SPLIT) al = __builtin_bit_cast(bf8, ld16(&lds[2 * LDSTILE + ar]));
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
          const int br = LDSTILE + (wn * 32 + bj * 16 + li) * LDSROW + boff;
          const bf8 bh = __builtin_bit_cast(bf8, ld16(&lds[br]));
          if (SPLIT) {
            const bf8 bl = __builtin_bit_cast(bf8, ld16(&lds[2 * LDSTILE + br]));
            // small terms first: lo*hi + hi*lo, then hi*hi
            acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[bi][bj], 0, 0, 0);
            acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[bi][bj], 0, 0, 0);
          }
          acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[bi][bj], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
}

template <int EPI>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs a) {
  __shared__ __attribute__((aligned(16))) unsigned char lds[4 * LDSTILE];
  __shared__ int colidx[64];
  __shared__ float red[2][64][NPART];

  // XCD-aware tile order: consecutive workgroups are dispatched round-robin
  // to the 8 XCDs, so workgroup L runs on XCD L % 8.  Each XCD takes a
  // contiguous band of row tiles, keeping its slice of the operator in its
  // own L2 across column tiles; the workgroups of one XCD that share a
  // column tile run side by side and share the B tile in L2.
  const int L = blockIdx.x, xcd = L & 7, j = L >> 3;
  const int RT = a.M / 64;
  const int r_lo = (xcd * RT) / 8, r_hi = ((xcd + 1) * RT) / 8, nr = r_hi - r_lo;
  if (nr <= 0) return;
  const int rt = r_lo + j % nr, ct = j / nr;
  const int i0 = rt * 64, slot0 = ct * 64;
  int nslots, prec;
  if (a.slot_col) {
    nslots = a.phase_off[NPHASE];
    prec = slot0 < a.phase_off[1] ? 0 : (slot0 < a.phase_off[2] ? 1 : 2);
  } else {
    nslots = a.n_cols;
    prec = a.prec;
  }
  if (slot0 >= nslots) return;  // uniform for the workgroup
  const int tid = threadIdx.x;
  if (tid < 64) {
    const int sl = slot0 + tid;
    colidx[tid] = (sl < nslots) ? (a.slot_col ? a.slot_col[sl] : sl) : -1;
  }
  __syncthreads();

  f4 acc[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = f4{0.f, 0.f, 0.f, 0.f};
  if (prec == PREC_F32) mainloop_f32(a, i0, colidx, lds, acc);
  else if (prec == PREC_BF16X3) mainloop_bf16<true>(a, i0, colidx, lds, acc);
  else mainloop_bf16<false>(a, i0, colidx, lds, acc);

  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1, li = lane & 15, q = lane >> 4;
  // ---- epilogue ----------------------------------------------------------
  // accumulator (bi, bj), register r: row i0 + wm*32 + bi*16 + 4q + r,
  // column slot wn*32 + bj*16 + li
  if (EPI == EPI_STORE) {
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      const int col = colidx[wn * 32 + bj * 16 + li];
      if (col < 0) continue;
      const float sc = a.col_scale ? a.col_scale[col] : 1.0f;
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = i0 + wm * 32 + bi * 16 + 4 * q + r;
          if (row < a.m_true) a.out[(long)col * a.ldo + row] = acc[bi][bj][r] * sc;
        }
    }
    return;
  }

  float part[2][NPART];
#pragma unroll
  for (int bj = 0; bj < 2; ++bj)
#pragma unroll
    for (int p = 0; p < NPART; ++p) part[bj][p] = 0.0f;

#pragma unroll
  for (int bj = 0; bj < 2; ++bj) {
    const int col = colidx[wn * 32 + bj * 16 + li];
    if (col < 0) continue;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
      const int row0 = i0 + wm * 32 + bi * 16 + 4 * q;
      const long idx = (long)col * a.lds + row0;
      const f4 c4 = *reinterpret_cast<const f4*>(a.C + idx);
      const f4 wo = *reinterpret_cast<const f4*>(a.W + idx);
      f4 wn4, un4;
      if (EPI == EPI_DALM) {
        const float bt = a.beta[col];
        const float ib = 1.0f / bt;
        const float zsc = a.zscale ? a.zscale[col] : 1.0f;
        const f4 vo = *reinterpret_cast<const f4*>(a.V + idx);
        f4 vn4;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = row0 + r;
          const bool ball = row >= a.e0;   // eps-ball block of the P_{1,2} splitting
          const float s = vo[r] + wo[r] * ib;
          const float z = ball ? s * zsc : clamp1(s);
          const float vn = acc[bi][bj][r] + c4[r];
          const float wn = wo[r] - bt * (z - vn);
          const float s2 = vn + wn * ib;
          const float z2 = ball ? s2 : clamp1(s2);  // ball rows: scaled after the column norm
          vn4[r] = vn;
          wn4[r] = wn;
          un4[r] = z2 - wn * ib;
          const float d = wn - wo[r];
          part[bj][0] += d * d;
          part[bj][1] += wn * wn;
          if (row < a.n_l1) {
            // complementarity term |w| - w v = |w| (1 - sign(w) v), summed
            // per element so that no two large sums cancel
            const float aw = fabsf(wn);
            part[bj][2] += aw;
            part[bj][3] += aw * (1.0f - copysignf(1.0f, wn) * vn);
          }
          if (ball) part[bj][4] += s2 * s2;
        }
        *reinterpret_cast<f4*>(a.V + idx) = vn4;
        *reinterpret_cast<f4*>(a.U + idx) = un4;
      } else {  // EPI_FISTA
        const float xi = a.beta[col];
        const float thr = a.inv_L / xi;
        const f4 zo = *reinterpret_cast<const f4*>(a.V + idx);  // current FISTA point
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float g = zo[r] + (c4[r] - acc[bi][bj][r]) * a.inv_L;
          const float wn = softf(g, thr);
          wn4[r] = wn;
          un4[r] = wn + a.gamma * (wn - wo[r]);
          const float d = wn - wo[r];
          part[bj][0] += d * d;
          part[bj][1] += wn * wn;
        }
        *reinterpret_cast<f4*>(a.out + idx) = un4;  // next FISTA point
      }
      *reinterpret_cast<f4*>(a.W + idx) = wn4;
    }
  }
  // reduce the partial sums over the 4 lane groups of each column ...
#pragma unroll
  for (int bj = 0; bj < 2; ++bj)
#pragma unroll
    for (int p = 0; p < NPART; ++p) {
      float v = part[bj][p];
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      part[bj][p] = v;
    }
  // ... and over the two waves that share the columns, in a fixed order
  if (q == 0) {
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int p = 0; p < NPART; ++p) red[wm][wn * 32 + bj * 16 + li][p] = part[bj][p];
  }
  __syncthreads();
  if (tid < 64) {
    const int col = colidx[tid];
    if (col >= 0) {
#pragma unroll
      for (int p = 0; p < NPART; ++p)
        a.partial[(long)(rt * NPART + p) * a.ldp + col] = red[0][tid][p] + red[1][tid][p];
    }
  }
}

void launch_gemm(hipStream_t s, int epi, const GemmArgs& a, int n_col_tiles) {
  if (n_col_tiles <= 0 || a.M <= 0) return;
  const int RT = a.M / 64;
  const int per_xcd = (RT + 7) / 8;
  const unsigned grid = 8u * per_xcd * n_col_tiles;
  if (epi == EPI_STORE) gemm_kernel<EPI_STORE><<<grid, 256, 0, s>>>(a);
  else if (epi == EPI_DALM) gemm_kernel<EPI_DALM><<<grid, 256, 0, s>>>(a);
  else gemm_kernel<EPI_FISTA><<<grid, 256, 0, s>>>(a);
  L1_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
__global__ void iota_kernel(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = i;
}
void fill_iota(hipStream_t s, int* p, int n) {
  if (n <= 0) return;
  iota_kernel<<<(n + 255) / 256, 256, 0, s>>>(p, n);
  L1_HIP(hipGetLastError());
}
__global__ void fill_f32_kernel(float* p, long n, float v) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
void fill_f32(hipStream_t s, float* p, long n, float v) {
  if (n <= 0) return;
  fill_f32_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n, v);
  L1_HIP(hipGetLastError());
}

}  // namespace l1
