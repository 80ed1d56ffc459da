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
#include "dalm_test.h"

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
// LDS byte offset of 16-byte chunk c of tile row r.  Rows are unpadded and the
// chunk index is XORed with bits 1..3 of the row, so that the 16 lanes of a
// fragment read (rows r..r+15, one chunk) and the 16 lanes of a staging write
// (two rows, eight chunks) each touch 16 distinct 16-byte bank groups.
__device__ inline int lo(int r, int c) { return r * ROWB + ((c ^ ((r >> 1) & 7)) << 4); }

__device__ inline float clamp1(float x) { return fminf(fmaxf(x, -1.0f), 1.0f); }
__device__ inline float softf(float x, float a) {
  const float m = fabsf(x) - a;
  return m > 0.0f ? copysignf(m, x) : 0.0f;
}
__device__ inline u4 ld16(const void* p) { return *reinterpret_cast<const u4*>(p); }
__device__ inline void st16(void* p, u4 v) { *reinterpret_cast<u4*>(p) = v; }

// LDS tiles of one stage buffer: 0 = A (hi), 1 = B (hi), 2 = A lo, 3 = B lo;
// 64 rows of ROWB bytes each; two stage buffers
constexpr int LDSTILE = 64 * ROWB;
constexpr int STAGE = 4 * LDSTILE;
constexpr int GEMM_LDS = 2 * STAGE;
// row tiles of partial sums per lane loaded before the K loop (the rest after it)
constexpr int TEST_PRE = 8;

// The K loop of a workgroup is a chain of global-memory round trips; each
// takes ~1 us under load, far longer than the MFMA work on one slice.  Both
// main loops keep D slices in flight in registers and stage slices through
// two LDS buffers: in step k the workgroup multiplies slice k from buffer
// k & 1 while it moves slice k + 1 from registers into the other buffer and
// requests slice k + 1 + D into the registers just freed, so one barrier per
// step (at its start) both publishes slice k and frees the buffer written
// next.  Every load is unconditional (the slice index is clamped; an empty
// slot reads column 0, whose products are never stored: each output column
// depends on its own B column only, so no load result is masked, which would
// make the compiler wait for it at once) and the steady-state loop runs a
// multiple of D steps, so the wait inserted before a register set is
// consumed always leaves the younger D - 1 slices in flight, also across the
// loop back-edge.  D is a compile-time constant so every register set is
// statically indexed.

// ---- FP32 main loop: 32-element K slices, v_mfma_f32_16x16x4_f32 ----------
template <int D>
__device__ inline void mainloop_f32(const GemmArgs& a, int i0, const int* colidx,
                                    unsigned char* lds, f4 (&acc)[2][2], int kb, int ke) {
  const int tid = threadIdx.x;
  const int ch = tid & 7, rr = tid >> 3;
  const char* A = reinterpret_cast<const char*>(a.A32);
  const char* B = reinterpret_cast<const char*>(a.B);
  const long arow0 = (long)(i0 + rr) * a.lda * 4, arow1 = (long)(i0 + rr + 32) * a.lda * 4;
  const int bc0 = colidx[rr], bc1 = colidx[rr + 32];
  const long brow0 = (long)(bc0 >= 0 ? bc0 : 0) * a.ldb * 4;
  const long brow1 = (long)(bc1 >= 0 ? bc1 : 0) * a.ldb * 4;
  // [kb, ke) is given in 64-element units; FP32 slices hold 32 elements
  A += (long)kb * 256;
  B += (long)kb * 256;
  const int nk = 2 * (ke - kb);
  if (nk <= 0) return;
  u4 ra[D][2], rb[D][2];
#define L1_FETCH_F32(d, kt)                                   \
  {                                                           \
    const long off = (long)min((kt), nk - 1) * 128 + ch * 16; \
    ra[d][0] = ld16(A + arow0 + off);                         \
    ra[d][1] = ld16(A + arow1 + off);                         \
    rb[d][0] = ld16(B + brow0 + off);                         \
    rb[d][1] = ld16(B + brow1 + off);                         \
  }
#define L1_PUT_F32(d, buf)                                             \
  {                                                                    \
    unsigned char* st_ = lds + (buf) * STAGE;                          \
    st16(&st_[lo(rr, ch)], ra[d][0]);                                  \
    st16(&st_[lo(rr + 32, ch)], ra[d][1]);                             \
    st16(&st_[LDSTILE + lo(rr, ch)], rb[d][0]);                        \
    st16(&st_[LDSTILE + lo(rr + 32, ch)], rb[d][1]);                   \
  }
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1, li = lane & 15, q = lane >> 4;
  // step k: slice k + 1 sits in register set (k + 1) % D = dn
#define L1_STEP_F32(k, dn)                                                                   \
  {                                                                                          \
    __syncthreads();                                                                         \
    L1_PUT_F32(dn, ((k) + 1) & 1)                                                            \
    L1_FETCH_F32(dn, (k) + 1 + D)                                                            \
    const unsigned char* cur_ = lds + ((k) & 1) * STAGE;                                     \
    _Pragma("unroll") for (int kc = 0; kc < 2; ++kc) {                                       \
      u4 fa[2], fb[2];                                                                       \
      _Pragma("unroll") for (int i = 0; i < 2; ++i) {                                        \
        fa[i] = ld16(&cur_[lo(wm * 32 + i * 16 + li, kc * 4 + q)]);                          \
        fb[i] = ld16(&cur_[LDSTILE + lo(wn * 32 + i * 16 + li, kc * 4 + q)]);                \
      }                                                                                      \
      /* lane (li, q) holds k = 4q..4q+3 of this 16-wide chunk; MFMA step s takes  */        \
      /* element s from every lane, so the four steps cover the chunk             */        \
      _Pragma("unroll") for (int s = 0; s < 4; ++s)                                          \
      _Pragma("unroll") for (int bi = 0; bi < 2; ++bi)                                       \
      _Pragma("unroll") for (int bj = 0; bj < 2; ++bj)                                       \
        acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x4f32(                                  \
            __uint_as_float(fa[bi][s]), __uint_as_float(fb[bj][s]), acc[bi][bj], 0, 0, 0);   \
    }                                                                                        \
  }
#pragma unroll
  for (int d = 0; d < D; ++d) L1_FETCH_F32(d, d)
  L1_PUT_F32(0, 0)
  L1_FETCH_F32(0, D)
  const int nmain = nk - nk % D;
  for (int k0 = 0; k0 < nmain; k0 += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) L1_STEP_F32(k0 + d, (d + 1) % D)
  }
#pragma unroll
  for (int d = 0; d < D - 1; ++d)
    if (nmain + d < nk) L1_STEP_F32(nmain + d, (d + 1) % D)
  __syncthreads();  // the stage is free again
#undef L1_STEP_F32
#undef L1_PUT_F32
#undef L1_FETCH_F32
}

// ---- BF16 main loops: 64-element K slices, v_mfma_f32_16x16x32_bf16 -------
// Both operands arrive already split into BF16 hi (+ lo): the operator once
// per plan, the iterate by the previous iteration's epilogue.
template <bool SPLIT, int D>
__device__ inline void mainloop_bf16(const GemmArgs& a, int i0, const int* colidx,
                                     unsigned char* lds, f4 (&acc)[2][2], int kb, int ke) {
  const int tid = threadIdx.x;
  const int ch = tid & 7, rr = tid >> 3;    // 16-byte chunk, rows rr and rr + 32
  const char* Ah = reinterpret_cast<const char*>(a.Ahi);
  const char* Al = reinterpret_cast<const char*>(a.Alo);
  const char* Bh = reinterpret_cast<const char*>(a.Bhi);
  const char* Bl = reinterpret_cast<const char*>(a.Blo);
  const long arow0 = (long)(i0 + rr) * a.lda * 2, arow1 = (long)(i0 + rr + 32) * a.lda * 2;
  const int bc0 = colidx[rr], bc1 = colidx[rr + 32];
  const long brow0 = (long)(bc0 >= 0 ? bc0 : 0) * a.ldb * 2;
  const long brow1 = (long)(bc1 >= 0 ? bc1 : 0) * a.ldb * 2;
  Ah += (long)kb * 128;
  Bh += (long)kb * 128;
  if (SPLIT) {
    Al += (long)kb * 128;
    Bl += (long)kb * 128;
  }
  const int nk = ke - kb;
  if (nk <= 0) return;
  u4 rah[D][2], ral[D][2], rbh[D][2], rbl[D][2];
#define L1_FETCH_BF(d, kt)                                    \
  {                                                           \
    const long off = (long)min((kt), nk - 1) * 128 + ch * 16; \
    rah[d][0] = ld16(Ah + arow0 + off);                       \
    rah[d][1] = ld16(Ah + arow1 + off);                       \
    rbh[d][0] = ld16(Bh + brow0 + off);                       \
    rbh[d][1] = ld16(Bh + brow1 + off);                       \
    if (SPLIT) {                                              \
      ral[d][0] = ld16(Al + arow0 + off);                     \
      ral[d][1] = ld16(Al + arow1 + off);                     \
      rbl[d][0] = ld16(Bl + brow0 + off);                     \
      rbl[d][1] = ld16(Bl + brow1 + off);                     \
    }                                                         \
  }
#define L1_PUT_BF(d, buf)                                              \
  {                                                                    \
    unsigned char* st_ = lds + (buf) * STAGE;                          \
    st16(&st_[lo(rr, ch)], rah[d][0]);                                 \
    st16(&st_[lo(rr + 32, ch)], rah[d][1]);                            \
    st16(&st_[LDSTILE + lo(rr, ch)], rbh[d][0]);                       \
    st16(&st_[LDSTILE + lo(rr + 32, ch)], rbh[d][1]);                  \
    if (SPLIT) {                                                       \
      st16(&st_[2 * LDSTILE + lo(rr, ch)], ral[d][0]);                 \
      st16(&st_[2 * LDSTILE + lo(rr + 32, ch)], ral[d][1]);            \
      st16(&st_[3 * LDSTILE + lo(rr, ch)], rbl[d][0]);                 \
      st16(&st_[3 * LDSTILE + lo(rr + 32, ch)], rbl[d][1]);            \
    }                                                                  \
  }
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1, li = lane & 15, q = lane >> 4;
#define L1_STEP_BF(k, dn)                                                                     \
  {                                                                                           \
    __syncthreads();                                                                          \
    L1_PUT_BF(dn, ((k) + 1) & 1)                                                              \
    L1_FETCH_BF(dn, (k) + 1 + D)                                                              \
    const unsigned char* cur_ = lds + ((k) & 1) * STAGE;                                      \
    _Pragma("unroll") for (int kc = 0; kc < 2; ++kc) {                                        \
      bf8 ah[2], bh[2], al[2], bl[2];                                                         \
      _Pragma("unroll") for (int i = 0; i < 2; ++i) {                                         \
        const int ar = lo(wm * 32 + i * 16 + li, kc * 4 + q);                                 \
        const int br = LDSTILE + lo(wn * 32 + i * 16 + li, kc * 4 + q);                       \
        ah[i] = __builtin_bit_cast(bf8, ld16(&cur_[ar]));                                     \
        bh[i] = __builtin_bit_cast(bf8, ld16(&cur_[br]));                                     \
        if (SPLIT) {                                                                          \
          al[i] = __builtin_bit_cast(bf8, ld16(&cur_[2 * LDSTILE + ar]));                     \
          bl[i] = __builtin_bit_cast(bf8, ld16(&cur_[2 * LDSTILE + br]));                     \
        }                                                                                     \
      }                                                                                       \
      /* four independent accumulators, issued round by round; small terms first */          \
      if (SPLIT) {                                                                            \
        _Pragma("unroll") for (int bi = 0; bi < 2; ++bi)                                      \
        _Pragma("unroll") for (int bj = 0; bj < 2; ++bj)                                      \
          acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[bi], bh[bj], acc[bi][bj], 0, 0, 0); \
        _Pragma("unroll") for (int bi = 0; bi < 2; ++bi)                                      \
        _Pragma("unroll") for (int bj = 0; bj < 2; ++bj)                                      \
          acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[bi], bl[bj], acc[bi][bj], 0, 0, 0); \
      }                                                                                       \
      _Pragma("unroll") for (int bi = 0; bi < 2; ++bi)                                        \
      _Pragma("unroll") for (int bj = 0; bj < 2; ++bj)                                        \
        acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[bi], bh[bj], acc[bi][bj], 0, 0, 0); \
    }                                                                                         \
  }
#pragma unroll
  for (int d = 0; d < D; ++d) L1_FETCH_BF(d, d)
  L1_PUT_BF(0, 0)
  L1_FETCH_BF(0, D)
  const int nmain = nk - nk % D;
  for (int k0 = 0; k0 < nmain; k0 += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) L1_STEP_BF(k0 + d, (d + 1) % D)
  }
#pragma unroll
  for (int d = 0; d < D - 1; ++d)
    if (nmain + d < nk) L1_STEP_BF(nmain + d, (d + 1) % D)
  __syncthreads();  // the stage is free again
#undef L1_STEP_BF
#undef L1_PUT_BF
#undef L1_FETCH_BF
}

// FAM = 1: the BF16-family instantiation (BF16 and split-BF16 tiles only,
// the epilogue's loads after the K loop, fewer test loads ahead of it), held
// to 256 registers so that two workgroups share a compute unit: on batches
// with more column tiles than compute units one workgroup's K loop then
// covers the other's memory waits.
template <int EPI, int FAM = 0>
__global__ __launch_bounds__(256, FAM == 1 ? 2 : 1) void gemm_kernel(GemmArgs a) {
  constexpr int TP = FAM == 1 ? 4 : TEST_PRE;
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];   // GEMM_LDS bytes
  __shared__ int colidx[64];
  __shared__ float red[2][64][NPART];

  // XCD-aware tile order: consecutive workgroups are dispatched round-robin
  // to the 8 XCDs, so workgroup L runs on XCD L % 8.  Each XCD takes a
  // contiguous band of row tiles, keeping its slice of the operator in its
  // own L2 across column tiles.  Within the band the XCD's workgroups go
  // through groups of TGR row tiles, all column tiles of a group before the
  // next, rows fastest: the workgroups resident at once then cover about as
  // many row tiles as column tiles (8 x 8 at two per CU), so each operator
  // tile and each B tile fetched into L2 serves about 8 workgroups side by
  // side in K (with the band's rows fastest across all column tiles, a
  // 4800 x 2100 band of 13-14 row tiles met only 4-5 column tiles at a time).
  const int L = blockIdx.x, xcd = L & 7, j = L >> 3;
  const int RT = a.M / 64;
  // row tiles of partial sums the test adds (all of the iteration's, also
  // when it is split over two launches), and this launch's first one
  const int RTP = a.ptiles > 0 ? a.ptiles : RT, pt0 = a.row_off / 64;
  const int r_lo = (xcd * RT) / 8, r_hi = ((xcd + 1) * RT) / 8, nr = r_hi - r_lo;
  if (nr <= 0) return;
  const int ks = (EPI == EPI_PARTIAL) ? a.ksplit : 1;
  constexpr int TGR = 8;
  const int per = nr * a.n_ctiles, split = j / per, jj = j - split * per;
  if (split >= ks) return;
  const int gi = jj / (TGR * a.n_ctiles), gr = min(TGR, nr - gi * TGR);
  const int loc = jj - gi * TGR * a.n_ctiles;
  const int rt = r_lo + gi * TGR + loc % gr, ct = loc / gr;
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
  if (a.prec_mask && !((a.prec_mask >> prec) & 1)) return;
  const int tid = threadIdx.x;
  __shared__ float s_zsc[64];
  __shared__ int s_live;
  if (tid < 64) {
    const int sl = slot0 + tid;
    colidx[tid] = (sl < nslots) ? (a.slot_col ? a.slot_col[sl] : sl) : -1;
    s_zsc[tid] = 1.0f;
  }
  if (tid == 0) s_live = 0;
  __syncthreads();

  // Convergence test of the previous iteration (4 lanes per column).  Its
  // loads are issued here and its decision is taken after the product, so
  // that its memory round trips overlap the K loop: the product does not
  // depend on it, because every listed column is multiplied (a column that
  // has just finished is simply not updated) in the arithmetic of its phase
  // group as of the last compaction.  The partial sums are added in the
  // order of column_sums.
  const bool test = EPI != EPI_PARTIAL && a.state_in != nullptr;
  const int tsl = tid >> 2, tpart = tid & 3;
  const int tcol = colidx[tsl];
  const bool tload = test && tcol >= 0 && a.prev_partial != nullptr;
  int st0 = NPHASE, ar0 = 0;
  float wcap = INFINITY, dsc = 1.0f, gfl = 0.0f;
  float tv[TP][NPART];
  if (test) {
    // unconditional loads from clamped addresses (values masked when
    // summed); an absent per-instance array reads a stand-in (the partial
    // sums, at least 2N long) whose value is replaced after the K loop, so
    // that no load result is consumed (and waited for) before the K loop
    const float* pp = a.prev_partial ? a.prev_partial : a.partial;
    const int cc = tcol >= 0 ? tcol : 0;
    st0 = a.state_in[cc];
    ar0 = (a.arith_in ? a.arith_in : a.state_in)[cc];
    wcap = (a.wcap2 ? a.wcap2 : pp)[cc];
    dsc = (a.dscale2 ? a.dscale2 : pp)[2 * cc];
    gfl = (a.dscale2 ? a.dscale2 : pp)[2 * cc + 1];
#pragma unroll
    for (int i = 0; i < TP; ++i) {
      const int t = min(tpart + 4 * i, RTP - 1);
#pragma unroll
      for (int q = 0; q < NPART; ++q) tv[i][q] = pp[(long)(t * NPART + q) * a.ldp + cc];
    }
  }

  f4 acc[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = f4{0.f, 0.f, 0.f, 0.f};
  // DALM: the epilogue's state loads are issued here, so that their memory
  // round trip overlaps the K loop instead of following it (measured on the
  // 1200 x 700 cross-and-bouquet batch of 512: epilogue 5.6 -> 3.9 us per
  // launch); the K loop's waits cover them, being younger
  f4 pre_c[2][2], pre_w[2][2], pre_v[2][2], pre_r[2][2];
  if (EPI == EPI_DALM && FAM == 0) {
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1, ec = lane >> 2, eg = lane & 3;
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      const int cc = colidx[wn * 32 + bj * 16 + ec];
      const long cb = (long)(cc >= 0 ? cc : 0) * a.lds;   // idle slots read column 0, never stored
#pragma unroll
      for (int bi = 0; bi < 2; ++bi) {
        const long idx = cb + a.row_off + i0 + wm * 32 + bi * 16 + 4 * eg;
        pre_c[bi][bj] = *reinterpret_cast<const f4*>(a.C + idx);
        pre_w[bi][bj] = *reinterpret_cast<const f4*>(a.W + idx);
        pre_v[bi][bj] = *reinterpret_cast<const f4*>(a.V + idx);
        pre_r[bi][bj] = a.Wref ? *reinterpret_cast<const f4*>(a.Wref + idx) : f4{0.f, 0.f, 0.f, 0.f};
      }
    }
  }
  {
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1, ec = lane >> 2, eg = lane & 3;
    if (EPI != EPI_PARTIAL && a.ws) {
      // split-K reduction: sum the parts in a fixed order (stored in the
      // epilogue's lane layout)
      for (int sp = 0; sp < a.ksplit; ++sp)
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj) {
            const long o = ((long)sp * a.ws_slots + slot0 + wn * 32 + bj * 16 + ec) * a.M +
                           i0 + wm * 32 + bi * 16 + 4 * eg;
            acc[bi][bj] += *reinterpret_cast<const f4*>(a.ws + o);
          }
    } else {
      const int nk64 = a.K / 64;
      const int kb = (split * nk64) / ks, ke = ((split + 1) * nk64) / ks;
      // slices in flight per arithmetic, from a sweep of 2..8 on the
      // 1200 x 700 cross-and-bouquet operator (deeper split-BF16 prefetch
      // makes the compiler serialise the loads)
      if (FAM == 0 && (prec == PREC_F32 || (EPI == EPI_REFRESH))) mainloop_f32<8>(a, i0, colidx, lds, acc, kb, ke);
      else if (prec == PREC_BF16X3) mainloop_bf16<true, FAM == 1 ? 2 : 3>(a, i0, colidx, lds, acc, kb, ke);
      else mainloop_bf16<false, 4>(a, i0, colidx, lds, acc, kb, ke);
      // from the MFMA layout (lane li + 16 q: column li, rows 4q..4q+3 of a
      // 16 x 16 block) to the epilogue's (lane 4 c + g: column c, rows
      // 4g..4g+3), so that four consecutive lanes move 64 contiguous bytes of
      // one column instead of 16 bytes of four columns
      const int src = ((lane >> 2) + 16 * (lane & 3)) << 2;
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            acc[bi][bj][r] = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(acc[bi][bj][r])));
    }
    if (EPI == EPI_PARTIAL) {
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
          const long o = ((long)split * a.ws_slots + slot0 + wn * 32 + bj * 16 + ec) * a.M +
                         i0 + wm * 32 + bi * 16 + 4 * eg;
          *reinterpret_cast<f4*>(a.ws + o) = acc[bi][bj];
        }
      return;
    }
  }

  if (test) {
    // the loaded values enter the arithmetic only here: the empty asm keeps
    // the compiler from starting the sums (and so waiting for the loads)
    // before the K loop
    asm volatile("" : "+v"(st0));
    asm volatile("" : "+v"(ar0));
    asm volatile("" : "+v"(wcap));
    asm volatile("" : "+v"(dsc));
    asm volatile("" : "+v"(gfl));
#pragma unroll
    for (int i = 0; i < TP; ++i)
#pragma unroll
      for (int q = 0; q < NPART; ++q) asm volatile("" : "+v"(tv[i][q]));
    if (!a.arith_in) ar0 = NPHASE;
    if (!a.wcap2) wcap = INFINITY;
    if (!a.dscale2) {
      dsc = 1.0f;
      gfl = 0.0f;
    }
    float sm[NPART];
#pragma unroll
    for (int q = 0; q < NPART; ++q) sm[q] = 0.0f;
    const bool live0 = tcol >= 0 && st0 < NPHASE;
    if (tload && live0) {
#pragma unroll
      for (int i = 0; i < TP; ++i)
        if (tpart + 4 * i < RTP) {
#pragma unroll
          for (int q = 0; q < NPART; ++q) sm[q] += tv[i][q];
        }
      for (int t = tpart + 4 * TP; t < RTP; t += 4) {
        const float* pt = a.prev_partial + (long)t * NPART * a.ldp + tcol;
#pragma unroll
        for (int q = 0; q < NPART; ++q) sm[q] += pt[(long)q * a.ldp];
      }
    }
#pragma unroll
    for (int q = 0; q < NPART; ++q) {
      sm[q] += __shfl_xor(sm[q], 1);
      sm[q] += __shfl_xor(sm[q], 2);
    }
    int st = live0 ? st0 : NPHASE, stat_new = L1_MAXITER;
    float zs = 1.0f;
    if (live0 && a.prev_partial && a.test_kind == 1) {
      // FISTA inner loop: stop on the relative change of the shrink output
      const float t = a.tp_tol;
      if (!(isfinite(sm[0]) && isfinite(sm[1]))) st = NPHASE;
      else if (t >= 0.0f && sm[0] <= t * t * sm[1]) st = NPHASE;
    } else if (live0 && a.prev_partial) {
      TestParams tp;
      tp.tol = a.tp_tol;
      tp.sw = a.tp_sw;
      tp.final_phase = a.tp_final;
      tp.wcap2 = wcap;
      tp.dscale2 = dsc;
      tp.gfloor = gfl;
#pragma unroll
      for (int q = 0; q < NPHASE; ++q) tp.floor[q] = a.tp_floor[q];
      st = decide_in(tp, st0, ar0, sm, &stat_new);
      if (a.eps) zs = ball_scale(sm[4], a.eps[tcol], a.beta[tcol]);
    } else if (live0 && a.eps) {
      zs = a.zscale[tcol];
    }
    __syncthreads();  // the K loop has read colidx
    if (tpart == 0 && tcol >= 0) {
      if (st < NPHASE) {
        s_zsc[tsl] = zs;
        atomicAdd(&s_live, 1);
      } else {
        colidx[tsl] = -1;
      }
      if (rt == 0 && !a.test_passive) {
        a.state_out[tcol] = st;
        if (a.arith_out && st < NPHASE) a.arith_out[tcol] = prec;
        if (live0) {
          if (st >= NPHASE) {
            if (a.status) a.status[tcol] = stat_new;
          } else {
            a.iters[tcol] += 1;
          }
        }
      }
    }
    __syncthreads();
    if (s_live == 0) return;  // every column of the tile has finished
    if (rt == 0 && tid == 0 && a.stat && !a.test_passive) {
      atomicAdd((unsigned long long*)&a.stat[3 + prec], (unsigned long long)s_live);
      atomicAdd((unsigned long long*)&a.stat[prec], 1ull);
      if (a.ldt > 0) atomicAdd((unsigned long long*)&a.stat[6], (unsigned long long)s_live);
    }
  }

  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1, ec = lane >> 2, eg = lane & 3;
  // ---- epilogue ----------------------------------------------------------
  // accumulator (bi, bj), register r of lane 4 c + g: row
  // i0 + wm*32 + bi*16 + 4g + r, column slot wn*32 + bj*16 + c
  if (EPI == EPI_STORE) {
    if (a.Tq_hi && prec != PREC_F32) {
      // the first product of the dense structured form: t in the BF16 hi /
      // lo split the second product of a BF16 tile reads (all rows)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        const int col = colidx[wn * 32 + bj * 16 + ec];
        if (col < 0) continue;
#pragma unroll
        for (int bi = 0; bi < 2; ++bi) {
          us4 h, l;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const uint16_t hb = f2bf(acc[bi][bj][r]);
            h[r] = hb;
            l[r] = f2bf(acc[bi][bj][r] - bf2f(hb));
          }
          const long tix = (long)col * a.ldo + i0 + wm * 32 + bi * 16 + 4 * eg;
          *reinterpret_cast<us4*>(a.Tq_hi + tix) = h;
          *reinterpret_cast<us4*>(a.Tq_lo + tix) = l;
        }
      }
      return;
    }
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      const int col = colidx[wn * 32 + bj * 16 + ec];
      if (col < 0) continue;
      const float sc = a.col_scale ? a.col_scale[col] : 1.0f;
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = i0 + wm * 32 + bi * 16 + 4 * eg + r;
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
    const int col = colidx[wn * 32 + bj * 16 + ec];
    if (col < 0) continue;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
      const int row0 = i0 + wm * 32 + bi * 16 + 4 * eg;   // output row
      const int srow = a.row_off + row0;                  // state row
      const long idx = (long)col * a.lds + srow;
      const bool pre = EPI == EPI_DALM && FAM == 0;
      const f4 c4 = pre ? pre_c[bi][bj] : *reinterpret_cast<const f4*>(a.C + idx);
      const f4 wo = pre ? pre_w[bi][bj] : *reinterpret_cast<const f4*>(a.W + idx);
      f4 wn4, un4;
      if (EPI == EPI_REFRESH) {
        // w_ref = w, c_ref = (C0 - P w) / beta, and the next operand
        // u = clamp(v + w/beta) - (w - w_ref)/beta = clamp(v + w/beta)
        const float ib = 1.0f / a.beta[col];
        const f4 c0 = *reinterpret_cast<const f4*>(a.C0 + idx);
        const f4 vo = *reinterpret_cast<const f4*>(a.V + idx);
        f4 cr4;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          cr4[r] = (c0[r] - acc[bi][bj][r]) * ib;
          un4[r] = clamp1(vo[r] + wo[r] * ib);
        }
        *reinterpret_cast<f4*>(const_cast<float*>(a.C) + idx) = cr4;
        *reinterpret_cast<f4*>(a.Wref + idx) = wo;
        if (prec == PREC_F32 || !a.Uhi) *reinterpret_cast<f4*>(a.U + idx) = un4;
        if (a.Uhi && prec != PREC_F32) {
          us4 h, l;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const uint16_t hb = f2bf(un4[r]);
            h[r] = hb;
            l[r] = f2bf(un4[r] - bf2f(hb));
          }
          *reinterpret_cast<us4*>(a.Uhi + idx) = h;
          *reinterpret_cast<us4*>(a.Ulo + idx) = l;
        }
        continue;
      } else if (EPI == EPI_DALM) {
        const float bt = a.beta[col];
        const float ib = 1.0f / bt;
        const float zsc = s_zsc[wn * 32 + bj * 16 + ec];
        const f4 vo = pre ? pre_v[bi][bj] : *reinterpret_cast<const f4*>(a.V + idx);
        const f4 wr4 = pre ? pre_r[bi][bj]
                           : (a.Wref ? *reinterpret_cast<const f4*>(a.Wref + idx) : f4{0.f, 0.f, 0.f, 0.f});
        // structured form: the operand the product multiplied, in the
        // tile's arithmetic (BF16: hi; split: hi + lo; FP32: u)
        f4 ut = {0.f, 0.f, 0.f, 0.f};
        if (a.add_u || a.q_rows > 0) {
          if (prec == PREC_F32 || !a.Ucur_hi) {
            ut = *reinterpret_cast<const f4*>(a.Ucur + idx);
          } else {
            const us4 h = *reinterpret_cast<const us4*>(a.Ucur_hi + idx);
            const us4 l = *reinterpret_cast<const us4*>(a.Ucur_lo + idx);
#pragma unroll
            for (int r = 0; r < 4; ++r) ut[r] = bf2f(h[r]) + (prec == PREC_BF16X3 ? bf2f(l[r]) : 0.0f);
          }
        }
        if (a.q_rows > 0) {
          // q = u - (P u) on the first rows (K^{-1} (u_x - B^T u_e)), 0 below
          f4 q4;
#pragma unroll
          for (int r = 0; r < 4; ++r) q4[r] = (srow + r < a.q_rows) ? ut[r] - acc[bi][bj][r] : 0.0f;
          const long tix = (long)col * a.ldt + row0;
          if (prec == PREC_F32 || !a.Tq_hi) {
            *reinterpret_cast<f4*>(a.Tq + tix) = q4;
          } else {
            us4 h, l;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const uint16_t hb = f2bf(q4[r]);
              h[r] = hb;
              l[r] = f2bf(q4[r] - bf2f(hb));
            }
            *reinterpret_cast<us4*>(a.Tq_hi + tix) = h;
            *reinterpret_cast<us4*>(a.Tq_lo + tix) = l;
          }
        }
        f4 vn4;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = srow + r;
          const bool ball = row >= a.e0;   // eps-ball block of the P_{1,2} splitting
          const float s = vo[r] + wo[r] * ib;
          const float z = ball ? s * zsc : clamp1(s);
          const float vn = acc[bi][bj][r] + c4[r] + (a.add_u ? ut[r] : 0.0f);
          const float wn = wo[r] - bt * (z - vn);
          const float s2 = vn + wn * ib;
          const float z2 = ball ? s2 : clamp1(s2);  // ball rows: scaled after the column norm
          vn4[r] = vn;
          wn4[r] = wn;
          un4[r] = z2 - (wn - wr4[r]) * ib;
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
        // the next product reads u in the tile's arithmetic family (a phase
        // group never moves between the BF16 forms and FP32)
        if (prec == PREC_F32 || !a.Uhi) *reinterpret_cast<f4*>(a.U + idx) = un4;
        if (a.Uhi && prec != PREC_F32) {
          us4 h, l;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const uint16_t hb = f2bf(un4[r]);
            h[r] = hb;
            l[r] = f2bf(un4[r] - bf2f(hb));
          }
          *reinterpret_cast<us4*>(a.Uhi + idx) = h;
          *reinterpret_cast<us4*>(a.Ulo + idx) = l;
        }
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
        if (a.Uhi) {
          us4 h, l;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const uint16_t hb = f2bf(un4[r]);
            h[r] = hb;
            l[r] = f2bf(un4[r] - bf2f(hb));
          }
          *reinterpret_cast<us4*>(a.Uhi + idx) = h;
          *reinterpret_cast<us4*>(a.Ulo + idx) = l;
        }
      }
      *reinterpret_cast<f4*>(a.W + idx) = wn4;
    }
  }
  if (EPI == EPI_REFRESH) return;   // the partial sums of the last iteration stay
  // reduce the partial sums over the 4 lanes of each column ...
#pragma unroll
  for (int bj = 0; bj < 2; ++bj)
#pragma unroll
    for (int p = 0; p < NPART; ++p) {
      float v = part[bj][p];
      v += __shfl_xor(v, 1);
      v += __shfl_xor(v, 2);
      part[bj][p] = v;
    }
  // ... and over the two waves that share the columns, in a fixed order
  if (eg == 0) {
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int p = 0; p < NPART; ++p) red[wm][wn * 32 + bj * 16 + ec][p] = part[bj][p];
  }
  __syncthreads();
  if (tid < 64) {
    const int col = colidx[tid];
    if (col >= 0) {
#pragma unroll
      for (int p = 0; p < NPART; ++p)
        a.partial[(long)((rt + pt0) * NPART + p) * a.ldp + col] = red[0][tid][p] + red[1][tid][p];
    }
  }
}

void launch_gemm(hipStream_t s, int epi, const GemmArgs& a0, int n_col_tiles) {
  if (n_col_tiles <= 0 || a0.M <= 0) return;
  GemmArgs a = a0;
  a.n_ctiles = n_col_tiles;
  if (a.ksplit < 1) a.ksplit = 1;
  const int ks = (epi == EPI_PARTIAL) ? a.ksplit : 1;
  const int RT = a.M / 64;
  const int per_xcd = (RT + 7) / 8;
  const unsigned grid = 8u * per_xcd * n_col_tiles * ks;
  // the two stage buffers exceed the default dynamic LDS limit: raise it once
  static const bool lds_ok = [] {
    bool ok = true;
    for (const void* f : {reinterpret_cast<const void*>(gemm_kernel<EPI_STORE>),
                          reinterpret_cast<const void*>(gemm_kernel<EPI_DALM>),
                          reinterpret_cast<const void*>(gemm_kernel<EPI_FISTA>),
                          reinterpret_cast<const void*>(gemm_kernel<EPI_PARTIAL>),
                          reinterpret_cast<const void*>(gemm_kernel<EPI_REFRESH>),
                          reinterpret_cast<const void*>(gemm_kernel<EPI_DALM, 1>),
                          reinterpret_cast<const void*>(gemm_kernel<EPI_PARTIAL, 1>)})
      ok = ok && hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, GEMM_LDS) ==
                     hipSuccess;
    return ok;
  }();
  L1_REQUIRE(lds_ok, "cannot give the iteration GEMM its LDS stages");
  const bool fam1 = a.fam == 1 && (epi == EPI_DALM || epi == EPI_PARTIAL);
  if (fam1 && epi == EPI_DALM) gemm_kernel<EPI_DALM, 1><<<grid, 256, GEMM_LDS, s>>>(a);
  else if (fam1) gemm_kernel<EPI_PARTIAL, 1><<<grid, 256, GEMM_LDS, s>>>(a);
  else if (epi == EPI_STORE) gemm_kernel<EPI_STORE><<<grid, 256, GEMM_LDS, s>>>(a);
  else if (epi == EPI_DALM) gemm_kernel<EPI_DALM><<<grid, 256, GEMM_LDS, s>>>(a);
  else if (epi == EPI_FISTA) gemm_kernel<EPI_FISTA><<<grid, 256, GEMM_LDS, s>>>(a);
  else if (epi == EPI_REFRESH) gemm_kernel<EPI_REFRESH><<<grid, 256, GEMM_LDS, s>>>(a);
  else gemm_kernel<EPI_PARTIAL><<<grid, 256, GEMM_LDS, s>>>(a);
  L1_HIP(hipGetLastError());
}

void launch_product(hipStream_t s, int epi, GemmArgs a, int n_col_tiles, int ksplit) {
  if (ksplit > 1 && a.ws) {
    a.ksplit = ksplit;
    a.ws_slots = n_col_tiles * TILE;
    launch_gemm(s, EPI_PARTIAL, a, n_col_tiles);
    launch_gemm(s, epi, a, n_col_tiles);
  } else {
    a.ksplit = 1;
    a.ws = nullptr;
    launch_gemm(s, epi, a, n_col_tiles);
  }
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
