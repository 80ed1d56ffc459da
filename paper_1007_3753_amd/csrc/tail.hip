// The DALM tail kernel.
//
// When only a few instances are left, an iteration of the launch-per-
// iteration path costs the kernel boundaries and the latency of one short
// K chain, whatever the work.  This kernel runs the remaining iterations of
// up to TAIL_NC instances in one cooperative launch:
//   - workgroup g owns operator rows [16 g, 16 g + 16), held in registers,
//     and the matching entries of v and w of every listed instance, also in
//     registers, for the whole launch;
//   - per iteration it stages the B operand u (all rows, listed instances)
//     in LDS, computes its 16 x 16 block of P u with the K range split as the
//     iteration GEMM splits it (MFMA, parts added in a fixed order), applies
//     the dual ALM update of Algorithm 2 (the same arithmetic as the epilogue
//     of the iteration GEMM), and publishes its rows of the next u and its
//     partial sums; the next iteration starts with the convergence test of
//     this one (every workgroup computes it from the same sums, so all take
//     the same decisions and leave at the same iteration).
// Exchange without a grid barrier: every published 32-bit value travels in
// one 64-bit word with a tag, the index of the iteration that consumes it
// plus one, written and read as single 64-bit agent-scope atomics (which the
// memory system keeps coherent across the XCDs' L2 caches).  A consumer
// polls until every word it needs carries the tag it expects, so the data
// and its readiness arrive in the same memory round trip.  Two buffers by
// iteration parity make the reuse safe: a workgroup can write the buffer of
// iteration k + 1 only after it has read every row of iteration k, which the
// other workgroups publish only after they have finished reading iteration
// k - 1 from that same buffer.  The exchange memory is cleared before every
// launch, so no stale tag can match.  Every wait is bounded: a workgroup that
// gives up raises a flag that ends the others' waits too.
#include <algorithm>
#include <mutex>

#include "region_list.h"
#include "tail.h"

namespace l1 {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

__device__ inline uint16_t f2bf_t(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf2f_t(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
__device__ inline float clamp1_t(float x) { return fminf(fmaxf(x, -1.0f), 1.0f); }
__device__ inline u4 ld16(const void* p) { return *reinterpret_cast<const u4*>(p); }

__device__ inline unsigned long long ld8c(const void* p) {
  return __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline u4 ld16c(const void* p) {
  const unsigned long long a = ld8c(p);
  const unsigned long long b = ld8c(reinterpret_cast<const char*>(p) + 8);
  return u4{(unsigned)a, (unsigned)(a >> 32), (unsigned)b, (unsigned)(b >> 32)};
}
__device__ inline float ldfc(const float* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void stfc(float* p, float v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// staged u: column j of the f32 stage at j * ldu32 floats, of the split
// stage at j * ldu16 bf16 (hi) and (ncap + j) * ldu16 (lo); the row padding
// spreads the 16 lanes of one fragment read over distinct banks
__device__ inline int ldu32(int n_pad) { return n_pad + 4; }
__device__ inline int ldu16(int n_pad) { return n_pad + 8; }

__device__ inline unsigned long long tagged(uint32_t v, unsigned tag) {
  return (unsigned long long)v | ((unsigned long long)tag << 32);
}
__device__ inline void st8c(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// polls of one wait before a workgroup gives up (each after a short sleep)
constexpr unsigned TAIL_SPIN_LIMIT = 1u << 20;

}  // namespace

template <bool F32>
__global__ __launch_bounds__(256) void dalm_tail_kernel(TailArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char ustage[];
  __shared__ int s_col[TAIL_NC], s_st[TAIL_NC], s_nc, s_live;
  __shared__ float s_red[8][16][17];
  __shared__ float s_ps[NPART][16][TAIL_NC];
  __shared__ float s_ts[TAIL_NC][16][NPART];
  // the partial sums of the previous iteration, [instance][sum][row group]
  __shared__ float s_pp[TAIL_NC][NPART][16 * TAIL_TG];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, q = lane >> 4;
  const int g = blockIdx.x, G = gridDim.x;
  const int r0 = g * TAIL_ROWS;
  const int n_pad = a.n_pad, ncap = a.ncap;

  // the listed unfinished instances, in slot order (the same in every workgroup)
  if (tid == 0) {
    int nc = 0;
    const int* st_in = a.st[a.k0 & 1];
    for (int sl = 0; sl < a.phase_off[NPHASE] && nc < ncap; ++sl) {
      const int col = a.slot_col[sl];
      if (col >= 0 && st_in[col] < NPHASE) {
        s_col[nc] = col;
        s_st[nc] = st_in[col];
        ++nc;
      }
    }
    // the products of one launch use one arithmetic: that of the final phase
    for (int j = 0; j < nc; ++j)
      if (s_st[j] != a.tp.final_phase) nc = 0;
    s_nc = nc;
  }
  __syncthreads();
  const int nc = s_nc;
  if (nc == 0) {
    if (g == 0 && tid == 0) a.flag[1] = a.k0;   // declined: nothing done
    return;
  }
  // stage columns the instances do not use stay zero
  {
    const long words = F32 ? (long)ncap * ldu32(n_pad) : (long)ncap * ldu16(n_pad);  // 4-byte words
    for (long e = tid; e < words; e += 256) reinterpret_cast<float*>(ustage)[e] = 0.0f;
  }

  // ---- operator rows of this workgroup, in registers for the whole launch ----
  // The K range is split exactly as the launch-per-iteration path splits it
  // for this many instances (a.ks parts in 64-element units, each summed in
  // the order of the iteration GEMM's main loop, then added in part order),
  // so both paths produce the same bits.  Wave w computes parts w and w + 4;
  // its 64-element units are listed in order, part w first.
  const int nk64 = n_pad / 64, row = r0 + li;
  const int pa = wave, pb = wave + 4;
  const int kba = (pa * nk64) / a.ks, kea = pa < a.ks ? ((pa + 1) * nk64) / a.ks : kba;
  const int kbb = pb < a.ks ? (pb * nk64) / a.ks : 0, keb = pb < a.ks ? ((pb + 1) * nk64) / a.ks : 0;
  const int nua = kea - kba, nu = nua + (keb - kbb);
  // per 64-element unit, lane (li, q): FP32 - four 16-element steps (k = 4q..4q+3
  // of each); split BF16 - two 32-element steps (k = 8q..8q+7), hi and lo
  u4 areg[TAIL_MAXU][4];
#pragma unroll
  for (int u = 0; u < TAIL_MAXU; ++u) {
    if (u < nu) {
      const int unit = u < nua ? kba + u : kbb + (u - nua);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (F32) {
          areg[u][t] = ld16(a.P32 + (long)row * n_pad + unit * 64 + t * 16 + q * 4);
        } else {
          const uint16_t* base = (t & 1) ? a.Plo : a.Phi;
          areg[u][t] = ld16(base + (long)row * n_pad + unit * 64 + (t >> 1) * 32 + q * 8);
        }
      }
    }
  }
  // v and w of (row r0 + tid / 16, listed instance tid % 16), in registers
  const int er = tid >> 4, ej = tid & 15;
  const bool eown = ej < nc;
  const long eidx = eown ? (long)s_col[ej] * a.lds + r0 + er : 0;
  float vreg = eown ? a.V[eidx] : 0.0f, wreg = eown ? a.W[eidx] : 0.0f;
  const float creg = eown ? a.C[eidx] : 0.0f;
  const float wref = (eown && a.Wref) ? a.Wref[eidx] : 0.0f;
  const float bt = eown ? a.beta[s_col[ej]] : 1.0f;
  const float ib = 1.0f / bt;

  __shared__ int s_gaveup;
  if (tid == 0) s_gaveup = 0;
  int k = a.k0;
  for (;; ++k) {
    const bool first = (k == a.k0);
    const unsigned want = (unsigned)k + 1u;   // tag of the words iteration k consumes
    // ---- loads: u of iteration k and the partial sums of iteration k - 1 ------
    // every load of the phase is issued before the first is used (one memory
    // round trip when the data is ready): a thread moves at most TAIL_UV
    // 16-byte vectors of u and sums at most TAIL_TG groups of partial sums.
    // Only instances still running published u (the others' columns of the
    // stage keep stale values whose products are never used).
    const int tj = tid >> 4, sub = tid & 15;
    {
      // 16-byte vectors per instance: the launch path's FP32 or hi / lo
      // split layout (4 values), or two tagged words (2 values); staged in
      // rounds of TAIL_UR vectors per thread (registers), the partial sums
      // with the first round
      const int nv = first ? n_pad / 4 : n_pad / 2;
      const int nvec = nc * nv;
      const int nt = first ? a.ntiles : G;
      const unsigned long long* xu = a.xu[k & 1];
      const unsigned long long* xp = a.xpart[(k - 1) & 1];
      auto u_src_ok = [&](int e) { return e < nvec && s_st[e / nv] < NPHASE; };
      auto load_u = [&](int e) -> u4 {
        const int j = e / nv, w = e % nv;
        if (F32 && first) return ld16(a.U32 + (long)s_col[j] * a.lds + w * 4);
        if (first) {
          // the launch path's split: the first half of an instance's
          // vectors are hi, the second lo
          const int hl = w >= nv / 2, w8 = (w - hl * (nv / 2)) * 8;
          return ld16((hl ? a.Ulo : a.Uhi) + (long)s_col[j] * a.lds + w8);
        }
        return ld16c(xu + (long)j * n_pad + w * 2);
      };
      // partial sums: element f = (j NPART + p) 128 + t of [instance j][sum
      // p][row group t], TAIL_PR per thread, spread over the workgroup
      constexpr int PT = 16 * TAIL_TG;
      auto p_ok = [&](int f) {
        const int t = f % PT, jp = f / PT, j = jp / NPART;
        return j < nc && s_st[j] < NPHASE && t < nt;
      };
      auto p_addr = [&](int f) -> long {
        const int t = f % PT, jp = f / PT, j = jp / NPART, p = jp % NPART;
        return ((long)t * NPART + p) * TAIL_NC + j;
      };
      float pv[TAIL_PR];
      unsigned pstale = 0;   // partial sums still carrying an old tag
#pragma unroll
      for (int round = 0; round < TAIL_UV / TAIL_UR; ++round) {
        if (round > 0 && 256 * TAIL_UR * round >= nvec) break;
        u4 uv[TAIL_UR];
        unsigned ustale = 0;
#pragma unroll
        for (int i = 0; i < TAIL_UR; ++i) {
          const int e = tid + 256 * (TAIL_UR * round + i);
          if (u_src_ok(e)) uv[i] = load_u(e);
        }
        if (round == 0) {
#pragma unroll
          for (int i = 0; i < TAIL_PR; ++i) {
            const int f = tid + 256 * i;
            pv[i] = 0.0f;
            if (p_ok(f)) {
              if (first) {
                const int t = f % PT, jp = f / PT;
                pv[i] = a.reg_partial[((long)t * NPART + jp % NPART) * a.ldp + s_col[jp / NPART]];
              } else {
                const unsigned long long v = ld8c(xp + p_addr(f));
                pv[i] = __uint_as_float((uint32_t)v);
                if ((unsigned)(v >> 32) != want) pstale |= 1u << i;
              }
            }
          }
        }
        if (!first) {
#pragma unroll
          for (int i = 0; i < TAIL_UR; ++i) {
            const int e = tid + 256 * (TAIL_UR * round + i);
            if (u_src_ok(e) && (uv[i][1] != want || uv[i][3] != want)) ustale |= 1u << i;
          }
          // poll until every word this thread needs carries the expected tag
          unsigned spins = 0;
          while (ustale | pstale) {
            if (++spins > TAIL_SPIN_LIMIT ||
                __hip_atomic_load(a.flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
              atomicExch(a.flag, 1);
              s_gaveup = 1;
              break;
            }
            __builtin_amdgcn_s_sleep(1);
#pragma unroll
            for (int i = 0; i < TAIL_UR; ++i) {
              if (ustale & (1u << i)) {
                uv[i] = load_u(tid + 256 * (TAIL_UR * round + i));
                if (uv[i][1] == want && uv[i][3] == want) ustale &= ~(1u << i);
              }
            }
#pragma unroll
            for (int i = 0; i < TAIL_PR; ++i)
              if (pstale & (1u << i)) {
                const unsigned long long v = ld8c(xp + p_addr(tid + 256 * i));
                pv[i] = __uint_as_float((uint32_t)v);
                if ((unsigned)(v >> 32) == want) pstale &= ~(1u << i);
              }
          }
          if (ustale | pstale) break;   // gave up
        }
#pragma unroll
        for (int i = 0; i < TAIL_UR; ++i) {
          const int e = tid + 256 * (TAIL_UR * round + i);
          if (!u_src_ok(e)) continue;
          const int j = e / nv, w = e % nv;
          if (first) {
            if (F32) {
              *reinterpret_cast<u4*>(reinterpret_cast<float*>(ustage) + (long)j * ldu32(n_pad) + w * 4) = uv[i];
            } else {
              const int hl = w >= nv / 2, w8 = (w - hl * (nv / 2)) * 8;
              uint16_t* sh = reinterpret_cast<uint16_t*>(ustage) + (long)(hl * ncap + j) * ldu16(n_pad);
              *reinterpret_cast<u4*>(sh + w8) = uv[i];
            }
          } else if (F32) {
            // two tagged FP32 values: elements 2w, 2w + 1
            typedef unsigned int u2 __attribute__((ext_vector_type(2)));
            *reinterpret_cast<u2*>(reinterpret_cast<float*>(ustage) + (long)j * ldu32(n_pad) + w * 2) =
                u2{uv[i][0], uv[i][2]};
          } else {
            // two tagged (hi | lo << 16) words: the hi pair and the lo pair
            // of elements 2w, 2w + 1
            const uint32_t hi = (uv[i][0] & 0xffffu) | (uv[i][2] << 16);
            const uint32_t lo = (uv[i][0] >> 16) | (uv[i][2] & 0xffff0000u);
            uint16_t* sh = reinterpret_cast<uint16_t*>(ustage) + (long)j * ldu16(n_pad) + w * 2;
            *reinterpret_cast<uint32_t*>(sh) = hi;
            *reinterpret_cast<uint32_t*>(sh + (long)ncap * ldu16(n_pad)) = lo;
          }
        }
      }
#pragma unroll
      for (int i = 0; i < TAIL_PR; ++i) {
        const int f = tid + 256 * i;
        const int t = f % PT, jp = f / PT;
        if (jp < nc * NPART) s_pp[jp / NPART][jp % NPART][t] = pv[i];
      }
    }
    __syncthreads();
    if (s_gaveup) return;
    // per instance and sum, 16 threads add the row groups t = sub + 16 i
    {
      const bool tlive = tj < nc && s_st[tj] < NPHASE;
#pragma unroll
      for (int p = 0; p < NPART; ++p) {
        float v = 0.0f;
        if (tlive) {
#pragma unroll
          for (int i = 0; i < TAIL_TG; ++i) v += s_pp[tj][p][sub + 16 * i];
        }
        s_ts[tj][sub][p] = v;
      }
    }
    __syncthreads();
    if (s_gaveup) return;

    // ---- convergence test of iteration k - 1 (the same in every workgroup) ----
    if (tid < TAIL_NC) {
      const int j = tid;
      if (j < nc && s_st[j] < NPHASE) {
        float sm[NPART];
#pragma unroll
        for (int p = 0; p < NPART; ++p) {
          float v = 0.0f;
          for (int t = 0; t < 16; ++t) v += s_ts[j][t][p];
          sm[p] = v;
        }
        int stat_new = L1_MAXITER;
        // the first sums come from the launch-per-iteration path, whose
        // product may have run in a lower arithmetic than the final phase
        const int ar = (first && a.reg_arith) ? a.reg_arith[s_col[j]] : NPHASE;
        TestParams tp = a.tp;
        tp.wcap2 = a.wcap2 ? a.wcap2[s_col[j]] : INFINITY;
        tp.dscale2 = a.dscale2 ? a.dscale2[2 * s_col[j]] : 1.0f;
        tp.gfloor = a.dscale2 ? a.dscale2[2 * s_col[j] + 1] : 0.0f;
        const int st = decide_in(tp, s_st[j], ar, sm, &stat_new);
        if (g == 0) {
          if (st >= NPHASE) a.status[s_col[j]] = stat_new;
          else if (k < a.k_end) a.iters[s_col[j]] += 1;
        }
        s_st[j] = st;
      }
    }
    __syncthreads();
    if (tid == 0) {
      int live = 0;
      for (int j = 0; j < nc; ++j) live += (s_st[j] < NPHASE) ? 1 : 0;
      s_live = live;
      if (g == 0 && live && k < a.k_end && a.stat) {
        const int pc = F32 ? PREC_F32 : PREC_BF16X3;
        atomicAdd((unsigned long long*)&a.stat[3 + pc], (unsigned long long)live);
        atomicAdd((unsigned long long*)&a.stat[pc], 1ull);
      }
    }
    __syncthreads();
    if (s_live == 0 || k >= a.k_end) break;

    // ---- this workgroup's 16 x 16 block of P u -----------------------------------
    {
      const bool colok = li < ncap;
      f4 acca = {0.f, 0.f, 0.f, 0.f}, accb = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int u = 0; u < TAIL_MAXU; ++u) {
        if (u < nu) {
          const int unit = u < nua ? kba + u : kbb + (u - nua);
          f4 acc = u < nua ? acca : accb;
          if (F32) {
            const float* Br = reinterpret_cast<const float*>(ustage) +
                              (long)(colok ? li : 0) * ldu32(n_pad) + unit * 64 + q * 4;
#pragma unroll
            for (int st = 0; st < 4; ++st) {
              const u4 av = areg[u][st];
              const u4 bv = colok ? ld16(Br + st * 16) : u4{0u, 0u, 0u, 0u};
#pragma unroll
              for (int t = 0; t < 4; ++t)
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(av[t]),
                                                            __uint_as_float(bv[t]), acc, 0, 0, 0);
            }
          } else {
            const int ld = ldu16(n_pad);
            const uint16_t* Bh = reinterpret_cast<const uint16_t*>(ustage) + (long)(colok ? li : 0) * ld +
                                 unit * 64 + q * 8;
            const uint16_t* Bl = Bh + (long)ncap * ld;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const bf8 ah = __builtin_bit_cast(bf8, areg[u][2 * h]);
              const bf8 al = __builtin_bit_cast(bf8, areg[u][2 * h + 1]);
              const u4 z4 = {0u, 0u, 0u, 0u};
              const bf8 bh = __builtin_bit_cast(bf8, colok ? ld16(Bh + h * 32) : z4);
              const bf8 bl = __builtin_bit_cast(bf8, colok ? ld16(Bl + h * 32) : z4);
              // small terms first, as in the iteration GEMM
              acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
              acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
              acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
            }
          }
          if (u < nua) acca = acc;
          else accb = acc;
        }
      }
      // accumulator register r of lane (li, q): row 4q + r, column li
      if (pa < a.ks) {
#pragma unroll
        for (int r = 0; r < 4; ++r) s_red[pa][4 * q + r][li] = acca[r];
      }
      if (pb < a.ks) {
#pragma unroll
        for (int r = 0; r < 4; ++r) s_red[pb][4 * q + r][li] = accb[r];
      }
    }
    __syncthreads();

    // ---- update of Algorithm 2 for (row r0 + er, listed instance ej) -------------
    {
      float part[NPART] = {0.f, 0.f, 0.f, 0.f, 0.f};
      if (eown && s_st[ej] < NPHASE) {
        float pu = s_red[0][er][ej];
        for (int sp = 1; sp < a.ks; ++sp) pu += s_red[sp][er][ej];
        const int rw = r0 + er;
        const float vo = vreg, wo = wreg;
        const float s = vo + wo * ib;
        const float z = clamp1_t(s);
        const float vn = pu + creg;
        const float wn = wo - bt * (z - vn);
        const float s2 = vn + wn * ib;
        const float z2 = clamp1_t(s2);
        const float un = z2 - (wn - wref) * ib;
        vreg = vn;
        wreg = wn;
        // the next u, tagged for iteration k + 1
        const long xo = (long)ej * n_pad + rw;
        const unsigned tag = (unsigned)k + 2u;
        if (F32) {
          st8c(a.xu[(k + 1) & 1] + xo, tagged(__float_as_uint(un), tag));
        } else {
          const uint16_t h = f2bf_t(un);
          const uint32_t w = (uint32_t)h | ((uint32_t)f2bf_t(un - bf2f_t(h)) << 16);
          st8c(a.xu[(k + 1) & 1] + xo, tagged(w, tag));
        }
        const float d = wn - wo;
        part[0] = d * d;
        part[1] = wn * wn;
        if (rw < a.n_l1) {
          const float aw = fabsf(wn);
          part[2] = aw;
          part[3] = aw * (1.0f - copysignf(1.0f, wn) * vn);
        }
      }
#pragma unroll
      for (int p = 0; p < NPART; ++p) s_ps[p][er][ej] = part[p];
    }
    __syncthreads();
    if (tid < NPART * TAIL_NC) {
      const int p = tid / TAIL_NC, j = tid % TAIL_NC;
      float sum = 0.0f;
      for (int r = 0; r < 16; ++r) sum += s_ps[p][r][j];
      st8c(a.xpart[k & 1] + ((long)g * NPART + p) * TAIL_NC + j, tagged(__float_as_uint(sum), (unsigned)k + 2u));
    }
  }
  // v and w back to memory; final phases into both buffers; iteration count
  if (eown) {
    a.V[eidx] = vreg;
    a.W[eidx] = wreg;
  }
  if (g == 0) {
    if (tid < nc) {
      a.st[0][s_col[tid]] = s_st[tid];
      a.st[1][s_col[tid]] = s_st[tid];
    }
    if (tid == 0) a.flag[1] = k;
  }
}

int tail_capacity(int n_pad, int f32) {
  const size_t budget = 96 * 1024;    // LDS for the u stage
  const size_t per_col = f32 ? (size_t)(n_pad + 4) * 4 : (size_t)(n_pad + 8) * 2 * 2;
  const size_t by_loads = (size_t)256 * TAIL_UV / (size_t)(n_pad / 2);   // tagged u vectors per thread
  const size_t by_sums = (size_t)256 * TAIL_PR / (size_t)(NPART * 16 * TAIL_TG);  // partial sums per thread
  return (int)std::min<size_t>({(size_t)TAIL_NC, budget / per_col, by_loads, by_sums});
}

bool tail_fits(int n_pad, int ntiles, int ks) {
  const int G = n_pad / TAIL_ROWS;
  const int nk64 = n_pad / 64;
  if (ks < 1 || ks > 8) return false;
  // one round trip per iteration for the loads: bounded work per thread
  if (G > 16 * TAIL_TG || ntiles > 16 * TAIL_TG) return false;
  // the operator rows of a wave's K parts must fit its registers
  for (int w = 0; w < 4; ++w) {
    int units = 0;
    for (int sp = w; sp < ks; sp += 4) units += ((sp + 1) * nk64) / ks - (sp * nk64) / ks;
    if (units > TAIL_MAXU) return false;
  }
  return true;
}

bool launch_dalm_tail(hipStream_t s, const TailArgs& t0) {
  TailArgs t = t0;
  const int G = t.n_pad / TAIL_ROWS;
  if (!tail_fits(t.n_pad, t.ntiles, t.ks)) return false;
  if (t.ncap < 1 || t.ncap > tail_capacity(t.n_pad, t.f32)) return false;
  const size_t dyn = t.f32 ? (size_t)t.ncap * (t.n_pad + 4) * 4 : (size_t)t.ncap * (t.n_pad + 8) * 4;
  int dev = 0;
  L1_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  L1_HIP(hipGetDeviceProperties(&prop, dev));
  if (!prop.cooperativeLaunch || t.ncap < 1) return false;
  const void* fn = t.f32 ? reinterpret_cast<const void*>(dalm_tail_kernel<true>)
                        : reinterpret_cast<const void*>(dalm_tail_kernel<false>);
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  int per_cu = 0;
  L1_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, dyn));
  if ((long)per_cu * prop.multiProcessorCount < G) return false;
  void* args[] = {&t};
  L1_HIP(hipLaunchCooperativeKernel(fn, dim3(G), dim3(256), args, dyn, s));
  return true;
}

namespace {
constexpr int kMaxDev = 64;
RegionList& regions(int dev) {
  static RegionList lists[kMaxDev];
  return lists[dev];
}
}  // namespace

void* tail_region_get(size_t bytes, size_t* got) {
  *got = 0;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) return nullptr;
  const size_t want = std::max<size_t>(bytes, (size_t)8 << 20);
  return regions(dev).get(want, [](size_t n) -> void* {
    void* p = nullptr;
    if (hipExtMallocWithFlags(&p, n, hipDeviceMallocUncached) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return p;
  }, got);
}

void tail_region_put(int dev, void* p, size_t bytes) {
  if (!p || dev < 0 || dev >= kMaxDev) return;
  regions(dev).put(p, bytes);
}

}  // namespace l1
