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
//     partial sums;
//   - one grid barrier per iteration; the next iteration starts with the
//     convergence test of this one (every workgroup computes it, so all take
//     the same decisions).
// Published data are written and read with agent-scope (sc1) accesses, which
// the memory system keeps coherent across the XCDs' L2 caches, so the barrier
// needs no L2 writeback or invalidation: each wave waits for its own stores,
// the workgroup adds to a counter and waits (bounded) for the grid, then the
// compute unit's L1 is dropped.
#include <algorithm>
#include <mutex>

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

// grid barrier on a counter in device memory; false if it gave up
__device__ inline bool tail_sync(unsigned* bar, unsigned target, int* flag) {
  __shared__ int s_ok;
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicAdd(bar, 1u);
    int ok = 1;
    unsigned spins = 0;
    while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
          ++spins > (1u << 20)) {
        atomicExch(flag, 1);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    // drop this compute unit's vector L1 so the next loads of published data
    // (and of this workgroup's own rows) come from memory
    asm volatile("buffer_inv sc0\n\ts_waitcnt vmcnt(0)" ::: "memory");
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

}  // namespace

template <bool F32>
__global__ __launch_bounds__(256) void dalm_tail_kernel(TailArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char ustage[];
  __shared__ int s_col[TAIL_NC], s_st[TAIL_NC], s_nc, s_live;
  __shared__ float s_red[8][16][17];
  __shared__ float s_ps[NPART][16][TAIL_NC];
  __shared__ float s_ts[TAIL_NC][16][NPART];
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
  const float bt = eown ? a.beta[s_col[ej]] : 1.0f;
  const float ib = 1.0f / bt;

  unsigned gen = 0;
  int k = a.k0;
  for (;; ++k) {
    const bool first = (k == a.k0);
    // ---- loads: u of iteration k and the partial sums of iteration k - 1 ------
    // every load of the phase is issued before the first is used (one memory
    // round trip): a thread moves at most TAIL_UV 16-byte vectors of u and
    // sums at most TAIL_TG groups of partial sums
    const int tj = tid >> 4, sub = tid & 15;
    {
      const int nv = n_pad / 4;   // 16-byte vectors per instance (FP32, or hi + lo BF16)
      const int nvec = nc * nv;
      u4 uv[TAIL_UV];
#pragma unroll
      for (int i = 0; i < TAIL_UV; ++i) {
        const int e = tid + 256 * i;
        if (e < nvec) {
          const int j = e / nv, w = e % nv;
          const void* src;
          if (F32) {
            src = first ? (const void*)(a.U32 + (long)s_col[j] * a.lds + w * 4)
                        : (const void*)(a.xu32[k & 1] + (long)j * n_pad + w * 4);
          } else if (first) {
            // the launch path's split: the first half of an instance's
            // vectors are hi, the second lo
            const int hl = w >= nv / 2, w8 = (w - hl * (nv / 2)) * 8;
            src = (hl ? a.Ulo : a.Uhi) + (long)s_col[j] * a.lds + w8;
          } else {
            // packed words: vector w holds elements 4w .. 4w + 3
            src = a.xpk[k & 1] + (long)j * n_pad + w * 4;
          }
          uv[i] = first ? ld16(src) : ld16c(src);
        }
      }
      float tv[TAIL_TG][NPART];
      const bool tlive = tj < nc && s_st[tj] < NPHASE;
#pragma unroll
      for (int i = 0; i < TAIL_TG; ++i) {
        const int t = sub + 16 * i;
        const int nt = first ? a.ntiles : G;
#pragma unroll
        for (int p = 0; p < NPART; ++p) {
          float v = 0.0f;
          if (tlive && t < nt) {
            v = first ? a.reg_partial[((long)t * NPART + p) * a.ldp + s_col[tj]]
                      : ldfc(a.xpart[(k - 1) & 1] + ((long)t * NPART + p) * TAIL_NC + tj);
          }
          tv[i][p] = v;
        }
      }
#pragma unroll
      for (int i = 0; i < TAIL_UV; ++i) {
        const int e = tid + 256 * i;
        if (e < nvec) {
          const int j = e / nv, w = e % nv;
          if (F32) {
            *reinterpret_cast<u4*>(reinterpret_cast<float*>(ustage) + (long)j * ldu32(n_pad) + w * 4) = uv[i];
          } else if (first) {
            const int hl = w >= nv / 2, w8 = (w - hl * (nv / 2)) * 8;
            uint16_t* sh = reinterpret_cast<uint16_t*>(ustage) + (long)(hl * ncap + j) * ldu16(n_pad);
            *reinterpret_cast<u4*>(sh + w8) = uv[i];
          } else {
            // unpack four (hi, lo) words into four hi and four lo values
            const u4 v = uv[i];
            typedef unsigned int u2 __attribute__((ext_vector_type(2)));
            const u2 hi = {(v[0] & 0xffffu) | (v[1] << 16), (v[2] & 0xffffu) | (v[3] << 16)};
            const u2 lo = {(v[0] >> 16) | (v[1] & 0xffff0000u), (v[2] >> 16) | (v[3] & 0xffff0000u)};
            uint16_t* sh = reinterpret_cast<uint16_t*>(ustage) + (long)j * ldu16(n_pad) + w * 4;
            *reinterpret_cast<u2*>(sh) = hi;
            *reinterpret_cast<u2*>(sh + (long)ncap * ldu16(n_pad)) = lo;
          }
        }
      }
#pragma unroll
      for (int p = 0; p < NPART; ++p) {
        float v = 0.0f;
#pragma unroll
        for (int i = 0; i < TAIL_TG; ++i) v += tv[i][p];
        s_ts[tj][sub][p] = v;
      }
    }
    __syncthreads();

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
        const int st = decide_in(a.tp, s_st[j], ar, sm, &stat_new);
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
        const float un = z2 - wn * ib;
        vreg = vn;
        wreg = wn;
        const long xo = (long)ej * n_pad + rw;
        const int nb = (k + 1) & 1;
        if (F32) {
          stfc(a.xu32[nb] + xo, un);
        } else {
          const uint16_t h = f2bf_t(un);
          const uint32_t w = (uint32_t)h | ((uint32_t)f2bf_t(un - bf2f_t(h)) << 16);
          __hip_atomic_store(a.xpk[nb] + xo, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
      stfc(a.xpart[k & 1] + ((long)g * NPART + p) * TAIL_NC + j, sum);
    }
    if (!tail_sync(a.bar, (unsigned)G * ++gen, a.flag)) return;
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
  const size_t budget = 128 * 1024;   // LDS for the u stage
  const size_t per_col = f32 ? (size_t)(n_pad + 4) * 4 : (size_t)(n_pad + 8) * 2 * 2;
  const size_t by_loads = (size_t)256 * TAIL_UV / (size_t)(n_pad / 4);   // u vectors per thread
  return (int)std::min<size_t>({(size_t)TAIL_NC, budget / per_col, by_loads});
}

bool launch_dalm_tail(hipStream_t s, const TailArgs& t0) {
  TailArgs t = t0;
  const int G = t.n_pad / TAIL_ROWS;
  const int nk64 = t.n_pad / 64;
  if (t.ks < 1 || t.ks > 8) return false;
  // one round trip per iteration for the loads: bounded work per thread
  if (G > 16 * TAIL_TG || t.ntiles > 16 * TAIL_TG) return false;
  if (t.ncap < 1 || t.ncap > tail_capacity(t.n_pad, t.f32)) return false;
  for (int w = 0; w < 4; ++w) {
    int units = 0;
    for (int sp = w; sp < t.ks; sp += 4) units += ((sp + 1) * nk64) / t.ks - (sp * nk64) / t.ks;
    if (units > TAIL_MAXU) return false;
  }
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

void* tail_pool(size_t bytes) {
  // one pool per device, grown by replacement only when a larger one is
  // needed; a replaced pool is kept (uncached memory is not freed)
  static std::mutex mu;
  static void* pool[64] = {nullptr};
  static size_t size[64] = {0};
  std::lock_guard<std::mutex> lock(mu);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  if (size[dev] >= bytes) return pool[dev];
  void* p = nullptr;
  const size_t want = std::max<size_t>(bytes, (size_t)8 << 20);
  if (hipExtMallocWithFlags(&p, want, hipDeviceMallocUncached) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  pool[dev] = p;
  size[dev] = want;
  return p;
}

}  // namespace l1
