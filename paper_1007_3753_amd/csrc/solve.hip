// Solve drivers.  All work of a solve runs on a plan-private stream that is
// ordered after the caller's stream at entry and before it at exit, so the
// iteration blocks can be captured into HIP graphs whatever stream the caller
// uses.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "plan.h"
#include "steps.h"
#include "tail.h"

namespace l1 {

namespace {

struct StreamGuard {
  hipStream_t user, own;
  hipEvent_t ev;
  StreamGuard(hipStream_t u) : user(u) {
    L1_HIP(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
    L1_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    L1_HIP(hipEventRecord(ev, user));
    L1_HIP(hipStreamWaitEvent(own, ev, 0));
  }
  ~StreamGuard() {
    (void)hipEventRecord(ev, own);
    (void)hipStreamWaitEvent(user, ev, 0);
    (void)hipStreamSynchronize(own);
    (void)hipEventDestroy(ev);
    (void)hipStreamDestroy(own);
  }
};

Lists lists_of(Plan* p) {
  const int Np = p->N_pad;
  int* q = p->ints;
  Lists L;
  L.state = q;                                     // phase buffer 0 (buffer 1 at q + 5 Np + 256)
  L.iters = q + Np;
  L.status = q + 2 * Np;
  L.slot_col = q + 3 * Np;                         // Np + NPHASE*TILE entries
  L.phase_off = q + 4 * Np + NPHASE * TILE;        // NPHASE + 1 entries
  L.n_total = L.phase_off + NPHASE + 1;
  L.cnt = L.n_total + 1;
  return L;
}

bool graphs_enabled() {
  const char* e = std::getenv("L1ALM_GRAPH");
  return !(e && e[0] == '0');
}

void check_common(Plan* p, const SolveArgs& a) {
  L1_REQUIRE(a.N >= 0 && a.N <= p->d.max_batch, "N must be in [0, max_batch]");
  if (a.N == 0) return;
  L1_REQUIRE(a.b != nullptr && a.x != nullptr, "b and x must be non-NULL");
  L1_REQUIRE(a.ldb >= p->m, "ldb < m");
  L1_REQUIRE(a.ldx >= std::max(p->nd, 1), "ldx < n_dict");
  L1_REQUIRE(a.e == nullptr || a.lde >= p->m, "lde < m");
  L1_REQUIRE(a.y == nullptr || a.ldy >= p->m, "ldy < m");
  L1_REQUIRE(p->d.problem != L1_P12 || a.eps != nullptr, "P_{1,2} needs eps (N radii)");
  L1_REQUIRE(a.max_iter != 0, "max_iter must be nonzero");
  L1_REQUIRE(std::isfinite(a.tol) && a.tol >= 0.0f, "tol must be finite and >= 0");
  L1_REQUIRE(!(a.pen && p->d.problem == L1_QPLAMBDA && p->d.method == L1_DALM),
             "DALM on QP_lambda takes beta from the plan (it enters the factor): pen must be NULL");
}

}  // namespace

// ---------------------------------------------------------------------------
// Precision schedule: the first phase, the final phase and the floors of the
// stopping test (where the rounding of the products stalls it).
static void dalm_phases(int precision, bool fixed, int* first, int* last) {
  if (precision == L1_FP32) *first = *last = PREC_F32;
  else if (precision == L1_BF16X3) *first = *last = PREC_BF16X3;
  else {
    *first = PREC_BF16;
    *last = PREC_BF16X3;
  }
  (void)fixed;
}

int dalm_ksplit(const Plan* p, int active, int phases_used) {
  const int RT = p->n_pad / TILE, nk64 = p->n_pad / 64;
  const int ctiles = col_tiles_for(active);
  const int est = (active + TILE - 1) / TILE + phases_used - 1;
  // split only when the launch would leave most compute units idle
  int ks = (RT * est >= p->ks_target) ? 1 : (p->ks_target + RT * est - 1) / (RT * est);
  // a tuned choice for this many active column tiles replaces the heuristic
  const int at = (active + TILE - 1) / TILE;
  if (at >= 1 && at <= 8 && p->ks_table[at] > 0) ks = p->ks_table[at];
  ks = std::min({ks, p->ks_max, nk64, std::max(1, p->ws_tiles / ctiles)});
  return std::max(ks, 1);
}

void solve_dalm(Plan* p, const SolveArgs& a) {
  check_common(p, a);
  if (a.N == 0) return;
  const auto t_start = std::chrono::steady_clock::now();
  const bool fixed = a.max_iter < 0;
  L1_REQUIRE(!(fixed && p->d.record_tape) ||
                 (p->d.problem != L1_P12 && p->d.precision == L1_FP32),
             "recording a tape needs an FP32 plan for P1 or QP_lambda");
  const int cap = fixed ? -a.max_iter : a.max_iter;
  StreamGuard sg(a.s);
  hipStream_t s = sg.own;
  const int N = a.N, m = p->m, nd = p->nd, n = p->n, lds = p->lds;
  const int ntc = (N + TILE - 1) / TILE;
  const int ctiles = col_tiles_for(N);
  const bool p12 = p->d.problem == L1_P12;
  int first, last;
  dalm_phases(p->d.precision, fixed, &first, &last);
  // BF16 phase threshold: low where the operand's reference point is
  // refreshed (more than one column tile), so that the iteration bound below
  // ends the phase; smaller batches hand over at 3e-3 (held in BF16 longer,
  // measured 13-20 % slower on 8- and 40-instance batches)
  const float sw = (p->d.refine_switch > 0) ? (float)p->d.refine_switch : (N > TILE ? 1e-4f : 3e-3f);

  // b, penalties, c = A^T G^{-1} b / beta
  L1_HIP(hipMemsetAsync(p->bb, 0, sizeof(float) * p->m_pad * N, s));
  L1_HIP(hipMemcpy2DAsync(p->bb, sizeof(float) * p->m_pad, a.b, sizeof(float) * a.ldb,
                          sizeof(float) * m, N, hipMemcpyDeviceToDevice, s));
  penalties(s, N, m, p->bb, p->m_pad, a.pen, p->d.beta > 0 ? (float)p->d.beta : 0.0f, 0,
            default_beta_scale(p, N), p->split && p->d.problem == L1_P1 ? 0.25f : 0.0f, div_factor(p),
            p->pen, p->ipen, p->wcap2, p->dscale2);
  {
    GemmArgs g{};
    g.A32 = p->Cop;
    g.lda = p->m_pad;
    g.B = p->bb;
    g.ldb = p->m_pad;
    g.M = p->n_pad;
    g.K = p->m_pad;
    g.n_cols = N;
    g.prec = PREC_F32;
    g.m_true = p->n_pad;
    g.out = p->C;
    g.ldo = lds;
    g.col_scale = p->ipen;
    launch_gemm(s, EPI_STORE, g, ntc);
    // the same product unscaled, C0 = A^T G^{-1} b, from which each refresh
    // of the operand's reference point forms c_ref = (C0 - P w_ref) / beta
    g.out = p->C0;
    g.col_scale = nullptr;
    launch_gemm(s, EPI_STORE, g, ntc);
  }
  // reference point of the operand u = z - (w - w_ref)/beta: 0 until the
  // first refresh (then c_ref = c)
  L1_HIP(hipMemsetAsync(p->Wref, 0, sizeof(float) * (size_t)lds * N, s));
  float* eps = nullptr;
  if (p12) {
    eps = p->tscal;
    L1_HIP(hipMemcpyAsync(eps, a.eps, sizeof(float) * N, hipMemcpyDeviceToDevice, s));
  }
  // initial state (Algorithm 2 input: w = 0, y = 0, or a warm start)
  L1_HIP(hipMemsetAsync(p->W, 0, sizeof(float) * (size_t)lds * N, s));
  L1_HIP(hipMemsetAsync(p->V, 0, sizeof(float) * (size_t)lds * N, s));
  if (a.w0) copy_in(s, n, N, a.w0, n, p->W, lds, 0);
  if (a.y0) {
    L1_HIP(hipMemsetAsync(p->aux, 0, sizeof(float) * p->m_pad * N, s));
    copy_in(s, m, N, a.y0, m, p->aux, p->m_pad, 0);
    if (nd > 0) {
      GemmArgs g{};
      g.A32 = p->Acol;
      g.lda = p->m_pad;
      g.B = p->aux;
      g.ldb = p->m_pad;
      g.M = p->nd_pad;
      g.K = p->m_pad;
      g.n_cols = N;
      g.prec = PREC_F32;
      g.m_true = nd;
      g.out = p->V;
      g.ldo = lds;
      launch_gemm(s, EPI_STORE, g, ntc);
    }
    if (p->split) copy_in(s, m, N, a.y0, m, p->V, lds, nd);
  }
  {
    DalmInit di{};
    di.n = n;
    di.n_pad = p->n_pad;
    di.lds = lds;
    di.e0 = p12 ? nd : (1 << 30);
    di.V = p->V;
    di.W = p->W;
    di.beta = p->pen;
    di.eps = eps;
    di.zscale = p->zscale;
    di.U = p->Uf[0];
    di.Uhi = p->Uh[0];
    di.Ulo = p->Ul[0];
    dalm_init_u(s, N, di);
  }
  const Lists L = lists_of(p);
  int* stbuf[2] = {L.state, p->ints + 5 * p->N_pad + 256};
  // arithmetic of each column's product: iteration k writes arbuf[k & 1]
  int* arbuf[2] = {p->ints + 6 * p->N_pad + 256, p->ints + 7 * p->N_pad + 256};
  init_lists(s, N, first, L, stbuf[1], p->stat);

  // tape: checkpoints of (W, V) every k iterations of a fixed-count solve
  const bool tape = fixed && p->d.record_tape;
  const int every = p->d.checkpoint_every > 0 ? p->d.checkpoint_every : 10;
  if (tape) {
    for (void* q : p->tape) (void)hipFree(q);
    p->tape.clear();
    const int nck = (cap + every - 1) / every;  // states at iterations 0, k, 2k, ... < cap
    p->tape_N = 0;
    for (int i = 0; i < 2 * nck + 2; ++i) {
      void* q = nullptr;
      if (hipMalloc(&q, sizeof(float) * (size_t)lds * N) != hipSuccess) {
        (void)hipGetLastError();
        set_error("out of device memory for the tape");
        throw Fail{L1_ENOMEM};
      }
      p->tape.push_back(q);
    }
    p->tape_K = cap;
    p->tape_every = every;
    p->tape_b = reinterpret_cast<float*>(p->tape[2 * nck]);      // b, ld m_pad
    p->tape_pen = reinterpret_cast<float*>(p->tape[2 * nck + 1]);  // beta, 1/beta
    L1_HIP(hipMemcpyAsync(p->tape_b, p->bb, sizeof(float) * p->m_pad * N,
                          hipMemcpyDeviceToDevice, s));
    L1_HIP(hipMemcpyAsync(p->tape_pen, p->pen, sizeof(float) * N, hipMemcpyDeviceToDevice, s));
    L1_HIP(hipMemcpyAsync(p->tape_pen + N, p->ipen, sizeof(float) * N, hipMemcpyDeviceToDevice, s));
  }

  const float tol = fixed ? -1.0f : a.tol;
  const float floors[NPHASE] = {1.0f, 4e-6f, 2e-6f};  // BF16 (never final), split BF16, FP32
  float* part[2] = {p->partial, p->partial + (size_t)p->ntiles * NPART * p->N_pad};
  GemmArgs it{};
  it.A32 = p->P32;
  it.Ahi = p->Phi;
  it.Alo = p->Plo;
  it.lda = p->n_pad;
  it.ldb = lds;
  it.M = p->n_pad;
  it.K = p->n_pad;
  it.slot_col = L.slot_col;
  it.phase_off = L.phase_off;
  it.n_cols = N;
  it.lds = lds;
  it.V = p->V;
  it.W = p->W;
  it.C = p->C;
  it.beta = p->pen;
  it.ldp = p->N_pad;
  it.n_l1 = p->n_l1;
  it.e0 = p12 ? nd : (1 << 30);
  it.zscale = p12 ? p->zscale : nullptr;
  it.iters = L.iters;
  it.status = L.status;
  it.tp_tol = tol;
  it.tp_sw = sw;
  for (int q = 0; q < NPHASE; ++q) it.tp_floor[q] = floors[q];
  it.tp_final = last;
  it.eps = p12 ? eps : nullptr;
  it.wcap2 = p->wcap2;
  it.dscale2 = p->dscale2;
  it.Wref = p->Wref;
  it.stat = p->stat;
  it.ws = p->ws;
  // BF16 plans never run an FP32 iteration tile (the refresh is its own launch)
  it.fam = (p->d.precision != L1_FP32) ? 1 : 0;
  DalmCheck ck{};
  ck.N = N;
  ck.ldp = p->N_pad;
  ck.ntiles = p->ntiles;
  ck.tol = tol;
  for (int q = 0; q < NPHASE; ++q) ck.floor[q] = floors[q];
  ck.sw = sw;
  ck.final_phase = last;
  // the BF16 phase ends after 2000 iterations at the latest: with the FP32
  // refresh of the operand's reference point, BF16 iterations progress as
  // fast as split ones until BF16 rounding holds the gap near 1e-4 relative
  // (about there on the 1200 x 700 and 4800 x 2100 cross-and-bouquet
  // batches), and instances that end the phase together keep the launches
  // in one arithmetic (1000 - 4000 measured, 2000 best on both)
  ck.low_cap = 2000;
  ck.L = L;
  ck.eps = eps;
  ck.beta = p->pen;
  ck.wcap2 = p->wcap2;
  ck.dscale2 = p->dscale2;
  ck.stat = p->stat;
  P12Fix fx{};
  fx.n = n;
  fx.e0 = nd;
  fx.lds = lds;
  fx.ldp = p->N_pad;
  fx.ntiles = p->ntiles;
  fx.slot_col = L.slot_col;
  fx.phase_off = L.phase_off;
  fx.V = p->V;
  fx.W = p->W;
  fx.beta = p->pen;
  fx.eps = eps;

  constexpr int BLK = 16;  // iterations per host poll (and per graph replay; even)
  // time_kernels: HIP events on the solve stream around every block of BLK
  // iterations (graph replay or uncaptured launches; the block's compaction
  // included), so the timed launches run exactly as untimed ones do
  const bool timing = p->d.time_kernels != 0;
  std::vector<hipEvent_t> ev;     // ev[0..1]: the tail launch; tev: the blocks, two slots
  hipEvent_t* tev = nullptr;
  hipEvent_t cev[2] = {nullptr, nullptr};  // the blocks' count copies
  for (auto& e : cev) L1_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  if (timing) {
    ev.resize(6);
    for (auto& e : ev) L1_HIP(hipEventCreate(&e));
    tev = ev.data() + 2;
  }
  // Launch shape of a block of iterations, from the number of unfinished
  // instances polled before it (the count only shrinks inside a block):
  // split the K range when few column tiles are active, so that enough
  // workgroups run and each walks a shorter chain of K slices.
  const int phases_used = (first == last) ? 1 : 2;
  struct Shape {
    int ctiles, ks;
    bool st;   // structured form (two launches per iteration)
  };
  // The structured form (cross-and-bouquet with n_dict < m, or a dense
  // dictionary with m < n_dict) runs the BF16 and FP32 tiles; split-BF16
  // tiles stay on the dense operator.  Its second
  // product passes the rounding of the first through B (||B|| ~ 30 on face
  // dictionaries): split BF16's 16 bits then miss the 1e-4 accuracy of the
  // converged solution, and even FP32's rounding lifts the relative change
  // of w above the stopping test's threshold for some instances.  So the
  // automatic rule takes it for FP32 plans only, and only while the
  // unfinished instances fill at least ST_MIN_TILES column tiles: as the
  // batch drains, the last instances converge on the dense operator
  // (measured on the 4800 x 2100 workload, 2048 instances: FP32 6.9 ->
  // 5.0 s; BF16 + refinement gains nothing, its split phase dominating).
  // The same holds on a dense dictionary (A with m < n_dict): A^T spreads
  // the first product's rounding by ||A|| (3 for the Gaussian 2000 x 8000
  // workload, whose 64 QP_lambda instances then stop by the iteration cap
  // under the FP32 floor of the test).  Asked for explicitly, it runs
  // whenever it applies.  Never while a tape is recorded (the backward
  // replays the dense form).
  constexpr int ST_MIN_TILES = 16;
  const bool st_plan = p->st_ok && !tape && p->d.precision != L1_BF16X3;
  auto shape_for = [&](int active) {
    Shape sh;
    sh.ctiles = col_tiles_for(active);
    sh.ks = dalm_ksplit(p, active, phases_used);
    sh.st = st_plan && (p->d.iteration_form == 2 ||
                        (p->d.precision == L1_FP32 && (active + TILE - 1) / TILE >= ST_MIN_TILES));
    if (sh.st) sh.ks = 1;
    return sh;
  };
  // the two launches of the structured form: the first R1 rows of P u (and
  // q = u - (P u) on the x rows), then v_e = u_e + B q on the rows from R1 on
  GemmArgs st1 = it, st2 = it;
  if (p->st_ok == 2) {
    // dense dictionary: t = Rop u in the tile's operand format (no test, no
    // state), then the iteration launch with A^T and t
    st1 = GemmArgs{};
    st1.A32 = p->R32;
    st1.Ahi = p->Rhi;
    st1.Alo = p->Rlo;
    st1.lda = p->n_pad;
    st1.M = p->m_pad;
    st1.K = p->n_pad;
    st1.ldb = lds;
    st1.slot_col = L.slot_col;
    st1.phase_off = L.phase_off;
    st1.n_cols = N;
    st1.m_true = p->m_pad;
    st1.out = p->Tf;
    st1.ldo = p->ldt;
    st1.Tq_hi = p->Th;
    st1.Tq_lo = p->Tl;
    st2.A32 = p->Bq32;
    st2.Ahi = p->Bqhi;
    st2.Alo = p->Bqlo;
    st2.lda = p->m_pad;
    st2.K = p->m_pad;
    st2.ldb = p->ldt;
    st2.ldt = p->ldt;
    st2.q_rows = 0;
    st1.prec_mask = st2.prec_mask = (1 << PREC_BF16) | (1 << PREC_F32);
  } else if (p->st_ok == 1) {
    st1.M = p->R1;
    st1.ptiles = p->n_pad / TILE;
    st1.Tq = p->Tf;
    st1.Tq_hi = p->Th;
    st1.Tq_lo = p->Tl;
    st1.q_rows = nd;
    st1.ldt = p->nd_pad;
    const size_t boff = (size_t)(p->R1 - nd) * p->nd_pad;
    st2.A32 = p->Bq32 + boff;
    st2.Ahi = p->Bqhi ? p->Bqhi + boff : nullptr;
    st2.Alo = p->Bqlo ? p->Bqlo + boff : nullptr;
    st2.lda = p->nd_pad;
    st2.M = p->n_pad - p->R1;
    st2.K = p->nd_pad;
    st2.ldb = p->nd_pad;
    st2.row_off = p->R1;
    st2.ptiles = p->n_pad / TILE;
    st2.test_passive = 1;
    st2.add_u = 1;
    st1.prec_mask = st2.prec_mask = (1 << PREC_BF16) | (1 << PREC_F32);
  }

  // iteration k (0-based) reads the phases and partial sums left by
  // iteration k - 1 and writes its own into the other buffers
  auto one_iter = [&](int k, const Shape& sh) {
    const int cur = k & 1;
    it.B = p->Uf[cur];
    it.Bhi = p->Uh[cur];
    it.Blo = p->Ul[cur];
    it.U = p->Uf[1 - cur];
    it.Uhi = p->Uh[1 - cur];
    it.Ulo = p->Ul[1 - cur];
    it.state_in = stbuf[cur];
    it.state_out = stbuf[1 - cur];
    it.arith_in = arbuf[1 - cur];
    it.arith_out = arbuf[cur];
    it.prev_partial = (k == 0) ? nullptr : part[1 - cur];
    it.partial = part[cur];
    if (sh.st && p->st_ok == 2) {
      st1.B = it.B;
      st1.Bhi = it.Bhi;
      st1.Blo = it.Blo;
      launch_gemm(s, EPI_STORE, st1, sh.ctiles);
      st2.state_in = it.state_in;
      st2.state_out = it.state_out;
      st2.arith_in = it.arith_in;
      st2.arith_out = it.arith_out;
      st2.prev_partial = it.prev_partial;
      st2.partial = it.partial;
      st2.U = it.U;
      st2.Uhi = it.Uhi;
      st2.Ulo = it.Ulo;
      st2.B = p->Tf;
      st2.Bhi = p->Th;
      st2.Blo = p->Tl;
      launch_product(s, EPI_DALM, st2, sh.ctiles, 1);
    } else if (sh.st) {
      for (GemmArgs* g : {&st1, &st2}) {
        g->state_in = it.state_in;
        g->state_out = it.state_out;
        g->arith_in = it.arith_in;
        g->arith_out = it.arith_out;
        g->prev_partial = it.prev_partial;
        g->partial = it.partial;
        g->U = it.U;
        g->Uhi = it.Uhi;
        g->Ulo = it.Ulo;
        g->Ucur = it.B;
        g->Ucur_hi = it.Bhi;
        g->Ucur_lo = it.Blo;
      }
      st1.B = it.B;
      st1.Bhi = it.Bhi;
      st1.Blo = it.Blo;
      st2.B = p->Tf;
      st2.Bhi = p->Th;
      st2.Blo = p->Tl;
      launch_product(s, EPI_DALM, st1, sh.ctiles, 1);
      launch_product(s, EPI_DALM, st2, sh.ctiles, 1);
    }
    if (sh.st) {
      if (p->d.precision == L1_BF16_REFINE) {
        // the split-BF16 tiles, on the dense operator
        GemmArgs g = it;
        g.prec_mask = 1 << PREC_BF16X3;
        launch_product(s, EPI_DALM, g, sh.ctiles, 1);
      }
      return;
    }
    launch_product(s, EPI_DALM, it, sh.ctiles, sh.ks);
    if (p12) {
      fx.state = stbuf[1 - cur];
      fx.partial = part[cur];
      fx.U = p->Uf[1 - cur];
      fx.Uhi = p->Uh[1 - cur];
      fx.Ulo = p->Ul[1 - cur];
      p12_fix(s, sh.ctiles * TILE, fx);
    }
  };
  // the phases after iteration k live in stbuf[(k + 1) & 1]
  auto compact_after = [&](int k) {
    const int nb = (k + 1) & 1;
    ck.L.state = stbuf[nb];
    ck.state_other = stbuf[1 - nb];
    dalm_compact(s, ck);
  };
  // FP32 refresh of the operand's reference point after iteration k (a block
  // end, after its compaction): w_ref = w, c_ref = (C0 - P w)/beta and the
  // next operand u = clamp(v + w/beta), for the listed instances.  Exact in
  // exact arithmetic (v = P u + c_ref = P (z - w/beta) + c either way); it
  // keeps the low-precision products' operand O(1).  Not for P_{1,2} (the
  // ball block's operand is fixed up separately) nor for recorded tapes (the
  // backward recomputes segments from (w, v) alone), and only while the
  // active instances span two or more column tiles (refresh_min below).
  const bool recentre = !p12 && !(fixed && p->d.record_tape);
  GemmArgs rf{};
  rf.A32 = p->P32;
  rf.lda = p->n_pad;
  rf.B = p->W;
  rf.ldb = lds;
  rf.M = p->n_pad;
  rf.K = p->n_pad;
  rf.slot_col = L.slot_col;
  rf.phase_off = L.phase_off;
  rf.n_cols = N;
  rf.lds = lds;
  rf.V = p->V;
  rf.W = p->W;
  rf.C = p->C;
  rf.C0 = p->C0;
  rf.beta = p->pen;
  rf.Wref = p->Wref;
  rf.force_f32 = 1;
  auto refresh_after = [&](int k, int ctiles) {
    const int nb = (k + 1) & 1;
    rf.U = p->Uf[nb];
    rf.Uhi = p->Uh[nb];
    rf.Ulo = p->Ul[nb];
    launch_gemm(s, EPI_REFRESH, rf, ctiles);
  };

  // captured blocks of BLK iterations, one per launch shape met; the first
  // block (no test in its first launch) and tape recording run uncaptured
  struct Captured {
    Shape sh;
    bool refresh;
    hipGraph_t g;
    hipGraphExec_t x;
  };
  std::vector<Captured> graphs;
  bool graphs_ok = graphs_enabled() && !tape && cap >= 4 * BLK;
  auto graph_for = [&](const Shape& sh, bool refresh) -> hipGraphExec_t {
    for (auto& c : graphs)
      if (c.sh.ctiles == sh.ctiles && c.sh.ks == sh.ks && c.sh.st == sh.st && c.refresh == refresh)
        return c.x;
    Captured c{sh, refresh, nullptr, nullptr};
    bool ok = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
      try {
        for (int t = 0; t < BLK; ++t) one_iter(BLK + t, sh);  // any k > 0 of even block start
        compact_after(2 * BLK - 1);
        if (refresh) refresh_after(2 * BLK - 1, sh.ctiles);
      } catch (const Fail&) {
        ok = false;
      }
      const hipError_t e = hipStreamEndCapture(s, &c.g);
      ok = ok && e == hipSuccess && hipGraphInstantiate(&c.x, c.g, nullptr, nullptr, 0) == hipSuccess;
    }
    if (!ok) {
      (void)hipGetLastError();
      if (c.x) (void)hipGraphExecDestroy(c.x);
      if (c.g) (void)hipGraphDestroy(c.g);
      return nullptr;
    }
    graphs.push_back(c);
    return c.x;
  };
  auto release = [&]() {
    for (auto& c : graphs) {
      (void)hipGraphExecDestroy(c.x);
      (void)hipGraphDestroy(c.g);
    }
    graphs.clear();
    for (auto e : ev) (void)hipEventDestroy(e);
    ev.clear();
    for (auto& e : cev)
      if (e) {
        (void)hipEventDestroy(e);
        e = nullptr;
      }
  };

  long long hstat[8] = {0};
  double timed_ms = 0.0;
  long long timed_n = 0;
  int done = 0, active = N;
  // tail kernel: once few instances are left, the remaining iterations run
  // in one cooperative launch (it also runs the test of the last iteration)
  const int tail_f32 = (last == PREC_F32) ? 1 : 0;
  const int tail_cap = tail_capacity(p->n_pad, tail_f32);
  // the operand's reference point is refreshed while the active instances
  // span at least two column tiles: a rule of the launch shape, like the
  // K split, so that an instance's arithmetic depends on the shape only (a
  // batch that fits one tile runs as each of its instances alone would, and
  // the tail kernel, which never refreshes, takes over within one tile)
  const int refresh_min = TILE;
  bool tail_ok = !tape && !p12 && (p->n_pad % (TAIL_ROWS * 4) == 0) && tail_cap >= 1 &&
                 (tail_f32 || p->Phi != nullptr);
  if (const char* e = std::getenv("L1ALM_TAIL")) tail_ok = tail_ok && e[0] != '0';
  bool tail_done = false;
  int tail_retry = 0;
  // The host keeps one block of iterations queued ahead of the block whose
  // unfinished-instance count it reads: the shape of a block comes from the
  // count after the block before the previous one.  The count never grows,
  // so a stale count still covers every unfinished instance (and a tail
  // launch chosen from it has room for all of them); at worst one block too
  // many is launched, whose launches find no listed instance.
  int* hcnt = p->h_total + 4;   // two pinned count slots
  int pend = -1, pend_blk = 0, nslot = 0;
  auto retire = [&]() {
    if (pend < 0) return;
    L1_HIP(hipEventSynchronize(cev[pend]));
    active = hcnt[pend];
    if (timing) {
      float ms = 0.0f;
      L1_HIP(hipEventElapsedTime(&ms, tev[2 * pend], tev[2 * pend + 1]));
      timed_ms += ms;
      timed_n += pend_blk;
    }
    pend = -1;
  };
  try {
    while (done < cap) {
      const int blk = std::min(BLK, cap - done);
      const Shape sh = shape_for(std::max(active, 1));
      if (tail_ok && done > 0 && done >= tail_retry && active <= tail_cap) {
        retire();
        const int G = p->n_pad / TAIL_ROWS;
        // tagged 8-byte words: u [TAIL_NC][n_pad] and partial sums
        // [G][NPART][TAIL_NC], two of each; flags in the first 256 bytes
        const size_t xu = (size_t)TAIL_NC * p->n_pad * 8;
        const size_t xp = (size_t)G * NPART * TAIL_NC * 8;
        const size_t need = 256 + 2 * xu + 2 * xp;
        if (p->tail_bytes < need) {
          tail_region_put(p->dev, p->tail_mem, p->tail_bytes);
          p->tail_mem = tail_region_get(need, &p->tail_bytes);
        }
        unsigned char* pool = reinterpret_cast<unsigned char*>(p->tail_mem);
        if (!pool) {
          tail_ok = false;
        } else {
          TailArgs ta{};
          ta.P32 = p->P32;
          ta.Phi = p->Phi;
          ta.Plo = p->Plo;
          ta.n_pad = p->n_pad;
          ta.n_l1 = p->n_l1;
          ta.lds = lds;
          ta.f32 = tail_f32;
          ta.ncap = tail_cap;
          ta.V = p->V;
          ta.W = p->W;
          ta.C = p->C;
          ta.Wref = p->Wref;
          ta.beta = p->pen;
          ta.wcap2 = p->wcap2;
          ta.dscale2 = p->dscale2;
          ta.st[0] = stbuf[0];
          ta.st[1] = stbuf[1];
          ta.iters = L.iters;
          ta.status = L.status;
          ta.slot_col = L.slot_col;
          ta.phase_off = L.phase_off;
          ta.reg_partial = part[(done - 1) & 1];
          ta.reg_arith = arbuf[(done - 1) & 1];
          ta.ldp = p->N_pad;
          ta.ntiles = p->ntiles;
          ta.U32 = p->Uf[done & 1];
          ta.Uhi = p->Uh[done & 1];
          ta.Ulo = p->Ul[done & 1];
          ta.tp.tol = tol;
          ta.tp.sw = sw;
          ta.tp.final_phase = last;
          for (int q = 0; q < NPHASE; ++q) ta.tp.floor[q] = floors[q];
          unsigned char* c = pool + 256;
          for (int b = 0; b < 2; ++b) {
            ta.xu[b] = reinterpret_cast<unsigned long long*>(c);
            c += xu;
          }
          for (int b = 0; b < 2; ++b) {
            ta.xpart[b] = reinterpret_cast<unsigned long long*>(c);
            c += xp;
          }
          ta.flag = reinterpret_cast<int*>(pool + 64);
          ta.k0 = done;
          ta.k_end = cap;
          ta.ks = std::min(sh.ks, 8);
          ta.stat = p->stat;
          // no tag of an earlier launch may match: clear flags and words
          L1_HIP(hipMemsetAsync(pool, 0, need, s));
          if (timing) L1_HIP(hipEventRecord(ev[0], s));
          if (launch_dalm_tail(s, ta)) {
            if (timing) L1_HIP(hipEventRecord(ev[1], s));
            L1_HIP(hipMemcpyAsync(p->h_total + 2, ta.flag, sizeof(int) * 2, hipMemcpyDeviceToHost, s));
            L1_HIP(hipStreamSynchronize(s));
            if (p->h_total[2] != 0) {
              set_error("the grid barrier of the tail kernel gave up");
              throw Fail{L1_EHIP};
            }
            const int kd = p->h_total[3];
            if (kd == done) {
              // declined (an instance is not yet in the final phase): go on
              // launching per iteration and try again after the next block
              tail_retry = done + BLK;
            } else {
            if (timing) {
              float ms = 0.0f;
              L1_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
              timed_ms += ms;
              timed_n += kd - done;
            }
            done = kd;
            tail_done = true;
            compact_after(done - 1);
            L1_HIP(hipMemcpyAsync(p->h_total, L.n_total, sizeof(int), hipMemcpyDeviceToHost, s));
            L1_HIP(hipStreamSynchronize(s));
            active = *p->h_total;
            break;
            }
          } else {
            tail_ok = false;  // not co-resident on this device: launch per iteration
          }
        }
      }
      const bool refresh = recentre && active > refresh_min;
      hipGraphExec_t gx = nullptr;
      if (graphs_ok && blk == BLK && done > 0) {
        gx = graph_for(sh, refresh);
        if (!gx) graphs_ok = false;
      }
      const int slot = nslot;
      nslot ^= 1;
      if (timing) L1_HIP(hipEventRecord(tev[2 * slot], s));
      if (gx) {
        L1_HIP(hipGraphLaunch(gx, s));
      } else {
        for (int t = 0; t < blk; ++t) {
          const int k = done + t;
          if (tape && k % every == 0) {
            const int ci = k / every;
            L1_HIP(hipMemcpyAsync(p->tape[2 * ci], p->W, sizeof(float) * (size_t)lds * N,
                                  hipMemcpyDeviceToDevice, s));
            L1_HIP(hipMemcpyAsync(p->tape[2 * ci + 1], p->V, sizeof(float) * (size_t)lds * N,
                                  hipMemcpyDeviceToDevice, s));
          }
          one_iter(k, sh);
        }
        compact_after(done + blk - 1);
        if (refresh) refresh_after(done + blk - 1, sh.ctiles);
      }
      if (timing) L1_HIP(hipEventRecord(tev[2 * slot + 1], s));
      done += blk;
      L1_HIP(hipMemcpyAsync(hcnt + slot, L.n_total, sizeof(int), hipMemcpyDeviceToHost, s));
      L1_HIP(hipEventRecord(cev[slot], s));
      retire();  // the block before this one (this one keeps the device busy)
      pend = slot;
      pend_blk = blk;
      if (!fixed && active == 0) break;
    }
    retire();
  } catch (...) {
    release();
    throw;
  }
  release();
  // the test of the last iteration (its launch only tested the one before;
  // the tail kernel runs it itself)
  if (!tail_done) {
    const int klast = done - 1;
    ck.L.state = stbuf[(klast + 1) & 1];
    ck.partial = part[klast & 1];
    ck.arith = arbuf[klast & 1];
    dalm_final_test(s, ck);
  }
  L1_HIP(hipMemcpyAsync(hstat, p->stat, sizeof(hstat), hipMemcpyDeviceToHost, s));

  // outputs
  copy_block(s, nd, N, p->W, lds, 0, a.x, a.ldx);
  if (p->split && a.e) copy_block(s, m, N, p->W, lds, nd, a.e, a.lde);
  if (a.y) {
    if (p->split) {
      copy_block(s, m, N, p->V, lds, nd, a.y, a.ldy);
    } else {
      GemmArgs g{};
      g.A32 = p->Yop;
      g.lda = p->n_pad;
      g.B = p->V;
      g.ldb = lds;
      g.M = p->m_pad;
      g.K = p->n_pad;
      g.n_cols = N;
      g.prec = PREC_F32;
      g.m_true = m;
      g.out = a.y;
      g.ldo = a.ldy;
      launch_gemm(s, EPI_STORE, g, ntc);
    }
  }
  finish_status(s, N, fixed ? cap : 0, L.iters, L.status, a.iters, a.status);
  L1_HIP(hipStreamSynchronize(s));
  if (tape) p->tape_N = N;
  // stats: header order FP32, BF16, split; internal precision order BF16, split, FP32
  const int map[3] = {PREC_F32, PREC_BF16, PREC_BF16X3};
  for (int i = 0; i < 14; ++i) p->last_stats[i] = 0.0;
  for (int i = 0; i < 3; ++i) {
    p->last_stats[i] = (double)hstat[map[i]];
    p->last_stats[3 + i] = (double)hstat[3 + map[i]];
  }
  p->last_stats[6] = timed_ms;
  p->last_stats[7] = (double)timed_n;
  p->last_stats[8] = (double)hstat[7];
  p->last_stats[9] =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  p->last_stats[12] = (double)hstat[6];
}


}  // namespace l1
