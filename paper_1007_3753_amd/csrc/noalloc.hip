// l1_alm_kkt_noalloc: the FP64 optimality report of l1_alm_kkt for callers
// that cannot allocate device memory (code under HIP graph capture, tight
// serving loops, harnesses that forbid allocation).  It needs no plan: the
// caller passes the dictionary itself, and the kernel's only scratch (the
// FP64 residual b - A w of the instances of one launch) lives in a static
// device array of fixed size, which the instances use chunk by chunk.
#include <mutex>

#include "internal.h"

namespace l1 {

// FP64 residual rows for the instances of one launch (8 MiB per device,
// held until the process ends)
constexpr long NOALLOC_SCRATCH_DOUBLES = L1_KKT_NOALLOC_MAX_M;
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];

namespace {

constexpr int kMaxDev = 64;

// The device address of `scratch` on the current device, looked up once per
// device with that device current (each device has its own copy; host code
// must never pass the array's name itself to a kernel).
double* scratch_ptr() {
  static std::mutex mu;
  static double* ptr[kMaxDev] = {nullptr};
  int dev = 0;
  L1_HIP(hipGetDevice(&dev));
  L1_REQUIRE(dev >= 0 && dev < kMaxDev, "device index out of range");
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    L1_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    ptr[dev] = reinterpret_cast<double*>(p);
  }
  return ptr[dev];
}

}  // namespace

void kkt_noalloc(hipStream_t s, int problem, int structure, int m, int nd, const float* A, int lda,
                 const float* b, int ldb, int N, const float* eps, double lambda, const float* x, int ldx,
                 const float* e, int lde, const float* y, int ldy, double* report) {
  L1_REQUIRE(m >= 1 && (long)m <= NOALLOC_SCRATCH_DOUBLES,
             "m exceeds the scratch of l1_alm_kkt_noalloc (1048576 rows)");
  double* rbuf = scratch_ptr();
  // instances per launch: as many residual rows as the scratch holds; the
  // launches run in stream order, so each reuses the scratch after the last
  const int chunk = (int)std::min<long>((long)N, NOALLOC_SCRATCH_DOUBLES / m);
  const int split = structure == L1_CAB ? 1 : 0;
  for (int j0 = 0; j0 < N; j0 += chunk) {
    const int nj = std::min(chunk, N - j0);
    kkt64(s, problem, m, nd, split, A, lda, b + (long)j0 * ldb, ldb, x + (long)j0 * ldx, ldx,
          e ? e + (long)j0 * lde : nullptr, lde, y ? y + (long)j0 * ldy : nullptr, ldy,
          eps ? eps + j0 : nullptr, lambda, nj, rbuf, report + 4L * j0);
  }
}

}  // namespace l1

using namespace l1;

extern "C" int l1_alm_kkt_noalloc(const float* A_dev, int m, int n_dict, int lda, int problem, int structure,
                                  double lambda, const float* b_dev, int ldb, int N, const float* eps_dev,
                                  const float* x_dev, int ldx, const float* e_dev, int lde, const float* y_dev,
                                  int ldy, double* report_dev, void* stream) {
  try {
    L1_REQUIRE(N >= 0, "N must be >= 0");
    L1_REQUIRE(problem >= 0 && problem <= 2, "unknown problem");
    L1_REQUIRE(structure == L1_DENSE || structure == L1_CAB, "unknown structure");
    L1_REQUIRE(!(structure == L1_CAB && problem != L1_P1),
               "QP_lambda and P_{1,2} are defined on a dense dictionary (structure L1_DENSE)");
    L1_REQUIRE(m >= 1 && n_dict >= 0 && lda >= m, "bad sizes: need m >= 1, n_dict >= 0, lda >= m");
    L1_REQUIRE(structure == L1_CAB || n_dict >= 1, "a dense dictionary needs n_dict >= 1");
    L1_REQUIRE(problem != L1_QPLAMBDA || lambda > 0, "QP_lambda needs lambda > 0");
    if (N == 0) return L1_OK;
    L1_REQUIRE(b_dev && x_dev && report_dev && (A_dev || n_dict == 0), "A, b, x and report must be non-NULL");
    L1_REQUIRE(ldb >= m && ldx >= std::max(n_dict, 1), "bad leading dimension");
    L1_REQUIRE(problem == L1_QPLAMBDA || y_dev != nullptr, "y is needed for P1 and P_{1,2}");
    L1_REQUIRE(problem != L1_P12 || eps_dev != nullptr, "P_{1,2} needs eps");
    L1_REQUIRE(structure != L1_CAB || e_dev != nullptr, "CAB needs e");
    if (y_dev) L1_REQUIRE(ldy >= m, "bad ldy");
    if (e_dev) L1_REQUIRE(lde >= m, "bad lde");
    kkt_noalloc(reinterpret_cast<hipStream_t>(stream), problem, structure, m, n_dict, A_dev, lda, b_dev, ldb, N,
                eps_dev, lambda, x_dev, ldx, e_dev, lde, y_dev, ldy, report_dev);
    return L1_OK;
  } catch (const Fail& f) {
    return f.code;
  } catch (const std::exception& e) {
    set_error(e.what());
    return L1_EHIP;
  }
}
