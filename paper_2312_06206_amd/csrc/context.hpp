// Internal: the solver context and helpers shared by the single-instance and the
// batched entry points.  Not part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <initializer_list>
#include <string>
#include <utility>
#include <vector>

#include "../../include/sadi.h"
#include "kernels.hpp"
#include "setup_device.hpp"

namespace sadi_impl {
// record msg as the calling thread's last error and return st
sadi_status fail(sadi_status st, const std::string& msg);
sadi_status check_launch();
bool finite_all(std::initializer_list<double> v);
bool supported_n(int n);
// host threads for the set-up maths of the calling thread (0: all hardware threads)
extern thread_local int g_setup_threads;
// set-up on this thread skips the run state buffers (contexts that only take batched steps)
extern thread_local bool g_setup_no_run_state;
// set-up on this thread leaves the device line tables (N + 1 = M) to the caller, who runs
// them for many contexts in one launch (sadi_ctx::gs_pending)
extern thread_local bool g_setup_defer_gs;
// argument checks of sadi_setup (allow2: alpha = 2 accepted, for injected tables)
sadi_status validate_problem(double alpha, double kappa, int n, double tau, const double* domain, bool allow2);
}  // namespace sadi_impl

#define SADI_HIP(call)                                                                                  \
  do {                                                                                                  \
    hipError_t e_ = (call);                                                                             \
    if (e_ != hipSuccess)                                                                               \
      return sadi_impl::fail(SADI_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_));         \
  } while (0)
// the same, returning on_error(status) (a clean-up that passes the status through)
#define SADI_HIP_OR(call, on_error)                                                                     \
  do {                                                                                                  \
    hipError_t e_ = (call);                                                                             \
    if (e_ != hipSuccess)                                                                               \
      return on_error(sadi_impl::fail(SADI_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_))); \
  } while (0)

struct sadi_ctx {
  int n = 0, m = 0;
  int r = 1;                   // M - N: rank of the correction from H_M^-1 to H_N^-1
  double alpha = 0, kappa = 0, tau = 0, a = 0, b = 0, h = 0, h_alpha = 0, beta = 0;
  sadi_g_kind g = SADI_G_NEG_SIN;
  double g_param = 0.0;
  sadi_precision prec = SADI_FP64;
  hipStream_t stream = nullptr;
  int magic = 0x5AD1;
  long long device_bytes = 0;

  // device data
  double2* rootM = nullptr;    // T entries
  double2* rootS = nullptr;    // E entries
  double2* root2M = nullptr;   // M entries, e^{-2 pi i k / 2M}
  double2* lam_s = nullptr;
  double2* lam_c = nullptr;
  double* f = nullptr;         // N
  double* lam2d = nullptr;     // (M+1) rows x ldlam
  int ldlam = 0;
  double2* S = nullptr;        // N rows x ldS complex
  int ldS = 0;
  double* X = nullptr;         // N rows x ldX (M rows when the correction is a GEMM)
  int ldX = 0;
  // Corrections of rank r > kTailGemmMinRank: the line solves leave the bordered solution of
  // size M and one matrix-core product per sweep applies the rank-r correction to all lines.
  // X then keeps plain rows (the product addresses it as a matrix); otherwise rows are
  // paired.  Measured: the per-line correction costs 0.03 ms/step at r = 2 (N = 4094) but
  // 0.2 ms at r = 8 and 1.0 ms at r = 32, where the product path costs 0.12-0.14 ms.
  static constexpr int kTailGemmMinRank = 3;
  bool tail_gemm = false;
  bool x_paired = true;
  // mixed precision: FP32 copies of the FFT and Gohberg-Semencul tables, FP64 eigenvalues
  // of the 2M-circulant embedding of beta T(a) (even / odd frequencies, scaled by 1/(2M))
  float2* rootM32 = nullptr;
  float2* rootS32 = nullptr;
  float2* q32 = nullptr;
  float2* lam_s32 = nullptr;
  float2* lam_c32 = nullptr;
  float* f32 = nullptr;
  double* sig_e = nullptr;
  double* sig_o = nullptr;
  double* partial = nullptr;   // 4 N partial sums (adjoint inner products)
  // sadi_run's copies of the two state arrays in paired rows (N + 1 rows of pitch N each),
  // or null (the run then works on the caller's arrays in plain rows)
  double* run_state[2] = {nullptr, nullptr};
  // set up with the device line tables deferred: their job (the tables lam_s, lam_c, f and
  // copies are not yet written while gs_pending)
  bool gs_pending = false;
  sadi::GsJob gs_job{};
  // device the context was set up on, and that device's static work space of
  // sadi_step_noalloc (null if its address could not be resolved)
  int device = 0;
  void* scratch = nullptr;

  std::vector<void*> allocs;

  // per-kernel timing: events[5*s + k] precedes kernel k of timed step s (k = 4: end)
  bool timing = false;
  std::vector<hipEvent_t> events;
  int timed_steps = 0;
  static constexpr int kMaxTimedSteps = 8192;

  sadi_status alloc(void** p, size_t bytes) {
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
      *p = nullptr;
      return sadi_impl::fail(SADI_E_NOMEM, std::string("hipMalloc(") + std::to_string(bytes) + "): " + hipGetErrorString(e));
    }
    allocs.push_back(*p);
    device_bytes += (long long)bytes;
    return SADI_OK;
  }
  void release() {
    for (void* p : allocs) (void)hipFree(p);
    allocs.clear();
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
    events.clear();
  }
  // event k of the current timed step (creating it on demand); null when not timing
  hipEvent_t mark(int k) {
    if (!timing || timed_steps >= kMaxTimedSteps) return nullptr;
    const size_t idx = (size_t)timed_steps * 5 + k;
    while (events.size() <= idx) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      events.push_back(e);
    }
    return events[idx];
  }
};

namespace sadi {
// The node rows ive(k, x_q) of the a_ij quadrature on the current device (setup_device.hip):
// rows[q * ld + k] for k < ld, and their first kLapLowOrders orders on the host,
// low[q * kLapLowOrders + k].  Built on first use per device, kept until the process ends.
sadi_status quadrature_table(const double** rows, int* ld, const double** low);
}  // namespace sadi

namespace sadi_impl {

inline bool ctx_ok(const sadi_ctx* c) { return c != nullptr && c->magic == 0x5AD1; }

// ---------------------------------------------------------------------------------
// dispatch on M
template <template <int> class F, class... A>
void dispatch_m(int m, A&&... args) {
  switch (m) {
#define SADI_CASE(MM) \
  case MM:            \
    F<MM>::run(std::forward<A>(args)...); \
    break;
    SADI_FOR_EACH_M(SADI_CASE)
#undef SADI_CASE
    default:
      break;
  }
}

template <int M> int threads_per_line() { return M / sadi::Shape<M>::E; }
template <int M> int e_of() { return sadi::Shape<M>::E; }
template <int M> int p2_of() { return sadi::Shape<M>::P2; }

struct ShapeInfo {
  int E, P2, T;
};
inline ShapeInfo shape_of(int m) {
  switch (m) {
#define SADI_SH(MM) \
  case MM:          \
    return ShapeInfo{sadi::Shape<MM>::E, sadi::Shape<MM>::P2, MM / sadi::Shape<MM>::E};
    SADI_FOR_EACH_M(SADI_SH)
#undef SADI_SH
    default:
      return ShapeInfo{0, 0, 0};
  }
}

inline sadi::FFTTables<double> tables(const sadi_ctx* c) { return sadi::FFTTables<double>{c->rootM, c->rootS, c->root2M}; }
inline sadi::GSTables64 gs_tables(const sadi_ctx* c) {
  return sadi::GSTables64{c->root2M, c->lam_s, c->lam_c, c->f, c->r};
}
// tables of the time step's sweeps: r = 0 when the correction is left to the GEMM
inline sadi::GSTables64 step_gs_tables(const sadi_ctx* c) {
  return sadi::GSTables64{c->root2M, c->lam_s, c->lam_c, c->f, c->tail_gemm ? 0 : c->r};
}


inline sadi::StepScalars scalars(const sadi_ctx* c, bool first) {
  sadi::StepScalars sc{};
  const double t2 = c->tau * c->tau;
  const double w = first ? 0.5 : 1.0;
  sc.sigma = -w * t2 * c->kappa * c->h_alpha;   // h_alpha = h^-alpha
  sc.gamma = w * t2;
  sc.tau = c->tau;
  sc.gkind = (int)c->g;
  sc.gparam = c->g_param;
  return sc;
}

}  // namespace sadi_impl
