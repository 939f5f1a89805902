// C ABI of the S-ADI solver: context, setup, and the entry points of include/sadi.h.
#include "../../include/sadi.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <exception>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "context.hpp"
#include "kernels.hpp"
#include "setup_math.hpp"

namespace sadi_impl {

thread_local std::string g_last_error;
thread_local int g_setup_threads = 0;
thread_local bool g_setup_no_run_state = false;
thread_local bool g_setup_defer_gs = false;

sadi_status fail(sadi_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

sadi_status check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(SADI_E_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
  return SADI_OK;
}

bool finite_all(std::initializer_list<double> v) {
  for (double x : v)
    if (!std::isfinite(x)) return false;
  return true;
}

bool supported_n(int n) { return n >= 15 && n <= 4095; }

sadi_status validate_problem(double alpha, double kappa, int n, double tau, const double* domain, bool allow2) {
  if (!domain) return fail(SADI_E_INVALID, "domain is NULL");
  if (!finite_all({alpha, kappa, tau, domain[0], domain[1]}))
    return fail(SADI_E_INVALID, "non-finite parameter");
  if (!(alpha > 1.0 && (alpha < 2.0 || (allow2 && alpha <= 2.0))))
    return fail(SADI_E_INVALID, "alpha must lie in (1, 2)");
  if (!(kappa > 0.0)) return fail(SADI_E_INVALID, "kappa must be positive");
  if (!(tau > 0.0)) return fail(SADI_E_INVALID, "tau must be positive");
  if (!(domain[1] > domain[0])) return fail(SADI_E_INVALID, "domain must satisfy b > a");
  if (n < 1) return fail(SADI_E_INVALID, "N must be >= 1");
  if (!supported_n(n)) return fail(SADI_E_UNSUPPORTED, "N must lie in [15, 4095]");
  return SADI_OK;
}

}  // namespace sadi_impl

using namespace sadi_impl;

namespace {

// Work space of sadi_step_noalloc: the half spectrum S and the x-sweep result X of one step,
// in a static device array instead of the context's buffers.  Every GPU that loads the
// library holds its own copy until the process ends.  In host code `scratch` only names the
// symbol; its device address is looked up once per device (resolve_scratch, called by
// set-up with the context's device current) and only that address is used.
constexpr size_t kScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_addr[kMaxDevices] = {};

// device address of `scratch` on the current device (nullptr if it cannot be resolved)
void* resolve_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
      (void)hipGetLastError();   // leave no error behind for the next call
      return nullptr;
    }
    g_scratch_addr[dev] = p;
  }
  return g_scratch_addr[dev];
}

// Streams for set-up work, per device: taken for the length of one set-up and returned, so
// that contexts set up one after another (or on a pool of host threads) reuse them instead
// of creating and destroying two streams each.  Kept until the process ends; at most as
// many as set-ups ran at once.
std::mutex g_setup_stream_mutex;
std::vector<hipStream_t> g_setup_streams[kMaxDevices];

hipError_t take_setup_stream(int dev, hipStream_t* s) {
  if (dev >= 0 && dev < kMaxDevices) {
    std::lock_guard<std::mutex> lock(g_setup_stream_mutex);
    if (!g_setup_streams[dev].empty()) {
      *s = g_setup_streams[dev].back();
      g_setup_streams[dev].pop_back();
      return hipSuccess;
    }
  }
  return hipStreamCreateWithFlags(s, hipStreamNonBlocking);
}

// s must be idle (synchronised) when it is returned
void return_setup_stream(int dev, hipStream_t s) {
  if (!s) return;
  if (dev >= 0 && dev < kMaxDevices) {
    std::lock_guard<std::mutex> lock(g_setup_stream_mutex);
    g_setup_streams[dev].push_back(s);
    return;
  }
  (void)hipStreamDestroy(s);
}

// bytes of the step's work space in the static array: S (rows in pairs), 256-byte aligned,
// then X
size_t noalloc_s_bytes(const sadi_ctx* c) {
  return (sizeof(double2) * (size_t)(c->n + 1) * c->ldS + 255) & ~size_t(255);
}
size_t noalloc_bytes(const sadi_ctx* c) { return noalloc_s_bytes(c) + sizeof(double) * (size_t)(c->n + 1) * c->ldX; }

template <int M> struct RowsFwd {
  static void run(const sadi_ctx* c, const double* u, double* lf_prev) {
    sadi::launch_rows_fwd<M>(u, lf_prev, lf_prev ? c->X : nullptr, c->ldX, c->n, c->S, c->ldS, c->n, tables(c),
                             c->root2M, c->stream);
  }
};
template <int M> struct ColsConv {
  static void run(const sadi_ctx* c) {
    sadi::launch_cols_conv<M>(c->S, c->ldS, c->n, c->lam2d, c->ldlam, tables(c), c->root2M, c->stream);
  }
};
template <int M> struct RowsRhs {
  static void run(const sadi_ctx* c, int mode, const double* u, const double* phi2, double* X, int ldx,
                  const sadi::StepScalars& sc, bool u_paired = false) {
    sadi::launch_rows_rhs_gs<M>(mode, c->S, c->ldS, u, c->n, phi2, X, ldx, c->x_paired, c->n, sc, tables(c),
                                step_gs_tables(c), c->root2M, c->stream, u_paired);
  }
};
template <int M> struct ColsGS {
  static void run(const sadi_ctx* c, int mode, const double* ucur, const double* uprev, double* uout) {
    sadi::launch_cols_gs<M>(mode, c->X, c->ldX, ucur, uprev, uout, c->n, c->n, tables(c), step_gs_tables(c),
                            c->stream);
  }
};
template <int M> struct ColsGSFwd {   // y-sweep, update into the transposed layout, next row pass
  static void run(const sadi_ctx* c, const double* ucur, double* prev_t, bool fwd, bool u_paired) {
    sadi::launch_cols_gs_fwd<M>(c->X, c->ldX, ucur, prev_t, c->n, c->S, c->ldS, fwd, tables(c), step_gs_tables(c),
                                c->root2M, c->stream, u_paired);
  }
};
template <int M> struct ColsGSPitched {   // in-place y-line solves of an N x ldX buffer
  static void run(const sadi_ctx* c, double* buf) {
    sadi::launch_cols_gs<M>(2, buf, c->ldX, nullptr, nullptr, nullptr, c->n, c->n, tables(c), gs_tables(c),
                            c->stream);
  }
};
template <int M> struct RowsFwdPitched {  // spectrum of a grid function with row pitch ld
  static void run(const sadi_ctx* c, const double* u, int ld) {
    sadi::launch_rows_fwd<M>(u, nullptr, nullptr, c->ldX, ld, c->S, c->ldS, c->n, tables(c), c->root2M, c->stream);
  }
};
template <int M> struct BccbEig {   // work_real may be lam2d itself (see launch_bccb_eigenvalues)
  static void run(const sadi_ctx* c, const double* a2d, double* work_real, double* g0, double2* spec) {
    sadi::launch_bccb_eigenvalues<M>(a2d, c->n, work_real, c->ldlam, g0, spec, c->ldS, c->lam2d, c->ldlam, tables(c),
                                     c->stream);
  }
};
template <int M> struct RowsGS {
  static void run(const sadi_ctx* c, double* lines, int ld, int nlines) {
    sadi::launch_rows_gs<M>(lines, ld, nlines, c->n, tables(c), gs_tables(c), c->stream);
  }
};

sadi::MixedTables mixed_tables(const sadi_ctx* c) {
  sadi::MixedTables mx{};
  mx.tab32 = sadi::FFTTables<float>{c->rootM32, c->rootS32, c->q32};
  mx.gs32 = sadi::GSTables<float>{c->q32, c->lam_s32, c->lam_c32, c->f32, 1};
  mx.toe = sadi::ToeplitzTables64{c->sig_e, c->sig_o};
  mx.q64 = c->root2M;
  mx.refine = c->prec == SADI_FP32_REFINE ? 1 : 0;
  return mx;
}
template <int M> struct RowsRhsMixed {
  static void run(const sadi_ctx* c, int mode, const double* u, const double* phi2, const sadi::StepScalars& sc,
                  bool u_paired = false) {
    sadi::launch_rows_rhs_mixed<M>(mode, c->S, c->ldS, u, c->n, phi2, c->X, c->ldX, c->n, sc, tables(c),
                                   mixed_tables(c), c->root2M, c->stream, u_paired);
  }
};
template <int M> struct ColsGSMixed {
  static void run(const sadi_ctx* c, int mode, const double* ucur, const double* uprev, double* uout) {
    sadi::launch_cols_gs_mixed<M>(mode, c->X, c->ldX, ucur, uprev, uout, c->n, c->n, tables(c), mixed_tables(c),
                                  c->stream);
  }
};
template <int M> struct ColsGSFwdMixed {   // mixed y-sweep, update into the transposed layout, next row pass
  static void run(const sadi_ctx* c, const double* ucur, double* prev_t, bool fwd, bool u_paired) {
    sadi::launch_cols_gs_fwd_mixed<M>(c->X, c->ldX, ucur, prev_t, c->n, c->S, c->ldS, fwd, tables(c), mixed_tables(c),
                                      c->root2M, c->stream, u_paired);
  }
};
template <int M> struct RowsGSMixed {
  static void run(const sadi_ctx* c, double* lines, int ld, int nlines) {
    sadi::launch_rows_gs_mixed<M>(lines, ld, nlines, c->n, tables(c), mixed_tables(c), c->stream);
  }
};

// Rank-r correction of every line of X from its bordered solution w (size M, the step's
// sweeps ran with r = 0): x = w[0:N] - F w[N:M] with F stored as r rows of N (section
// "Fast implementation based on GS formula" solves at size M; the Schur complement of the
// bordered matrix gives H_N^-1).  One matrix-core product per sweep:
//   rows:    X[y][k] -= sum_j X[y][N + j] F[j][k]   (C = X[:, 0:N], A = X[:, N:M], B = F)
//   columns: X[k][c] -= sum_j F[j][k] X[N + j][c]   (C = X[0:N, :], A = F^T, B = X[N:M, :])
sadi_status tail_correct(sadi_ctx* c, bool columns) {
  const int n = c->n, r = c->r, ld = c->ldX;
  if (!columns)
    sadi::launch_dgemm(n, n, r, sadi::GemmPtrs{c->X + n, c->f, c->X}, nullptr, 1, true, ld, n, ld, -1.0, 1.0,
                       c->stream);
  else
    sadi::launch_dgemm(n, n, r, sadi::GemmPtrs{c->f, c->X + (size_t)n * ld, c->X}, nullptr, 1, false, n, ld, ld,
                       -1.0, 1.0, c->stream);
  return check_launch();
}

// one step of the delta form on the device; mode 0: uout = 2 ucur - uprev + Uhat,
// mode 1 (start-up): uout = ucur + Uhat with phi2.
// Deferred update (FP64 runs): cols_mode 2 leaves Uhat in X instead of forming uout, and a
// non-null lf_prev makes the row transform first finish the previous step's update,
// lf_prev <- 2 ucur - lf_prev + X; the step then advances the state now held in lf_prev.
sadi_status enqueue_step(sadi_ctx* c, int mode, const double* ucur, const double* uprev, const double* phi2,
                         double* uout, int cols_mode = -1, double* lf_prev = nullptr) {
  auto mark = [&](int k) {
    hipEvent_t e = c->mark(k);
    if (e) (void)hipEventRecord(e, c->stream);
  };
  if (cols_mode < 0) cols_mode = mode;
  mark(0);
  dispatch_m<RowsFwd>(c->m, c, ucur, lf_prev);
  if (lf_prev) ucur = lf_prev;
  mark(1);
  dispatch_m<ColsConv>(c->m, c);
  mark(2);
  const sadi::StepScalars sc = scalars(c, mode == 1);
  if (c->prec == SADI_FP64) {
    dispatch_m<RowsRhs>(c->m, c, mode, ucur, phi2, c->X, c->ldX, sc);
    if (c->tail_gemm) {
      sadi_status st = tail_correct(c, false);
      if (st != SADI_OK) return st;
    }
  } else {
    dispatch_m<RowsRhsMixed>(c->m, c, mode, ucur, phi2, sc);
  }
  mark(3);
  if (c->prec == SADI_FP64 && c->tail_gemm) {
    // Uhat into X, its correction, then the update unless the next row pass applies it
    dispatch_m<ColsGS>(c->m, c, 2, ucur, uprev, uout);
    sadi_status st = tail_correct(c, true);
    if (st != SADI_OK) return st;
    if (cols_mode != 2)
      sadi::launch_leapfrog(cols_mode == 0 ? 0 : 1, const_cast<double*>(ucur), const_cast<double*>(uprev), c->X,
                            c->ldX, uout, c->n, c->stream);
  } else if (c->prec == SADI_FP64) {
    dispatch_m<ColsGS>(c->m, c, cols_mode, ucur, uprev, uout);
  } else
    dispatch_m<ColsGSMixed>(c->m, c, mode, ucur, uprev, uout);
  mark(4);
  if (c->timing && c->timed_steps < sadi_ctx::kMaxTimedSteps) ++c->timed_steps;
  return check_launch();
}

// a2: the coefficient table a_ij (N x N), or empty with ls: the alpha-dependent parts of its
// quadrature, combined on the device with the node rows of quadrature_table
sadi_status build_ctx(double alpha, double kappa, int n, double tau, const double* domain,
                      const std::vector<double>& a1, const std::vector<double>& a2, const sadi::LapSetup* ls,
                      sadi_ctx** out) {
  sadi_ctx* c = new (std::nothrow) sadi_ctx();
  if (!c) return fail(SADI_E_NOMEM, "host allocation failed");
  c->n = n;
  c->m = sadi::line_size(n);
  c->r = c->m - n;
  c->tail_gemm = c->r > sadi_ctx::kTailGemmMinRank;
  c->x_paired = !c->tail_gemm;
  c->alpha = alpha;
  c->kappa = kappa;
  c->tau = tau;
  c->a = domain[0];
  c->b = domain[1];
  c->h = (c->b - c->a) / (n + 1);
  c->h_alpha = std::pow(c->h, -alpha);
  c->beta = kappa * tau * tau * c->h_alpha / 2.0;
  const int m = c->m;
  const ShapeInfo sh = shape_of(m);
  auto bail = [&](sadi_status st) {
    c->release();
    delete c;
    return st;
  };

  // ---- host tables.  The Gohberg-Semencul data of H_M come from the device when N + 1 = M
  // (Levinson-Durbin in double-double, gs_tables_kernel), else from the host (gs_data, which
  // also forms the rank-(M - N) correction); the host receives the first column of H_M in
  // extended precision either way.
  const bool device_gs = c->r == 1;
  sadi::GSData gsd;
  std::vector<double> t_hi(m), t_lo(m);
  for (int k = 0; k < m; ++k) {
    const long double tk = (k == 0 ? 1.0L : 0.0L) + (long double)c->beta * a1[k];
    t_hi[k] = (double)tk;
    t_lo[k] = (double)(tk - (long double)t_hi[k]);
  }
  if (device_gs) {
    gsd.n = n;
    gsd.m = m;
    gsd.r = 1;
    gsd.lam_s.assign(m, {0.0, 0.0});
    gsd.lam_c.assign(m, {0.0, 0.0});
    gsd.f.assign(n, 0.0);
  } else {
    try {
      gsd = sadi::gs_data(a1, n, c->m, c->beta, g_setup_threads);
    } catch (const std::exception& e) {
      return bail(fail(SADI_E_INVALID, std::string("line matrix: ") + e.what()));
    }
  }
  const long double pi = 3.14159265358979323846264338327950288L;
  std::vector<double2> hrootM(sh.T), hrootS(sh.E), hroot2M(m);
  for (int j = 0; j < sh.T; ++j) {
    const long double a = -2.0L * pi * j / m;
    hrootM[j] = make_double2((double)std::cos(a), (double)std::sin(a));
  }
  for (int j = 0; j < sh.E; ++j) {
    const long double a = -2.0L * pi * j / (sh.E * sh.P2);
    hrootS[j] = make_double2((double)std::cos(a), (double)std::sin(a));
  }
  for (int k = 0; k < m; ++k) {
    const long double a = -pi * k / m;
    hroot2M[k] = make_double2((double)std::cos(a), (double)std::sin(a));
  }
  std::vector<double2> hls(m), hlc(m);
  for (int k = 0; k < m; ++k) {
    hls[k] = make_double2(gsd.lam_s[k].real(), gsd.lam_s[k].imag());
    hlc[k] = make_double2(gsd.lam_c[k].real(), gsd.lam_c[k].imag());
  }
  c->ldlam = m + 1 + ((8 - (m + 1) % 8) % 8);
  const size_t lam_elems = (size_t)(m + 1) * c->ldlam;

  // ---- mixed precision tables
  std::vector<float2> hrootM32(sh.T), hrootS32(sh.E), hq32(m), hls32(m), hlc32(m);
  std::vector<float> hf32(n);
  for (int j = 0; j < sh.T; ++j) hrootM32[j] = make_float2((float)hrootM[j].x, (float)hrootM[j].y);
  for (int j = 0; j < sh.E; ++j) hrootS32[j] = make_float2((float)hrootS[j].x, (float)hrootS[j].y);
  for (int k = 0; k < m; ++k) {
    hq32[k] = make_float2((float)hroot2M[k].x, (float)hroot2M[k].y);
    hls32[k] = make_float2((float)hls[k].x, (float)hls[k].y);
    hlc32[k] = make_float2((float)hlc[k].x, (float)hlc[k].y);
  }
  if (c->r == 1)
    for (int k = 0; k < n; ++k) hf32[k] = (float)gsd.f[k];   // FP32 solves: N = M - 1 only
  // beta T(a_0..a_{N-1}) embedded in a circulant of size P = 2M (first column a_0..a_{N-1},
  // three zeros, a_{N-1}..a_1); its eigenvalues split into even / odd frequencies
  std::vector<double> hsig_e(m), hsig_o(m);
  {
    const int p = 2 * m;
    std::vector<sadi::cld> cemb(p, sadi::cld(0, 0));
    for (int j = 0; j < n; ++j) {
      cemb[j] = a1[j];
      if (j > 0) cemb[p - j] = a1[j];
    }
    sadi::fft_inplace(cemb, -1);
    const long double sc = (long double)c->beta / p;
    for (int k = 0; k < m; ++k) {
      hsig_e[k] = (double)(cemb[2 * k].real() * sc);
      hsig_o[k] = (double)(cemb[2 * k + 1].real() * sc);
    }
  }

  // ---- device memory: one allocation.  The tables (and the set-up's temporary factors at
  // the start of S) are filled from one host staging buffer with one copy; during set-up X
  // holds a_ij, S the row transforms and lam2d the intermediate of the eigenvalue passes.
  c->ldS = m + 8;           // complex elements per row of the half spectrum (>= M+1); rows in pairs
  c->ldX = m;
  // X: N rows (paired rows: ceil(N / 2) pairs of 2 ldX values), or the M rows of the bordered
  // y-line solutions when the correction is a GEMM
  const size_t xrows = c->tail_gemm ? (size_t)m : (size_t)n + 1;
  // S: N rows stored in interleaved pairs; M + 2 rows during set-up (the eigenvalue passes)
  const size_t srows = std::max((size_t)n + 1, (size_t)m + 2);
  size_t off = 0;
  auto place = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return o;
  };
  const size_t o_rootM = place(sizeof(double2) * sh.T), o_rootS = place(sizeof(double2) * sh.E),
               o_root2M = place(sizeof(double2) * m), o_ls = place(sizeof(double2) * m),
               o_lc = place(sizeof(double2) * m), o_f = place(sizeof(double) * gsd.f.size()),
               o_rootM32 = place(sizeof(float2) * sh.T), o_rootS32 = place(sizeof(float2) * sh.E),
               o_q32 = place(sizeof(float2) * m), o_ls32 = place(sizeof(float2) * m),
               o_lc32 = place(sizeof(float2) * m), o_f32 = place(sizeof(float) * n),
               o_sige = place(sizeof(double) * m), o_sigo = place(sizeof(double) * m),
               o_partial = place(sizeof(double) * 4 * (size_t)n);
  // the set-up's factors of a_ij at the start of S: node weights, high-tail rows (for small N
  // they take more room than the spectrum)
  const size_t ft = ls ? (size_t)ls->ht * n : 0;
  const size_t fbytes = ls ? sizeof(double) * (ls->nq + 2 * ft) : 0;
  const size_t o_S = place(std::max(sizeof(double2) * srows * c->ldS, fbytes));
  const size_t o_X = place(sizeof(double) * xrows * c->ldX);
  const size_t o_lam = place(sizeof(double) * lam_elems);
  // sadi_run's paired-row copies of the state (three-kernel runs; not for batch members)
  const bool run_state = !c->tail_gemm && !g_setup_no_run_state;
  const size_t run_bytes = run_state ? sizeof(double) * (size_t)(n + 1) * n : 0;
  const size_t o_run0 = run_state ? place(run_bytes) : 0, o_run1 = run_state ? place(run_bytes) : 0;
  const size_t o_fw = o_S, o_fa = o_fw + sizeof(double) * (ls ? ls->nq : 0), o_fc = o_fa + sizeof(double) * ft;
  // the first column of H_M (double-double) for the device Levinson recursion and its
  // result c, in the adjoint's partial-sum space (4 N doubles, unused until a step), which
  // nothing else of the set-up touches: the recursion runs beside the a_ij products
  const size_t o_thi = o_partial, o_tlo = o_thi + sizeof(double) * m, o_cvec = o_tlo + sizeof(double) * m;
  const size_t staged = o_S + fbytes;
  sadi_status st;
  unsigned char* pool = nullptr;
  if ((st = c->alloc((void**)&pool, off)) != SADI_OK) return bail(st);
  c->rootM = (double2*)(pool + o_rootM);
  c->rootS = (double2*)(pool + o_rootS);
  c->root2M = (double2*)(pool + o_root2M);
  c->lam_s = (double2*)(pool + o_ls);
  c->lam_c = (double2*)(pool + o_lc);
  c->f = (double*)(pool + o_f);
  c->rootM32 = (float2*)(pool + o_rootM32);
  c->rootS32 = (float2*)(pool + o_rootS32);
  c->q32 = (float2*)(pool + o_q32);
  c->lam_s32 = (float2*)(pool + o_ls32);
  c->lam_c32 = (float2*)(pool + o_lc32);
  c->f32 = (float*)(pool + o_f32);
  c->sig_e = (double*)(pool + o_sige);
  c->sig_o = (double*)(pool + o_sigo);
  c->partial = (double*)(pool + o_partial);
  if (run_state) {
    c->run_state[0] = (double*)(pool + o_run0);
    c->run_state[1] = (double*)(pool + o_run1);
  }
  c->S = (double2*)(pool + o_S);
  c->X = (double*)(pool + o_X);
  c->lam2d = (double*)(pool + o_lam);
  {
    std::vector<unsigned char> host(staged, 0);
    auto put = [&](size_t o, const void* src, size_t bytes) {
      if (bytes) std::memcpy(host.data() + o, src, bytes);
    };
    put(o_rootM, hrootM.data(), sizeof(double2) * sh.T);
    put(o_rootS, hrootS.data(), sizeof(double2) * sh.E);
    put(o_root2M, hroot2M.data(), sizeof(double2) * m);
    put(o_ls, hls.data(), sizeof(double2) * m);
    put(o_lc, hlc.data(), sizeof(double2) * m);
    put(o_f, gsd.f.data(), sizeof(double) * gsd.f.size());
    put(o_rootM32, hrootM32.data(), sizeof(float2) * sh.T);
    put(o_rootS32, hrootS32.data(), sizeof(float2) * sh.E);
    put(o_q32, hq32.data(), sizeof(float2) * m);
    put(o_ls32, hls32.data(), sizeof(float2) * m);
    put(o_lc32, hlc32.data(), sizeof(float2) * m);
    put(o_f32, hf32.data(), sizeof(float) * n);
    put(o_sige, hsig_e.data(), sizeof(double) * m);
    put(o_sigo, hsig_o.data(), sizeof(double) * m);
    if (ls) {
      put(o_fw, ls->w.data(), sizeof(double) * ls->nq);
      put(o_fa, ls->tail_a.data(), sizeof(double) * ft);
      put(o_fc, ls->tail_c.data(), sizeof(double) * ft);
    }
    if (device_gs) {
      put(o_thi, t_hi.data(), sizeof(double) * m);
      put(o_tlo, t_lo.data(), sizeof(double) * m);
    }
    SADI_HIP_OR(hipMemcpy(pool, host.data(), staged, hipMemcpyHostToDevice), bail);
  }
  // set-up work runs on streams of its own (contexts set up concurrently on several host
  // threads overlap on the device), synchronised before returning
  int sdev = 0;
  if (hipGetDevice(&sdev) != hipSuccess) sdev = -1;
  hipStream_t sst = nullptr, sgs = nullptr;
  SADI_HIP_OR(take_setup_stream(sdev, &sst), bail);
  auto bail_s = [&](sadi_status e) {
    for (hipStream_t q : {sst, sgs})
      if (q) {
        (void)hipStreamSynchronize(q);
        (void)hipStreamDestroy(q);   // not returned: the stream may hold a failed launch
      }
    return bail(e);
  };
  if (device_gs && g_setup_defer_gs) {   // the caller runs the tables (with other contexts')
    c->gs_job = sadi::GsJob{(const double*)(pool + o_thi), (const double*)(pool + o_tlo), (double*)(pool + o_cvec),
                            c->root2M, c->lam_s, c->lam_c, c->f, c->lam_s32, c->lam_c32, c->f32, m};
    c->gs_pending = true;
  } else if (device_gs) {   // c = H_M^-1 e_1 (one workgroup, sequential in k), then the tables
    SADI_HIP_OR(take_setup_stream(sdev, &sgs), bail_s);
    sadi::launch_gs_generator((const double*)(pool + o_thi), (const double*)(pool + o_tlo), m,
                              (double*)(pool + o_cvec), c->root2M, c->lam_s, c->lam_c, c->f, c->lam_s32, c->lam_c32,
                              c->f32, sgs);
  }

  // ---- a_ij into X, on the device unless a table was given: the quadrature over the nodes
  // and the high tail as two matrix-core products, then the exact corner.  Then the
  // eigenvalues of the block-circulant embedding of L_h with the row transform: two passes
  // of even-extension DFTs through S, the intermediate in lam2d (its first column also after
  // a_ij in X).
  {
    double* a2d = c->X;
    const size_t nn = (size_t)n * n;
    if (ls) {
      const double* rows = nullptr;
      const double* low = nullptr;
      int ldr = 0;
      if ((st = sadi::quadrature_table(&rows, &ldr, &low)) != SADI_OK) return bail_s(st);
      const double* fw = (const double*)(pool + o_fw);
      const double* fa = (const double*)(pool + o_fa);
      const double* fc = (const double*)(pool + o_fc);
      // a2d[j n + i] = scale (sum_q R[q][j] w_q R[q][i] + sum_p C_p(j) A_p(i)), R the node rows
      sadi::launch_dgemm(n, n, ls->nq, sadi::GemmPtrs{rows, rows, a2d}, nullptr, 1, false, ldr, ldr, n, ls->scale,
                         0.0, sst, 0, fw);
      sadi::launch_dgemm(n, n, ls->ht, sadi::GemmPtrs{fc, fa, a2d}, nullptr, 1, false, n, n, n, ls->scale, 1.0,
                         sst);
      SADI_HIP_OR(hipGetLastError(), bail_s);
      SADI_HIP_OR(hipMemcpy2DAsync(a2d, sizeof(double) * n, ls->corner.data(), sizeof(double) * ls->nc,
                                   sizeof(double) * ls->nc, ls->nc, hipMemcpyHostToDevice, sst),
                  bail_s);
    } else {
      SADI_HIP_OR(hipMemcpyAsync(a2d, a2.data(), sizeof(double) * nn, hipMemcpyHostToDevice, sst), bail_s);
    }
    const hipStream_t own = c->stream;
    c->stream = sst;
    dispatch_m<BccbEig>(m, c, a2d, c->lam2d, a2d + nn, c->S);
    c->stream = own;
    SADI_HIP_OR(hipGetLastError(), bail_s);
    SADI_HIP_OR(hipStreamSynchronize(sst), bail_s);
    if (sgs) SADI_HIP_OR(hipStreamSynchronize(sgs), bail_s);
    return_setup_stream(sdev, sst);
    return_setup_stream(sdev, sgs);
  }
  // the static work space of sadi_step_noalloc on this device
  if (hipGetDevice(&c->device) != hipSuccess) return bail(fail(SADI_E_DEVICE, "hipGetDevice"));
  c->scratch = resolve_scratch(c->device);
  *out = c;
  return SADI_OK;
}

}  // namespace

extern "C" {

const char* sadi_last_error(void) { return sadi_impl::g_last_error.c_str(); }

sadi_status sadi_setup(double alpha, double kappa, int n, double tau, const double* domain, sadi_ctx** out) {
  if (!out) return fail(SADI_E_INVALID, "out is NULL");
  *out = nullptr;
  sadi_status st = validate_problem(alpha, kappa, n, tau, domain, false);
  if (st != SADI_OK) return st;
  try {
    const std::vector<double> a1 = sadi::riesz_coeffs(alpha, sadi::line_size(n));
    const double* rows = nullptr;
    const double* low = nullptr;
    int ldr = 0;
    st = sadi::quadrature_table(&rows, &ldr, &low);
    if (st != SADI_OK) return st;
    const sadi::LapSetup ls = sadi::laplacian_setup(alpha, n, low);
    return build_ctx(alpha, kappa, n, tau, domain, a1, {}, &ls, out);
  } catch (const std::bad_alloc&) {
    return fail(SADI_E_NOMEM, "host allocation failed in setup");
  } catch (const std::exception& e) {
    return fail(SADI_E_INVALID, std::string("setup: ") + e.what());
  }
}

sadi_status sadi_setup_with_coeffs(double alpha, double kappa, int n, double tau, const double* domain,
                                   const double* a1, const double* a2, sadi_ctx** out) {
  if (!out) return fail(SADI_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!a1 || !a2) return fail(SADI_E_INVALID, "coefficient table is NULL");
  sadi_status st = validate_problem(alpha, kappa, n, tau, domain, true);
  if (st != SADI_OK) return st;
  if (sadi::line_size(n) != n + 1)
    return fail(SADI_E_UNSUPPORTED, "injected coefficient tables need N + 1 to be a power of two");
  try {
    std::vector<double> v1(a1, a1 + n + 1), v2(a2, a2 + (size_t)n * n);
    return build_ctx(alpha, kappa, n, tau, domain, v1, v2, nullptr, out);
  } catch (const std::bad_alloc&) {
    return fail(SADI_E_NOMEM, "host allocation failed in setup");
  } catch (const std::exception& e) {
    return fail(SADI_E_INVALID, std::string("setup: ") + e.what());
  }
}

sadi_status sadi_set_options(sadi_ctx* c, sadi_g_kind g, double g_param, sadi_precision prec) {
  if (!ctx_ok(c)) return fail(SADI_E_STATE, "invalid context");
  if ((int)g < 0 || (int)g > 3) return fail(SADI_E_INVALID, "unknown g kind");
  if ((int)prec < 0 || (int)prec > 2) return fail(SADI_E_INVALID, "unknown precision");
  if (!std::isfinite(g_param)) return fail(SADI_E_INVALID, "g_param must be finite");
  if (prec != SADI_FP64 && c->r != 1)
    return fail(SADI_E_UNSUPPORTED, "float32 line solves need N + 1 to be a power of two");
  c->g = g;
  c->g_param = g_param;
  c->prec = prec;
  return SADI_OK;
}

sadi_status sadi_set_stream(sadi_ctx* c, void* s) {
  if (!ctx_ok(c)) return fail(SADI_E_STATE, "invalid context");
  c->stream = (hipStream_t)s;
  return SADI_OK;
}

sadi_status sadi_first_step(sadi_ctx* c, const double* phi1, const double* phi2, double* u1) {
  if (!ctx_ok(c)) return fail(SADI_E_STATE, "invalid context");
  if (!phi1 || !phi2 || !u1) return fail(SADI_E_INVALID, "NULL array");
  if (u1 == phi1 || u1 == phi2) return fail(SADI_E_INVALID, "u1 must not alias phi1 or phi2");
  return enqueue_step(c, 1, phi1, nullptr, phi2, u1);
}

sadi_status sadi_step(sadi_ctx* c, double* u_prev, const double* u_cur) {
  if (!ctx_ok(c)) return fail(SADI_E_STATE, "invalid context");
  if (!u_prev || !u_cur) return fail(SADI_E_INVALID, "NULL array");
  if (u_prev == u_cur) return fail(SADI_E_INVALID, "u_prev and u_cur must differ");
  return enqueue_step(c, 0, u_cur, u_prev, nullptr, u_prev);
}

sadi_status sadi_step_noalloc(sadi_ctx* c, double* u_prev, const double* u_cur) {
  if (!ctx_ok(c)) return fail(SADI_E_STATE, "invalid context");
  if (!u_prev || !u_cur) return fail(SADI_E_INVALID, "NULL array");
  if (u_prev == u_cur) return fail(SADI_E_INVALID, "u_prev and u_cur must differ");
  if (c->tail_gemm)
    return fail(SADI_E_UNSUPPORTED, "sadi_step_noalloc: M - N = " + std::to_string(c->r) +
                                        " > 3 (that correction runs as a library GEMM)");
  if (noalloc_bytes(c) > kScratchBytes)
    return fail(SADI_E_UNSUPPORTED, "sadi_step_noalloc: N = " + std::to_string(c->n) + " needs " +
                                        std::to_string(noalloc_bytes(c)) + " bytes of work space, more than the " +
                                        std::to_string(kScratchBytes) + " of the static array (N <= 1023)");
  int dev = -1;
  SADI_HIP(hipGetDevice(&dev));
  if (dev != c->device) return fail(SADI_E_INVALID, "sadi_step_noalloc: the context's device must be current");
  if (!c->scratch) return fail(SADI_E_DEVICE, "sadi_step_noalloc: the static work space has no device address");
  // the step's kernels take S and X from the context: point them at the static array for
  // this call (arguments are captured at launch) and restore the context's own buffers
  double2* own_s = c->S;
  double* own_x = c->X;
  const bool timing = c->timing;
  c->S = static_cast<double2*>(c->scratch);
  c->X = reinterpret_cast<double*>(static_cast<unsigned char*>(c->scratch) + noalloc_s_bytes(c));
  c->timing = false;   // no timing events: they are created on demand
  const sadi_status st = enqueue_step(c, 0, u_cur, u_prev, nullptr, u_prev);
  c->S = own_s;
  c->X = own_x;
  c->timing = timing;
  return st;
}

sadi_status sadi_run(sadi_ctx* c, double* u_prev, double* u_cur, int nsteps) {
  if (!ctx_ok(c)) return fail(SADI_E_STATE, "invalid context");
  if (!u_prev || !u_cur) return fail(SADI_E_INVALID, "NULL array");
  if (u_prev == u_cur) return fail(SADI_E_INVALID, "u_prev and u_cur must differ");
  if (nsteps < 0) return fail(SADI_E_INVALID, "nsteps must be >= 0");
  if (nsteps == 0) return SADI_OK;
  if (!c->tail_gemm) {
    // Three kernels per step: the y-sweep kernel also forms u^{n+1} and the next step's row
    // transform, on the transposed grid (x and y swap roles every step).  u^{n-1} starts in
    // the transposed layout; both arrays are back in the natural layout at the end.  The
    // float32 line solves take the same schedule, X in paired rows as well when the state is.
    auto mark = [&](int k) {
      hipEvent_t e = c->mark(k);
      if (e) (void)hipEventRecord(e, c->stream);
    };
    const sadi::StepScalars sc = scalars(c, false);
    // the state in paired rows for the run (the y-sweep then reads u^n by row pairs, as it
    // reads X), in the context's copies, when the context has them
    const bool paired = c->run_state[0] != nullptr;
    double* a = u_prev;   // u^{n-1}, transposed relative to b
    double* b = u_cur;    // u^n in this step's layout
    if (paired) {
      sadi::launch_state_to_paired(u_prev, c->run_state[0], c->n, true, c->stream);
      sadi::launch_state_to_paired(u_cur, c->run_state[1], c->n, false, c->stream);
      a = c->run_state[0];
      b = c->run_state[1];
    } else {
      sadi::launch_transpose_inplace(u_prev, c->n, c->stream);
    }
    for (int s = 0; s < nsteps; ++s) {
      mark(0);
      if (s == 0) dispatch_m<RowsFwd>(c->m, c, u_cur, nullptr);   // u^n in plain rows
      mark(1);
      dispatch_m<ColsConv>(c->m, c);
      mark(2);
      if (c->prec == SADI_FP64)
        dispatch_m<RowsRhs>(c->m, c, 0, b, nullptr, c->X, c->ldX, sc, paired);
      else
        dispatch_m<RowsRhsMixed>(c->m, c, 0, b, nullptr, sc, paired);
      mark(3);
      if (c->prec == SADI_FP64)
        dispatch_m<ColsGSFwd>(c->m, c, b, a, s + 1 < nsteps, paired);
      else
        dispatch_m<ColsGSFwdMixed>(c->m, c, b, a, s + 1 < nsteps, paired);
      mark(4);
      if (c->timing && c->timed_steps < sadi_ctx::kMaxTimedSteps) ++c->timed_steps;
      sadi_status st = check_launch();
      if (st != SADI_OK) return st;
      std::swap(a, b);
    }
    // b holds the newest state (transposed when nsteps is odd), a the one before
    if (paired) {
      sadi::launch_state_from_paired(b, u_cur, c->n, nsteps % 2 == 1, c->stream);
      sadi::launch_state_from_paired(a, u_prev, c->n, nsteps % 2 == 0, c->stream);
    } else if (nsteps % 2 == 0) {
      sadi::launch_transpose_inplace(a, c->n, c->stream);
    } else {
      sadi::launch_swap_transposed(u_cur, u_prev, c->n, c->stream);
    }
    return check_launch();
  }
  // corrections of rank above 3 (float64 only): four kernels per step in the natural layout,
  // the leapfrog update of step s riding on the row transform of step s + 1
  double* a = u_prev;
  double* b = u_cur;
  for (int s = 0; s < nsteps; ++s) {
    sadi_status st = s == 0 ? enqueue_step(c, 0, b, a, nullptr, a, 2)
                            : enqueue_step(c, 0, b, a, nullptr, a, 2, a);
    if (st != SADI_OK) return st;
    if (s > 0) std::swap(a, b);
  }
  // the pending update leaves the newest state in u_cur and the one before in u_prev
  if (b == u_cur)
    sadi::launch_leapfrog(2, b, a, c->X, c->ldX, nullptr, c->n, c->stream);
  else
    sadi::launch_leapfrog(0, b, a, c->X, c->ldX, a, c->n, c->stream);
  return check_launch();
}

sadi_status sadi_toeplitz_solve(sadi_ctx* c, double* lines, int nlines, int ld) {
  if (!ctx_ok(c)) return fail(SADI_E_STATE, "invalid context");
  if (nlines < 0) return fail(SADI_E_INVALID, "nlines must be >= 0");
  if (nlines == 0) return SADI_OK;
  if (!lines) return fail(SADI_E_INVALID, "NULL array");
  if (ld < c->n) return fail(SADI_E_INVALID, "ld must be >= N");
  if (c->prec == SADI_FP64)
    dispatch_m<RowsGS>(c->m, c, lines, ld, nlines);
  else
    dispatch_m<RowsGSMixed>(c->m, c, lines, ld, nlines);
  return check_launch();
}

sadi_status sadi_apply_lh(sadi_ctx* c, const double* u, double* out) {
  if (!ctx_ok(c)) return fail(SADI_E_STATE, "invalid context");
  if (!u || !out) return fail(SADI_E_INVALID, "NULL array");
  if (u == out) return fail(SADI_E_INVALID, "u and out must differ");
  dispatch_m<RowsFwd>(c->m, c, u, nullptr);
  dispatch_m<ColsConv>(c->m, c);
  sadi::StepScalars sc{};
  sc.sigma = c->h_alpha;
  dispatch_m<RowsRhs>(c->m, c, 2, u, (const double*)nullptr, out, c->n, sc);
  return check_launch();
}

sadi_status sadi_adjoint_step(sadi_ctx* c, int mode, const double* u_prev, const double* u_cur,
                              const double* u_next, const double* a_next, const double* a_next2, double* a_cur,
                              double* dkappa) {
  if (!ctx_ok(c)) return fail(SADI_E_STATE, "invalid context");
  if (mode != 0 && mode != 1) return fail(SADI_E_INVALID, "mode must be 0 (n >= 1) or 1 (start-up step)");
  if (!u_cur || !u_next || !a_next || !a_cur || !dkappa || (mode == 0 && !u_prev))
    return fail(SADI_E_INVALID, "NULL array");
  if (a_cur == a_next || a_cur == a_next2 || a_cur == u_cur)
    return fail(SADI_E_INVALID, "a_cur must not alias a_next, a_next2 or u_cur");
  if (c->prec != SADI_FP64) return fail(SADI_E_UNSUPPORTED, "the adjoint runs in float64 only");
  const int n = c->n;
  const size_t w = sizeof(double) * n;
  // Q = the first N x ldX doubles of the spectrum buffer, P = X
  double* P = c->X;
  double* Q = reinterpret_cast<double*>(c->S);
  SADI_HIP(hipMemcpy2DAsync(P, sizeof(double) * c->ldX, a_next, w, w, n, hipMemcpyDeviceToDevice, c->stream));
  SADI_HIP(hipMemcpy2DAsync(Q, sizeof(double) * c->ldX, a_next, w, w, n, hipMemcpyDeviceToDevice, c->stream));
  dispatch_m<RowsGS>(c->m, c, P, c->ldX, n);                      // p = H_x^-1 a
  dispatch_m<ColsGSPitched>(c->m, c, Q);                          // q = H_y^-1 a
  sadi::launch_adjoint_dots(mode, a_next, P, Q, c->ldX, u_prev, u_cur, u_next, n, c->partial, c->stream);
  dispatch_m<ColsGSPitched>(c->m, c, P);                          // z = H_y^-1 H_x^-1 a
  dispatch_m<RowsFwdPitched>(c->m, c, P, c->ldX);                 // L_h z into a_cur
  dispatch_m<ColsConv>(c->m, c);
  sadi::StepScalars sc{};
  sc.sigma = c->h_alpha;
  dispatch_m<RowsRhs>(c->m, c, 2, (const double*)P, (const double*)nullptr, a_cur, n, sc);
  const double t2 = c->tau * c->tau;
  const double c2 = mode == 0 ? t2 : 0.5 * t2;
  const double ca = mode == 0 ? 2.0 : 1.0;
  sadi::launch_adjoint_combine(ca, c2, c->kappa, (int)c->g, c->g_param, a_next, a_next2, P, c->ldX, u_cur, a_cur, n,
                               c->partial, c->stream);
  sadi::launch_adjoint_finish(c->partial, n, c2, c->kappa, dkappa, c->stream);
  return check_launch();
}

sadi_status sadi_set_kernel_timing(sadi_ctx* c, int enable) {
  if (!ctx_ok(c)) return fail(SADI_E_STATE, "invalid context");
  c->timing = enable != 0;
  c->timed_steps = 0;
  return SADI_OK;
}

sadi_status sadi_get_kernel_times(sadi_ctx* c, double* ms, long long* count) {
  if (!ctx_ok(c)) return fail(SADI_E_STATE, "invalid context");
  if (!ms || !count) return fail(SADI_E_INVALID, "NULL output");
  SADI_HIP(hipStreamSynchronize(c->stream));
  for (int k = 0; k < 4; ++k) {
    ms[k] = 0.0;
    count[k] = 0;
  }
  for (int s = 0; s < c->timed_steps; ++s)
    for (int k = 0; k < 4; ++k) {
      float t = 0.0f;
      SADI_HIP(hipEventElapsedTime(&t, c->events[(size_t)s * 5 + k], c->events[(size_t)s * 5 + k + 1]));
      ms[k] += t;
      count[k] += 1;
    }
  return SADI_OK;
}

sadi_status sadi_get_line_tables(const sadi_ctx* c, double* lam_s, double* lam_c, double* f) {
  if (!ctx_ok(c)) return fail(SADI_E_STATE, "invalid context");
  const size_t fsize = (size_t)c->r * c->n;
  if (lam_s) SADI_HIP(hipMemcpy(lam_s, c->lam_s, sizeof(double2) * c->m, hipMemcpyDeviceToHost));
  if (lam_c) SADI_HIP(hipMemcpy(lam_c, c->lam_c, sizeof(double2) * c->m, hipMemcpyDeviceToHost));
  if (f) SADI_HIP(hipMemcpy(f, c->f, sizeof(double) * fsize, hipMemcpyDeviceToHost));
  return SADI_OK;
}

sadi_status sadi_get_info(const sadi_ctx* c, int* n, int* m, long long* bytes) {
  if (!ctx_ok(c)) return fail(SADI_E_STATE, "invalid context");
  if (n) *n = c->n;
  if (m) *m = c->m;
  if (bytes) *bytes = c->device_bytes;
  return SADI_OK;
}

sadi_status sadi_destroy(sadi_ctx* c) {
  if (!c) return SADI_OK;
  if (!ctx_ok(c)) return fail(SADI_E_STATE, "invalid context");
  hipError_t e = hipStreamSynchronize(c->stream);
  c->magic = 0;
  c->release();
  delete c;
  if (e != hipSuccess) return fail(SADI_E_DEVICE, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
  return SADI_OK;
}

// ---- host-only helpers ------------------------------------------------------------
sadi_status sadi_host_riesz_coeffs(double alpha, int count, double* out) {
  if (!out || count < 0) return fail(SADI_E_INVALID, "bad arguments");
  if (!(alpha > 0.0 && alpha <= 2.0) || !std::isfinite(alpha)) return fail(SADI_E_INVALID, "alpha out of range");
  const std::vector<double> a = sadi::riesz_coeffs(alpha, count);
  std::memcpy(out, a.data(), sizeof(double) * a.size());
  return SADI_OK;
}

sadi_status sadi_host_laplacian_coeffs(double alpha, int n, double* out) {
  if (!out || n < 1) return fail(SADI_E_INVALID, "bad arguments");
  if (!(alpha > 1.0 && alpha < 2.0)) return fail(SADI_E_INVALID, "alpha must lie in (1, 2)");
  if (n > 8192) return fail(SADI_E_UNSUPPORTED, "n too large");
  try {
    const std::vector<double> a = sadi::laplacian_coeffs(alpha, n);
    std::memcpy(out, a.data(), sizeof(double) * a.size());
  } catch (const std::bad_alloc&) {
    return fail(SADI_E_NOMEM, "host allocation failed");
  }
  return SADI_OK;
}

sadi_status sadi_host_line_tables(double alpha, double kappa, int n, double tau, const double* domain,
                                  double* lam_s, double* lam_c, double* f) {
  if (!lam_s || !lam_c || !f) return fail(SADI_E_INVALID, "NULL output");
  sadi_status st = validate_problem(alpha, kappa, n, tau, domain, false);
  if (st != SADI_OK) return st;
  try {
    const int m = sadi::line_size(n);
    const double h = (domain[1] - domain[0]) / (n + 1);
    const double beta = kappa * tau * tau * std::pow(h, -alpha) / 2.0;
    const sadi::GSData g = sadi::gs_data(sadi::riesz_coeffs(alpha, m), n, m, beta);
    for (int k = 0; k < m; ++k) {
      lam_s[2 * k] = g.lam_s[k].real();
      lam_s[2 * k + 1] = g.lam_s[k].imag();
      lam_c[2 * k] = g.lam_c[k].real();
      lam_c[2 * k + 1] = g.lam_c[k].imag();
    }
    std::copy(g.f.begin(), g.f.end(), f);
  } catch (const std::exception& e) {
    return fail(SADI_E_INVALID, std::string("line tables: ") + e.what());
  }
  return SADI_OK;
}

sadi_status sadi_host_line_generator(double alpha, double kappa, int n, double tau, const double* domain,
                                     double* out) {
  if (!out) return fail(SADI_E_INVALID, "out is NULL");
  sadi_status st = validate_problem(alpha, kappa, n, tau, domain, false);
  if (st != SADI_OK && st != SADI_E_UNSUPPORTED) return st;
  try {
    const double h = (domain[1] - domain[0]) / (n + 1);
    const double beta = kappa * tau * tau * std::pow(h, -alpha) / 2.0;
    const std::vector<double> a1 = sadi::riesz_coeffs(alpha, n + 1);
    std::vector<long double> t(n + 1);
    for (int k = 0; k <= n; ++k) t[k] = (k == 0 ? 1.0L : 0.0L) + (long double)beta * a1[k];
    const std::vector<long double> cc = sadi::toeplitz_first_column_inverse(t);
    for (int k = 0; k <= n; ++k) out[k] = (double)cc[k];
  } catch (const std::exception& e) {
    return fail(SADI_E_INVALID, std::string("line generator: ") + e.what());
  }
  return SADI_OK;
}

}  // extern "C"
