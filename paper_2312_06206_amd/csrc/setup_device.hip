// Device part of the set-up of the 2D coefficients a_ij: the node rows of their quadrature.
//
// a_ij is a quadrature over nodes t_q of ive(i, 2 t_q) ive(j, 2 t_q) (the subordination
// integral of the symbol of L_h; see setup_math.cpp).  The rows ive(k, x_q), x_q = 2 t_q,
// k < kTableRows, do not depend on alpha or N (a row for fewer orders is a prefix of it), so
// one table per GPU serves every context: it is built on first use, one thread per node,
// and kept until the process ends (about 20 MB).  The alpha-dependent rest (node weights,
// high-tail rows, the exact corner) is set up on the host from the table's first orders,
// and the product itself runs on the matrix cores (gemm.hip).
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "context.hpp"
#include "kernels.hpp"
#include "setup_device.hpp"
#include "setup_math.hpp"

namespace sadi {

namespace {

constexpr double kIveHankelX = 1.0e8;   // x above this: Hankel series (x >> k^2 for every k < 4096)
constexpr int kIveHankelTerms = 24;
constexpr int kTableRows = 4096;        // orders k < 4096 cover every N <= 4095

// Double-double arithmetic (a value is hi + lo with |lo| <= ulp(hi)/2), enough to carry the
// backward recurrence below through ~1e5 steps without the float64 rounding that would
// otherwise accumulate where the recurrence neither grows nor decays (orders k << sqrt(x)).
// The error-free sums and products below hold only if every operation is rounded on its own:
// a product fused into the following sum (HIP's default contraction) would turn the low part
// of a product into a double count of its rounding error, so contraction is off in this file.
#pragma clang fp contract(off)
struct DD {
  double hi, lo;
};
__host__ __device__ inline DD dd_quick(double s, double e) {
  const double h = s + e;
  return DD{h, e - (h - s)};
}
__host__ __device__ inline DD dd_add(DD a, DD b) {
  const double s = a.hi + b.hi;
  const double bb = s - a.hi;
  const double e = (a.hi - (s - bb)) + (b.hi - bb) + a.lo + b.lo;
  return dd_quick(s, e);
}
__host__ __device__ inline DD dd_mul(DD a, DD b) {
  const double p = a.hi * b.hi;
  const double e = fma(a.hi, b.hi, -p) + (a.hi * b.lo + a.lo * b.hi);
  return dd_quick(p, e);
}
__host__ __device__ inline DD dd_scale(DD a, int e2) { return DD{ldexp(a.hi, e2), ldexp(a.lo, e2)}; }

// e^-x I_k(x) for k < nrows (x > 0), in double-double arithmetic rounded to float64.
// Miller's backward recurrence I_{k-1} = (2k/x) I_k + I_{k+1} from an order above the
// wanted ones and above the bulk of the normalisation sum e^-x (I_0 + 2 sum_k I_k) = 1 (its
// terms fall like e^{-k^2/2x}); orders whose value lies below the double range start the
// recurrence just above them and are returned as zero.  Above kIveHankelX the Hankel
// large-argument series (float64) is used instead.
__host__ __device__ void ive_row_fp64(double x, int nrows, double* out) {
  if (x > kIveHankelX) {
    for (int k = 0; k < nrows; ++k) {
      const double mu = 4.0 * k * k;
      double term = 1.0, acc = 1.0;
      for (int m = 1; m <= kIveHankelTerms; ++m) {
        term *= -(mu - (double)(2 * m - 1) * (2 * m - 1)) / (m * 8.0 * x);
        acc += term;
        if (fabs(term) < 1e-18 * fabs(acc)) break;
      }
      out[k] = acc / sqrt(2.0 * 3.14159265358979323846 * x);
    }
    return;
  }
  int kstart = nrows + 40 + (int)(12.0 * sqrt(x));
  // log(e^-x I_k(x)) <= k log(x/2) - log(k!): start where that falls below -760 (k > x)
  {
    const double lx = log(0.5 * x);
    int k0 = (int)x + 1;
    if (k0 < kstart) {
      double lfact = lgamma((double)k0);   // log((k0 - 1)!)
      for (int k = k0; k < kstart; ++k) {
        lfact += log((double)k);
        if (k * lx - lfact < -760.0) {
          kstart = k + 30;
          break;
        }
      }
    }
  }
  const int nstore = nrows < kstart ? nrows : kstart;
  const double inv_x = 1.0 / x;
  const DD rx{inv_x, fma(-inv_x, x, 1.0) * inv_x};   // 1/x in double-double
  DD rp1{0.0, 0.0}, r{1.0, 0.0}, sum{0.0, 0.0};
  constexpr int kRescale = 800;                     // powers of two: exact rescaling
  const double big = ldexp(1.0, kRescale);
  for (int k = kstart; k >= 1; --k) {
    const DD c = dd_mul(DD{2.0 * k, 0.0}, rx);      // 2k / x
    const DD rm1 = dd_add(dd_mul(c, r), rp1);
    if (k < nstore) out[k] = r.hi + r.lo;
    sum = dd_add(sum, DD{2.0 * r.hi, 2.0 * r.lo});
    rp1 = r;
    r = rm1;
    if (r.hi > big) {   // rescale everything seen so far
      r = dd_scale(r, -kRescale);
      rp1 = dd_scale(rp1, -kRescale);
      sum = dd_scale(sum, -kRescale);
      for (int q = k; q < nstore; ++q) out[q] = ldexp(out[q], -kRescale);
    }
  }
  out[0] = r.hi + r.lo;   // I_0 (scaled)
  sum = dd_add(sum, r);
  const double s = sum.hi + sum.lo;
  for (int k = 0; k < nrows; ++k) out[k] = k < nstore ? out[k] / s : 0.0;
}

__global__ void __launch_bounds__(64) ive_rows_kernel(const double* __restrict__ x, int nq, int nrows, double* out,
                                                     int ld) {
  const int q = blockIdx.x * 64 + threadIdx.x;
  if (q < nq) ive_row_fp64(x[q], nrows, out + (size_t)q * ld);
}

struct DeviceTable {
  std::mutex mu;
  double* rows = nullptr;          // nq x kTableRows
  std::vector<double> low;         // nq x kLapLowOrders, host copy
};
constexpr int kMaxDevices = 64;
DeviceTable g_tables[kMaxDevices];

// ---- Gohberg-Semencul data of the line matrix H_M (N + 1 = M) on the device ----------------

__host__ __device__ inline DD dd_sub(DD a, DD b) { return dd_add(a, DD{-b.hi, -b.lo}); }
// 1 / a in double-double: one Newton step on the float64 reciprocal
__host__ __device__ inline DD dd_recip(DD a) {
  const double q = 1.0 / a.hi;
  const DD r = dd_sub(DD{1.0, 0.0}, dd_mul(a, DD{q, 0.0}));
  return dd_add(DD{q, 0.0}, DD{r.hi * q, 0.0});
}

constexpr int kLevThreads = 1024;
constexpr int kLevMaxM = 4096;

// sum of v over the workgroup (red: kLevThreads / 64 entries of LDS).  After one barrier
// every wave reduces the waves' partial sums itself (a butterfly over groups of lanes) and
// takes lane 0's result, so all threads get the same total.  The caller synchronises
// before red is written again.
__device__ DD block_sum_dd(DD v, DD* red) {
  constexpr int W = kLevThreads / 64;
  static_assert((W & (W - 1)) == 0 && W <= 64, "waves per workgroup: a power of two");
  for (int off = 32; off > 0; off >>= 1) v = dd_add(v, DD{__shfl_down(v.hi, off), __shfl_down(v.lo, off)});
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  DD p = red[threadIdx.x & (W - 1)];
#pragma unroll
  for (int off = W / 2; off > 0; off >>= 1) p = dd_add(p, DD{__shfl_xor(p.hi, off), __shfl_xor(p.lo, off)});
  return DD{__shfl(p.hi, 0), __shfl(p.lo, 0)};
}

// Levinson-Durbin recursion for T c = e_1, T the SPD Toeplitz matrix of first column t (given
// as double-double t_hi + t_lo, m <= 4096 entries), in double-double arithmetic by one
// workgroup: with f the solution at size k (T_k f = e_1), e = sum_{i<k} t[k-i] f[i] and
// [f; 0] updated to ([f; 0] - e [0; J f]) / (1 - e^2), pairs (i, k - i) in place.  The
// thread that forms the new f[i] also adds its terms of the next e, so each step needs one
// barrier (the block sum's; its partials alternate between two buffers).  c = f rounded.
__device__ __forceinline__ void levinson_body(const double* __restrict__ t_hi, const double* __restrict__ t_lo, int m,
                                              double* __restrict__ c) {
  __shared__ double fh[kLevMaxM], fl[kLevMaxM], th[kLevMaxM], tl[kLevMaxM];
  __shared__ DD red[2][kLevThreads / 64];
  for (int i = threadIdx.x; i < m; i += kLevThreads) {
    th[i] = t_hi[i];
    tl[i] = t_lo[i];
    fh[i] = 0.0;
    fl[i] = 0.0;
  }
  __syncthreads();
  DD acc{0.0, 0.0};   // this thread's terms of the next e
  if (threadIdx.x == 0) {
    const DD f0 = dd_recip(DD{th[0], tl[0]});
    fh[0] = f0.hi;
    fl[0] = f0.lo;
    if (m > 1) acc = dd_mul(DD{th[1], tl[1]}, f0);
  }
  for (int k = 1; k < m; ++k) {
    const DD e = block_sum_dd(acc, red[k & 1]);
    const DD inv = dd_recip(dd_sub(DD{1.0, 0.0}, dd_mul(e, e)));
    acc = DD{0.0, 0.0};
    const bool next = k + 1 < m;
    for (int i = threadIdx.x; 2 * i <= k; i += kLevThreads) {
      const int j = k - i;                       // f[k] is still 0 here
      const DD a{fh[i], fl[i]}, b{fh[j], fl[j]};
      const DD na = dd_mul(dd_sub(a, dd_mul(e, b)), inv);
      const DD nb = dd_mul(dd_sub(b, dd_mul(e, a)), inv);
      fh[i] = na.hi;
      fl[i] = na.lo;
      if (next) acc = dd_add(acc, dd_mul(DD{th[k + 1 - i], tl[k + 1 - i]}, na));
      if (j != i) {
        fh[j] = nb.hi;
        fl[j] = nb.lo;
        if (next) acc = dd_add(acc, dd_mul(DD{th[i + 1], tl[i + 1]}, nb));
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < m; i += kLevThreads) c[i] = fh[i] + fl[i];
}
__global__ void __launch_bounds__(kLevThreads)
levinson_kernel(const double* __restrict__ t_hi, const double* __restrict__ t_lo, int m, double* __restrict__ c) {
  levinson_body(t_hi, t_lo, m, c);
}
// one workgroup per job
__global__ void __launch_bounds__(kLevThreads) levinson_batched(const GsJob* __restrict__ jobs) {
  const GsJob& j = jobs[blockIdx.x];
  levinson_body(j.t_hi, j.t_lo, j.m, j.c);
}

// The tables of Algorithm 1 from c = H_M^-1 e_1 (p1 = c[0]), by direct DFTs summed in
// double-double: lam_c[k] = fft(c)[k] / M and lam_s[k] = fft(Q s)[k] / (2 p1 M) with
// s = (p1, -c[M-1], ..., -c[1]) and Q = diag(e^{-i pi j / M}); the correction f[k] =
// c[M-1-k] / p1 (k < N = M - 1); and their float32 copies.  q[j] = e^{-i pi j / M}, j < M.
// Frequency k (< m) of those tables.
__device__ __forceinline__ void gs_tables_body(const double* __restrict__ c, int m, const double2* __restrict__ q,
                                               double2* __restrict__ lam_s, double2* __restrict__ lam_c,
                                               double* __restrict__ f, float2* __restrict__ lam_s32,
                                               float2* __restrict__ lam_c32, float* __restrict__ f32, int k) {
  const int two_m = 2 * m;
  // e^{-i pi idx / M} for 0 <= idx < 2M
  auto w = [&](int idx) -> double2 {
    const double2 v = q[idx < m ? idx : idx - m];
    return idx < m ? v : double2{-v.x, -v.y};
  };
  auto mac = [](DD& re, DD& im, double x, double2 wv) {   // (re, im) += x wv
    re = dd_add(re, dd_mul(DD{x, 0.0}, DD{wv.x, 0.0}));
    im = dd_add(im, dd_mul(DD{x, 0.0}, DD{wv.y, 0.0}));
  };
  const double p1 = c[0];
  DD cr{0.0, 0.0}, ci{0.0, 0.0}, sr{0.0, 0.0}, si{0.0, 0.0};
  // exponent indices j 2k and j (2k + 1) modulo 2M, advanced with j
  int ic = 0, is = 0;
  for (int j = 0; j < m; ++j) {
    const double cj = c[j];
    const double sj = j == 0 ? p1 : -c[m - j];
    mac(cr, ci, cj, w(ic));     // e^{-2 pi i j k / M}
    mac(sr, si, sj, w(is));     // e^{-i pi j (2k + 1) / M}
    ic += 2 * k;
    if (ic >= two_m) ic -= two_m;
    is += 2 * k + 1;
    if (is >= two_m) is -= two_m;
  }
  const double rm = 1.0 / m, rs = 1.0 / (2.0 * p1 * m);
  const double2 lc{(cr.hi + cr.lo) * rm, (ci.hi + ci.lo) * rm};
  const double2 ls{(sr.hi + sr.lo) * rs, (si.hi + si.lo) * rs};
  lam_c[k] = lc;
  lam_s[k] = ls;
  lam_c32[k] = float2{(float)lc.x, (float)lc.y};
  lam_s32[k] = float2{(float)ls.x, (float)ls.y};
  if (k < m - 1) {
    const double fk = c[m - 1 - k] / p1;
    f[k] = fk;
    f32[k] = (float)fk;
  }
}
__global__ void __launch_bounds__(256)
gs_tables_kernel(const double* __restrict__ c, int m, const double2* __restrict__ q, double2* __restrict__ lam_s,
                 double2* __restrict__ lam_c, double* __restrict__ f, float2* __restrict__ lam_s32,
                 float2* __restrict__ lam_c32, float* __restrict__ f32) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= m) return;
  gs_tables_body(c, m, q, lam_s, lam_c, f, lam_s32, lam_c32, f32, k);
}
// job blockIdx.y, frequencies blockIdx.x * 256 + threadIdx.x
__global__ void __launch_bounds__(256) gs_tables_batched(const GsJob* __restrict__ jobs) {
  const GsJob& j = jobs[blockIdx.y];
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= j.m) return;
  gs_tables_body(j.c, j.m, j.q, j.lam_s, j.lam_c, j.f, j.lam_s32, j.lam_c32, j.f32, k);
}

}  // namespace

void launch_gs_generator(const double* t_hi, const double* t_lo, int m, double* c, const double2* q, double2* lam_s,
                         double2* lam_c, double* f, float2* lam_s32, float2* lam_c32, float* f32, hipStream_t st) {
  hipLaunchKernelGGL(levinson_kernel, dim3(1), dim3(kLevThreads), 0, st, t_hi, t_lo, m, c);
  hipLaunchKernelGGL(gs_tables_kernel, dim3((m + 255) / 256), dim3(256), 0, st, c, m, q, lam_s, lam_c, f, lam_s32,
                     lam_c32, f32);
}

void launch_gs_generator_batched(const GsJob* jobs, int njobs, int max_m, hipStream_t st) {
  if (njobs <= 0) return;
  hipLaunchKernelGGL(levinson_batched, dim3(njobs), dim3(kLevThreads), 0, st, jobs);
  hipLaunchKernelGGL(gs_tables_batched, dim3((max_m + 255) / 256, njobs), dim3(256), 0, st, jobs);
}

// The node table of the current device (built on first use; host-synchronous then).
sadi_status quadrature_table(const double** rows, int* ld, const double** low) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return sadi_impl::fail(SADI_E_DEVICE, "quadrature table: no usable current device");
  DeviceTable& tb = g_tables[dev];
  std::lock_guard<std::mutex> lock(tb.mu);
  if (!tb.rows) {
    const int nq = lap_node_count();
    std::vector<double> hx(nq);
    for (int q = 0; q < nq; ++q) hx[q] = lap_node_x(q);
    double* dx = nullptr;
    double* drows = nullptr;
    hipStream_t st = nullptr;
    auto bail = [&](const std::string& what, hipError_t e) {
      if (dx) (void)hipFree(dx);
      if (drows) (void)hipFree(drows);
      if (st) (void)hipStreamDestroy(st);
      return sadi_impl::fail(SADI_E_DEVICE, "quadrature table: " + what + ": " + hipGetErrorString(e));
    };
    hipError_t e;
    if ((e = hipStreamCreate(&st)) != hipSuccess) return bail("hipStreamCreate", e);
    if ((e = hipMalloc(&dx, sizeof(double) * nq)) != hipSuccess) return bail("hipMalloc", e);
    if ((e = hipMalloc(&drows, sizeof(double) * (size_t)nq * kTableRows)) != hipSuccess) return bail("hipMalloc", e);
    if ((e = hipMemcpyAsync(dx, hx.data(), sizeof(double) * nq, hipMemcpyHostToDevice, st)) != hipSuccess)
      return bail("hipMemcpyAsync", e);
    hipLaunchKernelGGL(ive_rows_kernel, dim3((nq + 63) / 64), dim3(64), 0, st, dx, nq, kTableRows, drows,
                       kTableRows);
    if ((e = hipGetLastError()) != hipSuccess) return bail("launch", e);
    tb.low.assign((size_t)nq * kLapLowOrders, 0.0);
    if ((e = hipMemcpy2DAsync(tb.low.data(), sizeof(double) * kLapLowOrders, drows, sizeof(double) * kTableRows,
                              sizeof(double) * kLapLowOrders, nq, hipMemcpyDeviceToHost, st)) != hipSuccess)
      return bail("hipMemcpy2DAsync", e);
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return bail("hipStreamSynchronize", e);
    (void)hipFree(dx);
    (void)hipStreamDestroy(st);
    tb.rows = drows;
  }
  *rows = tb.rows;
  *ld = kTableRows;
  *low = tb.low.data();
  return SADI_OK;
}

}  // namespace sadi

extern "C" sadi_status sadi_host_quadrature_rows(int nrows, int fp64, int* nodes, double* x, double* rows) {
  if (nrows < 1 || nrows > sadi::kTableRows) return sadi_impl::fail(SADI_E_INVALID, "nrows must lie in [1, 4096]");
  const int nq = sadi::lap_node_count();
  if (nodes) *nodes = nq;
  if (x)
    for (int q = 0; q < nq; ++q) x[q] = sadi::lap_node_x(q);
  if (!rows) return SADI_OK;
  if (fp64) {
    for (int q = 0; q < nq; ++q) sadi::ive_row_fp64(sadi::lap_node_x(q), nrows, rows + (size_t)q * nrows);
  } else {
    const std::vector<double> r = sadi::ive_node_rows(nrows);
    std::copy(r.begin(), r.end(), rows);
  }
  return SADI_OK;
}
