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
#include "setup_math.hpp"

namespace sadi {

namespace {

constexpr double kIveHankelX = 1.0e8;   // x above this: Hankel series (x >> k^2 for every k < 4096)
constexpr int kIveHankelTerms = 24;
constexpr int kTableRows = 4096;        // orders k < 4096 cover every N <= 4095

// Double-double arithmetic (a value is hi + lo with |lo| <= ulp(hi)/2), enough to carry the
// backward recurrence below through ~1e5 steps without the float64 rounding that would
// otherwise accumulate where the recurrence neither grows nor decays (orders k << sqrt(x)).
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

}  // namespace

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
