// Host-side setup mathematics of the S-ADI solver.
//
// 1D coefficients a_k: the closed form (-1)^k Gamma(alpha+1) / (Gamma(alpha/2-k+1)
// Gamma(alpha/2+k+1)) of section 2 satisfies a_{k+1} = a_k (k - alpha/2)/(k + alpha/2 + 1)
// (Gamma(z+1) = z Gamma(z)); evaluated in long double.
//
// 2D coefficients a_ij (Fourier coefficients of s^beta, s = 4 sin^2(eta/2) +
// 4 sin^2(xi/2), beta = alpha/2), through the identity
//     s^beta = beta/Gamma(1-beta) int_0^inf (1 - e^{-ts}) t^{-1-beta} dt
// and e^{-2t(1 - cos eta)} = sum_k ive(k, 2t) e^{ik eta}, ive(k,x) = e^{-x} I_k(x):
//     a_ij = beta/Gamma(1-beta) int_0^inf (delta_{i0} delta_{j0} - ive(i,2t) ive(j,2t)) t^{-1-beta} dt.
// With t = e^s this is an integral over the real line of an analytic function, for
// which the trapezoidal rule converges geometrically in 1/step; the nodes outside a
// finite window are summed in closed form from the small-t power series and the
// large-t Hankel series.  ive(k, x) for all k < n at once: Miller's backward
// recurrence normalised by e^{-x}(I_0 + 2 sum I_k) = 1, or the Hankel series for
// very large x.  The sum over nodes is a rank-Q symmetric product B^T B.
#include "setup_math.hpp"

#include <algorithm>
#include <cmath>
#include <stdexcept>
#include <thread>

namespace sadi {

namespace {

constexpr double kStep = 0.1;      // trapezoid step in s = log t
constexpr double kSLo = -18.0;     // window [kSLo, kSHi]; outside: closed-form sums
constexpr double kSHi = 42.0;
constexpr double kXHankel = 1.0e8; // x = 2t above this: Hankel series for ive
constexpr int kHankelTerms = 24;
constexpr int kSeriesDeg = 40;

int worker_count(int requested) {
  if (requested > 0) return requested;
  unsigned h = std::thread::hardware_concurrency();
  return h == 0 ? 4 : (int)std::min(h, 32u);
}

template <class F>
void parallel_for(int count, int nthreads, F f) {
  nthreads = std::max(1, std::min(nthreads, count));
  std::vector<std::thread> pool;
  for (int w = 0; w < nthreads; ++w)
    pool.emplace_back([=] {
      for (int i = w; i < count; i += nthreads) f(i);
    });
  for (auto& th : pool) th.join();
}

// e^-x I_k(x), k = 0..n-1, Miller's backward recurrence (x > 0).  Orders whose value is
// below the double range are set to zero and the recurrence starts just above them.
void ive_miller(double x, int n, double* out) {
  // start: beyond both the orders wanted and the bulk of the normalisation sum
  // (terms ~ e^{-k^2/2x}), but not far into the underflow region for small x
  int kstart = n + 40 + (int)(12.0 * std::sqrt(x));
  {
    // log(e^-x I_k(x)) <= k log(x/2) - log(k!) for k >= 0; stop where < -760
    const double lx = std::log(0.5 * x);
    double lfact = 0.0;
    for (int k = 1; k < kstart; ++k) {
      lfact += std::log((double)k);
      if (k > x && k * lx - lfact < -760.0) {
        kstart = k + 30;
        break;
      }
    }
  }
  const int nstore = std::min(n, kstart);
  long double rp1 = 0.0L, r = 1.0e-300L, sum = 0.0L;
  std::vector<long double> tmp(std::max(nstore, 1), 0.0L);
  for (int k = kstart; k >= 1; --k) {
    const long double rm1 = (2.0L * k / x) * r + rp1;
    if (k < nstore) tmp[k] = r;
    sum += 2.0L * r;
    rp1 = r;
    r = rm1;
    if (r > 1.0e300L) {  // rescale everything seen so far
      const long double sc = 1.0e-300L;
      r *= sc;
      rp1 *= sc;
      sum *= sc;
      for (int q = k; q < nstore; ++q) tmp[q] *= sc;
    }
  }
  tmp[0] = r;  // I_0 (scaled)
  sum += r;
  for (int k = 0; k < n; ++k) out[k] = k < nstore ? (double)(tmp[k] / sum) : 0.0;
}

// Hankel large-x series of e^-x I_k(x) (x >> k^2)
double ive_hankel(int k, double x) {
  const long double mu = 4.0L * k * k;
  long double term = 1.0L, acc = 1.0L;
  for (int m = 1; m <= kHankelTerms; ++m) {
    term *= -(mu - (long double)(2 * m - 1) * (2 * m - 1)) / (m * 8.0L * x);
    acc += term;
    if (std::fabs(term) < 1e-22L * std::fabs(acc)) break;
  }
  return (double)(acc / std::sqrt(2.0L * 3.14159265358979323846264338327950288L * x));
}

void ive_all(double x, int n, double* out) {
  if (x <= kXHankel) {
    ive_miller(x, n, out);
  } else {
    for (int k = 0; k < n; ++k) out[k] = ive_hankel(k, x);
  }
}

// sum_{q>=1} step * exp(rate * (edge + dir*q*step)) for the decaying direction
long double geom_tail(long double rate, long double edge, int dir) {
  const long double x = -dir * rate * kStep;  // > 0
  return kStep * std::exp(rate * edge) / std::expm1(x);
}

// power series (in t) of e^{-a t} I_i(2t) I_j(2t) (j < 0: omit that factor), degree kSeriesDeg
std::vector<long double> series_product(long double a, int i, int j) {
  const int D = kSeriesDeg;
  std::vector<long double> e(D + 1), bi(D + 1, 0.0L), bj(D + 1, 0.0L), out(D + 1, 0.0L);
  long double f = 1.0L;
  for (int p = 0; p <= D; ++p) {
    if (p > 0) f *= -a / p;
    e[p] = f;
  }
  auto ibess = [&](int k, std::vector<long double>& b) {
    // I_k(2t) = sum_m t^{2m+k} / (m! (m+k)!)
    long double c = 1.0L;
    for (int q = 1; q <= k; ++q) c /= q;
    for (int m = 0; 2 * m + k <= D; ++m) {
      if (m > 0) c /= (long double)m * (m + k);
      b[2 * m + k] = c;
    }
  };
  ibess(i, bi);
  std::vector<long double> t1(D + 1, 0.0L);
  for (int p = 0; p <= D; ++p)
    for (int q = 0; p + q <= D; ++q) t1[p + q] += e[p] * bi[q];
  if (j < 0) return t1;
  ibess(j, bj);
  for (int p = 0; p <= D; ++p)
    for (int q = 0; p + q <= D; ++q) out[p + q] += t1[p] * bj[q];
  return out;
}

// trapezoid nodes below kSLo of f(t) t^-beta where f has power series c (c[0] excluded)
long double low_tail(const std::vector<long double>& c, long double beta, bool skip_const) {
  long double tot = 0.0L;
  for (int p = skip_const ? 1 : 0; p < (int)c.size(); ++p)
    if (c[p] != 0.0L && p - beta > 0) tot += c[p] * geom_tail(p - beta, kSLo, -1);
  return tot;
}

// 1 - (e^{-2t} I_0(2t))^2 without cancellation
long double one_minus_ive0_sq(double t, double ive0) {
  if (t < 1.0) {
    long double term = 1.0L, i0m1 = 0.0L;
    for (int m = 1; m < 60; ++m) {
      term *= (long double)t * t / ((long double)m * m);
      i0m1 += term;
      if (term < 1e-22L * i0m1) break;
    }
    return -std::expm1(2.0L * (std::log1p(i0m1) - 2.0L * t));
  }
  return -std::expm1(2.0L * std::log((long double)ive0));
}

}  // namespace

std::vector<double> riesz_coeffs(double alpha, int count) {
  std::vector<double> a(std::max(count, 0));
  if (count <= 0) return a;
  const long double al = alpha, b = al / 2;
  long double v = std::tgamma(al + 1.0L) / (std::tgamma(b + 1.0L) * std::tgamma(b + 1.0L));
  for (int k = 0; k < count; ++k) {
    a[k] = (double)v;
    v *= ((long double)k - b) / ((long double)k + b + 1.0L);
  }
  return a;
}

int lap_node_count() { return (int)std::lround((kSHi - kSLo) / kStep) + 1; }

double lap_node_x(int q) { return 2.0 * std::exp(kSLo + q * kStep); }

LapSetup laplacian_setup(double alpha, int n, const double* ive_low) {
  LapSetup f;
  if (n <= 0) return f;
  const long double beta = (long double)alpha / 2;
  const long double cb = beta / std::tgamma(1.0L - beta);
  const int nq = lap_node_count();
  const int HT = kLapTailTerms;
  f.n = n;
  f.nq = nq;
  f.ht = HT;
  f.scale = (double)(-cb);
  f.w.resize(nq);

  // node weights (trapezoid step times t^-beta) and the origin integrand (1 - ive0^2) t^-beta
  long double acc0 = 0.0L;
  for (int q = 0; q < nq; ++q) {
    const double sq = kSLo + q * kStep;
    const long double w = kStep * std::exp(-beta * sq);
    f.w[q] = (double)w;
    acc0 += w * one_minus_ive0_sq(std::exp(sq), ive_low[(size_t)q * kLapLowOrders]);
  }

  // Hankel coefficients A_m(k) of ive(k, 2t) = (4 pi t)^-1/2 sum_m A_m(k) t^-m, for the high
  // tail: rows p of tail_a hold A_p and of tail_c C_p with C[p][j] = sum_r Wt[p][r] A_r(j),
  // so that the high tail of (i, j) is sum_p A_p(i) C[p][j] (Wt depends on p + r only)
  f.tail_a.assign((size_t)HT * n, 0.0);
  f.tail_c.assign((size_t)HT * n, 0.0);
  double* A = f.tail_a.data();
  for (int k = 0; k < n; ++k) {
    const long double mu = 4.0L * k * k;
    long double term = 1.0L;
    A[k] = 1.0;
    for (int m = 1; m < HT; ++m) {
      term *= -(mu - (long double)(2 * m - 1) * (2 * m - 1)) / (m * 16.0L);
      A[(size_t)m * n + k] = (double)term;
    }
  }
  const long double pi = 3.14159265358979323846264338327950288L;
  std::vector<long double> Wt(HT * HT, 0.0L);
  for (int p = 0; p < HT; ++p)
    for (int r = 0; p + r < HT; ++r) Wt[p * HT + r] = geom_tail(-(1.0L + beta + p + r), kSHi, +1) / (4.0L * pi);
  double* Cht = f.tail_c.data();
  for (int p = 0; p < HT; ++p)
    for (int j = 0; j < n; ++j) {
      long double sacc = 0.0L;
      for (int r = 0; p + r < HT; ++r) sacc += Wt[p * HT + r] * A[(size_t)r * n + j];
      Cht[(size_t)p * n + j] = (double)sacc;
    }

  // corner i, j < nc: the factor product plus the low tail (small i + j) and the origin
  const int nc = std::min(n, kLapLowOrders);
  f.nc = nc;
  f.corner.assign((size_t)nc * nc, 0.0);
  for (int i = 0; i < nc; ++i)
    for (int j = 0; j < nc; ++j) {
      long double acc = 0.0L;
      for (int q = 0; q < nq; ++q)
        acc += (long double)f.w[q] * ive_low[(size_t)q * kLapLowOrders + i] * ive_low[(size_t)q * kLapLowOrders + j];
      for (int p = 0; p < HT; ++p) acc += (long double)A[(size_t)p * n + i] * Cht[(size_t)p * n + j];
      long double v = -cb * acc;
      if (i + j > 0 && i + j < kLapLowOrders)
        v += -cb * low_tail(series_product(4.0L, std::min(i, j), std::max(i, j)), beta, false);
      f.corner[(size_t)j * nc + i] = (double)v;
    }
  {
    std::vector<long double> c = series_product(4.0L, 0, 0);
    for (auto& v : c) v = -v;
    c[0] = 0.0L;
    acc0 += low_tail(c, beta, true);
    long double hi00 = 0.0L;
    for (int p = 0; p < HT; ++p)
      for (int r = 0; p + r < HT; ++r) hi00 += Wt[p * HT + r] * A[(size_t)p * n] * A[(size_t)r * n];
    acc0 += geom_tail(-beta, kSHi, +1) - hi00;
    f.corner[0] = (double)(cb * acc0);
  }
  return f;
}

std::vector<double> ive_node_rows(int nrows, int nthreads) {
  const int nq = lap_node_count();
  std::vector<double> rows((size_t)nq * nrows);
  parallel_for(nq, worker_count(nthreads), [&](int q) { ive_all(lap_node_x(q), nrows, &rows[(size_t)q * nrows]); });
  return rows;
}

LapFactors laplacian_factors(double alpha, int n, int nthreads) {
  LapFactors f;
  if (n <= 0) return f;
  const int nq = lap_node_count();
  // node rows ive(k, 2 t_q), k < n, on the host (long double Miller recurrence)
  const std::vector<double> rows = ive_node_rows(n, nthreads);
  std::vector<double> low((size_t)nq * kLapLowOrders, 0.0);
  for (int q = 0; q < nq; ++q)
    for (int k = 0; k < std::min(n, kLapLowOrders); ++k) low[(size_t)q * kLapLowOrders + k] = rows[(size_t)q * n + k];
  const LapSetup ls = laplacian_setup(alpha, n, low.data());
  f.n = n;
  f.k = nq + ls.ht;
  f.nc = ls.nc;
  f.scale = ls.scale;
  f.corner = ls.corner;
  f.L.assign((size_t)f.k * n, 0.0);
  f.R.assign((size_t)f.k * n, 0.0);
  // node rows: L[q][k] = R[q][k] = sqrt(w_q) ive(k, 2 t_q); then the high-tail rows
  for (int q = 0; q < nq; ++q) {
    const double sw = std::sqrt(ls.w[q]);
    for (int k = 0; k < n; ++k) f.L[(size_t)q * n + k] = f.R[(size_t)q * n + k] = sw * rows[(size_t)q * n + k];
  }
  std::copy(ls.tail_a.begin(), ls.tail_a.end(), f.L.begin() + (size_t)nq * n);
  std::copy(ls.tail_c.begin(), ls.tail_c.end(), f.R.begin() + (size_t)nq * n);
  return f;
}

std::vector<double> laplacian_coeffs(double alpha, int n, int nthreads) {
  if (n <= 0) return {};
  const LapFactors f = laplacian_factors(alpha, n, nthreads);
  const int nw = worker_count(nthreads);
  std::vector<double> out((size_t)n * n);
  // rank-k symmetric product in blocks of rows; the upper triangle j >= i is computed and
  // mirrored
  constexpr int RB = 16;
  const int nblk = (n + RB - 1) / RB;
  parallel_for(nblk, nw, [&](int blk) {
    const int i0 = blk * RB, i1 = std::min(n, i0 + RB);
    std::vector<double> acc((size_t)RB * n, 0.0);
    for (int q = 0; q < f.k; ++q) {
      const double* lrow = &f.L[(size_t)q * n];
      const double* rrow = &f.R[(size_t)q * n];
      for (int i = i0; i < i1; ++i) {
        const double li = lrow[i];
        if (li == 0.0) continue;
        double* a = &acc[(size_t)(i - i0) * n];
        for (int j = i; j < n; ++j) a[j] += li * rrow[j];
      }
    }
    for (int i = i0; i < i1; ++i)
      for (int j = i; j < n; ++j) {
        const double v = f.scale * acc[(size_t)(i - i0) * n + j];
        out[(size_t)j * n + i] = v;
        out[(size_t)i * n + j] = v;
      }
  });
  for (int j = 0; j < f.nc; ++j)
    for (int i = 0; i < f.nc; ++i) out[(size_t)j * n + i] = f.corner[(size_t)j * f.nc + i];
  return out;
}

std::vector<long double> toeplitz_first_column_inverse(const std::vector<long double>& t) {
  const int m = (int)t.size();
  std::vector<long double> f(m, 0.0L), nf(m, 0.0L);
  if (m == 0) return f;
  if (!(t[0] > 0.0L)) throw std::runtime_error("Toeplitz matrix is not positive definite");
  f[0] = 1.0L / t[0];
  for (int k = 1; k < m; ++k) {
    // T_{k+1} [f; 0] = e_1 + ef e_{k+1};  T_{k+1} [0; J f] = ef e_1 + e_{k+1}
    long double ef = 0.0L;
    for (int i = 0; i < k; ++i) ef += t[k - i] * f[i];
    const long double den = 1.0L - ef * ef;
    if (!(den > 0.0L)) throw std::runtime_error("Levinson recursion broke down (matrix not SPD)");
    for (int i = 0; i <= k; ++i) {
      const long double fi = i < k ? f[i] : 0.0L;
      const long double bi = i > 0 ? f[k - i] : 0.0L;   // [0; J f]_i = f[k-i]
      nf[i] = (fi - ef * bi) / den;
    }
    std::copy(nf.begin(), nf.begin() + k + 1, f.begin());
  }
  return f;
}

void fft_inplace(std::vector<cld>& a, int sign) {
  const int n = (int)a.size();
  if (n & (n - 1)) throw std::runtime_error("fft length must be a power of two");
  for (int i = 1, j = 0; i < n; ++i) {
    int bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[i], a[j]);
  }
  const long double pi = 3.14159265358979323846264338327950288L;
  for (int len = 2; len <= n; len <<= 1) {
    const int half = len / 2;
    std::vector<cld> w(half);
    for (int k = 0; k < half; ++k) {
      const long double ang = sign * 2.0L * pi * k / len;
      w[k] = cld(std::cos(ang), std::sin(ang));
    }
    for (int i = 0; i < n; i += len)
      for (int k = 0; k < half; ++k) {
        const cld u = a[i + k], v = a[i + k + half] * w[k];
        a[i + k] = u + v;
        a[i + k + half] = u - v;
      }
  }
}

GSData gs_data(const std::vector<double>& a1, int n, int m, double beta, int nthreads) {
  GSData g;
  g.n = n;
  g.m = m;
  g.r = m - n;
  if (g.r < 1 || (int)a1.size() < m) throw std::invalid_argument("line size must exceed N");
  std::vector<long double> t(m);
  for (int k = 0; k < m; ++k) t[k] = (k == 0 ? 1.0L : 0.0L) + (long double)beta * a1[k];
  g.c = toeplitz_first_column_inverse(t);
  const long double p1 = g.c[0];
  const long double pi = 3.14159265358979323846264338327950288L;
  // lam_c = fft(c); lam_s = fft(Q s), s = (p1, -p_M, ..., -p_2), Q = diag(e^{-i pi k / M})
  std::vector<cld> vc(m), vs(m);
  for (int k = 0; k < m; ++k) {
    vc[k] = g.c[k];
    const long double sk = k == 0 ? p1 : -g.c[m - k];
    const long double ang = -pi * k / m;
    vs[k] = cld(std::cos(ang), std::sin(ang)) * sk;
  }
  fft_inplace(vc, -1);
  fft_inplace(vs, -1);
  g.lam_c.resize(m);
  g.lam_s.resize(m);
  for (int k = 0; k < m; ++k) {
    const cld lc = vc[k] / (long double)m;
    const cld ls = vs[k] / (2.0L * p1 * m);
    g.lam_c[k] = std::complex<double>((double)lc.real(), (double)lc.imag());
    g.lam_s[k] = std::complex<double>((double)ls.real(), (double)ls.imag());
  }
  if (g.r == 1) {
    g.f.resize(n);
    for (int k = 0; k < n; ++k) g.f[k] = (double)(g.c[m - 1 - k] / p1);
    return g;
  }
  // F = -H_N^-1 B column by column, H_N^-1 by the Gohberg-Semencul formula at size N:
  //   H_N^-1 = (L(x) L(x)^T - L(y) L(y)^T) / x_0,  x = H_N^-1 e_1,  y = (0, x_{N-1}, ..., x_1)
  // with L(v) the lower-triangular Toeplitz matrix of first column v
  std::vector<long double> tn(t.begin(), t.begin() + n);
  const std::vector<long double> xl = toeplitz_first_column_inverse(tn);
  std::vector<double> x(n), y(n, 0.0);
  for (int k = 0; k < n; ++k) x[k] = (double)xl[k];
  for (int k = 1; k < n; ++k) y[k] = x[n - k];
  const double x0 = x[0];
  g.f.assign((size_t)g.r * n, 0.0);
  parallel_for(g.r, worker_count(nthreads), [&](int j) {
    std::vector<double> b(n), u(n), v(n), out(n);
    for (int k = 0; k < n; ++k) b[k] = beta * a1[n + j - k];   // column j of H_M[0:N, N:M]
    // u = L(x)^T b, v = L(y)^T b
    for (int i = 0; i < n; ++i) {
      double su = 0.0, sv = 0.0;
      for (int k = i; k < n; ++k) {
        su += x[k - i] * b[k];
        sv += y[k - i] * b[k];
      }
      u[i] = su;
      v[i] = sv;
    }
    // out = L(x) u - L(y) v
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int k = 0; k <= i; ++k) s += x[i - k] * u[k] - y[i - k] * v[k];
      out[i] = s / x0;
    }
    for (int k = 0; k < n; ++k) g.f[(size_t)j * n + k] = -out[k];
  });
  return g;
}

int line_size(int n) {
  int m = 16;
  while (m < n + 1) m *= 2;
  return m;
}


}  // namespace sadi
