// Host-side setup mathematics of the S-ADI solver (no GPU code).
#pragma once
#include <complex>
#include <vector>

namespace sadi {

using cld = std::complex<long double>;

// a_k, k = 0..count-1 (1D fractional centred difference, closed form via its
// Gamma-ratio recurrence, extended precision).
std::vector<double> riesz_coeffs(double alpha, int count);

// a_ij for 0 <= i,j < n, stored [j*n + i] (symmetric).  Subordination integral with
// a whole-line trapezoidal rule in s = log t; nthreads workers (0 = hardware).
std::vector<double> laplacian_coeffs(double alpha, int n, int nthreads = 0);

// The same a_ij as a rank-k product: a_ij = scale * sum_q L[q][i] R[q][j] (rows q of n: the
// quadrature nodes, then the high-tail Hankel terms), except for the corner i, j < nc,
// given exactly in corner[j*nc + i] (low-tail series and the origin).
struct LapFactors {
  int n = 0, k = 0, nc = 0;
  double scale = 0.0;
  std::vector<double> L, R, corner;
};
LapFactors laplacian_factors(double alpha, int n, int nthreads = 0);

// The same quadrature split by where its parts are computed.  The node rows ive(k, x_q),
// x_q = 2 t_q (q < lap_node_count()), do not depend on alpha; everything else does and is
// cheap: LapSetup holds the node weights w_q (a_ij gets w_q ive(i, x_q) ive(j, x_q) from node
// q), the high-tail rows (a_ij gets sum_p tail_a[p][i] tail_c[p][j]), the overall factor
// `scale`, and the exact corner i, j < nc.  ive_low: ive(k, x_q) for k < kLapLowOrders at
// ive_low[q * kLapLowOrders + k].
constexpr int kLapLowOrders = 12;   // low-tail series needed only for i + j < this
constexpr int kLapTailTerms = 16;   // Hankel terms of the high tail
struct LapSetup {
  int n = 0, nq = 0, ht = 0, nc = 0;
  double scale = 0.0;
  std::vector<double> w, tail_a, tail_c, corner;
};
int lap_node_count();
double lap_node_x(int q);
LapSetup laplacian_setup(double alpha, int n, const double* ive_low);
// ive(k, x_q) for k < nrows at every node (host, long double recurrence): [q * nrows + k]
std::vector<double> ive_node_rows(int nrows, int nthreads = 0);

// First column of T^-1 for the SPD Toeplitz T with first column t[0..m-1]
// (Levinson-Durbin, extended precision).
std::vector<long double> toeplitz_first_column_inverse(const std::vector<long double>& t);

// In-place radix-2 FFT of length n (power of two), sign -1 forward, +1 inverse
// (unnormalised), extended precision.
void fft_inplace(std::vector<cld>& a, int sign);

// Gohberg-Semencul data of the bordered line matrix H_M (M = N+1):
//   lam_s = fft(Q s) / (2 p1 M), lam_c = fft(c) / M, f[k] = c[M-1-k] / p1 (k < N)
// Gohberg-Semencul data of the line matrix H_M = I + beta T(a_0..a_{M-1}) (M a power of two,
// M >= N + 1) and the correction from H_M^-1 to H_N^-1: with w = H_M^-1 [v; 0],
//   H_N^-1 v = w[0:N] - F w[N:M],   F = A12 A22^-1 = -H_N^-1 B   (A = H_M^-1, B = H_M[0:N, N:M]).
// r = M - N = 1: F is the vector f (f[k] = c[M-1-k] / c[0]); otherwise F is stored as r rows
// of N (row j = column j of F).
struct GSData {
  int n = 0, m = 0, r = 0;
  std::vector<long double> c;            // H_M^-1 e_1
  std::vector<std::complex<double>> lam_s, lam_c;
  std::vector<double> f;                 // r * n entries
};
GSData gs_data(const std::vector<double>& a1, int n, int m, double beta, int nthreads = 0);


// Line size for N interior nodes: the smallest power of two M >= max(N + 1, 16).
int line_size(int n);

}  // namespace sadi
