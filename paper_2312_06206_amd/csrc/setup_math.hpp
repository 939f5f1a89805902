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

// First column of T^-1 for the SPD Toeplitz T with first column t[0..m-1]
// (Levinson-Durbin, extended precision).
std::vector<long double> toeplitz_first_column_inverse(const std::vector<long double>& t);

// In-place radix-2 FFT of length n (power of two), sign -1 forward, +1 inverse
// (unnormalised), extended precision.
void fft_inplace(std::vector<cld>& a, int sign);

// Gohberg-Semencul data of the bordered line matrix H_M (M = N+1):
//   lam_s = fft(Q s) / (2 p1 M), lam_c = fft(c) / M, f[k] = c[M-1-k] / p1 (k < N)
struct GSData {
  int n = 0, m = 0;
  std::vector<long double> c;            // H_M^-1 e_1
  std::vector<std::complex<double>> lam_s, lam_c;
  std::vector<double> f;
};
GSData gs_data(const std::vector<double>& a1, int n, double beta);

// Eigenvalues of the P x P (P = 2M) block-circulant embedding of the N x N BTTB with
// coefficients a2, divided by P^2, for kx, ky in [0, M].  Row kx of the result
// (length M+1, at out[kx*ld ...]) is [Lam(kx, 0), Lam(kx, 2), ..., Lam(kx, M)]
// followed by [Lam(kx, 1), Lam(kx, 3), ..., Lam(kx, M-1)] (even then odd ky).
void bccb_eigenvalues(const std::vector<double>& a2, int n, double* out, int ld, int nthreads = 0);

}  // namespace sadi
