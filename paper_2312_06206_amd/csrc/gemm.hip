// Dense FP64 matrix products on the matrix cores of gfx950 (v_mfma_f64_16x16x4_f64).
//
// C = alpha A B + beta C, C row-major (C(i, j) at C[i ldc + j]), B with contiguous rows
// (B(k, j) at B[k ldb + j]), A either with contiguous rows (AK: A(i, k) at A[i lda + k])
// or contiguous columns (A(i, k) at A[k lda + i]).  Blocks of 256 threads compute 64 x 64
// tiles of C: four waves in a 2 x 2 arrangement, each wave a 32 x 32 quarter as 2 x 2 MFMA
// tiles of 16 x 16.  K advances in slices of 16 staged through LDS, double buffered: the
// global loads of slice s + 1 are in flight while the matrix cores work on slice s.
// Batches: blockIdx.z indexes an array of (A, B, C) pointer triples; without the array
// the single triple passed by value is used.
//
// Operand layout of v_mfma_f64_16x16x4_f64 (wave64, measured on gfx950): lane l supplies
// A(l % 16, l / 16) and B(l / 16, l % 16) of the 16 x 4 and 4 x 16 operands, and holds
// D(4 r + l / 16, l % 16) in accumulator register r (r < 4).
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace sadi {

namespace {

constexpr int kBM = 64, kBN = 64, kBK = 16;
constexpr int kPad = 1;   // LDS row padding (doubles)

using acc4 = __attribute__((__vector_size__(4 * sizeof(double)))) double;

// A slice (kBM rows x kBK columns of op(A)) and a B slice (kBK x kBN) staged in registers,
// 4 values of each per thread.  Loads run along the contiguous direction: AK: 16 lanes per
// row of A (128 bytes), rows t / 16 + 16 q; otherwise 64 lanes along a column of A (512
// bytes), columns t / 64 + 4 q.  B: 64 lanes along a row, rows t / 64 + 4 q.
template <bool AK>
struct Stage {
  double a[4], b[4];

  __device__ __forceinline__ void load(const double* __restrict__ A, long lda, const double* __restrict__ B,
                                       long ldb, int m, int n, int k, int i0, int j0, int k0, int t) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = AK ? i0 + (t >> 4) + 16 * q : i0 + (t & 63);
      const int kk = AK ? k0 + (t & 15) : k0 + (t >> 6) + 4 * q;
      const bool in = i < m && kk < k;
      a[q] = in ? (AK ? A[(long)i * lda + kk] : A[(long)kk * lda + i]) : 0.0;
      const int kb = k0 + (t >> 6) + 4 * q, j = j0 + (t & 63);
      b[q] = (kb < k && j < n) ? B[(long)kb * ldb + j] : 0.0;
    }
  }

  // into LDS, both k-major: As[kk][i], Bs[kk][j]
  __device__ __forceinline__ void store(double (*As)[kBM + kPad], double (*Bs)[kBN + kPad], int t) const {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if constexpr (AK) As[t & 15][(t >> 4) + 16 * q] = a[q];
      else As[(t >> 6) + 4 * q][t & 63] = a[q];
      Bs[(t >> 6) + 4 * q][t & 63] = b[q];
    }
  }
};

template <bool AK>
__global__ void __launch_bounds__(256)
dgemm_mfma_kernel(int m, int n, int k, GemmPtrs single, const GemmPtrs* __restrict__ batch, long lda, long ldb,
                  long ldc, double alpha, double beta) {
  __shared__ double As[2][kBK][kBM + kPad];
  __shared__ double Bs[2][kBK][kBN + kPad];
  const GemmPtrs p = batch ? batch[blockIdx.z] : single;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;      // the wave's 32 x 32 quarter
  const int i0 = blockIdx.y * kBM, j0 = blockIdx.x * kBN;

  acc4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = acc4{0.0, 0.0, 0.0, 0.0};

  Stage<AK> st;
  st.load(p.A, lda, p.B, ldb, m, n, k, i0, j0, 0, t);
  st.store(As[0], Bs[0], t);
  __syncthreads();
  const int nslices = (k + kBK - 1) / kBK;
  const int fr = lane & 15, fk = lane >> 4;     // fragment row / k of this lane
  for (int s = 0; s < nslices; ++s) {
    const int cur = s & 1;
    if (s + 1 < nslices) st.load(p.A, lda, p.B, ldb, m, n, k, i0, j0, (s + 1) * kBK, t);
#pragma unroll
    for (int kk = 0; kk < kBK; kk += 4) {
      const double a0 = As[cur][kk + fk][wm * 32 + fr];
      const double a1 = As[cur][kk + fk][wm * 32 + 16 + fr];
      const double b0 = Bs[cur][kk + fk][wn * 32 + fr];
      const double b1 = Bs[cur][kk + fk][wn * 32 + 16 + fr];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    if (s + 1 < nslices) {
      st.store(As[cur ^ 1], Bs[cur ^ 1], t);   // the other buffer: last read one slice ago
      __syncthreads();
    }
  }

  // D(4 r + lane / 16, lane % 16) of each 16 x 16 tile
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      const int j = j0 + wn * 32 + 16 * y + fr;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wm * 32 + 16 * x + 4 * r + fk;
        if (i < m && j < n) {
          double* c = p.C + (long)i * ldc + j;
          const double v = alpha * acc[x][y][r];
          *c = beta == 0.0 ? v : fma(beta, *c, v);
        }
      }
    }
}

}  // namespace

void launch_dgemm(int m, int n, int k, const GemmPtrs& single, const GemmPtrs* batch, int count, bool a_rows,
                  long lda, long ldb, long ldc, double alpha, double beta, hipStream_t st) {
  if (m <= 0 || n <= 0 || count <= 0) return;
  const dim3 grid((n + kBN - 1) / kBN, (m + kBM - 1) / kBM, batch ? count : 1);
  if (a_rows)
    hipLaunchKernelGGL(dgemm_mfma_kernel<true>, grid, dim3(256), 0, st, m, n, k, single, batch, lda, ldb, ldc, alpha,
                       beta);
  else
    hipLaunchKernelGGL(dgemm_mfma_kernel<false>, grid, dim3(256), 0, st, m, n, k, single, batch, lda, ldb, ldc, alpha,
                       beta);
}

}  // namespace sadi
