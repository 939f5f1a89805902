// Dense matrix products on the matrix cores of gfx950: FP64 (v_mfma_f64_16x16x4_f64) and
// FP32 operands (v_mfma_f32_16x16x4_f32, FP32 accumulation, C in FP32 or FP64).
//
// C = alpha A diag(s) B + beta C (s optional), C row-major (C(i, j) at C[i ldc + j]), B with
// contiguous rows (B(k, j) at B[k ldb + j]), A either with contiguous rows (AK: A(i, k) at A[i lda + k])
// or contiguous columns (A(i, k) at A[k lda + i]).  A block of WM x WN waves computes a
// (32 WM) x (32 WN) tile of C, each wave a 32 x 32 part as 2 x 2 MFMA tiles of 16 x 16; two
// shapes are built, 64 x 64 (four waves) and 32 x 32 (one wave, for products with few
// tiles).  K advances in slices of 16 staged through LDS, double buffered: the global loads
// of slice s + 1 are in flight while the matrix cores work on slice s.
// Batches: blockIdx.z indexes an array of (A, B, C) pointer triples; without the array
// the single triple passed by value is used.
//
// Operand layouts (wave64, measured on gfx950): lane l supplies A(l % 16, l / 16) and
// B(l / 16, l % 16) of the 16 x 4 and 4 x 16 operands for both instructions; accumulator
// register r (r < 4) holds D(4 r + l / 16, l % 16) for the FP64 instruction and
// D(4 (l / 16) + r, l % 16) for the FP32 one.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace sadi {

namespace {

constexpr int kBK = 16;
constexpr int kPad = 1;   // LDS row padding (doubles)

// Slices of A (BM x 16 of op(A)) and B (16 x BN) staged in registers.  Loads run along the
// contiguous direction: AK: 16 lanes per row of A (128 bytes); otherwise BM lanes along a
// column of A; B: BN lanes along a row.
template <typename TI, bool AK, int BM, int BN, int NT>
struct Stage {
  static constexpr int QA = BM * kBK / NT, QB = BN * kBK / NT;
  TI a[QA], b[QB];

  __device__ __forceinline__ void load(const TI* __restrict__ A, long lda, const TI* __restrict__ B, long ldb,
                                       const double* __restrict__ bscale, int m, int n, int k, int i0, int j0,
                                       int k0, int t) {
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int i = AK ? i0 + t / 16 + (NT / 16) * q : i0 + t % BM;
      const int kk = AK ? k0 + t % 16 : k0 + t / BM + (NT / BM) * q;
      a[q] = (i < m && kk < k) ? (AK ? A[(long)i * lda + kk] : A[(long)kk * lda + i]) : TI(0);
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int kb = k0 + t / BN + (NT / BN) * q, j = j0 + t % BN;
      b[q] = (kb < k && j < n) ? B[(long)kb * ldb + j] : TI(0);
      if (bscale && kb < k) b[q] = (TI)(b[q] * bscale[kb]);
    }
  }

  // into LDS, both k-major: As[kk][i], Bs[kk][j]
  __device__ __forceinline__ void store(TI (*As)[BM + kPad], TI (*Bs)[BN + kPad], int t) const {
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      if constexpr (AK) As[t % 16][t / 16 + (NT / 16) * q] = a[q];
      else As[t / BM + (NT / BM) * q][t % BM] = a[q];
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) Bs[t / BN + (NT / BN) * q][t % BN] = b[q];
  }
};

// one MFMA step of a 16 x 16 tile and the row of C its accumulator register r holds
template <typename TI> struct Mfma;
template <> struct Mfma<double> {
  using acc = __attribute__((__vector_size__(4 * sizeof(double)))) double;
  static __device__ __forceinline__ acc step(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int r, int fk) { return 4 * r + fk; }
};
template <> struct Mfma<float> {
  using acc = __attribute__((__vector_size__(4 * sizeof(float)))) float;
  static __device__ __forceinline__ acc step(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int r, int fk) { return 4 * fk + r; }
};

template <typename TI, typename P, bool AK, int WM, int WN>
__global__ void __launch_bounds__(64 * WM * WN)
gemm_mfma_kernel(int m, int n, int k, P single, const P* __restrict__ batch, long lda, long ldb, long ldc,
                 double alpha, double beta, const double* __restrict__ bscale) {
  constexpr int BM = 32 * WM, BN = 32 * WN, NT = 64 * WM * WN;
  using MF = Mfma<TI>;
  __shared__ TI As[2][kBK][BM + kPad];
  __shared__ TI Bs[2][kBK][BN + kPad];
  const P p = batch ? batch[blockIdx.z] : single;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = wave / WN, wn = wave % WN;     // the wave's 32 x 32 part
  const int i0 = blockIdx.y * BM, j0 = blockIdx.x * BN;

  typename MF::acc acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = typename MF::acc{0, 0, 0, 0};

  Stage<TI, AK, BM, BN, NT> st;
  st.load(p.A, lda, p.B, ldb, bscale, m, n, k, i0, j0, 0, t);
  st.store(As[0], Bs[0], t);
  __syncthreads();
  const int nslices = (k + kBK - 1) / kBK;
  const int fr = lane & 15, fk = lane >> 4;     // fragment row / k of this lane
  for (int s = 0; s < nslices; ++s) {
    const int cur = s & 1;
    if (s + 1 < nslices) st.load(p.A, lda, p.B, ldb, bscale, m, n, k, i0, j0, (s + 1) * kBK, t);
#pragma unroll
    for (int kk = 0; kk < kBK; kk += 4) {
      const TI a0 = As[cur][kk + fk][wm * 32 + fr];
      const TI a1 = As[cur][kk + fk][wm * 32 + 16 + fr];
      const TI b0 = Bs[cur][kk + fk][wn * 32 + fr];
      const TI b1 = Bs[cur][kk + fk][wn * 32 + 16 + fr];
      acc[0][0] = MF::step(a0, b0, acc[0][0]);
      acc[0][1] = MF::step(a0, b1, acc[0][1]);
      acc[1][0] = MF::step(a1, b0, acc[1][0]);
      acc[1][1] = MF::step(a1, b1, acc[1][1]);
    }
    if (s + 1 < nslices) {
      st.store(As[cur ^ 1], Bs[cur ^ 1], t);   // the other buffer: last read one slice ago
      __syncthreads();
    }
  }

#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      const int j = j0 + wn * 32 + 16 * y + fr;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wm * 32 + 16 * x + MF::row(r, fk);
        if (i < m && j < n) {
          auto* c = p.C + (long)i * ldc + j;
          const double v = alpha * (double)acc[x][y][r];
          *c = beta == 0.0 ? v : fma(beta, (double)*c, v);
        }
      }
    }
}

template <typename TI, typename P, int WM, int WN>
void launch_shape(int m, int n, int k, const P& single, const P* batch, int count, bool a_rows, long lda, long ldb,
                  long ldc, double alpha, double beta, const double* bscale, hipStream_t st) {
  const dim3 grid((n + 32 * WN - 1) / (32 * WN), (m + 32 * WM - 1) / (32 * WM), batch ? count : 1);
  const dim3 blk(64 * WM * WN);
  if (a_rows)
    hipLaunchKernelGGL((gemm_mfma_kernel<TI, P, true, WM, WN>), grid, blk, 0, st, m, n, k, single, batch, lda, ldb,
                       ldc, alpha, beta, bscale);
  else
    hipLaunchKernelGGL((gemm_mfma_kernel<TI, P, false, WM, WN>), grid, blk, 0, st, m, n, k, single, batch, lda, ldb,
                       ldc, alpha, beta, bscale);
}

// 64 x 64 (four waves per block) unless that leaves fewer blocks than half the 256 CUs;
// measured on the rank-225 correction at N = 799 (169 blocks): 64 x 64 is the faster
int pick_tile(int m, int n, long batches) {
  const long big = (long)((m + 63) / 64) * ((n + 63) / 64) * batches;
  return big >= 128 ? 64 : 32;
}

template <typename TI, typename P>
void launch_any(int m, int n, int k, const P& single, const P* batch, int count, bool a_rows, long lda, long ldb,
                long ldc, double alpha, double beta, hipStream_t st, int tile, const double* bscale) {
  if (m <= 0 || n <= 0 || count <= 0) return;
  if (tile == 0) tile = pick_tile(m, n, batch ? count : 1);
  if (tile == 64)
    launch_shape<TI, P, 2, 2>(m, n, k, single, batch, count, a_rows, lda, ldb, ldc, alpha, beta, bscale, st);
  else
    launch_shape<TI, P, 1, 1>(m, n, k, single, batch, count, a_rows, lda, ldb, ldc, alpha, beta, bscale, st);
}

// ---- element-wise helpers of the dense paths -------------------------------------------
__global__ void __launch_bounds__(256) to_fp32_kernel(const CvtPtrs* __restrict__ b, int n, long lds) {
  const CvtPtrs p = b[blockIdx.y];
  const size_t nn = (size_t)n * n;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < nn; e += (size_t)gridDim.x * 256) {
    const size_t i = e / n, j = e % n;
    p.dst[e] = (float)p.src[i * lds + j];
  }
}
__global__ void __launch_bounds__(256) copy_fp64_kernel(const CopyPtrs* __restrict__ b, int n, long lds, long ldd) {
  const CopyPtrs p = b[blockIdx.y];
  const size_t nn = (size_t)n * n;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < nn; e += (size_t)gridDim.x * 256) {
    const size_t i = e / n, j = e % n;
    p.dst[i * ldd + j] = p.src[i * lds + j];
  }
}
__global__ void __launch_bounds__(256) toeplitz_fill_kernel(const ToeplitzPtrs* __restrict__ b, int n) {
  const ToeplitzPtrs p = b[blockIdx.y];
  const size_t nn = (size_t)n * n;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < nn; e += (size_t)gridDim.x * 256) {
    const int i = (int)(e / n), j = (int)(e % n);
    p.H[e] = p.t[i > j ? i - j : j - i];
  }
}

int elementwise_grid(int n) {
  const size_t blocks = ((size_t)n * n + 255) / 256;
  return blocks > 1024 ? 1024 : (int)blocks;
}

}  // namespace

void launch_dgemm(int m, int n, int k, const GemmPtrs& single, const GemmPtrs* batch, int count, bool a_rows,
                  long lda, long ldb, long ldc, double alpha, double beta, hipStream_t st, int tile,
                  const double* bscale) {
  launch_any<double, GemmPtrs>(m, n, k, single, batch, count, a_rows, lda, ldb, ldc, alpha, beta, st, tile, bscale);
}

void launch_sgemm(int m, int n, int k, const GemmPtrs32<float>* batch, int count, bool a_rows, long lda, long ldb,
                  long ldc, double alpha, double beta, hipStream_t st, int tile) {
  launch_any<float, GemmPtrs32<float>>(m, n, k, GemmPtrs32<float>{}, batch, count, a_rows, lda, ldb, ldc, alpha,
                                       beta, st, tile, nullptr);
}

void launch_sgemm(int m, int n, int k, const GemmPtrs32<double>* batch, int count, bool a_rows, long lda, long ldb,
                  long ldc, double alpha, double beta, hipStream_t st, int tile) {
  launch_any<float, GemmPtrs32<double>>(m, n, k, GemmPtrs32<double>{}, batch, count, a_rows, lda, ldb, ldc, alpha,
                                        beta, st, tile, nullptr);
}

void launch_to_fp32(const CvtPtrs* batch, int count, int n, long lds, hipStream_t st) {
  if (count > 0 && n > 0)
    hipLaunchKernelGGL(to_fp32_kernel, dim3(elementwise_grid(n), count), dim3(256), 0, st, batch, n, lds);
}
void launch_copy_fp64(const CopyPtrs* batch, int count, int n, long lds, long ldd, hipStream_t st) {
  if (count > 0 && n > 0)
    hipLaunchKernelGGL(copy_fp64_kernel, dim3(elementwise_grid(n), count), dim3(256), 0, st, batch, n, lds, ldd);
}
void launch_toeplitz_fill(const ToeplitzPtrs* batch, int count, int n, hipStream_t st) {
  if (count > 0 && n > 0)
    hipLaunchKernelGGL(toeplitz_fill_kernel, dim3(elementwise_grid(n), count), dim3(256), 0, st, batch, n);
}

}  // namespace sadi
