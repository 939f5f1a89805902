// Internal interface between the C ABI layer and the device kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "fft_core.hpp"

namespace sadi {

// supported line lengths M = N + 1
#define SADI_FOR_EACH_M(X) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096)

// tables of the Gohberg-Semencul line solve (R = double, or float for the FP32 solves)
template <typename R> struct GSTables {
  const V2<R>* q;        // Q = diag(e^{-i pi k / M}), k < M
  const V2<R>* lam_s;    // fft(Q s) / (2 p_1 M)
  const V2<R>* lam_c;    // fft(c) / M
  const R* f;            // correction to H_N^-1: r = 1: (J c)[k] / p_1, k < N; else F, r rows of N
  int r;                 // M - N; 0: no correction (the bordered solution of size M is left)
};
using GSTables64 = GSTables<double>;

// FP64 product with beta T(a_0..a_{N-1}) (residual of the FP32 solves): eigenvalues of its
// 2M-point circulant embedding, even and odd frequencies, times beta / (2M)
struct ToeplitzTables64 {
  const double* sig_e;
  const double* sig_o;
};

// per-call scalars of the right-hand side B = sigma (L u) h^alpha + gamma g(u) [+ tau phi2]
struct StepScalars {
  double sigma;   // multiplies the BTTB convolution (carries -kappa tau^2 h^-alpha etc.)
  double gamma;   // multiplies g(u)
  double tau;     // start-up step: multiplies phi2
  int gkind;      // 0: 0, 1: -sin u, 2: -u^3, 3: -gparam * u
  double gparam;
};

// sin x in FP64 for |x| <= kSinFastMax: Cody-Waite reduction x = k pi + r, |r| <= pi/2,
// with pi split into three doubles (fused multiply-adds, one rounding per term), then
// sin x = (-1)^k sin r with the Taylor series of sin r to r^23, whose truncation error is
// below 1e-20 on |r| <= pi/2.  About 18 instructions instead of the general routine's ~110.
// Larger arguments, infinities and NaN must go to the library sin (see rhs_phase): for
// them the reduced argument is not small (|x| above about 5e30 overflows the series, and
// k leaves the int range above 2^31 pi), so the result is not used.
constexpr double kSinFastMax = 1.0e5;
__device__ __forceinline__ double sin_fp64(double x) {
  constexpr double kPi_1 = 0x1.921fb54442d18p+1, kPi_2 = 0x1.1a62633145c07p-53,
                   kPi_3 = -0x1.f1976b7ed8fbcp-109, kOneOverPi = 0x1.45f306dc9c883p-2;
  const double k = rint(x * kOneOverPi);
  double r = fma(-k, kPi_1, x);
  r = fma(-k, kPi_2, r);
  r = fma(-k, kPi_3, r);
  const double r2 = r * r;
  double ps = -1.0 / 25852016738884976640000.0;  // -1/23!
  ps = fma(ps, r2, 1.0 / 51090942171709440000.0);  // 1/21!
  ps = fma(ps, r2, -1.0 / 121645100408832000.0);   // -1/19!
  ps = fma(ps, r2, 1.0 / 355687428096000.0);       // 1/17!
  ps = fma(ps, r2, -1.0 / 1307674368000.0);        // -1/15!
  ps = fma(ps, r2, 1.0 / 6227020800.0);            // 1/13!
  ps = fma(ps, r2, -1.0 / 39916800.0);             // -1/11!
  ps = fma(ps, r2, 1.0 / 362880.0);                // 1/9!
  ps = fma(ps, r2, -1.0 / 5040.0);                 // -1/7!
  ps = fma(ps, r2, 1.0 / 120.0);                   // 1/5!
  ps = fma(ps, r2, -1.0 / 6.0);                    // -1/3!
  const double s = fma(r * r2, ps, r);
  return ((int)k & 1) ? -s : s;
}

// launch shapes per kernel family (measured over N = 127..4095 and the uneven batch)
// row line kernels: one line per workgroup from T = 128 threads per line, else 128 threads
// with the lines' lanes interleaved (the rows of a pair of S then share every request)
template <int M> struct RowCfg {
  static constexpr int T = M / Shape<M>::E;
  static constexpr int LPW = T >= 128 ? 1 : 128 / T;
  static constexpr bool LINE_FAST = LPW > 1;
  static constexpr int SPLIT = 2;
  using Line = sadi::Line<M, double, LPW, LINE_FAST, SPLIT>;
  static constexpr int NT = Line::NT;
  static constexpr int LDS_BYTES = Line::LDS_BYTES;
};

// forward row transforms: at T = 256 both rows of a pair of the half spectrum in one
// workgroup, lanes interleaved, so that every store covers whole cache lines of S
template <int M> struct RowFwdCfg {
  static constexpr int T = M / Shape<M>::E;
  static constexpr int LPW = T >= 256 ? 2 : 256 / T;
  static constexpr bool LINE_FAST = T >= 256;
  static constexpr int SPLIT = 2;
  using Line = sadi::Line<M, double, LPW, LINE_FAST, SPLIT>;
  static constexpr int NT = Line::NT;
  static constexpr int LDS_BYTES = Line::LDS_BYTES;
};

// two lines (even / odd frequency halves) per column; 256 threads per workgroup (512 at
// M = 4096, one column).  Small workgroups spread the few columns of small N over all CUs.
template <int M> struct ColConvCfg {
  static constexpr int T = M / Shape<M>::E;
  static constexpr int LPW = (256 / T) < 2 ? 2 : 256 / T;
  static constexpr bool LINE_FAST = true;
  static constexpr int SPLIT = 2;
  using Line = sadi::Line<M, double, LPW, LINE_FAST, SPLIT>;
  static constexpr int NT = Line::NT;
  static constexpr int LDS_BYTES = Line::LDS_BYTES;
};

// adjacent columns in adjacent lanes; 256 threads per workgroup (512 at M = 4096)
template <int M> struct ColGSCfg {
  static constexpr int T = M / Shape<M>::E;
  static constexpr int LPW = (256 / T) < 2 ? 2 : 256 / T;
  static constexpr bool LINE_FAST = true;
  static constexpr int SPLIT = 2;
  using Line = sadi::Line<M, double, LPW, LINE_FAST, SPLIT>;
  static constexpr int NT = Line::NT;
  static constexpr int LDS_BYTES = Line::LDS_BYTES;
};

// mixed precision (FP32 solves, optional FP64 residual correction): 2 waves per SIMD,
// 256 threads per workgroup.  Beyond the exchange region (LDS_BYTES), KEEP_BYTES hold M
// doubles per line that the solve keeps across its stages (keep(smem, line)).
template <int M, bool FAST> struct MixCfg {
  static constexpr int T = M / Shape<M>::E;
  static constexpr int LPW = T >= 256 ? 1 : 256 / T;
  static constexpr bool LINE_FAST = FAST;
  using Line = sadi::Line<M, double, LPW, LINE_FAST, 2>;
  using Line32 = sadi::Line<M, float, LPW, LINE_FAST, 1>;
  static constexpr int NT = Line::NT;
  static constexpr int LDS_BYTES = Line::LDS_BYTES > Line32::LDS_BYTES ? Line::LDS_BYTES : Line32::LDS_BYTES;
  static constexpr int KEEP_BYTES = LPW * M * (int)sizeof(double);
  static __device__ __forceinline__ double* keep(unsigned char* smem, int line) {
    return reinterpret_cast<double*>(smem + LDS_BYTES) + (size_t)line * M;
  }
};
template <int M> using MixRowCfg = MixCfg<M, false>;
template <int M> using MixColCfg = MixCfg<M, true>;

// everything the mixed-precision line solve needs
struct MixedTables {
  FFTTables<float> tab32;
  GSTables<float> gs32;
  ToeplitzTables64 toe;
  const double2* q64;      // e^{-i pi k / M} (FP64), k < M
  int refine;              // 1: one FP64 residual correction
};

// One instance of a batch.  The instances of one launch share N, the pitches of S, X and
// Lambda, and the FFT tables (rootM, rootS, root2M; root2M also serves as Q).
struct BatchInst {
  double* u[2];             // the two state buffers, N x N (pitch N), caller-owned
  const double* phi2;       // start-up velocity, N x N, or null
  double2* S;               // half spectrum, N rows
  double* X;                // line-solve workspace, N rows
  const double* lam2d;      // BCCB eigenvalues, M + 1 rows
  const double2* lam_s;     // Gohberg-Semencul tables of this instance's H
  const double2* lam_c;
  const double* f;
  int r;                    // M - N (the same for every instance of a launch)
  StepScalars sc;           // sigma, gamma carry this instance's kappa, h^-alpha, tau
  // for launches that mix instances of different sizes (work lists): this instance's grid,
  // line length, pitches of S (complex), X (doubles) and Lambda, and its line tables
  int n, m, lds, ldx, ldlam;
  FFTTables<double> tab;
};

// One workgroup's share of a work-list launch: instance `inst` of the descriptor array and
// its block `blk` in the single-instance numbering of that phase; inst < 0: nothing to do.
struct WorkItem {
  int inst;
  int blk;
};
// Work lists cover line lengths M <= kWorkListMaxM (their workgroup size is the same for all).
constexpr int kWorkListMaxM = 2048;
// Blocks of one instance in each phase of the batched step (0: column convolution,
// 1: row pass with the x-sweep, 2: y-sweep with the next row transform) and a relative cost
// per block (lines x M log2 M) for balancing.
void worklist_shape(int m, int n, int blocks[3], double cost[3]);
// One launch of phase `phase` over the work list (nitems entries).  iu: the state buffer the
// step advances (phase 1, 2); ip: the other one (phase 2).
void launch_worklist(int phase, const BatchInst* bi, const WorkItem* items, int nitems, int iu, int ip,
                     hipStream_t st);

// Dense FP64 products on the matrix cores: C = alpha A B + beta C (k may be 0: C = beta C).
// C(i, j) at C[i ldc + j]; B(k, j) at B[k ldb + j]; A(i, k) at A[i lda + k] (a_rows) or at
// A[k lda + i].  batch: device array of count pointer triples (blockIdx.z), or null to use
// `single`.  No element of C may also be an element of A or B (they may share a buffer).
// tile: 64 or 32 (square tile of C per workgroup), 0 picks by the number of tiles.  bscale:
// optional k-vector s, C = alpha A diag(s) B + beta C.
struct GemmPtrs {
  const double* A;
  const double* B;
  double* C;
};
void launch_dgemm(int m, int n, int k, const GemmPtrs& single, const GemmPtrs* batch, int count, bool a_rows,
                  long lda, long ldb, long ldc, double alpha, double beta, hipStream_t st, int tile = 0,
                  const double* bscale = nullptr);
// The same with FP32 operands on the FP32 matrix cores (v_mfma_f32_16x16x4_f32), FP32
// accumulation, and C in FP32 or FP64 (alpha, beta and the update of C in FP64).  Batched only.
template <typename TC> struct GemmPtrs32 {
  const float* A;
  const float* B;
  TC* C;
};
void launch_sgemm(int m, int n, int k, const GemmPtrs32<float>* batch, int count, bool a_rows, long lda, long ldb,
                  long ldc, double alpha, double beta, hipStream_t st, int tile = 0);
void launch_sgemm(int m, int n, int k, const GemmPtrs32<double>* batch, int count, bool a_rows, long lda, long ldb,
                  long ldc, double alpha, double beta, hipStream_t st, int tile = 0);
// Element-wise helpers of the dense paths, over `count` n x n matrices (blockIdx.y):
// dst = (float) src (src pitch lds, dst pitch n); dst = src (FP64, pitches lds and ldd);
// H = the symmetric Toeplitz matrix of first column t (pitch n).
struct CvtPtrs {
  const double* src;
  float* dst;
};
struct CopyPtrs {
  const double* src;
  double* dst;
};
struct ToeplitzPtrs {
  const double* t;
  double* H;
};
void launch_to_fp32(const CvtPtrs* batch, int count, int n, long lds, hipStream_t st);
void launch_copy_fp64(const CopyPtrs* batch, int count, int n, long lds, long ldd, hipStream_t st);
void launch_toeplitz_fill(const ToeplitzPtrs* batch, int count, int n, hipStream_t st);

// Gohberg-Semencul data of H_M (M = m <= 4096, N = M - 1) on the device: c = H_M^-1 e_1 by a
// double-double Levinson-Durbin recursion (t = t_hi + t_lo, the first column of H_M; one
// workgroup), then lam_s, lam_c, f (and float32 copies) as in Algorithm 1; q[j] = e^{-i pi j/M}.
// c: m doubles of work space.
void launch_gs_generator(const double* t_hi, const double* t_lo, int m, double* c, const double2* q, double2* lam_s,
                         double2* lam_c, double* f, float2* lam_s32, float2* lam_c32, float* f32, hipStream_t st);

// hat == nullptr: transform u.  Otherwise first u <- 2 u - uprev + hat (stored into uprev),
// hat in plain rows of pitch ldx
template <int M>
void launch_rows_fwd(const double* u, double* uprev, const double* hat, int ldx, int ldu, double2* S, int lds_,
                     int n, const FFTTables<double>& tab, const double2* root2M, hipStream_t st);
void launch_leapfrog(int mode, double* ucur, double* uprev, const double* hat, int ldx, double* out, int n,
                     hipStream_t st);
template <int M>
void launch_cols_conv(double2* S, int lds_, int n, const double* lam, int ldlam, const FFTTables<double>& tab,
                      const double2* root2M, hipStream_t st);
template <int M>
void launch_rows_rhs_gs(int mode, const double2* S, int lds_, const double* u, int ldu, const double* phi2, double* X,
                        int ldx, bool x_paired, int n, const StepScalars& sc, const FFTTables<double>& tab,
                        const GSTables64& gs, const double2* root2M, hipStream_t st, bool u_paired = false);
template <int M>
void launch_rows_gs(double* lines, int ld, int nlines, int n, const FFTTables<double>& tab, const GSTables64& gs,
                    hipStream_t st);
template <int M>
void launch_cols_gs(int mode, const double* X, int ldx, const double* ucur, const double* uprev, double* uout,
                    int ldu, int n, const FFTTables<double>& tab, const GSTables64& gs, hipStream_t st);
// y-line solves of X (paired rows), the update into prev_t's rows (transposed layout) and,
// with fwd, the next step's row transform of the new state into S.  u_paired: both state
// arrays in paired rows (launch_state_to_paired) instead of plain rows.
template <int M>
void launch_cols_gs_fwd(const double* X, int ldx, const double* ucur, double* prev_t, int n, double2* S, int lds_,
                        bool fwd, const FFTTables<double>& tab, const GSTables64& gs, const double2* root2M,
                        hipStream_t st, bool u_paired = false);
// N x N: A <- A^T; (cur, prev) <- (prev^T, cur); A <- I (dense row-major, pitch N)
void launch_transpose_inplace(double* A, int n, hipStream_t st);
// plain grid (pitch N) <-> paired rows (pitch N, room for N + 1 rows), optionally transposed
void launch_state_to_paired(const double* u, double* p, int n, bool trans, hipStream_t st);
void launch_state_from_paired(const double* p, double* u, int n, bool trans, hipStream_t st);
void launch_identity(double* A, int n, hipStream_t st);
void launch_swap_transposed(double* cur, double* prev, int n, hipStream_t st);
// batched forms (instances in blockIdx.y; iu / ip select u[0] or u[1]).  Row pass modes:
// 0 / 1 step / start-up with the x-sweep, 3 / 4 the same without it (X = B)
template <int M>
void launch_batch_rows_fwd(int lf, const BatchInst* bi, int count, int iu, int ip, int ldx, int lds_, int n,
                           const FFTTables<double>& tab, hipStream_t st);
template <int M>
void launch_batch_cols_conv(const BatchInst* bi, int count, int lds_, int n, int ldlam, const FFTTables<double>& tab,
                            hipStream_t st);
template <int M>
void launch_batch_rows_rhs(int mode, const BatchInst* bi, int count, int iu, int lds_, int ldx, int n,
                           const FFTTables<double>& tab, hipStream_t st);
template <int M>
void launch_batch_cols_gs(const BatchInst* bi, int count, int ldx, int n, const FFTTables<double>& tab,
                          hipStream_t st);
void launch_batch_leapfrog(int mode, const BatchInst* bi, int count, int ic, int ip, int ldx, int n, hipStream_t st);
// y-line solves of X (plain rows), update into u[ip] in the transposed layout and the next
// step's row transform into S, for every instance
template <int M>
void launch_batch_cols_gs_fwd(const BatchInst* bi, int count, int ic, int ip, int ldx, int lds_, int n,
                              const FFTTables<double>& tab, hipStream_t st);
// every instance: u[which] <- u[which]^T; (u[1], u[0]) <- (u[0]^T, u[1])
void launch_batch_transpose(const BatchInst* bi, int count, int which, int n, hipStream_t st);
void launch_batch_swap_transposed(const BatchInst* bi, int count, int n, hipStream_t st);

// set-up: eigenvalues of the block-circulant embedding of the N x N coefficients a2 (device,
// row-major, pitch N) into lam ((M+1) rows, pitch ldlam, even ky then odd ky per row kx,
// scaled 1/P^2).  work_real: (M+1) x ldg doubles (ldg >= N; may be lam itself); g0: M+1
// doubles; work_spec: M+2 rows of ldt complex (ldt >= M+1), rows in pairs.  None of them may
// overlap a2 except as stated.
template <int M>
void launch_bccb_eigenvalues(const double* a2, int n, double* work_real, int ldg, double* g0, double2* work_spec,
                             int ldt, double* lam, int ldlam, const FFTTables<double>& tab, hipStream_t st);

// adjoint of a step (per-row partial sums in partial[4 j + k], then one finishing block)
void launch_adjoint_dots(int mode, const double* a, const double* p, const double* q, int ldx, const double* uprev,
                         const double* ucur, const double* unext, int n, double* partial, hipStream_t st);
void launch_adjoint_combine(double ca, double c2, double kappa, int gkind, double gparam, const double* anext,
                            const double* anext2, const double* z, int ldx, const double* ucur, double* acur, int n,
                            double* partial, hipStream_t st);
void launch_adjoint_finish(const double* partial, int nrows, double c2, double kappa, double* dkappa,
                           hipStream_t st);

// mixed-precision x-sweep (modes 0 / 1 as launch_rows_rhs_gs).  u_paired (run steps, mode 0):
// the state in paired rows, and X written in paired rows for launch_cols_gs_fwd_mixed
template <int M>
void launch_rows_rhs_mixed(int mode, const double2* S, int lds_, const double* u, int ldu, const double* phi2,
                           double* X, int ldx, int n, const StepScalars& sc, const FFTTables<double>& tab,
                           const MixedTables& mx, const double2* root2M, hipStream_t st, bool u_paired = false);
template <int M>
void launch_rows_gs_mixed(double* lines, int ld, int nlines, int n, const FFTTables<double>& tab,
                          const MixedTables& mx, hipStream_t st);
template <int M>
void launch_cols_gs_mixed(int mode, const double* X, int ldx, const double* ucur, const double* uprev, double* uout,
                          int ldu, int n, const FFTTables<double>& tab, const MixedTables& mx, hipStream_t st);
// mixed-precision y-line solves of X, the update into prev_t's rows and, with fwd, the next
// step's row transform (as launch_cols_gs_fwd).  u_paired: X and both state arrays in paired
// rows; otherwise all in plain rows
template <int M>
void launch_cols_gs_fwd_mixed(const double* X, int ldx, const double* ucur, double* prev_t, int n, double2* S,
                              int lds_, bool fwd, const FFTTables<double>& tab, const MixedTables& mx,
                              const double2* root2M, hipStream_t st, bool u_paired = false);

}  // namespace sadi
