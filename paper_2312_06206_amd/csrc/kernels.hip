// Device kernels of the S-ADI time step (FP64 path).
//
// Grid layout: an N x N grid function u(x_i, y_j) is stored with x fastest,
// element (i, j) at u[j * ld + i] (row j = the x-line y = y_j).  M is the smallest power
// of two >= N + 1; P = 2M >= 2N - 1 is the size of the block-circulant embedding of the
// BTTB operator L_h (section "Fast implementation based on GS formula": L_h u by
// embedding in a block circulant with circulant blocks and 2D FFT).
//
// Kernels of one step (delta form H Uhat H = B of that section):
//   rows_fwd   : rFFT_P of every zero-padded x-line          u -> S (N x (M+1) complex)
//   cols_conv  : per x-frequency column, FFT_P over y, times the BCCB eigenvalues,
//                inverse FFT_P, first N rows kept             S -> S
//   rows_rhs_gs: inverse rFFT_P of every row -> (L_h u) h^alpha; B = sigma L u + gamma g(u)
//                (+ tau phi2 in the start-up step); x-line solve H^-1 B -> X
//   cols_gs    : y-line solve H^-1 on every column of X, then the leapfrog update
//                u^{n+1} = 2u^n - u^{n-1} + Uhat (start-up: u^1 = u^0 + Uhat)
// In a run, cols_gs_fwd replaces cols_gs and the next step's rows_fwd: the grid is
// transposed from one step to the next (x and y swap roles), so the column it solves is
// a row of the next step's grid.
// Line solves use the Gohberg-Semencul formula (Proposition 1 / Algorithm 1 of that
// section) on the bordered system of size M, whose first N unknowns follow from a
// rank-(M - N) correction (Schur complement of the bordered matrix).
#include <hip/hip_runtime.h>

#include "fft_core.hpp"
#include "kernels.hpp"

namespace sadi {

using V = double2;

// at least 4 waves per SIMD: <= 128 VGPRs, several workgroups per CU to overlap barriers
#define SADI_OCC4 __attribute__((amdgpu_waves_per_eu(4, 8)))
// mixed-precision kernels hold more per-line state: 2 waves per SIMD, <= 256 VGPRs
#define SADI_OCC2 __attribute__((amdgpu_waves_per_eu(2, 8)))

// ----------------------------------------------------------------------------------
// Paired row layout: rows y and y + 1 (y even) interleaved, element (y, k) at
// ((y >> 1) ld + k) 2 + (y & 1) for a row pitch of ld elements.  A column pass then fetches
// two rows of a column per memory request.  The half spectrum S always uses it; the y-sweep
// increment X of a single instance uses it too (XS = 1), while batched instances and the
// pitched buffers of the adjoint keep plain rows (XS = 0).  pair_row(y) is the offset of
// element (y, 0); the elements of a row then lie 2 apart.
__device__ __forceinline__ size_t pair_row(int y, int ld) { return (size_t)(y >> 1) * 2 * ld + (y & 1); }
template <int XS>
__device__ __forceinline__ size_t x_row(int y, int ld) { return XS ? pair_row(y, ld) : (size_t)y * ld; }

// Row kernels of one row per workgroup: blocks 16 q + j and 16 q + 8 + j (j < 8) take rows
// 2 (8 q + j) and 2 (8 q + j) + 1, and dispatch sends both to the same XCD, whose L2 then
// holds the whole lines of S that the pair shares.  The grid is a multiple of 16.
__device__ __forceinline__ int paired_row_block() {
  const int b = blockIdx.x;
  return (((b >> 4) << 3) | (b & 7)) * 2 + ((b >> 3) & 1);
}

// XCD-aware block order for column kernels: consecutive dispatch slots go to the 8
// XCDs round robin, so give the blocks of one XCD adjacent column groups (their row
// segments then share L2 lines).
__device__ __forceinline__ int xcd_group(int nblocks_used) {
  const int per = (nblocks_used + 7) / 8;
  const int b = blockIdx.x;
  return (b % 8) * per + b / 8;
}

// ----------------------------------------------------------------------------------
// Line access in canonical layout for lines of n < M values (stride `st` elements): slot m
// holds index k = t + T m; indices k >= n lie outside the line and read as zero.  Loads
// use the clamped index min(k, n-1), so every address stays inside the line.
// d[m] = (v[k], v[M-1-k]) with v[k] = 0 for k >= n: the Gohberg-Semencul input v + i J v.
template <int M, int E, int T>
__device__ __forceinline__ void load_line_pair(V* d, const double* __restrict__ v, int st, int t, int n) {
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int k = t + T * m, kr = (T - 1 - t) + T * (E - 1 - m);
    const double xf = (v + T * m * st)[(min(k, n - 1) - T * m) * st];
    const double xr = (v + T * (E - 1 - m) * st)[(min(kr, n - 1) - T * (E - 1 - m)) * st];
    d[m].x = k < n ? xf : 0.0;
    d[m].y = kr < n ? xr : 0.0;
  }
}

template <int M, int E, int T>
__device__ __forceinline__ void store_line(const V* d, double* __restrict__ v, int st, int t, int n) {
#pragma unroll
  for (int m = 0; m < E; ++m)
    if (t + T * m < n) (v + T * m * st)[t * st] = d[m].x;
}

// Same pairs for column `col` of an array with row pitch ld (paired rows when XS = 1): each
// element is loaded once, the reversed copy comes through LDS.  T m is even, so slot m's
// rows start at the uniform offset T m ld in both layouts.
template <int M, int E, int T, int XS, class L_t>
__device__ __forceinline__ void load_column_pair(const L_t& L, V* d, const double* __restrict__ X, int col, int ld,
                                                 void* lds, int n) {
  const int t = L.t;
  double a[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int k = t + T * m, kc = min(k, n - 1);
    const double x = (X + T * m * ld)[((kc - T * m) >> XS) * (ld << XS) + (col << XS) + (kc & XS)];
    a[m] = k < n ? x : 0.0;
  }
  double* buf = reinterpret_cast<double*>(lds);
#pragma unroll
  for (int m = 0; m < E; ++m) L.put_real(buf, t + T * m, a[m]);
  __syncthreads();
#pragma unroll
  for (int m = 0; m < E; ++m) d[m] = V{a[m], L.get_real(buf, (T - 1 - t) + T * (E - 1 - m))};
  __syncthreads();
}

// ----------------------------------------------------------------------------------
// Gohberg-Semencul solve on a line in canonical layout.  On entry slot m holds
// v1[k] = v[k] + i v[M-1-k], k = t + T m (v the bordered right-hand side, v[M-1] = 0).
// On exit slot m holds w[k] = (H_M^-1 [v;0])[k] minus the bordering correction,
// i.e. (H_N^-1 v)[k] for k < N.  lam_s carries the 1/(2 p_1) and both 1/M.
// d[m] *= tab[t + T m] (CONJ: times the conjugate), loads issued in groups of four so
// that at most four table values are live at once.
template <int E, int T, bool CONJ, typename VV>
__device__ __forceinline__ void pointwise(VV* d, const VV* __restrict__ tab, int t) {
  // groups of four, the next group's loads issued before the current group is used
  VV w[4], nx[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) w[j] = (tab + T * j)[t];
#pragma unroll
  for (int g = 0; g < E; g += 4) {
    if (g + 4 < E) {
#pragma unroll
      for (int j = 0; j < 4; ++j) nx[j] = (tab + T * (g + 4 + j))[t];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) d[g + j] = CONJ ? cmulc(d[g + j], w[j]) : cmul(d[g + j], w[j]);
    asm volatile("" ::: "memory");
#pragma unroll
    for (int j = 0; j < 4; ++j) w[j] = nx[j];
  }
}

// d[m] *= tab[t + T m] for a real table
template <int E, int T, typename VV, typename R>
__device__ __forceinline__ void pointwise_real(VV* d, const R* __restrict__ tab, int t) {
#pragma unroll
  for (int g = 0; g < E; g += 4) {
    R w[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) w[j] = (tab + T * (g + j))[t];
#pragma unroll
    for (int j = 0; j < 4; ++j) d[g + j] = cscale(d[g + j], w[j]);
    asm volatile("" ::: "memory");
  }
}

template <class LineT>
__device__ __forceinline__ void gs_solve(const LineT& L, V2<typename LineT::Real>* d, void* lds,
                                         const FFTTables<typename LineT::Real>& tab,
                                         const GSTables<typename LineT::Real>& gs, int n) {
  using R = typename LineT::Real;
  constexpr int M = LineT::M, E = LineT::E, T = LineT::T;
  const int t = L.t;
  // v2 = Q^H ifft(lam_s o fft(Q v1)); Q = diag(e^{-i pi k/M}) rides on the transform
  L.template transform<-1, -1>(d, lds, tab);
  pointwise<E, T, false>(d, gs.lam_s, t);
  L.template transform<+1>(d, lds, tab);
  // v3 = ifft(lam_c o fft(v2)), the Q^H of v2 again folded into the transform
  L.template transform<-1, +1>(d, lds, tab);
  pointwise<E, T, false>(d, gs.lam_c, t);
  L.template transform<+1>(d, lds, tab);
  // w = Re(v3) + J Im(v3); correction to H_N^-1: w[:N] - F w[N:M]
  R* buf = reinterpret_cast<R*>(lds);
  constexpr int SC = LineT::LINE_FAST_ ? LineT::LPW_ : 1;
  const int wb = L.lds_index(t), rb = L.lds_index(T - 1 - t);
#pragma unroll
  for (int m = 0; m < E; ++m) buf[wb + SC * T * m] = d[m].y;
  if (gs.r != 1) {
    // N < M - 1: w for every slot, then w[N..M-1] through LDS, then the rank-r correction.
    // r = 0: stop at w (all M slots); the caller corrects all lines at once.
    __syncthreads();
#pragma unroll
    for (int m = 0; m < E; ++m) d[m].x += buf[rb + SC * T * (E - 1 - m)];
    __syncthreads();
    if (gs.r == 0) return;
#pragma unroll
    for (int m = 0; m < E; ++m)
      if (t + T * m >= n) buf[wb + SC * T * m] = d[m].x;
    __syncthreads();
#pragma unroll 1
    for (int j = 0; j < gs.r; ++j) {
      const R wj = L.get_real(buf, n + j);
      const R* Fj = gs.f + (size_t)j * n;
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int k = t + T * m;
        const R fk = (Fj + T * m)[min(k, n - 1) - T * m];
        if (k < n) d[m].x -= fk * wj;
      }
    }
    __syncthreads();
    return;
  }
  if (t == T - 1) L.put_real(buf, M, d[E - 1].x);   // Re v3[M-1]
  __syncthreads();
  const R wN = L.get_real(buf, M) + L.get_real(buf, 0);
  // (J Im v3)[k] = Im v3[M-1-k], M-1-k = (T-1-t) + T (E-1-m)
#pragma unroll
  for (int g = 0; g < E; g += 4) {
    R f[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int m = g + j;
      f[j] = (gs.f + T * m)[m == E - 1 ? min(t, T - 2) : t];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int m = g + j;
      const R fm = (m == E - 1 && t == T - 1) ? R(0) : f[j];   // k = N: no correction
      d[m].x = d[m].x + buf[rb + SC * T * (E - 1 - m)] - fm * wN;
    }
    asm volatile("" ::: "memory");
  }
  __syncthreads();
}

// y[k] = (beta T(a) x)[k], k = t + T m, for a real line x (FP64): the 2M-point circulant
// embedding of beta T(a), whose eigenvalues s (real, even: s[k + M] = s[M - k]) are stored
// as even / odd frequencies scaled by 1/(2M).  The real input of length 2M (x, then zeros)
// is packed as z[j] = x[2j] + i x[2j+1], so one length-M transform each way suffices.
// With Z = fft(z), E = (Z[k] + conj Z[M-k]) / 2, O = (Z[k] - conj Z[M-k]) / (2i) and
// W = e^{-i pi/M}: X[k] = E + W^k O and X[k+M] = E - W^k O are the 2M-point spectrum,
// Y = s X, and Z'[k] = (Y[k] + Y[k+M]) / 2 + i W^-k (Y[k] - Y[k+M]) / 2 gives
// ifft(Z')[j] = M (y[2j] + i y[2j+1]); the factor 2 sig_(e|o) = s / M absorbs the M.
template <class LineT>
__device__ __forceinline__ void toeplitz_apply64(const LineT& L, const float* x, double* y, void* lds,
                                                 const FFTTables<double>& tab, const ToeplitzTables64& toe,
                                                 const double2* __restrict__ q) {
  constexpr int M = LineT::M, E = LineT::E, T = LineT::T;
  const int t = L.t;
  double* buf = reinterpret_cast<double*>(lds);
  V* zb = reinterpret_cast<V*>(lds);
  // pack: slot c < E/2 holds z[j], j = t + T c; the other slots are the zero half
#pragma unroll
  for (int m = 0; m < E; ++m) L.put_real(buf, t + T * m, (double)x[m]);
  __syncthreads();
  V d[E];
#pragma unroll
  for (int c = 0; c < E; ++c) {
    const int j = t + T * c;
    d[c] = c < E / 2 ? V{L.get_real(buf, 2 * j), L.get_real(buf, 2 * j + 1)} : V{0.0, 0.0};
  }
  __syncthreads();
  L.template transform<-1>(d, lds, tab);
  // s[k] / M for 0 <= k <= M
  auto sig = [&](int k) -> double { return 2.0 * ((k & 1) ? toe.sig_o[k >> 1] : toe.sig_e[k >> 1]); };
  // Z'[k] from Z[k] and Z[M-k]
  auto zprime = [&](int k, V zk, V zmk) -> V {
    const V zm = cconj(zmk);
    const V e = cscale(cadd(zk, zm), 0.5);
    const V io = cscale(csub(zk, zm), 0.5);   // i O
    const V o = V{io.y, -io.x};
    const V w = k < M ? q[k] : V{-1.0, 0.0};   // W^k
    const V wo = cmul(w, o);
    const V ya = cscale(cadd(e, wo), sig(k));       // Y[k]
    const V yb = cscale(csub(e, wo), sig(M - k));   // Y[k + M]
    const V ep = cscale(cadd(ya, yb), 0.5);
    const V op = cmulc(cscale(csub(ya, yb), 0.5), w);
    return V{ep.x - op.y, ep.y + op.x};
  };
  // pairs (k, M - k) through a half-length complex buffer: slots c >= E/2 hold k >= M/2.
  // The upper half publishes Z; each lower k (0 < k < M/2) forms Z'[k] and Z'[M - k] and
  // leaves the latter in its partner's place; k = 0 and k = M/2 pair with themselves.
#pragma unroll
  for (int c = E / 2; c < E; ++c) zb[L.cidx(t + T * c - M / 2)] = d[c];
  __syncthreads();
#pragma unroll
  for (int c = 0; c < E / 2; ++c) {
    const int k = t + T * c;
    if (k == 0) {
      d[c] = zprime(0, d[c], d[c]);
    } else {
      const int pm = L.cidx(M - k - M / 2);
      const V zmk = zb[pm];
      zb[pm] = zprime(M - k, zmk, d[c]);
      d[c] = zprime(k, d[c], zmk);
    }
  }
  __syncthreads();
#pragma unroll
  for (int c = E / 2; c < E; ++c) {
    const int k = t + T * c;
    d[c] = k == M / 2 ? zprime(k, d[c], d[c]) : zb[L.cidx(k - M / 2)];
  }
  __syncthreads();
  L.template transform<+1>(d, lds, tab);
  // unpack: y[2j] = Re, y[2j+1] = Im for j = t + T c < M/2, back to the canonical slots
#pragma unroll
  for (int c = 0; c < E / 2; ++c) {
    const int j = t + T * c;
    L.put_real(buf, 2 * j, d[c].x);
    L.put_real(buf, 2 * j + 1, d[c].y);
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < E; ++m) y[m] = L.get_real(buf, t + T * m);
  __syncthreads();
}

// Mixed-precision line solve.  On entry dv[m] = (v[k], v[M-1-k]) (FP64, v[N] = 0); on exit
// dv[m].x = x[k] with x = x0 + x1, x0 = GS32(v), x1 = GS32(v - H x0) (FP64 residual) when
// refining, else x = x0.  keep: this line's M doubles of LDS outside the exchange region,
// which hold v and then x0 across the solves instead of registers (each thread touches only
// its own entries k = t + T m, so no barrier is needed around them).
template <class Line64, class Line32>
__device__ __forceinline__ void mixed_solve(const Line64& L, const Line32& Lf, V* dv, void* lds, double* keep,
                                            const FFTTables<double>& tab, const MixedTables& mx) {
  constexpr int M = Line64::M, E = Line64::E, T = Line64::T;
  const int t = L.t;
  float2 df[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    df[m] = float2{(float)dv[m].x, (float)dv[m].y};
    if (mx.refine) (keep + T * m)[t] = dv[m].x;
  }
  gs_solve(Lf, df, lds, mx.tab32, mx.gs32, M - 1);
  if (!mx.refine) {
#pragma unroll
    for (int m = 0; m < E; ++m) dv[m].x = (double)df[m].x;
    return;
  }
  float x0[E];
  double r[E];
#pragma unroll
  for (int m = 0; m < E; ++m) x0[m] = df[m].x;
  if (t == T - 1) x0[E - 1] = 0.0f;   // slot k = N holds the bordering unknown, not x
  // r = v - x0 - beta T x0  (FP64, x0 is exactly representable), r[N] = 0; x0 then takes
  // v's place in LDS
  toeplitz_apply64(L, x0, r, lds, tab, mx.toe, mx.q64);
#pragma unroll
  for (int m = 0; m < E; ++m) {
    r[m] = (keep + T * m)[t] - (double)x0[m] - r[m];
    if (m == E - 1 && t == T - 1) r[m] = 0.0;
    (keep + T * m)[t] = (double)x0[m];
  }
  // reversed copy of r through LDS
  double* buf = reinterpret_cast<double*>(lds);
#pragma unroll
  for (int m = 0; m < E; ++m) L.put_real(buf, t + T * m, r[m]);
  __syncthreads();
#pragma unroll
  for (int m = 0; m < E; ++m)
    df[m] = float2{(float)r[m], (float)L.get_real(buf, (T - 1 - t) + T * (E - 1 - m))};
  __syncthreads();
  gs_solve(Lf, df, lds, mx.tab32, mx.gs32, M - 1);
#pragma unroll
  for (int m = 0; m < E; ++m) dv[m].x = (keep + T * m)[t] + (double)df[m].x;
  (void)M;
}

// Half spectrum of a real line of length P = 2M (zero beyond N) from its packed form:
// on entry slot c holds z[j] = x[2j] + i x[2j+1], j = t + T c.  One complex transform of
// length M, then X[k] = FE[k] + W_P^k FO[k] for k = 0..M, stored to out[2 k] (a row of the
// paired-row spectrum) when `live`.
template <class L_t>
__device__ __forceinline__ void real_transform_store(const L_t& L, V* d, void* smem, V* __restrict__ out, bool live,
                                                     const FFTTables<double>& tab, const V* __restrict__ root2M) {
  constexpr int M = L_t::M, E = L_t::E, T = L_t::T;
  L.template transform<-1>(d, smem, tab);
  // pair Z[k] with Z[M-k] through a half-length complex buffer in two rounds: slots
  // m < E/2 hold k < M/2, the others k >= M/2; k = 0 and k = M/2 are their own partners.
  V* zb = reinterpret_cast<V*>(smem);
  auto emit = [&](int k, V zk, V zmk) {
    const V zm = cconj(zmk);
    const V ev = cscale(cadd(zk, zm), 0.5);
    const V od = cscale(csub(zk, zm), 0.5);        // = i * FO[k]
    const V fo = V{od.y, -od.x};                   // X[k] = FE[k] + W_P^k FO[k]
    if (live) out[2 * k] = cadd(ev, cmul(fo, root2M[k]));
  };
#pragma unroll
  for (int round = 0; round < 2; ++round) {
#pragma unroll
    for (int c = 0; c < E; ++c) {
      const bool lower = c < E / 2;
      if (lower == (round == 0)) {
        const int k = L.t + T * c;
        zb[L.cidx(lower ? k : k - M / 2)] = d[c];
      }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < E; ++c) {
      const bool lower = c < E / 2;
      const int k = L.t + T * c;
      if (lower != (round == 0)) {
        if (k == 0) {
          emit(0, d[c], d[c]);
          if (live) out[2 * M] = V{d[c].x - d[c].y, 0.0};   // X[M] = Re Z0 - Im Z0
        } else if (k == M / 2) {
          emit(k, d[c], d[c]);
        } else {
          const int km = M - k;
          emit(k, d[c], zb[L.cidx(lower ? km - M / 2 : km)]);
        }
      }
    }
    __syncthreads();
  }
}

// ----------------------------------------------------------------------------------
// rows_fwd: S[y][k] = sum_{n<N} u[y][n] e^{-2 pi i k n / P}, k = 0..M.
// LF = 1 first completes the previous step's update: u = 2 u + (-uprev) + hat, with
// u = ucur, hat = the increment left in X by the y-sweep; the result overwrites uprev.
template <int M, int LF, int XS>
__device__ __forceinline__ void rows_fwd_body(const double* __restrict__ u, double* __restrict__ uprev, const double* __restrict__ hat, int ldx,
                int ldu, V* __restrict__ S, int lds_, int n, FFTTables<double> tab, const V* __restrict__ root2M,
                int nrows) {
  using L_t = typename RowFwdCfg<M>::Line;
  constexpr int E = L_t::E, T = L_t::T;
  __shared__ __align__(16) unsigned char smem[RowFwdCfg<M>::LDS_BYTES];
  const L_t L(threadIdx.x);
  const int y = blockIdx.x * RowFwdCfg<M>::LPW + L.line;
  const bool live = y < nrows;   // rows of n values each
  const int yy = live ? y : 0;
  const double* row = u + (size_t)yy * ldu;
  double* prow = LF ? uprev + (size_t)yy * ldu : nullptr;
  const double* hrow = LF ? hat + x_row<XS>(yy, ldx) : nullptr;
  const int t = L.t;
  V d[E];
  // z[j] = x[2j] + i x[2j+1], j = t + T c, x[i] = 0 for i >= N (N <= M - 1): slots c >= E/2
  // are zero; loads use the clamped index min(i, N-1)
#pragma unroll
  for (int c = 0; c < E; ++c) {
    if (c < E / 2) {
      const int i0 = 2 * (t + T * c), base = 2 * T * c;
      const bool ve = i0 < n, vo = i0 + 1 < n;
      const int ie = min(i0, n - 1) - base, io = min(i0 + 1, n - 1) - base;   // offsets from 2 T c
      double xe = (row + base)[ie];
      double xo = (row + base)[io];
      if constexpr (LF == 1) {
        xe = 2.0 * xe - (prow + base)[ie] + (hrow + (base << XS))[ie << XS];
        xo = 2.0 * xo - (prow + base)[io] + (hrow + (base << XS))[io << XS];
        if (live) {
          if (ve) (prow + base)[ie] = xe;
          if (vo) (prow + base)[io] = xo;
        }
      }
      d[c].x = ve ? xe : 0.0;
      d[c].y = vo ? xo : 0.0;
    } else {
      d[c] = V{0.0, 0.0};
    }
  }
  real_transform_store(L, d, smem, S + pair_row(live ? y : 0, lds_), live, tab, root2M);
}

// f(integral_constant<int, C>) for every slot C, in order
template <typename F, int... C>
__device__ __forceinline__ void for_slots(F f, std::integer_sequence<int, C...>) {
  (f(std::integral_constant<int, C>{}), ...);
}

// d[c] *= e^{-i pi c/E} where `odd` (per lane), else unchanged
template <int E, typename VV, int... C>
__device__ __forceinline__ void shift_odd_slots(VV* d, bool odd, std::integer_sequence<int, C...>) {
  ((d[C] = odd ? shift16<-1, C * (16 / E)>(d[C]) : d[C]), ...);
}
template <typename VV, int... C>
__device__ __forceinline__ void shift_odd_slots(VV* d, bool odd, std::integer_sequence<int, C...> seq) {
  shift_odd_slots<(int)sizeof...(C)>(d, odd, seq);
}

// ----------------------------------------------------------------------------------
// cols_conv: for every x-frequency column kx (0..M): c[y] = S[y][kx] (y < N, zero to P),
// out = IFFT_P(Lambda[kx] o FFT_P(c)), first N rows.  The length-P transform is split
// into its even and odd frequencies (two length-M transforms of c and W_P^y c), each
// handled by its own line of the workgroup (lines 2g / 2g+1 for column group g).
// grp: this workgroup's column group (< the number of groups); smem: ColConvCfg<M>::LDS_BYTES
// bytes of LDS.
template <int M>
__device__ __forceinline__ void cols_conv_body(V* __restrict__ S, int lds_, int n, const double* __restrict__ lam, int ldlam,
                 FFTTables<double> tab, const V* __restrict__ root2M, int grp, unsigned char* smem) {
  using Cfg = ColConvCfg<M>;
  using L_t = typename Cfg::Line;
  constexpr int E = L_t::E, T = L_t::T;
  constexpr int CPW = Cfg::LPW / 2;  // columns per workgroup
  const L_t L(threadIdx.x);
  const int col = grp * CPW + L.line / 2;
  const int odd = L.line & 1;
  const bool live = col <= M;   // M + 1 columns
  const int colc = live ? col : M;
  V d[E];
  const int t = L.t;
  // Addresses: uniform base (per slot) + one per-lane offset.
  // y = N (m = E-1, t = T-1) is the zero padding row; odd lines take W_P^y c[y]
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int y = t + T * m;   // rows y >= N are the zero padding (clamped, unused load)
    const int yc = min(y, n - 1);
    // S(yc, colc) from the uniform base of rows T m (T m is even)
    const V v = (S + T * m * lds_)[((yc - T * m) >> 1) * 2 * lds_ + 2 * colc + (yc & 1)];
    d[m] = y < n ? v : V{0.0, 0.0};
  }
  // odd lines: W_P^y = e^{-i pi y/M} on the input, y = t + T m: the per-slot part
  // e^{-i pi m/E} here, the per-thread part e^{-i pi t/M} on the first twiddle
  shift_odd_slots(d, odd, std::make_integer_sequence<int, E>{});
  const V s0 = root2M[t];
  L.template transform_scaled<-1>(d, smem, tab, odd ? s0 : V{1.0, 0.0});
  // eigenvalues of the embedding, row kx: [Lam_e(0..M/2), Lam_o(0..M/2-1)] (even in ky):
  //   k < M/2 : even Lam_e[k],       odd Lam_o[k]           -> k + odd (M/2 + 1)
  //   k >= M/2: even Lam_e[M-k],     odd Lam_o[M-1-k]       -> M - k + odd (M/2)
  const int lo = colc * ldlam + t + odd * (M / 2 + 1);
  const int hi = colc * ldlam - t + odd * (M / 2);
#pragma unroll
  for (int g = 0; g < E; g += 4) {
    double sv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int m = g + j;
      sv[j] = (m < E / 2) ? (lam + T * m)[lo] : (lam + (M - T * m))[hi];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) d[g + j] = cscale(d[g + j], sv[j]);
    asm volatile("" ::: "memory");
  }
  L.template transform<+1>(d, smem, tab);
  // combine: out[y] = even[y] + W_P^{-y} odd[y]; the two lines of a column share
  // their exchange space as one complex buffer (complex index y * CPW + column slot)
  V* xb = reinterpret_cast<V*>(smem);
  static_assert(Cfg::LINE_FAST, "column pairing assumes interleaved lines");
  const int xo = t * CPW + L.line / 2;
  if (odd) {
    // W_P^{-y}, y = t + T m: e^{i pi t/M} (conjugate of s0) times e^{i pi m/E}
#pragma unroll
    for (int m = 0; m < E; ++m) d[m] = cmulc(d[m], s0);
    shift_slots<+1, 16 / E>(d, std::make_integer_sequence<int, E>{});
#pragma unroll
    for (int m = 0; m < E; ++m) (xb + T * CPW * m)[xo] = d[m];
  }
  __syncthreads();
  if (!odd && live) {
    const int wo = (t >> 1) * 2 * lds_ + 2 * col + (t & 1);   // S(t + T m, col)
#pragma unroll
    for (int m = 0; m < E; ++m) {
      if (t + T * m < n) (S + T * m * lds_)[wo] = cadd(d[m], (xb + T * CPW * m)[xo]);
    }
  }
}

// ----------------------------------------------------------------------------------
// rows_rhs_gs: x[n] = inverse rFFT_P of S row (Lambda carries 1/(P M)); B = sigma x +
// gamma g(u) [+ tau phi2]; X = H^-1 B on the x-line.  MODE: 0 = step (n >= 1),
// 1 = start-up step (n = 0, adds tau phi2), 2 = L_h only (X = sigma x, no solve).
//
// rhs_phase: everything before the line solve.  Returns false for MODE 2 (output written);
// otherwise d[m] = (B[k], B[M-1-k]) with B[k] = 0 for k >= N.
// B[k] += gamma g(u[k]) (+ tau phi2[k] for the start-up step) for this thread's k < N, in
// place in LDS; returns whether some sine argument lies beyond the fast reduction's range
template <int MODE, int GK, int US, class L_t>
__device__ __forceinline__ bool add_pointwise(const L_t& L, double* buf, const double* __restrict__ urow,
                                              const double* __restrict__ prow, const StepScalars& sc, int n) {
  constexpr int E = L_t::E, T = L_t::T;
  const int t = L.t;
  bool far = false;
#pragma unroll
  for (int m = 0; m < E / 2; ++m) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (2 * (t + T * m) + h >= n) continue;   // B[k] = 0 outside the line
      const int lane_off = 2 * t + h;
      const double uv = (urow + ((2 * T * m) << US))[lane_off << US];
      double gv = 0.0;
      if constexpr (GK == 1) {
        // far arguments (and inf / NaN) contribute nothing here: the fast reduction is not
        // valid for them, and the library sine is added in a separate pass
        const bool f = !(fabs(uv) <= kSinFastMax);
        far |= f;
        gv = f ? 0.0 : -sin_fp64(uv);
      } else if constexpr (GK == 2) {
        gv = -uv * uv * uv;
      } else if constexpr (GK == 3) {
        gv = -sc.gparam * uv;
      }
      double b = sc.gamma * gv;
      if constexpr (MODE == 1) b += sc.tau * (prow + 2 * T * m)[lane_off];
      const int k = 2 * (t + T * m) + h;
      L.put_real(buf, k, L.get_real(buf, k) + b);
    }
    if (m % 2 == 1) asm volatile("" ::: "memory");   // bound the live sine temporaries
  }
  return far;
}

template <int MODE, int US, class L_t>
__device__ __forceinline__ bool rhs_phase(const L_t& L, V* d, void* smem, const V* __restrict__ srow,
                                          const double* __restrict__ urow, const double* __restrict__ prow,
                                          double* __restrict__ xo, bool live, const StepScalars& sc,
                                          const FFTTables<double>& tab, const V* __restrict__ root2M, int n) {
  constexpr int M = L_t::M, E = L_t::E, T = L_t::T;
  const int t = L.t;
  // c2r pre-processing: Z[k] = FE[k] + i FO[k], FE = (X[k] + conj X[M-k])/2,
  // FO = W_P^{-k} (X[k] - conj X[M-k])/2 ; the 1/2 is folded into Lambda.
  // X[M-k] with M-k = (M - T m) - t: uniform base minus the lane index (srow elements 2 apart)
  // W_P^{-k}, k = t + T m: e^{i pi t/M} (conjugate of root2M[t]) times e^{i pi m/E}
  const V s0 = root2M[t];
  for_slots([&](auto mc) {
    constexpr int m = decltype(mc)::value;
    const V xk = (srow + 2 * T * m)[2 * t];
    const V c = cconj((srow + 2 * (M - T * m))[-2 * t]);
    const V fe = cadd(xk, c);
    const V fo = shift16<+1, m * (16 / E)>(cmulc(csub(xk, c), s0));
    d[m] = V{fe.x - fo.y, fe.y + fo.x};
    if constexpr (m % 4 == 3) asm volatile("" ::: "memory");
  }, std::make_integer_sequence<int, E>{});
  L.template transform<+1>(d, smem, tab);
  // slot m holds z[j], j = t + T m: x[2j] = Re, x[2j+1] = Im; only j < M/2 (slots
  // m < E/2) carry x[i] with i < M, and x[i] with i >= N is outside the grid
  double* buf = reinterpret_cast<double*>(smem);
  if constexpr (MODE == 2) {
    if (live) {
#pragma unroll
      for (int m = 0; m < E / 2; ++m) {
        const int j = t + T * m;
        if (2 * j < n) xo[2 * j] = sc.sigma * d[m].x;
        if (2 * j + 1 < n) xo[2 * j + 1] = sc.sigma * d[m].y;
      }
    }
    return false;
  } else {
    // x[2j + h], j = t + T m: uniform base 2 T m, lane offset 2 t + h; B[k] = 0 for k >= N
    // first sigma x (frees the transform's registers), then the pointwise terms are added
    // in place: each thread only touches its own LDS entries, so no barrier in between
#pragma unroll
    for (int m = 0; m < E / 2; ++m) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int k = 2 * (t + T * m) + h;
        const double xv = h ? d[m].y : d[m].x;
        L.put_real(buf, k, k < n ? sc.sigma * xv : 0.0);
      }
    }
    // one loop per kind of g (the kind is uniform: no per-element branches)
    bool far = false;   // some sin argument beyond the fast reduction's range
    switch (sc.gkind) {
      case 1: far = add_pointwise<MODE, 1, US>(L, buf, urow, prow, sc, n); break;
      case 2: add_pointwise<MODE, 2, US>(L, buf, urow, prow, sc, n); break;
      case 3: add_pointwise<MODE, 3, US>(L, buf, urow, prow, sc, n); break;
      default: add_pointwise<MODE, 0, US>(L, buf, urow, prow, sc, n); break;
    }
    if (sc.gkind == 1 && far) {
      // rare: the library sine for the far arguments of this lane (their fast-sine term
      // was left out above)
#pragma unroll 1
      for (int i = 0; i < E; ++i) {
        const int m = i >> 1, h = i & 1;
        if (2 * (t + T * m) + h >= n) continue;
        const double uv = (urow + ((2 * T * m) << US))[(2 * t + h) << US];
        if (!(fabs(uv) <= kSinFastMax)) {
          const int k = 2 * (t + T * m) + h;
          L.put_real(buf, k, L.get_real(buf, k) - sc.gamma * sin(uv));
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < E; ++m)   // v[k], v[M-1-k] with M-1-k = (T-1-t) + T (E-1-m)
      d[m] = V{L.get_real(buf, t + T * m), L.get_real(buf, (T - 1 - t) + T * (E - 1 - m))};
    __syncthreads();
    return true;
  }
}

// rowblk: this workgroup's block of RowCfg<M>::LPW rows; smem: RowCfg<M>::LDS_BYTES bytes.
template <int M, int MODE, int XS, int US = 0>
__device__ __forceinline__ void rows_rhs_gs_body(const V* __restrict__ S, int lds_, const double* __restrict__ u, int ldu,
                   const double* __restrict__ phi2, double* __restrict__ X, int ldx, int n,
                   StepScalars sc, FFTTables<double> tab, GSTables64 gs, const V* __restrict__ root2M, int rowblk,
                   unsigned char* smem) {
  using L_t = typename RowCfg<M>::Line;
  constexpr int E = L_t::E, T = L_t::T;
  const L_t L(threadIdx.x);
  const int y = rowblk * RowCfg<M>::LPW + L.line;
  if (RowCfg<M>::LPW == 1 && y >= n) return;   // a whole workgroup past the last row
  const bool live = y < n;
  const int yy = live ? y : 0;
  // MODE 3 / 4: as 0 / 1 but X = B (no line solve; the dense-inverse path follows)
  constexpr int RMODE = MODE >= 3 ? MODE - 3 : MODE;
  static_assert(RMODE != 2 || XS == 0, "L_h output rows are plain");
  V d[E];
  static_assert(US == 0 || RMODE == 0, "paired state rows only in run steps");
  if (!rhs_phase<RMODE, US>(L, d, smem, S + pair_row(yy, lds_), u + (US ? pair_row(yy, ldu) : (size_t)yy * ldu),
                        RMODE == 1 ? phi2 + (size_t)yy * ldu : nullptr, X + (size_t)yy * ldx, live, sc, tab,
                        root2M, n))
    return;
  if constexpr (MODE < 3) gs_solve(L, d, smem, tab, gs, n);
  if (live) {
    // X rows have M >= N + 1 slots: the value at k = N lands in the row padding.  The lane
    // offset is recomputed from an opaque copy of the lane index (register pressure).
    double* xo = X + x_row<XS>(yy, ldx);
    int tt = L.t;
    asm volatile("" : "+v"(tt));
#pragma unroll
    for (int m = 0; m < E; ++m) (xo + ((T * m) << XS))[tt << XS] = d[m].x;
  }
}

// Mixed precision variant (MODE 0 / 1): FP32 solves, optional FP64 residual correction
template <int M, int MODE, int US>
__global__ void __launch_bounds__(MixRowCfg<M>::NT) SADI_OCC2
rows_rhs_mixed_kernel(const V* __restrict__ S, int lds_, const double* __restrict__ u, int ldu,
                      const double* __restrict__ phi2, double* __restrict__ X, int ldx, int n,
                      StepScalars sc, FFTTables<double> tab, MixedTables mx, const V* __restrict__ root2M) {
  using Cfg = MixRowCfg<M>;
  using L_t = typename Cfg::Line;
  using L32 = typename Cfg::Line32;
  constexpr int E = L_t::E, T = L_t::T;
  __shared__ __align__(16) unsigned char smem[Cfg::LDS_BYTES + Cfg::KEEP_BYTES];
  const L_t L(threadIdx.x);
  const L32 Lf(threadIdx.x);
  // at one row per workgroup the two rows of a pair go to one XCD at about the same time
  // (paired_row_block): they share the L2 lines of S they read and, in runs, of X they write
  const int blk = Cfg::LPW == 1 ? paired_row_block() : (int)blockIdx.x;
  const int y = blk * Cfg::LPW + L.line;
  const bool live = y < n;
  const int yy = live ? y : 0;
  // run steps (US): X in paired rows, as the run's y-sweep reads it
  double* xo = X + (US ? pair_row(yy, ldx) : (size_t)yy * ldx);
  V d[E];
  rhs_phase<MODE, US>(L, d, smem, S + pair_row(yy, lds_), u + (US ? pair_row(yy, ldu) : (size_t)yy * ldu),
                  MODE == 1 ? phi2 + (size_t)yy * ldu : nullptr, xo, live, sc, tab, root2M, n);
  mixed_solve(L, Lf, d, smem, Cfg::keep(smem, L.line), tab, mx);
  if (live) {
#pragma unroll
    for (int m = 0; m < E; ++m) (xo + ((T * m) << US))[L.t << US] = d[m].x;
  }
}

// ----------------------------------------------------------------------------------
// rows_gs: in-place H^-1 on nlines lines of length N (stride ld).
template <int M>
__global__ void __launch_bounds__(RowCfg<M>::NT) SADI_OCC4
rows_gs_kernel(double* __restrict__ lines, int ld, int nlines, int n, FFTTables<double> tab, GSTables64 gs) {
  using L_t = typename RowCfg<M>::Line;
  constexpr int E = L_t::E, T = L_t::T;
  __shared__ __align__(16) unsigned char smem[RowCfg<M>::LDS_BYTES];
  const L_t L(threadIdx.x);
  const int y = blockIdx.x * RowCfg<M>::LPW + L.line;
  const bool live = y < nlines;
  double* row = lines + (size_t)(live ? y : 0) * ld;
  V d[E];
  load_line_pair<M, E, T>(d, row, 1, L.t, n);
  gs_solve(L, d, smem, tab, gs, n);
  if (live) store_line<M, E, T>(d, row, 1, L.t, n);
}

// ----------------------------------------------------------------------------------
// cols_gs: y-line solves on the columns of X and the leapfrog update.
// MODE 0: uout = 2 ucur - uprev + Uhat (uout may alias uprev); MODE 1: uout = ucur + Uhat.
template <int M, int MODE, int XS>
__device__ __forceinline__ void cols_gs_body(double* X, int ldx, const double* ucur, const double* uprev,
               double* uout, int ldu, int n, FFTTables<double> tab, GSTables64 gs, int ngroups) {
  using Cfg = ColGSCfg<M>;
  using L_t = typename Cfg::Line;
  constexpr int E = L_t::E, T = L_t::T;
  __shared__ __align__(16) unsigned char smem[Cfg::LDS_BYTES];
  const int grp = xcd_group(ngroups);
  if (grp >= ngroups) return;
  const L_t L(threadIdx.x);
  const int col = grp * Cfg::LPW + L.line;
  const bool live = col < n;
  const int cc = live ? col : 0;
  const int t = L.t;
  V d[E];
  load_column_pair<M, E, T, XS>(L, d, X, cc, ldx, smem, n);
  gs_solve(L, d, smem, tab, gs, n);
  if (!live) return;
  // row offsets below come from an opaque copy of the lane index, so they are not kept
  // live across the solve from the column load (register pressure)
  int tt = t;
  asm volatile("" : "+v"(tt));
  const int o = tt * ldu + col;
  if constexpr (MODE == 2) {
    // the increment stays in X (the next row pass applies the update)
    // with the correction deferred (r = 0) the bordered rows N..M-1 are kept as well
    const int ox = (tt >> XS) * (ldx << XS) + (col << XS) + (tt & XS);
    const int nst = gs.r == 0 ? M : n;
#pragma unroll
    for (int m = 0; m < E; ++m)
      if (tt + T * m < nst) (X + T * m * ldx)[ox] = d[m].x;
  } else {
    // rows k = t + T m >= N: clamped loads, no store
    double uc[E], up[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int oc = (min(tt + T * m, n - 1) - T * m) * ldu + col;
      uc[m] = (ucur + T * m * ldu)[oc];
      if constexpr (MODE == 0) up[m] = (uprev + T * m * ldu)[oc];
    }
#pragma unroll
    for (int m = 0; m < E; ++m) {
      if (tt + T * m < n) {
        if constexpr (MODE == 0) (uout + T * m * ldu)[o] = 2.0 * uc[m] - up[m] + d[m].x;
        else (uout + T * m * ldu)[o] = uc[m] + d[m].x;
      }
    }
  }
}

// ----------------------------------------------------------------------------------
// cols_gs_fwd: one kernel for the end of a step and the start of the next, with the grid
// transposed from one step to the next.  The scheme is symmetric in x and y (square grid,
// one line matrix H, Lambda symmetric in (kx, ky), g pointwise), so a step on the
// transposed state gives the transposed result.  For column c of this step's grid:
//   Uhat = y-line solve of column c of X (paired rows),
//   u^{n+1}[k][c] = 2 u^n[k][c] - u^{n-1}[k][c] + Uhat[k],
// with ucur = u^n in this step's layout (column c read with stride N) and prev_t =
// u^{n-1} in the transposed layout (its row c is column c here, contiguous).  The new
// column is stored as row c of prev_t: u^{n+1} in the transposed layout, the layout of the
// next step.  With `fwd` the same column is then transformed along its length, which is
// the next step's row transform: its half spectrum goes to row c of S.  XS: X in paired
// rows (single instances) or plain rows (batch members).
// The end of a run's step for column cc of this step's grid, after its y-line solve: slot m
// of d holds Uhat[k] in .x, k = t + T m.  u^{n+1}[k][cc] = 2 u^n[k][cc] - u^{n-1}[k][cc] + Uhat[k]
// with ucur = u^n in this step's layout (column cc read with stride N) and prev_t = u^{n-1}
// in the transposed layout (its row cc is column cc here, contiguous); the new column is
// stored as row cc of prev_t.  With `fwd` it is then transformed along its length (the next
// step's row transform): its half spectrum goes to row cc of S.
template <int US, class L_t>
__device__ __forceinline__ void update_transposed_and_forward(const L_t& L, V* d, unsigned char* smem,
                                                              const double* __restrict__ ucur,
                                                              double* __restrict__ prev_t, int n, int cc, bool live,
                                                              V* __restrict__ S, int lds_, const FFTTables<double>& tab,
                                                              const V* __restrict__ root2M, int fwd) {
  constexpr int E = L_t::E, T = L_t::T;
  const int t = L.t;
  // an opaque copy of the lane index: the row indices below are recomputed rather than
  // kept live across the solve from the column load (register pressure)
  int tt = t;
  asm volatile("" : "+v"(tt));
  // k = t + T m; rows k >= N are outside the grid (clamped loads, zero values).  Each new
  // value goes straight to memory and, for the transform, to LDS (the solve has finished
  // its LDS reads).
  // US: both state arrays in paired rows (pitch N): element (y, x) at pair_row(y, N) + 2 x;
  // T m is even, so slot m's rows start at the uniform offset T m N in either layout
  const double* uc = ucur + (cc << US);
  double* up = prev_t + (US ? pair_row(cc, n) : (size_t)cc * n);
  double* buf = reinterpret_cast<double*>(smem);
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int k = tt + T * m, kc = min(k, n - 1);
    // uniform base of slot m plus a 32-bit lane offset (negative only for clamped rows)
    const int ro = kc - T * m;
    const double a = (uc + (size_t)T * m * n)[US ? (ro >> 1) * 2 * n + (kc & 1) : ro * n];
    const double b = (up + ((T * m) << US))[US ? 2 * ro : ro];   // ro < 0 for clamped rows
    const double v = k < n ? 2.0 * a - b + d[m].x : 0.0;
    if (live && k < n) (up + ((T * m) << US))[tt << US] = v;
    if (fwd) L.put_real(buf, k, v);
  }
  if (!fwd) return;   // uniform
  // z[j] = x[2j] + i x[2j+1], j = t + T c (c < E/2; the other slots are zero)
  __syncthreads();
#pragma unroll
  for (int c = 0; c < E; ++c) {
    if (c < E / 2) {
      const int j = t + T * c;
      d[c] = V{L.get_real(buf, 2 * j), L.get_real(buf, 2 * j + 1)};
    } else {
      d[c] = V{0.0, 0.0};
    }
  }
  __syncthreads();
  real_transform_store(L, d, smem, S + pair_row(cc, lds_), live, tab, root2M);
}

// grp: this workgroup's group of ColGSCfg<M>::LPW columns; smem: ColGSCfg<M>::LDS_BYTES bytes.
template <int M, int XS, int US = 0>
__device__ __forceinline__ void cols_gs_fwd_body(const double* __restrict__ X, int ldx, const double* __restrict__ ucur,
                                                 double* __restrict__ prev_t, int n, V* __restrict__ S, int lds_,
                                                 FFTTables<double> tab, GSTables64 gs, const V* __restrict__ root2M,
                                                 int grp, int fwd, unsigned char* smem) {
  using Cfg = ColGSCfg<M>;
  using L_t = typename Cfg::Line;
  constexpr int E = L_t::E, T = L_t::T;
  const L_t L(threadIdx.x);
  const int col = grp * Cfg::LPW + L.line;
  const bool live = col < n;
  const int cc = live ? col : 0;
  V d[E];
  load_column_pair<M, E, T, XS>(L, d, X, cc, ldx, smem, n);
  gs_solve(L, d, smem, tab, gs, n);
  update_transposed_and_forward<US>(L, d, smem, ucur, prev_t, n, cc, live, S, lds_, tab, root2M, fwd);
}

// Mixed-precision form of cols_gs_fwd: the y-line solve of column cc of X (paired rows with US,
// as the run's x-sweep writes it; plain rows otherwise) in float32 with one float64 residual
// correction (or none), then the same update and next row transform.
template <int M, int US>
__global__ void __launch_bounds__(MixColCfg<M>::NT) SADI_OCC2
cols_gs_fwd_mixed_kernel(const double* __restrict__ X, int ldx, const double* __restrict__ ucur,
                         double* __restrict__ prev_t, int n, V* __restrict__ S, int lds_, FFTTables<double> tab,
                         MixedTables mx, const V* __restrict__ root2M, int ngroups, int fwd) {
  using Cfg = MixColCfg<M>;
  using L_t = typename Cfg::Line;
  constexpr int E = L_t::E, T = L_t::T;
  __shared__ __align__(16) unsigned char smem[Cfg::LDS_BYTES + Cfg::KEEP_BYTES];
  const int grp = xcd_group(ngroups);
  if (grp >= ngroups) return;   // whole workgroup
  const L_t L(threadIdx.x);
  const typename Cfg::Line32 Lf(threadIdx.x);
  const int col = grp * Cfg::LPW + L.line;
  const bool live = col < n;
  const int cc = live ? col : 0;
  V d[E];
  load_column_pair<M, E, T, US>(L, d, X, cc, ldx, smem, n);
  mixed_solve(L, Lf, d, smem, Cfg::keep(smem, L.line), tab, mx);
  update_transposed_and_forward<US>(L, d, smem, ucur, prev_t, n, cc, live, S, lds_, tab, root2M, fwd);
}

// ----------------------------------------------------------------------------------
// Square N x N transposes in 32 x 32 tiles; block (I, J) with I <= J handles the tile pair
// {(I, J), (J, I)} (blocks with I > J exit).  transpose_inplace: A <- A^T.  swap_transposed:
// (cur, prev) <- (prev^T, cur).
__device__ __forceinline__ void transpose_inplace_tiles(double* A, int n) {
  const int I = blockIdx.y, J = blockIdx.x;
  if (I > J) return;
  __shared__ double ta[32][33], tb[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = ty + 8 * q;
    const int ra = I * 32 + r, ca = J * 32 + tx;   // tile (I, J)
    const int rb = J * 32 + r, cb = I * 32 + tx;   // tile (J, I)
    ta[r][tx] = (ra < n && ca < n) ? A[(size_t)ra * n + ca] : 0.0;
    tb[r][tx] = (rb < n && cb < n) ? A[(size_t)rb * n + cb] : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = ty + 8 * q;
    const int ra = I * 32 + r, ca = J * 32 + tx;   // (I, J) <- (J, I)^T
    const int rb = J * 32 + r, cb = I * 32 + tx;   // (J, I) <- (I, J)^T
    if (ra < n && ca < n) A[(size_t)ra * n + ca] = tb[tx][r];
    if (I != J && rb < n && cb < n) A[(size_t)rb * n + cb] = ta[tx][r];
  }
}

__device__ __forceinline__ void swap_transposed_tiles(double* cur, double* prev, int n) {
  const int I = blockIdx.y, J = blockIdx.x;
  if (I > J) return;
  __shared__ double ta[32][33], tb[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  double ca_v[4], cb_v[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = ty + 8 * q;
    const int ra = I * 32 + r, ca = J * 32 + tx;
    const int rb = J * 32 + r, cb = I * 32 + tx;
    const bool ia = ra < n && ca < n, ib = rb < n && cb < n;
    ta[r][tx] = ia ? prev[(size_t)ra * n + ca] : 0.0;
    tb[r][tx] = ib ? prev[(size_t)rb * n + cb] : 0.0;
    ca_v[q] = ia ? cur[(size_t)ra * n + ca] : 0.0;
    cb_v[q] = ib ? cur[(size_t)rb * n + cb] : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = ty + 8 * q;
    const int ra = I * 32 + r, ca = J * 32 + tx;
    const int rb = J * 32 + r, cb = I * 32 + tx;
    if (ra < n && ca < n) {
      cur[(size_t)ra * n + ca] = tb[tx][r];
      prev[(size_t)ra * n + ca] = ca_v[q];
    }
    if (I != J && rb < n && cb < n) {
      cur[(size_t)rb * n + cb] = ta[tx][r];
      prev[(size_t)rb * n + cb] = cb_v[q];
    }
  }
}

__global__ void __launch_bounds__(256) transpose_inplace_kernel(double* A, int n) { transpose_inplace_tiles(A, n); }
__global__ void __launch_bounds__(256) identity_kernel(double* A, int n) {
  const size_t nn = (size_t)n * n;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < nn; i += (size_t)gridDim.x * 256)
    A[i] = (i % (size_t)(n + 1)) == 0 ? 1.0 : 0.0;
}
__global__ void __launch_bounds__(256) swap_transposed_kernel(double* cur, double* prev, int n) {
  swap_transposed_tiles(cur, prev, n);
}

// Plain N x N grid u (pitch N) <-> paired rows p (pitch N, N + 1 rows of room): element (y, x)
// of p at pair_row(y, N) + 2 x.  trans: p holds the transpose of u.  32 x 32 tiles through
// LDS, so that both sides are read and written along rows (for p, along both rows of a pair).
template <bool TO_P>
__global__ void __launch_bounds__(256) paired_state_kernel(const double* __restrict__ src, double* __restrict__ dst,
                                                           int n, int trans) {
  __shared__ double tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  const int y0 = blockIdx.y * 32, x0 = blockIdx.x * 32;
  // read: element (y0 + r, x0 + tx) of the source grid in its own layout
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int r = ty + 8 * j, y = y0 + r, x = x0 + tx;
    if (y < n && x < n) tile[r][tx] = TO_P ? src[(size_t)y * n + x] : src[pair_row(y, n) + 2 * (size_t)x];
  }
  __syncthreads();
  // write: without trans the same element; with trans element (x0 + r, y0 + c) takes (c, r)
  // of the tile.  For p the lanes run over (row parity, column) so that each wave writes the
  // two rows of a pair together.
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    int r, c;
    if (TO_P) {               // lanes: c = (lane / 2), parity = lane % 2
      const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;   // 4 waves
      const int q = w + 4 * j;                                     // pair index in the tile, 0..15
      r = 2 * q + (lane & 1);
      c = lane >> 1;
    } else {
      r = ty + 8 * j;
      c = tx;
    }
    const int yd = (trans ? x0 : y0) + r, xd = (trans ? y0 : x0) + c;   // destination (row, column)
    if (yd < n && xd < n) {
      const double v = trans ? tile[c][r] : tile[r][c];
      if (TO_P) dst[pair_row(yd, n) + 2 * (size_t)xd] = v;
      else dst[(size_t)yd * n + xd] = v;
    }
  }
}
// batched (instance blockIdx.z): u[which] <- u[which]^T; (u[1], u[0]) <- (u[0]^T, u[1])
__global__ void __launch_bounds__(256) transpose_inplace_batched(const BatchInst* __restrict__ bi, int which, int n) {
  transpose_inplace_tiles(bi[blockIdx.z].u[which], n);
}
__global__ void __launch_bounds__(256) swap_transposed_batched(const BatchInst* __restrict__ bi, int n) {
  swap_transposed_tiles(bi[blockIdx.z].u[1], bi[blockIdx.z].u[0], n);
}

// ----------------------------------------------------------------------------------
// mixed-precision in-place line solves and y-sweep
template <int M>
__global__ void __launch_bounds__(MixRowCfg<M>::NT) SADI_OCC2
rows_gs_mixed_kernel(double* __restrict__ lines, int ld, int nlines, int n, FFTTables<double> tab, MixedTables mx) {
  using Cfg = MixRowCfg<M>;
  using L_t = typename Cfg::Line;
  constexpr int E = L_t::E, T = L_t::T;
  __shared__ __align__(16) unsigned char smem[Cfg::LDS_BYTES + Cfg::KEEP_BYTES];
  const L_t L(threadIdx.x);
  const typename Cfg::Line32 Lf(threadIdx.x);
  const int y = blockIdx.x * Cfg::LPW + L.line;
  const bool live = y < nlines;
  double* row = lines + (size_t)(live ? y : 0) * ld;
  V d[E];
  load_line_pair<M, E, T>(d, row, 1, L.t, M - 1);
  mixed_solve(L, Lf, d, smem, Cfg::keep(smem, L.line), tab, mx);
  if (live) store_line<M, E, T>(d, row, 1, L.t, M - 1);
}

template <int M, int MODE>
__global__ void __launch_bounds__(MixColCfg<M>::NT) SADI_OCC2
cols_gs_mixed_kernel(const double* __restrict__ X, int ldx, const double* ucur, const double* uprev,
                     double* uout, int ldu, int n, FFTTables<double> tab, MixedTables mx, int ngroups) {
  using Cfg = MixColCfg<M>;
  using L_t = typename Cfg::Line;
  constexpr int E = L_t::E, T = L_t::T;
  __shared__ __align__(16) unsigned char smem[Cfg::LDS_BYTES + Cfg::KEEP_BYTES];
  const int grp = xcd_group(ngroups);
  if (grp >= ngroups) return;
  const L_t L(threadIdx.x);
  const typename Cfg::Line32 Lf(threadIdx.x);
  const int col = grp * Cfg::LPW + L.line;
  const bool live = col < n;
  const int cc = live ? col : 0;
  V d[E];
  load_line_pair<M, E, T>(d, X + cc, ldx, L.t, M - 1);
  mixed_solve(L, Lf, d, smem, Cfg::keep(smem, L.line), tab, mx);
  if (live) {
    const int o = L.t * ldu + col;
    const int oe = min(L.t, T - 2) * ldu + col;
#pragma unroll
    for (int m = 0; m < E; ++m) {
      if (m < E - 1 || L.t < T - 1) {
        const double uc = (ucur + T * m * ldu)[m == E - 1 ? oe : o];
        if constexpr (MODE == 0) (uout + T * m * ldu)[o] = 2.0 * uc - (uprev + T * m * ldu)[o] + d[m].x;
        else (uout + T * m * ldu)[o] = uc + d[m].x;
      }
    }
  }
}


// ----------------------------------------------------------------------------------
// kernels: one instance (pointer arguments) and batched (instance blockIdx.y of an
// array of BatchInst sharing N, pitches and line tables; iu / ip pick the state buffers)
template <int M, int LF, int XS>
__global__ void __launch_bounds__(RowFwdCfg<M>::NT) SADI_OCC4
rows_fwd_kernel(const double* __restrict__ u, double* __restrict__ uprev, const double* __restrict__ hat, int ldx,
                int ldu, V* __restrict__ S, int lds_, int n, FFTTables<double> tab, const V* __restrict__ root2M) {
  rows_fwd_body<M, LF, XS>(u, uprev, hat, ldx, ldu, S, lds_, n, tab, root2M, n);
}
template <int M, int LF>
__global__ void __launch_bounds__(RowFwdCfg<M>::NT) SADI_OCC4
rows_fwd_batched(const BatchInst* __restrict__ bi, int iu, int ip, int ldx, int lds_, int n, FFTTables<double> tab) {
  const BatchInst& p = bi[blockIdx.y];
  rows_fwd_body<M, LF, 0>(p.u[iu], p.u[ip], p.X, ldx, n, p.S, lds_, n, tab, tab.root2M, n);
}

template <int M>
__global__ void __launch_bounds__(ColConvCfg<M>::NT) SADI_OCC4
cols_conv_kernel(V* __restrict__ S, int lds_, int n, const double* __restrict__ lam, int ldlam,
                 FFTTables<double> tab, const V* __restrict__ root2M, int ngroups) {
  __shared__ __align__(16) unsigned char smem[ColConvCfg<M>::LDS_BYTES];
  const int grp = xcd_group(ngroups);
  if (grp >= ngroups) return;
  cols_conv_body<M>(S, lds_, n, lam, ldlam, tab, root2M, grp, smem);
}
template <int M>
__global__ void __launch_bounds__(ColConvCfg<M>::NT) SADI_OCC4
cols_conv_batched(const BatchInst* __restrict__ bi, int lds_, int n, int ldlam, FFTTables<double> tab, int ngroups) {
  __shared__ __align__(16) unsigned char smem[ColConvCfg<M>::LDS_BYTES];
  const int grp = xcd_group(ngroups);
  if (grp >= ngroups) return;
  const BatchInst& p = bi[blockIdx.y];
  cols_conv_body<M>(p.S, lds_, n, p.lam2d, ldlam, tab, tab.root2M, grp, smem);
}

// blocks of rows_rhs_gs with one row per block are launched in paired order (multiple of 16)
template <int M>
__device__ __forceinline__ int rhs_row_block() {
  return RowCfg<M>::LPW == 1 ? paired_row_block() : (int)blockIdx.x;
}

template <int M, int MODE, int XS, int US>
__global__ void __launch_bounds__(RowCfg<M>::NT) SADI_OCC4
rows_rhs_gs_kernel(const V* __restrict__ S, int lds_, const double* __restrict__ u, int ldu,
                   const double* __restrict__ phi2, double* __restrict__ X, int ldx, int n,
                   StepScalars sc, FFTTables<double> tab, GSTables64 gs, const V* __restrict__ root2M) {
  __shared__ __align__(16) unsigned char smem[RowCfg<M>::LDS_BYTES];
  rows_rhs_gs_body<M, MODE, XS, US>(S, lds_, u, ldu, phi2, X, ldx, n, sc, tab, gs, root2M, rhs_row_block<M>(), smem);
}
template <int M, int MODE>
__global__ void __launch_bounds__(RowCfg<M>::NT) SADI_OCC4
rows_rhs_gs_batched(const BatchInst* __restrict__ bi, int iu, int lds_, int ldx, int n, FFTTables<double> tab) {
  __shared__ __align__(16) unsigned char smem[RowCfg<M>::LDS_BYTES];
  const BatchInst& p = bi[blockIdx.y];
  const GSTables64 gs{tab.root2M, p.lam_s, p.lam_c, p.f, p.r};
  rows_rhs_gs_body<M, MODE, MODE == 0 ? 1 : 0>(p.S, lds_, p.u[iu], n, p.phi2, p.X, ldx, n, p.sc, tab, gs, tab.root2M,
                               rhs_row_block<M>(), smem);
}

template <int M, int MODE, int XS>
__global__ void __launch_bounds__(ColGSCfg<M>::NT) SADI_OCC4
cols_gs_kernel(double* X, int ldx, const double* ucur, const double* uprev,
               double* uout, int ldu, int n, FFTTables<double> tab, GSTables64 gs, int ngroups) {
  cols_gs_body<M, MODE, XS>(X, ldx, ucur, uprev, uout, ldu, n, tab, gs, ngroups);
}
template <int M>
__global__ void __launch_bounds__(ColGSCfg<M>::NT) SADI_OCC4
cols_gs_batched(const BatchInst* __restrict__ bi, int ldx, int n, FFTTables<double> tab, int ngroups) {
  const BatchInst& p = bi[blockIdx.y];
  const GSTables64 gs{tab.root2M, p.lam_s, p.lam_c, p.f, p.r};
  cols_gs_body<M, 2, 0>(p.X, ldx, nullptr, nullptr, nullptr, n, n, tab, gs, ngroups);
}

template <int M, int US>
__global__ void __launch_bounds__(ColGSCfg<M>::NT) SADI_OCC4
cols_gs_fwd_kernel(const double* __restrict__ X, int ldx, const double* __restrict__ ucur, double* __restrict__ prev_t,
                   int n, V* __restrict__ S, int lds_, FFTTables<double> tab, GSTables64 gs,
                   const V* __restrict__ root2M, int ngroups, int fwd) {
  __shared__ __align__(16) unsigned char smem[ColGSCfg<M>::LDS_BYTES];
  const int grp = xcd_group(ngroups);
  if (grp >= ngroups) return;   // whole workgroup
  cols_gs_fwd_body<M, 1, US>(X, ldx, ucur, prev_t, n, S, lds_, tab, gs, root2M, grp, fwd, smem);
}
// batched: instance blockIdx.y; u[ic] = u^n in this step's layout, u[ip] = u^{n-1} transposed
template <int M>
__global__ void __launch_bounds__(ColGSCfg<M>::NT) SADI_OCC4
cols_gs_fwd_batched(const BatchInst* __restrict__ bi, int ic, int ip, int ldx, int lds_, int n,
                    FFTTables<double> tab, int ngroups) {
  __shared__ __align__(16) unsigned char smem[ColGSCfg<M>::LDS_BYTES];
  const int grp = xcd_group(ngroups);
  if (grp >= ngroups) return;   // whole workgroup
  const BatchInst& p = bi[blockIdx.y];
  const GSTables64 gs{tab.root2M, p.lam_s, p.lam_c, p.f, p.r};
  cols_gs_fwd_body<M, 1>(p.X, ldx, p.u[ic], p.u[ip], n, p.S, lds_, tab, gs, tab.root2M, grp, 1, smem);
}

// ----------------------------------------------------------------------------------
// Work lists: one launch per phase of the batched step for all instances with M <= 2048,
// whatever their sizes.  Each workgroup takes (instance, block) from items[blockIdx.x] and
// runs the single-instance body of that instance's M (a uniform branch); the launch uses the
// largest LDS footprint of the bodies.  The host orders the list for the XCDs.
#define SADI_WL_CASES(F) F(16) F(32) F(64) F(128) F(256) F(512) F(1024) F(2048)

constexpr int cmax() { return 0; }
template <typename... A> constexpr int cmax(int a, A... b) {
  const int r = cmax(b...);
  return a > r ? a : r;
}
#define SADI_WL_LDS(C, MM) , C<MM>::LDS_BYTES
#define SADI_WL_CONV_LDS(MM) SADI_WL_LDS(ColConvCfg, MM)
#define SADI_WL_ROW_LDS(MM) SADI_WL_LDS(RowCfg, MM)
#define SADI_WL_GS_LDS(MM) SADI_WL_LDS(ColGSCfg, MM)
constexpr int kWlConvLds = cmax(0 SADI_WL_CASES(SADI_WL_CONV_LDS));
constexpr int kWlRowLds = cmax(0 SADI_WL_CASES(SADI_WL_ROW_LDS));
constexpr int kWlGsLds = cmax(0 SADI_WL_CASES(SADI_WL_GS_LDS));
constexpr int kWlConvNT = 256, kWlRowNT = 128, kWlGsNT = 256;
#define SADI_WL_CHECK(MM)                                                                   \
  static_assert(ColConvCfg<MM>::NT == kWlConvNT && RowCfg<MM>::NT == kWlRowNT &&            \
                    ColGSCfg<MM>::NT == kWlGsNT,                                            \
                "work-list phases need one workgroup size for every M");
SADI_WL_CASES(SADI_WL_CHECK)

__global__ void __launch_bounds__(kWlConvNT) SADI_OCC4
cols_conv_worklist(const BatchInst* __restrict__ bi, const WorkItem* __restrict__ items) {
  __shared__ __align__(16) unsigned char smem[kWlConvLds];
  const WorkItem w = items[blockIdx.x];
  if (w.inst < 0) return;
  const BatchInst& p = bi[w.inst];
  switch (p.m) {
#define SADI_WL_CONV(MM)                                                                          \
  case MM:                                                                                        \
    cols_conv_body<MM>(p.S, p.lds, p.n, p.lam2d, p.ldlam, p.tab, p.tab.root2M, w.blk, smem);    \
    break;
    SADI_WL_CASES(SADI_WL_CONV)
#undef SADI_WL_CONV
    default: break;
  }
}

__global__ void __launch_bounds__(kWlRowNT) SADI_OCC4
rows_rhs_gs_worklist(const BatchInst* __restrict__ bi, const WorkItem* __restrict__ items, int iu) {
  __shared__ __align__(16) unsigned char smem[kWlRowLds];
  const WorkItem w = items[blockIdx.x];
  if (w.inst < 0) return;
  const BatchInst& p = bi[w.inst];
  const GSTables64 gs{p.tab.root2M, p.lam_s, p.lam_c, p.f, p.r};
  switch (p.m) {
#define SADI_WL_ROW(MM)                                                                              \
  case MM:                                                                                           \
    rows_rhs_gs_body<MM, 0, 1>(p.S, p.lds, p.u[iu], p.n, p.phi2, p.X, p.ldx, p.n, p.sc, p.tab, gs,   \
                               p.tab.root2M, w.blk, smem);                                           \
    break;
    SADI_WL_CASES(SADI_WL_ROW)
#undef SADI_WL_ROW
    default: break;
  }
}

__global__ void __launch_bounds__(kWlGsNT) SADI_OCC4
cols_gs_fwd_worklist(const BatchInst* __restrict__ bi, const WorkItem* __restrict__ items, int ic, int ip) {
  __shared__ __align__(16) unsigned char smem[kWlGsLds];
  const WorkItem w = items[blockIdx.x];
  if (w.inst < 0) return;
  const BatchInst& p = bi[w.inst];
  const GSTables64 gs{p.tab.root2M, p.lam_s, p.lam_c, p.f, p.r};
  switch (p.m) {
#define SADI_WL_GS(MM)                                                                              \
  case MM:                                                                                          \
    cols_gs_fwd_body<MM, 1>(p.X, p.ldx, p.u[ic], p.u[ip], p.n, p.S, p.lds, p.tab, gs, p.tab.root2M, \
                            w.blk, 1, smem);                                                        \
    break;
    SADI_WL_CASES(SADI_WL_GS)
#undef SADI_WL_GS
    default: break;
  }
}

void worklist_shape(int m, int n, int blocks[3], double cost[3]) {
  blocks[0] = blocks[1] = blocks[2] = 0;
  cost[0] = cost[1] = cost[2] = 0.0;
  switch (m) {
#define SADI_WL_SHAPE(MM)                                                                     \
  case MM: {                                                                                  \
    constexpr int cpw = ColConvCfg<MM>::LPW / 2;                                              \
    const double ml = (double)MM * __builtin_ctz(MM);                                         \
    blocks[0] = (MM + 1 + cpw - 1) / cpw;                                                     \
    blocks[1] = (n + RowCfg<MM>::LPW - 1) / RowCfg<MM>::LPW;                                  \
    blocks[2] = (n + ColGSCfg<MM>::LPW - 1) / ColGSCfg<MM>::LPW;                              \
    cost[0] = ColConvCfg<MM>::LPW * ml;                                                       \
    cost[1] = RowCfg<MM>::LPW * ml;                                                           \
    cost[2] = ColGSCfg<MM>::LPW * ml;                                                         \
    break;                                                                                    \
  }
    SADI_WL_CASES(SADI_WL_SHAPE)
#undef SADI_WL_SHAPE
    default: break;
  }
}

void launch_worklist(int phase, const BatchInst* bi, const WorkItem* items, int nitems, int iu, int ip,
                     hipStream_t st) {
  if (nitems <= 0) return;
  if (phase == 0)
    hipLaunchKernelGGL(cols_conv_worklist, dim3(nitems), dim3(kWlConvNT), 0, st, bi, items);
  else if (phase == 1)
    hipLaunchKernelGGL(rows_rhs_gs_worklist, dim3(nitems), dim3(kWlRowNT), 0, st, bi, items, iu);
  else
    hipLaunchKernelGGL(cols_gs_fwd_worklist, dim3(nitems), dim3(kWlGsNT), 0, st, bi, items, iu, ip);
}

// batched update, instance blockIdx.z, row blockIdx.y:
//   mode 0: u[ip] = 2 u[ic] - u[ip] + X       (newest in the former previous buffer)
//   mode 1: u[ip] = u[ic] + X                 (start-up step)
//   mode 2: u[ic], u[ip] = 2 u[ic] - u[ip] + X, u[ic]   (newest in the current buffer)
__global__ void __launch_bounds__(256)
leapfrog_batched(const BatchInst* __restrict__ bi, int mode, int ic, int ip, int ldx, int n) {
  const BatchInst& p = bi[blockIdx.z];
  const int i = blockIdx.x * 256 + threadIdx.x, j = blockIdx.y;
  if (i >= n) return;
  const size_t o = (size_t)j * n + i;
  double* uc = p.u[ic];
  double* up = p.u[ip];
  const double h = p.X[(size_t)j * ldx + i];
  const double c = uc[o];
  if (mode == 1) {
    up[o] = c + h;
  } else {
    const double v = 2.0 * c - up[o] + h;
    if (mode == 0) {
      up[o] = v;
    } else {
      up[o] = c;
      uc[o] = v;
    }
  }
}


// ----------------------------------------------------------------------------------
// adjoint of a step: inner products and the combination (one workgroup per grid row,
// partial sums per row reduced in a fixed order, so results are deterministic)
template <int NV>
__device__ __forceinline__ void block_sums(double (&v)[NV], double* out) {
  __shared__ double red[NV][256];
#pragma unroll
  for (int k = 0; k < NV; ++k) red[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
#pragma unroll
      for (int k = 0; k < NV; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) out[k] = red[k][0];
  }
}

// row j: sums of a Uhat, p Uhat, q Uhat with Uhat = unext - 2 ucur + uprev (mode 0) or
// unext - ucur (mode 1); a, ucur, unext, uprev pitch n, p and q pitch ldx
__global__ void __launch_bounds__(256)
adjoint_dots_kernel(int mode, const double* __restrict__ a, const double* __restrict__ p, const double* __restrict__ q,
                    int ldx, const double* __restrict__ uprev, const double* __restrict__ ucur,
                    const double* __restrict__ unext, int n, double* __restrict__ partial) {
  const int j = blockIdx.x;
  double v[3] = {0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < n; i += 256) {
    const size_t o = (size_t)j * n + i, ox = (size_t)j * ldx + i;
    const double uh = mode == 0 ? unext[o] - 2.0 * ucur[o] + uprev[o] : unext[o] - ucur[o];
    v[0] += a[o] * uh;
    v[1] += p[ox] * uh;
    v[2] += q[ox] * uh;
  }
  block_sums<3>(v, partial + 4 * (size_t)j);
}

// acur = ca anext - anext2 + c2 (-kappa Lz + g'(ucur) z), with Lz read from acur (same
// element, read before write); partial[4 j + 3] = sum over row j of Lz ucur
__global__ void __launch_bounds__(256)
adjoint_combine_kernel(double ca, double c2, double kappa, int gkind, double gparam,
                       const double* __restrict__ anext, const double* __restrict__ anext2,
                       const double* __restrict__ z, int ldx, const double* __restrict__ ucur, double* acur, int n,
                       double* __restrict__ partial) {
  const int j = blockIdx.x;
  double v[1] = {0.0};
  for (int i = threadIdx.x; i < n; i += 256) {
    const size_t o = (size_t)j * n + i;
    const double lz = acur[o], zz = z[(size_t)j * ldx + i], u = ucur[o];
    double gp;
    switch (gkind) {
      case 1: gp = -cos(u); break;
      case 2: gp = -3.0 * u * u; break;
      case 3: gp = -gparam; break;
      default: gp = 0.0; break;
    }
    v[0] += lz * u;
    const double prev2 = anext2 ? anext2[o] : 0.0;
    acur[o] = ca * anext[o] - prev2 + c2 * (gp * zz - kappa * lz);
  }
  block_sums<1>(v, partial + 4 * (size_t)j + 3);
}

// dkappa += -c2 sum(Lz u) - (2 sum(a Uhat) - sum(p Uhat) - sum(q Uhat)) / kappa
__global__ void __launch_bounds__(256)
adjoint_finish_kernel(const double* __restrict__ partial, int nrows, double c2, double kappa,
                      double* __restrict__ dkappa) {
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int r = threadIdx.x; r < nrows; r += 256) {
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] += partial[4 * (size_t)r + k];
  }
  __shared__ double tot[4];
  block_sums<4>(v, tot);
  __syncthreads();
  if (threadIdx.x == 0) dkappa[0] += -c2 * tot[3] - (2.0 * tot[0] - tot[1] - tot[2]) / kappa;
}

void launch_adjoint_dots(int mode, const double* a, const double* p, const double* q, int ldx, const double* uprev,
                         const double* ucur, const double* unext, int n, double* partial, hipStream_t st) {
  hipLaunchKernelGGL(adjoint_dots_kernel, dim3(n), dim3(256), 0, st, mode, a, p, q, ldx, uprev, ucur, unext, n,
                     partial);
}

void launch_adjoint_combine(double ca, double c2, double kappa, int gkind, double gparam, const double* anext,
                            const double* anext2, const double* z, int ldx, const double* ucur, double* acur, int n,
                            double* partial, hipStream_t st) {
  hipLaunchKernelGGL(adjoint_combine_kernel, dim3(n), dim3(256), 0, st, ca, c2, kappa, gkind, gparam, anext, anext2,
                     z, ldx, ucur, acur, n, partial);
}

void launch_adjoint_finish(const double* partial, int nrows, double c2, double kappa, double* dkappa,
                           hipStream_t st) {
  hipLaunchKernelGGL(adjoint_finish_kernel, dim3(1), dim3(256), 0, st, partial, nrows, c2, kappa, dkappa);
}


// ----------------------------------------------------------------------------------
// Eigenvalues of the block-circulant embedding (set-up).  The embedding of a_ij is even in
// both directions, so each 1D transform of it is 2 Re(transform of the zero-padded half) -
// (the value at 0): first over j for every row i, then over i.
template <int M>
__global__ void __launch_bounds__(RowFwdCfg<M>::NT) SADI_OCC4
rows_fwd_rect_kernel(const double* __restrict__ u, int ldu, V* __restrict__ S, int lds_, int nrows, int nlen,
                     FFTTables<double> tab) {
  rows_fwd_body<M, 0, 0>(u, nullptr, nullptr, 0, ldu, S, lds_, nlen, tab, tab.root2M, nrows);
}

// G(i, k) = 2 Re S[i][k] - a_i0 for i < n, k <= M, stored transposed: GT[k][i]; its first
// column also in g0[k] = G(0, k)
__global__ void __launch_bounds__(256)
bccb_pass1_kernel(const V* __restrict__ S, int lds_, const double* __restrict__ a2, int n, int m,
                  double* __restrict__ GT, int ldg, double* __restrict__ g0) {
  const int k = blockIdx.x * 256 + threadIdx.x, i = blockIdx.y;
  if (k > m) return;
  const double v = 2.0 * S[pair_row(i, lds_) + 2 * k].x - a2[i];
  GT[(size_t)k * ldg + i] = v;
  if (i == 0) g0[k] = v;
}

// Lambda(kx, ky) = (2 Re T[ky][kx] - G(0, ky)) * scale, row kx of lam: even ky at ky/2, odd
// ky at M/2 + 1 + (ky - 1)/2
__global__ void __launch_bounds__(256)
bccb_pass2_kernel(const V* __restrict__ Tsp, int ldt, const double* __restrict__ g0, int m, double* __restrict__ lam,
                  int ldlam, double scale) {
  const int kx = blockIdx.x * 256 + threadIdx.x, ky = blockIdx.y;
  if (kx > m) return;
  const int pos = (ky % 2 == 0) ? ky / 2 : m / 2 + 1 + (ky - 1) / 2;
  lam[(size_t)kx * ldlam + pos] = (2.0 * Tsp[pair_row(ky, ldt) + 2 * kx].x - g0[ky]) * scale;
}

template <int M>
void launch_bccb_eigenvalues(const double* a2, int n, double* work_real, int ldg, double* g0, V* work_spec, int ldt,
                             double* lam, int ldlam, const FFTTables<double>& tab, hipStream_t st) {
  // pass 1: transforms of the rows of a2 (n rows of n) into work_spec (n rows, pitch ldt)
  hipLaunchKernelGGL(rows_fwd_rect_kernel<M>, dim3((n + RowFwdCfg<M>::LPW - 1) / RowFwdCfg<M>::LPW),
                     dim3(RowFwdCfg<M>::NT), 0, st, a2, n, work_spec, ldt, n, n, tab);
  hipLaunchKernelGGL(bccb_pass1_kernel, dim3((M + 1 + 255) / 256, n), dim3(256), 0, st, work_spec, ldt, a2, n, M,
                     work_real, ldg, g0);
  // pass 2: transforms of the M + 1 rows of G^T (n values each)
  hipLaunchKernelGGL(rows_fwd_rect_kernel<M>, dim3((M + 1 + RowFwdCfg<M>::LPW - 1) / RowFwdCfg<M>::LPW),
                     dim3(RowFwdCfg<M>::NT), 0, st, work_real, ldg, work_spec, ldt, M + 1, n, tab);
  const double p = 2.0 * M;
  hipLaunchKernelGGL(bccb_pass2_kernel, dim3((M + 1 + 255) / 256, M + 1), dim3(256), 0, st, work_spec, ldt, g0, M,
                     lam, ldlam, 1.0 / (p * p));
}

// ----------------------------------------------------------------------------------
// host-side launchers
template <int M>
void launch_rows_fwd(const double* u, double* uprev, const double* hat, int ldx, int ldu, V* S, int lds_, int n,
                     const FFTTables<double>& tab, const V* root2M, hipStream_t st) {
  const int grid = (n + RowFwdCfg<M>::LPW - 1) / RowFwdCfg<M>::LPW;
  const dim3 blk(RowFwdCfg<M>::NT);
  if (hat == nullptr)
    hipLaunchKernelGGL((rows_fwd_kernel<M, 0, 0>), dim3(grid), blk, 0, st, u, uprev, hat, ldx, ldu, S, lds_, n, tab,
                       root2M);
  else   // the deferred update reads X in plain rows
    hipLaunchKernelGGL((rows_fwd_kernel<M, 1, 0>), dim3(grid), blk, 0, st, u, uprev, hat, ldx, ldu, S, lds_, n, tab,
                       root2M);
}

// out = 2 ucur - uprev + hat (mode 0, out may alias uprev), out = ucur + hat (mode 1), or
// (ucur, uprev) <- (2 ucur - uprev + hat, ucur) (mode 2)
__global__ void __launch_bounds__(256)
leapfrog_kernel(int mode, double* ucur, double* uprev, const double* __restrict__ hat, int ldx, double* out,
                int n) {
  const int i = blockIdx.x * 256 + threadIdx.x, j = blockIdx.y;
  if (i >= n) return;
  const size_t o = (size_t)j * n + i;
  const double h = hat[(size_t)j * ldx + i];   // X in plain rows
  const double c = ucur[o];
  if (mode == 2) {           // newest into ucur, the current state into uprev
    const double v = 2.0 * c - uprev[o] + h;
    uprev[o] = c;
    ucur[o] = v;
  } else {
    out[o] = mode == 0 ? 2.0 * c - uprev[o] + h : c + h;
  }
}

void launch_leapfrog(int mode, double* ucur, double* uprev, const double* hat, int ldx, double* out, int n,
                     hipStream_t st) {
  hipLaunchKernelGGL(leapfrog_kernel, dim3((n + 255) / 256, n), dim3(256), 0, st, mode, ucur, uprev, hat, ldx, out, n);
}

template <int M>
void launch_cols_conv(V* S, int lds_, int n, const double* lam, int ldlam, const FFTTables<double>& tab,
                      const V* root2M, hipStream_t st) {
  constexpr int CPW = ColConvCfg<M>::LPW / 2;
  const int ngroups = (M + 1 + CPW - 1) / CPW;
  const int grid = ((ngroups + 7) / 8) * 8;
  hipLaunchKernelGGL(cols_conv_kernel<M>, dim3(grid), dim3(ColConvCfg<M>::NT), 0, st, S, lds_, n, lam, ldlam,
                     tab, root2M, ngroups);
}

// blocks of rows_rhs_gs: one row per block is launched in paired order (multiple of 16)
template <int M>
int rhs_grid(int n) {
  const int g = (n + RowCfg<M>::LPW - 1) / RowCfg<M>::LPW;
  return RowCfg<M>::LPW == 1 ? (g + 15) / 16 * 16 : g;
}

template <int M>
void launch_rows_rhs_gs(int mode, const V* S, int lds_, const double* u, int ldu, const double* phi2, double* X,
                        int ldx, bool x_paired, int n, const StepScalars& sc, const FFTTables<double>& tab,
                        const GSTables64& gs, const V* root2M, hipStream_t st, bool u_paired) {
  const int grid = rhs_grid<M>(n);
  const dim3 blk(RowCfg<M>::NT);
  // mode 2 (L_h only) writes plain rows; the state in paired rows only in run steps (mode 0)
  if (mode == 0 && x_paired && u_paired)
    hipLaunchKernelGGL((rows_rhs_gs_kernel<M, 0, 1, 1>), dim3(grid), blk, 0, st, S, lds_, u, ldu, phi2, X, ldx, n,
                       sc, tab, gs, root2M);
  else if (mode == 0 && x_paired)
    hipLaunchKernelGGL((rows_rhs_gs_kernel<M, 0, 1, 0>), dim3(grid), blk, 0, st, S, lds_, u, ldu, phi2, X, ldx, n, sc,
                       tab, gs, root2M);
  else if (mode == 0)
    hipLaunchKernelGGL((rows_rhs_gs_kernel<M, 0, 0, 0>), dim3(grid), blk, 0, st, S, lds_, u, ldu, phi2, X, ldx, n, sc,
                       tab, gs, root2M);
  else if (mode == 1 && x_paired)
    hipLaunchKernelGGL((rows_rhs_gs_kernel<M, 1, 1, 0>), dim3(grid), blk, 0, st, S, lds_, u, ldu, phi2, X, ldx, n, sc,
                       tab, gs, root2M);
  else if (mode == 1)
    hipLaunchKernelGGL((rows_rhs_gs_kernel<M, 1, 0, 0>), dim3(grid), blk, 0, st, S, lds_, u, ldu, phi2, X, ldx, n, sc,
                       tab, gs, root2M);
  else
    hipLaunchKernelGGL((rows_rhs_gs_kernel<M, 2, 0, 0>), dim3(grid), blk, 0, st, S, lds_, u, ldu, phi2, X, ldx, n, sc,
                       tab, gs, root2M);
}

template <int M>
void launch_rows_gs(double* lines, int ld, int nlines, int n, const FFTTables<double>& tab, const GSTables64& gs,
                    hipStream_t st) {
  const int grid = (nlines + RowCfg<M>::LPW - 1) / RowCfg<M>::LPW;
  hipLaunchKernelGGL(rows_gs_kernel<M>, dim3(grid), dim3(RowCfg<M>::NT), 0, st, lines, ld, nlines, n, tab, gs);
}

template <int M>
void launch_cols_gs(int mode, const double* X, int ldx, const double* ucur, const double* uprev, double* uout,
                    int ldu, int n, const FFTTables<double>& tab, const GSTables64& gs, hipStream_t st) {
  const int ngroups = (n + ColGSCfg<M>::LPW - 1) / ColGSCfg<M>::LPW;
  const int grid = ((ngroups + 7) / 8) * 8;
  double* Xw = const_cast<double*>(X);
  // modes 0 and 1 read a single step's X in paired rows; mode 2 works in place on plain
  // rows (the four-kernel run of GEMM-corrected contexts, the adjoint's buffers)
  if (mode == 0)
    hipLaunchKernelGGL((cols_gs_kernel<M, 0, 1>), dim3(grid), dim3(ColGSCfg<M>::NT), 0, st, Xw, ldx, ucur, uprev,
                       uout, ldu, n, tab, gs, ngroups);
  else if (mode == 1)
    hipLaunchKernelGGL((cols_gs_kernel<M, 1, 1>), dim3(grid), dim3(ColGSCfg<M>::NT), 0, st, Xw, ldx, ucur, uprev,
                       uout, ldu, n, tab, gs, ngroups);
  else
    hipLaunchKernelGGL((cols_gs_kernel<M, 2, 0>), dim3(grid), dim3(ColGSCfg<M>::NT), 0, st, Xw, ldx, ucur, uprev,
                       uout, ldu, n, tab, gs, ngroups);
}

template <int M>
void launch_rows_rhs_mixed(int mode, const V* S, int lds_, const double* u, int ldu, const double* phi2, double* X,
                           int ldx, int n, const StepScalars& sc, const FFTTables<double>& tab, const MixedTables& mx,
                           const V* root2M, hipStream_t st, bool u_paired) {
  const int grid = (n + MixRowCfg<M>::LPW - 1) / MixRowCfg<M>::LPW;
  // paired_row_block numbers blocks in groups of 16
  const int grid_p = MixRowCfg<M>::LPW == 1 ? (grid + 15) / 16 * 16 : grid;
  if (mode == 0 && u_paired)
    hipLaunchKernelGGL((rows_rhs_mixed_kernel<M, 0, 1>), dim3(grid_p), dim3(MixRowCfg<M>::NT), 0, st, S, lds_, u, ldu,
                       phi2, X, ldx, n, sc, tab, mx, root2M);
  else if (mode == 0)
    hipLaunchKernelGGL((rows_rhs_mixed_kernel<M, 0, 0>), dim3(grid_p), dim3(MixRowCfg<M>::NT), 0, st, S, lds_, u, ldu,
                       phi2, X, ldx, n, sc, tab, mx, root2M);
  else
    hipLaunchKernelGGL((rows_rhs_mixed_kernel<M, 1, 0>), dim3(grid_p), dim3(MixRowCfg<M>::NT), 0, st, S, lds_, u, ldu,
                       phi2, X, ldx, n, sc, tab, mx, root2M);
}

template <int M>
void launch_rows_gs_mixed(double* lines, int ld, int nlines, int n, const FFTTables<double>& tab,
                          const MixedTables& mx, hipStream_t st) {
  const int grid = (nlines + MixRowCfg<M>::LPW - 1) / MixRowCfg<M>::LPW;
  hipLaunchKernelGGL(rows_gs_mixed_kernel<M>, dim3(grid), dim3(MixRowCfg<M>::NT), 0, st, lines, ld, nlines, n, tab,
                     mx);
}

template <int M>
void launch_cols_gs_fwd(const double* X, int ldx, const double* ucur, double* prev_t, int n, V* S, int lds_, bool fwd,
                        const FFTTables<double>& tab, const GSTables64& gs, const V* root2M, hipStream_t st,
                        bool u_paired) {
  const int ngroups = (n + ColGSCfg<M>::LPW - 1) / ColGSCfg<M>::LPW;
  const int grid = ((ngroups + 7) / 8) * 8;
  if (u_paired)
    hipLaunchKernelGGL((cols_gs_fwd_kernel<M, 1>), dim3(grid), dim3(ColGSCfg<M>::NT), 0, st, X, ldx, ucur, prev_t, n,
                       S, lds_, tab, gs, root2M, ngroups, fwd ? 1 : 0);
  else
    hipLaunchKernelGGL((cols_gs_fwd_kernel<M, 0>), dim3(grid), dim3(ColGSCfg<M>::NT), 0, st, X, ldx, ucur, prev_t, n,
                       S, lds_, tab, gs, root2M, ngroups, fwd ? 1 : 0);
}

void launch_identity(double* A, int n, hipStream_t st) {
  const size_t nn = (size_t)n * n;
  const size_t blocks = (nn + 255) / 256;
  const int grid = blocks > 4096 ? 4096 : (int)blocks;
  if (grid > 0) hipLaunchKernelGGL(identity_kernel, dim3(grid), dim3(256), 0, st, A, n);
}

void launch_transpose_inplace(double* A, int n, hipStream_t st) {
  const int nt = (n + 31) / 32;
  hipLaunchKernelGGL(transpose_inplace_kernel, dim3(nt, nt), dim3(256), 0, st, A, n);
}

void launch_state_to_paired(const double* u, double* p, int n, bool trans, hipStream_t st) {
  const int nt = (n + 31) / 32;
  hipLaunchKernelGGL(paired_state_kernel<true>, dim3(nt, nt), dim3(256), 0, st, u, p, n, trans ? 1 : 0);
}

void launch_state_from_paired(const double* p, double* u, int n, bool trans, hipStream_t st) {
  const int nt = (n + 31) / 32;
  hipLaunchKernelGGL(paired_state_kernel<false>, dim3(nt, nt), dim3(256), 0, st, p, u, n, trans ? 1 : 0);
}

void launch_swap_transposed(double* cur, double* prev, int n, hipStream_t st) {
  const int nt = (n + 31) / 32;
  hipLaunchKernelGGL(swap_transposed_kernel, dim3(nt, nt), dim3(256), 0, st, cur, prev, n);
}

template <int M>
void launch_cols_gs_fwd_mixed(const double* X, int ldx, const double* ucur, double* prev_t, int n, V* S, int lds_,
                              bool fwd, const FFTTables<double>& tab, const MixedTables& mx, const V* root2M,
                              hipStream_t st, bool u_paired) {
  const int ngroups = (n + MixColCfg<M>::LPW - 1) / MixColCfg<M>::LPW;
  const int grid = ((ngroups + 7) / 8) * 8;
  if (u_paired)
    hipLaunchKernelGGL((cols_gs_fwd_mixed_kernel<M, 1>), dim3(grid), dim3(MixColCfg<M>::NT), 0, st, X, ldx, ucur,
                       prev_t, n, S, lds_, tab, mx, root2M, ngroups, fwd ? 1 : 0);
  else
    hipLaunchKernelGGL((cols_gs_fwd_mixed_kernel<M, 0>), dim3(grid), dim3(MixColCfg<M>::NT), 0, st, X, ldx, ucur,
                       prev_t, n, S, lds_, tab, mx, root2M, ngroups, fwd ? 1 : 0);
}

template <int M>
void launch_cols_gs_mixed(int mode, const double* X, int ldx, const double* ucur, const double* uprev, double* uout,
                          int ldu, int n, const FFTTables<double>& tab, const MixedTables& mx, hipStream_t st) {
  const int ngroups = (n + MixColCfg<M>::LPW - 1) / MixColCfg<M>::LPW;
  const int grid = ((ngroups + 7) / 8) * 8;
  if (mode == 0)
    hipLaunchKernelGGL((cols_gs_mixed_kernel<M, 0>), dim3(grid), dim3(MixColCfg<M>::NT), 0, st, X, ldx, ucur, uprev,
                       uout, ldu, n, tab, mx, ngroups);
  else
    hipLaunchKernelGGL((cols_gs_mixed_kernel<M, 1>), dim3(grid), dim3(MixColCfg<M>::NT), 0, st, X, ldx, ucur, uprev,
                       uout, ldu, n, tab, mx, ngroups);
}


// ---- batched launchers
template <int M>
void launch_batch_rows_fwd(int lf, const BatchInst* bi, int count, int iu, int ip, int ldx, int lds_, int n,
                           const FFTTables<double>& tab, hipStream_t st) {
  const dim3 grid((n + RowFwdCfg<M>::LPW - 1) / RowFwdCfg<M>::LPW, count);
  const dim3 blk(RowFwdCfg<M>::NT);
  if (lf)
    hipLaunchKernelGGL((rows_fwd_batched<M, 1>), grid, blk, 0, st, bi, iu, ip, ldx, lds_, n, tab);
  else
    hipLaunchKernelGGL((rows_fwd_batched<M, 0>), grid, blk, 0, st, bi, iu, ip, ldx, lds_, n, tab);
}

template <int M>
void launch_batch_cols_conv(const BatchInst* bi, int count, int lds_, int n, int ldlam, const FFTTables<double>& tab,
                            hipStream_t st) {
  constexpr int CPW = ColConvCfg<M>::LPW / 2;
  const int ngroups = (M + 1 + CPW - 1) / CPW;
  const dim3 grid(((ngroups + 7) / 8) * 8, count);
  hipLaunchKernelGGL(cols_conv_batched<M>, grid, dim3(ColConvCfg<M>::NT), 0, st, bi, lds_, n, ldlam, tab, ngroups);
}

template <int M>
void launch_batch_rows_rhs(int mode, const BatchInst* bi, int count, int iu, int lds_, int ldx, int n,
                           const FFTTables<double>& tab, hipStream_t st) {
  const dim3 grid(rhs_grid<M>(n), count);
  const dim3 blk(RowCfg<M>::NT);
  switch (mode) {
    case 0: hipLaunchKernelGGL((rows_rhs_gs_batched<M, 0>), grid, blk, 0, st, bi, iu, lds_, ldx, n, tab); break;
    case 1: hipLaunchKernelGGL((rows_rhs_gs_batched<M, 1>), grid, blk, 0, st, bi, iu, lds_, ldx, n, tab); break;
    case 3: hipLaunchKernelGGL((rows_rhs_gs_batched<M, 3>), grid, blk, 0, st, bi, iu, lds_, ldx, n, tab); break;
    default: hipLaunchKernelGGL((rows_rhs_gs_batched<M, 4>), grid, blk, 0, st, bi, iu, lds_, ldx, n, tab); break;
  }
}

template <int M>
void launch_batch_cols_gs(const BatchInst* bi, int count, int ldx, int n, const FFTTables<double>& tab,
                          hipStream_t st) {
  const int ngroups = (n + ColGSCfg<M>::LPW - 1) / ColGSCfg<M>::LPW;
  const dim3 grid(((ngroups + 7) / 8) * 8, count);
  hipLaunchKernelGGL(cols_gs_batched<M>, grid, dim3(ColGSCfg<M>::NT), 0, st, bi, ldx, n, tab, ngroups);
}

template <int M>
void launch_batch_cols_gs_fwd(const BatchInst* bi, int count, int ic, int ip, int ldx, int lds_, int n,
                              const FFTTables<double>& tab, hipStream_t st) {
  const int ngroups = (n + ColGSCfg<M>::LPW - 1) / ColGSCfg<M>::LPW;
  const dim3 grid(((ngroups + 7) / 8) * 8, count);
  hipLaunchKernelGGL(cols_gs_fwd_batched<M>, grid, dim3(ColGSCfg<M>::NT), 0, st, bi, ic, ip, ldx, lds_, n, tab,
                     ngroups);
}

void launch_batch_transpose(const BatchInst* bi, int count, int which, int n, hipStream_t st) {
  const int nt = (n + 31) / 32;
  hipLaunchKernelGGL(transpose_inplace_batched, dim3(nt, nt, count), dim3(256), 0, st, bi, which, n);
}

void launch_batch_swap_transposed(const BatchInst* bi, int count, int n, hipStream_t st) {
  const int nt = (n + 31) / 32;
  hipLaunchKernelGGL(swap_transposed_batched, dim3(nt, nt, count), dim3(256), 0, st, bi, n);
}

void launch_batch_leapfrog(int mode, const BatchInst* bi, int count, int ic, int ip, int ldx, int n, hipStream_t st) {
  hipLaunchKernelGGL(leapfrog_batched, dim3((n + 255) / 256, n, count), dim3(256), 0, st, bi, mode, ic, ip, ldx, n);
}

#define SADI_INSTANTIATE(M)                                                                                      \
  template void launch_rows_fwd<M>(const double*, double*, const double*, int, int, V*, int, int,              \
                                   const FFTTables<double>&, const V*, hipStream_t);                             \
  template void launch_cols_conv<M>(V*, int, int, const double*, int, const FFTTables<double>&, const V*,        \
                                    hipStream_t);                                                                \
  template void launch_rows_rhs_gs<M>(int, const V*, int, const double*, int, const double*, double*, int, bool, \
                                      int, const StepScalars&, const FFTTables<double>&, const GSTables64&,       \
                                      const V*, hipStream_t, bool);                                              \
  template void launch_rows_gs<M>(double*, int, int, int, const FFTTables<double>&, const GSTables64&,            \
                                  hipStream_t);                                                                  \
  template void launch_cols_gs<M>(int, const double*, int, const double*, const double*, double*, int, int,       \
                                  const FFTTables<double>&, const GSTables64&, hipStream_t);                     \
  template void launch_cols_gs_fwd<M>(const double*, int, const double*, double*, int, V*, int, bool,            \
                                      const FFTTables<double>&, const GSTables64&, const V*, hipStream_t, bool); \
  template void launch_rows_rhs_mixed<M>(int, const V*, int, const double*, int, const double*, double*, int,     \
                                         int, const StepScalars&, const FFTTables<double>&, const MixedTables&,  \
                                         const V*, hipStream_t, bool);                                           \
  template void launch_rows_gs_mixed<M>(double*, int, int, int, const FFTTables<double>&, const MixedTables&,     \
                                        hipStream_t);                                                            \
  template void launch_cols_gs_mixed<M>(int, const double*, int, const double*, const double*, double*, int, int, \
                                        const FFTTables<double>&, const MixedTables&, hipStream_t);                \
  template void launch_cols_gs_fwd_mixed<M>(const double*, int, const double*, double*, int, V*, int, bool,      \
                                            const FFTTables<double>&, const MixedTables&, const V*, hipStream_t,  \
                                            bool);                                                               \
  template void launch_batch_rows_fwd<M>(int, const BatchInst*, int, int, int, int, int, int,                     \
                                         const FFTTables<double>&, hipStream_t);                                  \
  template void launch_batch_cols_conv<M>(const BatchInst*, int, int, int, int, const FFTTables<double>&,         \
                                          hipStream_t);                                                           \
  template void launch_batch_rows_rhs<M>(int, const BatchInst*, int, int, int, int, int, const FFTTables<double>&, \
                                         hipStream_t);                                                            \
  template void launch_batch_cols_gs<M>(const BatchInst*, int, int, int, const FFTTables<double>&, hipStream_t); \
  template void launch_batch_cols_gs_fwd<M>(const BatchInst*, int, int, int, int, int, int,                      \
                                            const FFTTables<double>&, hipStream_t);                              \
  template void launch_bccb_eigenvalues<M>(const double*, int, double*, int, double*, V*, int, double*, int,     \
                                           const FFTTables<double>&, hipStream_t);

SADI_FOR_EACH_M(SADI_INSTANTIATE)

}  // namespace sadi
