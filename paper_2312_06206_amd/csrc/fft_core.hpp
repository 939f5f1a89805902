// Register/LDS FFT engine for gfx950: complex FFTs of length M = E * P2 * E
// (M = 16 ... 4096), one line per group of T = M / E threads, E elements per
// thread in registers.
//
// Canonical layout: thread t of a line holds element t + T*m in slot m (m < E).
// A transform keeps this layout from input to output, in natural order, so
// pointwise products (convolution symbols, Q twiddles) and inverse transforms can
// follow without any data movement.  Three register stages (radix E, P2, E) with
// two exchanges through LDS (one when P2 == 1):
//
//   n = a + E b + E P2 c,  k = k1 + E k2 + E P2 k3
//   stage 1 over c (thread t = a + E b):   Y1 = DFT_E(c -> k1) * W_M^{t k1}
//   stage 2 over b (butterfly a + E k1):   Y2 = DFT_P2(b -> k2) * W_{E P2}^{a k2}
//   stage 3 over a (thread k1 + E k2):     X[k1 + E k2 + T k3] = DFT_E(a -> k3)
//
// DIR = -1 is the forward transform (e^{-2 pi i nk/M}), DIR = +1 the unnormalised
// inverse.  Lines of a workgroup are either interleaved lane by lane (LINE_FAST,
// for column kernels: adjacent grid columns in adjacent lanes give coalesced
// row-strided accesses) or contiguous (rows).  Exchanges move either whole
// complex values (SPLIT = 1) or the real and imaginary parts in two rounds
// (SPLIT = 2, half the LDS footprint).
#pragma once
#include <hip/hip_runtime.h>

#include <utility>

namespace sadi {

template <typename R> struct vec2;
template <> struct vec2<double> { using type = double2; };
template <> struct vec2<float> { using type = float2; };
template <typename R> using V2 = typename vec2<R>::type;

template <typename V> __device__ __forceinline__ V cadd(V a, V b) { return V{a.x + b.x, a.y + b.y}; }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { return V{a.x - b.x, a.y - b.y}; }
template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
  return V{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename V> __device__ __forceinline__ V cmulc(V a, V b) {  // a * conj(b)
  return V{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename V, typename R> __device__ __forceinline__ V cscale(V a, R s) { return V{a.x * s, a.y * s}; }
template <typename V> __device__ __forceinline__ V cconj(V a) { return V{a.x, -a.y}; }

// a * e^{DIR i pi/2}
template <int DIR, typename V> __device__ __forceinline__ V mul_i(V a) {
  return DIR < 0 ? V{a.y, -a.x} : V{-a.y, a.x};
}
// a * (c + DIR i s) for constants c, s
template <int DIR, typename V, typename R>
__device__ __forceinline__ V mul_cs(V a, R c, R s) {
  const R ss = DIR < 0 ? -s : s;
  return V{a.x * c - a.y * ss, a.x * ss + a.y * c};
}

// cos / sin of pi*j/8, j = 0..8
#define SADI_C8_1 0.92387953251128675612818318939678828682L
#define SADI_S8_1 0.38268343236508977172845998403039886676L
#define SADI_R2 0.70710678118654752440084436210484903928L

// multiply by e^{DIR 2 pi i j / 16} for a compile-time j in [0, 16)
template <int DIR, int J, typename V>
__device__ __forceinline__ V tw16(V a) {
  using R = decltype(a.x);
  constexpr int j = J & 15;
  if constexpr (j == 0) return a;
  else if constexpr (j == 4) return mul_i<DIR>(a);
  else if constexpr (j == 8) return V{-a.x, -a.y};
  else if constexpr (j == 12) return mul_i<-DIR>(a);
  else if constexpr (j == 2) return mul_cs<DIR>(a, (R)SADI_R2, (R)SADI_R2);
  else if constexpr (j == 6) return mul_cs<DIR>(a, (R)-SADI_R2, (R)SADI_R2);
  else if constexpr (j == 10) return mul_cs<DIR>(a, (R)-SADI_R2, (R)-SADI_R2);
  else if constexpr (j == 14) return mul_cs<DIR>(a, (R)SADI_R2, (R)-SADI_R2);
  else if constexpr (j == 1) return mul_cs<DIR>(a, (R)SADI_C8_1, (R)SADI_S8_1);
  else if constexpr (j == 3) return mul_cs<DIR>(a, (R)SADI_S8_1, (R)SADI_C8_1);
  else if constexpr (j == 5) return mul_cs<DIR>(a, (R)-SADI_S8_1, (R)SADI_C8_1);
  else if constexpr (j == 7) return mul_cs<DIR>(a, (R)-SADI_C8_1, (R)SADI_S8_1);
  else if constexpr (j == 9) return mul_cs<DIR>(a, (R)-SADI_C8_1, (R)-SADI_S8_1);
  else if constexpr (j == 11) return mul_cs<DIR>(a, (R)-SADI_S8_1, (R)-SADI_C8_1);
  else if constexpr (j == 13) return mul_cs<DIR>(a, (R)SADI_S8_1, (R)-SADI_C8_1);
  else return mul_cs<DIR>(a, (R)SADI_C8_1, (R)-SADI_S8_1);  // 15
}

// cos(pi j/16), j = 0..8
#define SADI_C16_1 0.98078528040323044912618223613423903697L
#define SADI_C16_3 0.83146961230254523707878837761790575674L
#define SADI_C16_5 0.55557023301960222474283081394853287437L
#define SADI_C16_7 0.19509032201612826784828486847702224093L

template <int J> struct Cos16;   // cos(pi J / 16) for J in [0, 8]
template <> struct Cos16<0> { static constexpr long double v = 1.0L; };
template <> struct Cos16<1> { static constexpr long double v = SADI_C16_1; };
template <> struct Cos16<2> { static constexpr long double v = SADI_C8_1; };
template <> struct Cos16<3> { static constexpr long double v = SADI_C16_3; };
template <> struct Cos16<4> { static constexpr long double v = SADI_R2; };
template <> struct Cos16<5> { static constexpr long double v = SADI_C16_5; };
template <> struct Cos16<6> { static constexpr long double v = SADI_S8_1; };
template <> struct Cos16<7> { static constexpr long double v = SADI_C16_7; };
template <> struct Cos16<8> { static constexpr long double v = 0.0L; };

// multiply by e^{SH i pi j / 16} for a compile-time j in [0, 16), SH = +-1
template <int SH, int J, typename V>
__device__ __forceinline__ V shift16(V a) {
  using R = decltype(a.x);
  if constexpr (J == 0) return a;
  else if constexpr (J == 8) return mul_i<SH>(a);
  else {
    constexpr long double c = J < 8 ? Cos16<(J < 8 ? J : 0)>::v : -Cos16<(J > 8 ? 16 - J : 0)>::v;
    constexpr long double sn = J < 8 ? Cos16<(J < 8 ? 8 - J : 0)>::v : Cos16<(J > 8 ? J - 8 : 0)>::v;
    return mul_cs<SH>(a, (R)c, (R)sn);
  }
}

// d[c] *= e^{SH i pi c STEP / 16} for every slot c
template <int SH, int STEP, typename V, int... C>
__device__ __forceinline__ void shift_slots(V* d, std::integer_sequence<int, C...>) {
  ((d[C] = shift16<SH, C * STEP>(d[C])), ...);
}

// ---- in-register DFTs, natural order in and out ------------------------------
template <int DIR, typename V> __device__ __forceinline__ void dft2(V* a) {
  V t = a[0];
  a[0] = cadd(t, a[1]);
  a[1] = csub(t, a[1]);
}

template <int DIR, typename V> __device__ __forceinline__ void dft4(V* a) {
  V t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]);
  V t2 = cadd(a[1], a[3]), t3 = mul_i<DIR>(csub(a[1], a[3]));
  a[0] = cadd(t0, t2);
  a[2] = csub(t0, t2);
  a[1] = cadd(t1, t3);
  a[3] = csub(t1, t3);
}

template <int DIR, typename V> __device__ __forceinline__ void dft8(V* a) {
  V e[4] = {a[0], a[2], a[4], a[6]};
  V o[4] = {a[1], a[3], a[5], a[7]};
  dft4<DIR>(e);
  dft4<DIR>(o);
  o[1] = tw16<DIR, 2>(o[1]);
  o[2] = tw16<DIR, 4>(o[2]);
  o[3] = tw16<DIR, 6>(o[3]);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    a[k] = cadd(e[k], o[k]);
    a[k + 4] = csub(e[k], o[k]);
  }
}

// 16 = 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2
template <int DIR, typename V> __device__ __forceinline__ void dft16(V* a) {
  V b[4][4];  // b[n2][k1]
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
#pragma unroll
    for (int n1 = 0; n1 < 4; ++n1) b[n2][n1] = a[4 * n1 + n2];
    dft4<DIR>(b[n2]);
  }
  // twiddles W16^{n2 k1}
  b[1][1] = tw16<DIR, 1>(b[1][1]);
  b[1][2] = tw16<DIR, 2>(b[1][2]);
  b[1][3] = tw16<DIR, 3>(b[1][3]);
  b[2][1] = tw16<DIR, 2>(b[2][1]);
  b[2][2] = tw16<DIR, 4>(b[2][2]);
  b[2][3] = tw16<DIR, 6>(b[2][3]);
  b[3][1] = tw16<DIR, 3>(b[3][1]);
  b[3][2] = tw16<DIR, 6>(b[3][2]);
  b[3][3] = tw16<DIR, 9>(b[3][3]);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    V c[4] = {b[0][k1], b[1][k1], b[2][k1], b[3][k1]};
    dft4<DIR>(c);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) a[k1 + 4 * k2] = c[k2];
  }
}

template <int N, int DIR, typename V> __device__ __forceinline__ void dft(V* a) {
  if constexpr (N == 1) return;
  else if constexpr (N == 2) dft2<DIR>(a);
  else if constexpr (N == 4) dft4<DIR>(a);
  else if constexpr (N == 8) dft8<DIR>(a);
  else if constexpr (N == 16) dft16<DIR>(a);
  else static_assert(N == 16, "radix not supported");
}

// a[k] *= w^k, k = 0..N-1.  Powers by a running product restarted from w^4 every four
// steps (product depth <= 6, few live registers).
template <int N, typename V> __device__ __forceinline__ void twiddle_powers(V* a, V w) {
  if constexpr (N == 1) return;
  V p = w;
  a[1] = cmul(a[1], p);
  if constexpr (N >= 4) {
    V w2 = cmul(w, w);
    a[2] = cmul(a[2], w2);
    a[3] = cmul(a[3], cmul(w2, w));
    if constexpr (N >= 8) {
      const V w4 = cmul(w2, w2);
      V g = w4;
#pragma unroll
      for (int q = 1; q < N / 4; ++q) {
        if (q > 1) g = cmul(g, w4);
        a[4 * q] = cmul(a[4 * q], g);
        V r = cmul(g, w);
        a[4 * q + 1] = cmul(a[4 * q + 1], r);
        r = cmul(g, w2);
        a[4 * q + 2] = cmul(a[4 * q + 2], r);
        r = cmul(r, w);
        a[4 * q + 3] = cmul(a[4 * q + 3], r);
      }
    }
  }
}

// a[k] *= s w^k, k = 0..N-1 (the same product structure with every power scaled by s)
template <int N, typename V> __device__ __forceinline__ void twiddle_powers_s(V* a, V w, V s) {
  a[0] = cmul(a[0], s);
  if constexpr (N == 1) return;
  a[1] = cmul(a[1], cmul(s, w));
  if constexpr (N >= 4) {
    const V w2 = cmul(w, w);
    V r = cmul(s, w2);
    a[2] = cmul(a[2], r);
    a[3] = cmul(a[3], cmul(r, w));
    if constexpr (N >= 8) {
      const V w4 = cmul(w2, w2);
      V g = cmul(s, w4);
#pragma unroll
      for (int q = 1; q < N / 4; ++q) {
        if (q > 1) g = cmul(g, w4);
        a[4 * q] = cmul(a[4 * q], g);
        r = cmul(g, w);
        a[4 * q + 1] = cmul(a[4 * q + 1], r);
        r = cmul(g, w2);
        a[4 * q + 2] = cmul(a[4 * q + 2], r);
        r = cmul(r, w);
        a[4 * q + 3] = cmul(a[4 * q + 3], r);
      }
    }
  }
}

// e^{DIR 2 pi i j / N} from a table of forward roots e^{-2 pi i j / N}
template <int DIR, typename V> __device__ __forceinline__ V root(const V* tab, int j) {
  V w = tab[j];
  return DIR < 0 ? w : cconj(w);
}

// ---- the line transform --------------------------------------------------------
// Shape of a length-M transform.
template <int M_> struct Shape;
template <> struct Shape<16> { static constexpr int E = 4, P2 = 1; };
template <> struct Shape<32> { static constexpr int E = 4, P2 = 2; };
template <> struct Shape<64> { static constexpr int E = 8, P2 = 1; };
template <> struct Shape<128> { static constexpr int E = 8, P2 = 2; };
template <> struct Shape<256> { static constexpr int E = 16, P2 = 1; };
template <> struct Shape<512> { static constexpr int E = 8, P2 = 8; };
template <> struct Shape<1024> { static constexpr int E = 16, P2 = 4; };
template <> struct Shape<2048> { static constexpr int E = 16, P2 = 8; };
template <> struct Shape<4096> { static constexpr int E = 16, P2 = 16; };

// Per-line twiddle-root tables, forward direction (device constant data owned by
// the context): rootM[j] = e^{-2 pi i j/M} for j < T, rootS[j] = e^{-2 pi i j/(E P2)}
// for j < E.
template <typename R> struct FFTTables {
  const V2<R>* rootM;
  const V2<R>* rootS;
  const V2<R>* root2M;   // e^{-i pi j/M}, j < M (half-bin shifted transforms)
};

// LPW lines per workgroup.  LDS exchange region: SPLIT==1 -> V2<R> per element,
// SPLIT==2 -> R per element.  Row stride per line (in elements) is LINE_STRIDE.
template <int M_, typename R, int LPW, bool LINE_FAST, int SPLIT>
struct Line {
  using V = V2<R>;
  static constexpr int M = M_;
  static constexpr int E = Shape<M>::E;
  static constexpr int P2 = Shape<M>::P2;
  static constexpr int T = M / E;          // threads per line
  static constexpr int NT = T * LPW;       // threads per workgroup
  static constexpr int PAD = 1;
  static constexpr bool LINE_FAST_ = LINE_FAST;
  using Real = R;
  static constexpr int LPW_ = LPW;
  static_assert((M + E * PAD) % 2 == 0, "region must hold whole complex values");
  static constexpr int REGION = M + E * PAD;      // elements per line in the exchange
  static constexpr int LDS_ELEMS = REGION * LPW;
  static constexpr int LDS_BYTES = LDS_ELEMS * (SPLIT == 1 ? (int)sizeof(V) : (int)sizeof(R));
  static_assert(E * P2 * E == M, "bad shape");
  static_assert(P2 <= E, "stage-2 radix must not exceed E");

  int line;  // line index within the workgroup
  int t;     // thread index within the line

  __device__ __forceinline__ Line(int tid) {
    if (LINE_FAST) { line = tid % LPW; t = tid / LPW; }
    else { line = tid / T; t = tid % T; }
  }

  // LDS element address of (line, position p) in the exchange region
  __device__ __forceinline__ int lds_index(int p) const {
    return LINE_FAST ? p * LPW + line : line * REGION + p;
  }

  // write value v (all SPLIT rounds are handled by the caller through exchange())
  // SH = +-1: transform of x[n] e^{SH i pi n/M} instead of x[n] (a half-bin shift, e.g. the
  // skew-circulant diagonalisation).  With n = t + T c the factor splits into e^{SH i pi c/E}
  // per slot (constants, before the first DFT) and e^{SH i pi t/M} per thread, which starts
  // the running product of the first twiddle.
  template <int DIR, int SH = 0>
  __device__ __forceinline__ void transform(V* d, void* lds, const FFTTables<R>& tab) const {
    // ---- stage 1: DFT_E over c, twiddle W_M^{t k1}
    if constexpr (SH != 0) shift_slots<SH, 16 / E>(d, std::make_integer_sequence<int, E>{});
    dft<E, DIR>(d);
    if constexpr (SH == 0) twiddle_powers<E>(d, root<DIR>(tab.rootM, t));
    else twiddle_powers_s<E>(d, root<DIR>(tab.rootM, t), root<SH>(tab.root2M, t));
    stages23<DIR>(d, lds, tab);
  }

  // Same with a per-thread factor s on the first twiddle (the caller has applied any
  // per-slot factor): a half-bin shift that only some lines of a workgroup take.
  template <int DIR>
  __device__ __forceinline__ void transform_scaled(V* d, void* lds, const FFTTables<R>& tab, V s) const {
    dft<E, DIR>(d);
    twiddle_powers_s<E>(d, root<DIR>(tab.rootM, t), s);
    stages23<DIR>(d, lds, tab);
  }

  // exchanges, stage 2 and stage 3 (natural-order output in canonical layout)
  template <int DIR>
  __device__ __forceinline__ void stages23(V* d, void* lds, const FFTTables<R>& tab) const {
    if constexpr (P2 == 1) {
      // single exchange: writer t = a holds k1; reader t3 = k1 gathers a
      exchange(d, lds, [&](int k1) { return k1 + (T + PAD) * t; },
               [&](int a) { return t + (T + PAD) * a; });
    } else {
      // exchange 1: writer t (= a + E b) slot k1 -> address t + T k1
      // stage-2 butterflies: beta = t + T q (q < E/P2), beta = a + E k1; value b at
      //   address a + E b + T k1
      constexpr int NB = E / P2;
      exchange(d, lds, [&](int k1) { return t + T * k1; },
               [&](int s) {
                 const int q = s / P2, b = s % P2;
                 const int beta = t + T * q;
                 const int a = beta % E, k1 = beta / E;
                 return a + E * b + T * k1;
               });
      // ---- stage 2: per butterfly, DFT_P2 over b then twiddle W_{E P2}^{a k2}
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        dft<P2, DIR>(d + q * P2);
        const int beta = t + T * q;
        const int a = beta % E;
        twiddle_powers<P2>(d + q * P2, root<DIR>(tab.rootS, a));
      }
      // exchange 2: butterfly (a, k1) value k2 -> reader t3 = k1 + E k2 gathers a;
      //   address t3 + (T + PAD) a
      exchange(d, lds,
               [&](int s) {
                 const int q = s / P2, k2 = s % P2;
                 const int beta = t + T * q;
                 const int a = beta % E, k1 = beta / E;
                 return (k1 + E * k2) + (T + PAD) * a;
               },
               [&](int a) { return t + (T + PAD) * a; });
    }
    // ---- stage 3: DFT_E over a; slot k3 holds X[t + T k3]
    dft<E, DIR>(d);
  }

  // Exchange through LDS: element in slot s is written to address wr(s); slot s
  // is then reloaded from address rd(s).  Ends with all reads complete.
  template <typename WF, typename RF>
  __device__ __forceinline__ void exchange(V* d, void* lds, WF wr, RF rd) const {
    if constexpr (SPLIT == 1) {
      V* buf = reinterpret_cast<V*>(lds);
#pragma unroll
      for (int s = 0; s < E; ++s) buf[lds_index(wr(s))] = d[s];
      __syncthreads();
#pragma unroll
      for (int s = 0; s < E; ++s) d[s] = buf[lds_index(rd(s))];
      __syncthreads();
    } else {
      R* buf = reinterpret_cast<R*>(lds);
#pragma unroll
      for (int s = 0; s < E; ++s) buf[lds_index(wr(s))] = d[s].x;
      __syncthreads();
#pragma unroll
      for (int s = 0; s < E; ++s) d[s].x = buf[lds_index(rd(s))];
      __syncthreads();
#pragma unroll
      for (int s = 0; s < E; ++s) buf[lds_index(wr(s))] = d[s].y;
      __syncthreads();
#pragma unroll
      for (int s = 0; s < E; ++s) d[s].y = buf[lds_index(rd(s))];
      __syncthreads();
    }
  }

  // Publish one real value per element (canonical layout) into LDS, natural order;
  // then `get(k)` may read any element.  Uses the R view of the exchange region.
  // complex positions p < REGION/2 inside this line's share of the exchange region
  __device__ __forceinline__ int cidx(int p) const {
    return LINE_FAST ? p * LPW + line : line * (REGION / 2) + p;
  }

  __device__ __forceinline__ void put_real(R* buf, int k, R v) const { buf[lds_index(k)] = v; }
  __device__ __forceinline__ R get_real(const R* buf, int k) const { return buf[lds_index(k)]; }
};

}  // namespace sadi
