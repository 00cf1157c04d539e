// fft_core.h - mixed-radix in-place FFT building blocks (radix 2, 3, 4, 5, 7, 8, 9, 16).
//
// The spectral operators L = (Id - alpha Laplacian)^s and K = L^-1 (Section 2.1
// of the paper) are applied as forward FFT -> real symbol -> inverse FFT.  Since
// the symbol is pointwise, the spectrum never has to be in natural order:
//   forward  = decimation-in-frequency (Gentleman-Sande), natural input ->
//              digit-reversed output, twiddle after each butterfly;
//   inverse  = decimation-in-time (Cooley-Tukey), digit-reversed input ->
//              natural output, conjugate twiddle before each butterfly.
// Each stage updates its butterflies' elements in place (every element belongs
// to exactly one butterfly per stage), so a stage needs no staging copy, no
// register-resident sweep and only one barrier.
//
// All functions are __host__ __device__: kernels run them on LDS with one
// butterfly per thread, and a host program can run the very same stage code
// sequentially (a stage has no intra-stage hazards).
#pragma once

#include <hip/hip_runtime.h>

namespace lddmm {

#define LD_HD __host__ __device__ __forceinline__

template <typename T>
struct cplx {
  T x, y;
};

template <typename T>
LD_HD cplx<T> c_add(cplx<T> a, cplx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
LD_HD cplx<T> c_sub(cplx<T> a, cplx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
LD_HD cplx<T> c_mul(cplx<T> a, cplx<T> b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
// a * conj(b)
template <typename T>
LD_HD cplx<T> c_mulc(cplx<T> a, cplx<T> b) { return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y}; }
template <typename T>
LD_HD cplx<T> c_conj(cplx<T> a) { return {a.x, -a.y}; }
template <typename T>
LD_HD cplx<T> c_scale(cplx<T> a, T s) { return {a.x * s, a.y * s}; }
// a * (DIR i): DIR = +1 multiplies by i, DIR = -1 by -i.
template <int DIR, typename T>
LD_HD cplx<T> c_mul_i(cplx<T> a) {
  return DIR > 0 ? cplx<T>{-a.y, a.x} : cplx<T>{a.y, -a.x};
}

constexpr int kMaxFactors = 16;

// Factorisation of one transform length; radix[s] is used by DIF stage s.
struct FftPlan {
  int n;
  int nf;
  int radix[kMaxFactors];
};

// cos / sin of 2 pi m / R for the odd radices (m in [0, R)).
LD_HD constexpr double root_cos(int R, int m) {
  return R == 3 ? (m == 0 ? 1.0 : -0.5)
       : R == 5 ? (m == 0 ? 1.0 : (m == 1 || m == 4) ? 0.30901699437494742410 : -0.80901699437494742410)
       : (m == 0 ? 1.0
          : (m == 1 || m == 6) ? 0.62348980185873353053
          : (m == 2 || m == 5) ? -0.22252093395631440429
                               : -0.90096886790241912624);
}
LD_HD constexpr double root_sin(int R, int m) {
  return R == 3 ? (m == 0 ? 0.0 : m == 1 ? 0.86602540378443864676 : -0.86602540378443864676)
       : R == 5 ? (m == 0 ? 0.0
                   : m == 1 ? 0.95105651629515357212
                   : m == 2 ? 0.58778525229247312917
                   : m == 3 ? -0.58778525229247312917
                            : -0.95105651629515357212)
       : (m == 0 ? 0.0
          : m == 1 ? 0.78183148246802980871
          : m == 2 ? 0.97492791218182360702
          : m == 3 ? 0.43388373911755812048
          : m == 4 ? -0.43388373911755812048
          : m == 5 ? -0.97492791218182360702
                   : -0.78183148246802980871);
}

// In-register DFT of size R with kernel exp(DIR 2 pi i j k / R).
template <typename T, int R, int DIR>
struct Dft {
  // odd radix: pair j with R - j
  static LD_HD void run(cplx<T>* a) {
    constexpr int H = (R - 1) / 2;
    cplx<T> b[H + 1], d[H + 1];
#pragma unroll
    for (int j = 1; j <= H; ++j) {
      b[j] = c_add(a[j], a[R - j]);
      d[j] = c_sub(a[j], a[R - j]);
    }
    cplx<T> y0 = a[0];
#pragma unroll
    for (int j = 1; j <= H; ++j) y0 = c_add(y0, b[j]);
    cplx<T> out[R];
    out[0] = y0;
#pragma unroll
    for (int k = 1; k <= H; ++k) {
      cplx<T> A = a[0], B = {T(0), T(0)};
#pragma unroll
      for (int j = 1; j <= H; ++j) {
        const int m = (j * k) % R;
        const T cc = T(root_cos(R, m));
        const T ss = T(root_sin(R, m));
        A = c_add(A, c_scale(b[j], cc));
        B = c_add(B, c_scale(d[j], ss));
      }
      const cplx<T> iB = c_mul_i<DIR>(B);
      out[k] = c_add(A, iB);
      out[R - k] = c_sub(A, iB);
    }
#pragma unroll
    for (int k = 0; k < R; ++k) a[k] = out[k];
  }
};

template <typename T, int DIR>
struct Dft<T, 2, DIR> {
  static LD_HD void run(cplx<T>* a) {
    const cplx<T> t = a[0];
    a[0] = c_add(t, a[1]);
    a[1] = c_sub(t, a[1]);
  }
};

template <typename T, int DIR>
struct Dft<T, 4, DIR> {
  static LD_HD void run(cplx<T>* a) {
    const cplx<T> t0 = c_add(a[0], a[2]);
    const cplx<T> t1 = c_sub(a[0], a[2]);
    const cplx<T> t2 = c_add(a[1], a[3]);
    const cplx<T> t3 = c_mul_i<DIR>(c_sub(a[1], a[3]));
    a[0] = c_add(t0, t2);
    a[2] = c_sub(t0, t2);
    a[1] = c_add(t1, t3);
    a[3] = c_sub(t1, t3);
  }
};

template <typename T, int DIR>
struct Dft<T, 8, DIR> {
  // 8 = 2 x 4: radix-2 split of (a_j, a_{j+4}), twiddles W8^j, two DFT4s.
  static LD_HD void run(cplx<T>* a) {
    constexpr T r = T(0.70710678118654752440);
    cplx<T> b[4], c[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      b[j] = c_add(a[j], a[j + 4]);
      c[j] = c_sub(a[j], a[j + 4]);
    }
    // c1 *= (r, DIR r), c2 *= DIR i, c3 *= (-r, DIR r)
    c[1] = cplx<T>{r * (c[1].x - T(DIR) * c[1].y), r * (c[1].y + T(DIR) * c[1].x)};
    c[2] = c_mul_i<DIR>(c[2]);
    c[3] = cplx<T>{-r * (c[3].x + T(DIR) * c[3].y), r * (T(DIR) * c[3].x - c[3].y)};
    Dft<T, 4, DIR>::run(b);
    Dft<T, 4, DIR>::run(c);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      a[2 * k] = b[k];
      a[2 * k + 1] = c[k];
    }
  }
};

// 16 = 4 x 4: DFT4 over the four stride-4 groups, twiddles W16^(n2 k1), DFT4 over
// the groups again (Cooley-Tukey; W = exp(DIR 2 pi i / 16)).
template <typename T, int DIR>
struct Dft<T, 16, DIR> {
  // x * (re + DIR im i) for the constant root (re, im)
  static LD_HD cplx<T> rot(cplx<T> x, T re, T im) {
    const T si = T(DIR) * im;
    return {x.x * re - x.y * si, x.x * si + x.y * re};
  }
  static LD_HD void run(cplx<T>* a) {
    const T c1 = T(0.92387953251128675613), s1 = T(0.38268343236508977173), r = T(0.70710678118654752440);
    cplx<T> y[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      cplx<T> g[4] = {a[n2], a[4 + n2], a[8 + n2], a[12 + n2]};
      Dft<T, 4, DIR>::run(g);
#pragma unroll
      for (int k1 = 0; k1 < 4; ++k1) y[n2][k1] = g[k1];
    }
    y[1][1] = rot(y[1][1], c1, s1);    // W^1
    y[1][2] = cplx<T>{r * (y[1][2].x - T(DIR) * y[1][2].y), r * (y[1][2].y + T(DIR) * y[1][2].x)};  // W^2
    y[1][3] = rot(y[1][3], s1, c1);    // W^3
    y[2][1] = cplx<T>{r * (y[2][1].x - T(DIR) * y[2][1].y), r * (y[2][1].y + T(DIR) * y[2][1].x)};  // W^2
    y[2][2] = c_mul_i<DIR>(y[2][2]);   // W^4
    y[2][3] = cplx<T>{-r * (y[2][3].x + T(DIR) * y[2][3].y), r * (T(DIR) * y[2][3].x - y[2][3].y)};  // W^6
    y[3][1] = rot(y[3][1], s1, c1);    // W^3
    y[3][2] = cplx<T>{-r * (y[3][2].x + T(DIR) * y[3][2].y), r * (T(DIR) * y[3][2].x - y[3][2].y)};  // W^6
    y[3][3] = rot(y[3][3], -c1, -s1);  // W^9
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      cplx<T> h[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
      Dft<T, 4, DIR>::run(h);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) a[k1 + 4 * k2] = h[k2];
    }
  }
};

// 9 = 3 x 3: DFT3 over the three stride-3 groups, twiddles W9^(n2 k1), DFT3 over
// the groups again (Cooley-Tukey; W = exp(DIR 2 pi i / 9)).
template <typename T, int DIR>
struct Dft<T, 9, DIR> {
  // x * (re + DIR im i) for the constant root (re, im)
  static LD_HD cplx<T> rot(cplx<T> x, T re, T im) {
    const T si = T(DIR) * im;
    return {x.x * re - x.y * si, x.x * si + x.y * re};
  }
  static LD_HD void run(cplx<T>* a) {
    // cos and sin of 2 pi m / 9 for m = 1, 2, 4
    const T c1 = T(0.76604444311897803520), s1 = T(0.64278760968653932632);
    const T c2 = T(0.17364817766693034885), s2 = T(0.98480775301220805937);
    const T c4 = T(-0.93969262078590838405), s4 = T(0.34202014332566873304);
    cplx<T> y[3][3];
#pragma unroll
    for (int n2 = 0; n2 < 3; ++n2) {
      cplx<T> g[3] = {a[n2], a[3 + n2], a[6 + n2]};
      Dft<T, 3, DIR>::run(g);
#pragma unroll
      for (int k1 = 0; k1 < 3; ++k1) y[n2][k1] = g[k1];
    }
    y[1][1] = rot(y[1][1], c1, s1);  // W^1
    y[1][2] = rot(y[1][2], c2, s2);  // W^2
    y[2][1] = rot(y[2][1], c2, s2);  // W^2
    y[2][2] = rot(y[2][2], c4, s4);  // W^4
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) {
      cplx<T> h[3] = {y[0][k1], y[1][k1], y[2][k1]};
      Dft<T, 3, DIR>::run(h);
#pragma unroll
      for (int k2 = 0; k2 < 3; ++k2) a[k1 + 3 * k2] = h[k2];
    }
  }
};

// Twiddle powers w[q] = W^(j q), q = 1..R-1, from one table read W^j (the
// rest by complex products in registers: fewer LDS reads, a few ulp of error).
template <typename T, int R>
LD_HD void twiddle_powers(cplx<T>* w, int j, int twstep, const cplx<T>* tw) {
  w[1] = tw[j * twstep];
  if (R > 2) w[2] = c_mul(w[1], w[1]);
  if (R > 3) w[3] = c_mul(w[2], w[1]);
  if (R > 4) w[4] = c_mul(w[2], w[2]);
  if (R > 5) w[5] = c_mul(w[4], w[1]);
  if (R > 6) w[6] = c_mul(w[4], w[2]);
  if (R > 7) w[7] = c_mul(w[4], w[3]);
  if (R > 8) {
    w[8] = c_mul(w[4], w[4]);
#pragma unroll
    for (int q = 9; q < R; ++q) w[q] = c_mul(w[8], w[q - 8]);
  }
}

// One butterfly of DIF stage with sub-length L = R * stride.  Elements at
// base + t * step (t < R); j = position inside the sub-block; tw[m] =
// exp(-2 pi i m / n); twstep = n / L.  TW = false when the stride is 1 (the
// last DIF stage), where every twiddle is W^0 = 1.
template <typename T, int R, bool TW = true>
LD_HD void dif_butterfly(cplx<T>* buf, int base, int step, int j, int twstep, const cplx<T>* tw) {
  cplx<T> a[R];
#pragma unroll
  for (int t = 0; t < R; ++t) a[t] = buf[base + t * step];
  Dft<T, R, -1>::run(a);
  if constexpr (TW) {
    buf[base] = a[0];
    cplx<T> w[R];
    twiddle_powers<T, R>(w, j, twstep, tw);
#pragma unroll
    for (int q = 1; q < R; ++q) buf[base + q * step] = c_mul(a[q], w[q]);
  } else {
#pragma unroll
    for (int q = 0; q < R; ++q) buf[base + q * step] = a[q];
  }
}

// Inverse of dif_butterfly up to the factor R (conjugate twiddle, then DFT).
template <typename T, int R, bool TW = true>
LD_HD void dit_butterfly(cplx<T>* buf, int base, int step, int j, int twstep, const cplx<T>* tw) {
  cplx<T> a[R];
  if constexpr (TW) {
    a[0] = buf[base];
    cplx<T> w[R];
    twiddle_powers<T, R>(w, j, twstep, tw);
#pragma unroll
    for (int q = 1; q < R; ++q) a[q] = c_mulc(buf[base + q * step], w[q]);
  } else {
#pragma unroll
    for (int q = 0; q < R; ++q) a[q] = buf[base + q * step];
  }
  Dft<T, R, +1>::run(a);
#pragma unroll
  for (int t = 0; t < R; ++t) buf[base + t * step] = a[t];
}

// All butterflies of one stage over `count` sequences of length n; element e of
// sequence s sits at buf[s * ss + e * es].  Butterfly b of the stage is handled
// by the caller's index `b` in [0, count * n / R).  SEQ_FAST maps consecutive b
// to consecutive sequences (use when sequences are contiguous, es > 1);
// otherwise to consecutive butterflies of one sequence (es == 1).
template <typename T, int R, bool INV, bool SEQ_FAST>
LD_HD void fft_stage_item(cplx<T>* buf, int b, int n, int L, int count, int es, int ss, const cplx<T>* tw) {
  const int stride = L / R;
  const int nbf = n / R;
  int s, u;
  if (SEQ_FAST) {
    u = b / count;
    s = b - u * count;
  } else {
    s = b / nbf;
    u = b - s * nbf;
  }
  const int blk = u / stride;
  const int j = u - blk * stride;
  const int base = s * ss + (blk * L + j) * es;
  if (INV)
    dit_butterfly<T, R>(buf, base, stride * es, j, n / L, tw);
  else
    dif_butterfly<T, R>(buf, base, stride * es, j, n / L, tw);
}

// Sub-length of stage `st` (DIF order): n / (radix[0] ... radix[st-1]).
LD_HD int stage_length(const FftPlan& pl, int st) {
  int L = pl.n;
  for (int i = 0; i < st; ++i) L /= pl.radix[i];
  return L;
}

// Factor n into radices, largest power-of-two radices first (8s, then one 4 or
// 2), then a single 3 where 3 divides n an odd number of times, 5s, 7s, and the
// 3 x 3 pairs as radix 9 last (the stride-1 last stage takes no twiddles, so the
// largest odd radix goes there); with at least two 8s a trailing 8 x 2 becomes
// 16 and a trailing 8 x 8 x 4 becomes 16 x 16 (one stage fewer).  False if
// another prime divides n (or 3, 5, 7 more than 8, 5, 4 times).
inline bool make_plan(int n, FftPlan& pl) {
  pl.n = n;
  pl.nf = 0;
  for (int i = 0; i < kMaxFactors; ++i) pl.radix[i] = 0;
  if (n < 1) return false;
  int m = n;
  const int order[] = {8, 8, 8, 8, 8, 8, 8, 8, 8, 8, 4, 2};
  for (int r : order) {
    if (m % r != 0) continue;
    if (r == 2 && m % 4 == 0) continue;
    if (pl.nf >= kMaxFactors) return false;
    pl.radix[pl.nf++] = r;
    m /= r;
  }
  int c3 = 0, c5 = 0, c7 = 0;
  while (c3 < 8 && m % 3 == 0) ++c3, m /= 3;
  while (c5 < 5 && m % 5 == 0) ++c5, m /= 5;
  while (c7 < 4 && m % 7 == 0) ++c7, m /= 7;
  if (m != 1) return false;
  if (pl.nf + (c3 % 2) + c5 + c7 + c3 / 2 > kMaxFactors) return false;
  if (c3 % 2) pl.radix[pl.nf++] = 3;
  for (int i = 0; i < c5; ++i) pl.radix[pl.nf++] = 5;
  for (int i = 0; i < c7; ++i) pl.radix[pl.nf++] = 7;
  for (int i = 0; i < c3 / 2; ++i) pl.radix[pl.nf++] = 9;
  int n8 = 0;
  while (n8 < pl.nf && pl.radix[n8] == 8) ++n8;
  const int rest = n8 < pl.nf ? pl.radix[n8] : 1;
  if (n8 >= 2 && (rest == 2 || rest == 4)) {
    int out[kMaxFactors], k = 0;
    const int keep = rest == 2 ? n8 - 1 : n8 - 2;
    for (int i = 0; i < keep; ++i) out[k++] = 8;
    out[k++] = 16;
    if (rest == 4) out[k++] = 16;
    for (int i = n8 + 1; i < pl.nf; ++i) out[k++] = pl.radix[i];
    for (int i = 0; i < kMaxFactors; ++i) pl.radix[i] = i < k ? out[i] : 0;
    pl.nf = k;
  }
  return true;
}

// DIF output slot p holds frequency digit_reverse(p).
inline __host__ __device__ int digit_reverse(const FftPlan& pl, int p) {
  int k = 0, mult = 1, span = pl.n, rem = p;
  for (int s = 0; s < pl.nf; ++s) {
    span /= pl.radix[s];
    const int d = rem / span;
    rem -= d * span;
    k += d * mult;
    mult *= pl.radix[s];
  }
  return k;
}

}  // namespace lddmm

namespace lddmm {

// ---------------------------------------------------------------------------
// Compile-time plans.  For the power-of-two lengths of the common grids the
// radices, sub-lengths, strides and sequence counts are template constants, so
// every index of a butterfly is a shift or a constant multiply.  The radix
// order is the one make_plan produces, which keeps the digit-reversed slot
// tables of the runtime plan valid.
// ---------------------------------------------------------------------------
template <int N>
struct Pow2Plan {
  static_assert(N >= 2 && (N & (N - 1)) == 0, "power of two");
  static constexpr int n8 = __builtin_ctz(N) / 3;
  static constexpr int rest = N >> (3 * n8);  // 1, 2 or 4
  static constexpr bool g2 = rest == 2 && n8 >= 2;  // ... 8 x 2 -> 16
  static constexpr bool g4 = rest == 4 && n8 >= 2;  // ... 8 x 8 x 4 -> 16 x 16
  static constexpr int nf = (g2 || g4) ? n8 : n8 + (rest > 1 ? 1 : 0);
  static constexpr int radix(int i) {
    return g2 ? (i < n8 - 1 ? 8 : 16) : g4 ? (i < n8 - 2 ? 8 : 16) : (i < n8 ? 8 : rest);
  }
  static constexpr int length(int i) { return i == 0 ? N : length(i - 1) / radix(i - 1); }
};

// Explicit radix list (in DIF stage order) for the other lengths in use.
template <int N, int... Rs>
struct RadixPlan {
  static constexpr int nf = sizeof...(Rs);
  static constexpr int rs[sizeof...(Rs)] = {Rs...};
  static constexpr int radix(int i) { return rs[i]; }
  static constexpr int length(int i) { return i == 0 ? N : length(i - 1) / radix(i - 1); }
};

// Compile-time plan of length N: powers of two by rule, the mixed lengths of
// the supported grids listed (each equal to make_plan(N), checked on the host).
template <int N>
struct PlanOf {
  using type = Pow2Plan<N>;
};
#define LDDMM_PLAN(n, ...)                       template <>                                    struct PlanOf<n> {                               using type = RadixPlan<n, __VA_ARGS__>;      };
LDDMM_PLAN(40, 8, 5)
LDDMM_PLAN(48, 8, 2, 3)
LDDMM_PLAN(56, 8, 7)
LDDMM_PLAN(80, 8, 2, 5)
LDDMM_PLAN(90, 2, 5, 9)
LDDMM_PLAN(96, 8, 4, 3)
LDDMM_PLAN(108, 4, 3, 9)
LDDMM_PLAN(112, 8, 2, 7)
LDDMM_PLAN(180, 4, 5, 9)
LDDMM_PLAN(216, 8, 3, 9)
#undef LDDMM_PLAN

// Slot (DIF output position) that holds frequency k: the inverse of
// digit_reverse for the compile-time plan P.
template <class P>
LD_HD int slot_of(int k) {
  int p = 0, span = P::length(0);
#pragma unroll
  for (int i = 0; i < P::nf; ++i) {
    span /= P::radix(i);
    const int d = k % P::radix(i);
    k /= P::radix(i);
    p += d * span;
  }
  return p;
}

// True if the compile-time plan P has the runtime plan's radices.
template <class P>
inline bool plan_matches(const FftPlan& rt) {
  if (rt.n != P::length(0) || rt.nf != P::nf) return false;
  for (int i = 0; i < P::nf; ++i)
    if (rt.radix[i] != P::radix(i)) return false;
  return true;
}

// Butterfly b of DIF/DIT stage ST (plan P) over COUNT sequences; element e of
// sequence s at buf[s * SS + e * ES].
template <typename T, class P, int ST, bool INV, bool SEQ_FAST, int COUNT, int ES, int SS>
LD_HD void fft_stage_item_static(cplx<T>* buf, int b, const cplx<T>* tw) {
  constexpr int R = P::radix(ST);
  constexpr int L = P::length(ST);
  constexpr int stride = L / R;
  constexpr int nbf = P::length(0) / R;
  int s, u;
  if (SEQ_FAST) {
    u = b / COUNT;
    s = b - u * COUNT;
  } else {
    s = b / nbf;
    u = b - s * nbf;
  }
  const int blk = u / stride;
  const int j = u - blk * stride;
  const int base = s * SS + (blk * L + j) * ES;
  if (INV)
    dit_butterfly<T, R, (stride > 1)>(buf, base, stride * ES, j, P::length(0) / L, tw);
  else
    dif_butterfly<T, R, (stride > 1)>(buf, base, stride * ES, j, P::length(0) / L, tw);
}

}  // namespace lddmm
