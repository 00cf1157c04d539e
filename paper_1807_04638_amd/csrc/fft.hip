// fft.hip - spectral application of L = (Id - alpha Laplacian)^s and K = L^-1
// (Section 2.1 of the paper) on the periodic grid, with integer wavenumbers.
//
// Per component: real 3D FFT -> multiply by (1 + alpha |k|^2)^(+-s) / N -> inverse.
// Spectrum layout (per component): [x0 or k0 slot][k1 slot][k2 slot], M = N2/2 + 1
// columns; slots are digit-reversed positions of the DIF outputs (the symbol
// only needs |k|^2 of each slot, so the spectrum is never reordered).
//
// x2 (contiguous) real transform: the N2 reals of a row are read as N2/2
// complex pairs, transformed with length H = N2/2, and split into the H + 1
// non-negative frequencies (the even/odd half-length method); the inverse
// recombines them before a length-H inverse transform.
//
// Fused path (the (x1, x2) half-plane fits one workgroup's LDS):
//   pass 1  plane: rows (x2, real) + columns (x1)     real field  -> spectrum
//   pass 2  pencil: x0 forward, symbol, x0 inverse    spectrum in place
//   pass 3  plane: columns (x1) inverse + rows (x2)   spectrum    -> real field
// Split path: rows, x1 pencils, x0 pencils with symbol, x1 pencils, rows.
#include <cmath>
#include <cstring>

#include "lddmm.h"
#include "lddmm_internal.h"

namespace lddmm {

// --------------------------------------------------------------------------
// LDS drivers
// --------------------------------------------------------------------------
#define LDDMM_FFT_STAGE(R)                                                             \
  case R:                                                                              \
    for (int b = tid; b < total; b += nthr)                                            \
      fft_stage_item<T, R, INV, SEQ_FAST>(buf, b, n, L, count, es, ss, tw);            \
    break;

// Full transform (all stages) of `count` sequences held in LDS.  Ends with a
// barrier.  Forward = DIF (natural -> digit-reversed), inverse = DIT.
template <typename T, bool INV, bool SEQ_FAST>
__device__ void lds_fft(cplx<T>* buf, const FftPlan& pl, int count, int es, int ss, const cplx<T>* tw) {
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int n = pl.n;
  for (int i = 0; i < pl.nf; ++i) {
    const int st = INV ? pl.nf - 1 - i : i;
    const int r = pl.radix[st];
    const int L = stage_length(pl, st);
    const int total = count * (n / r);
    switch (r) {
      LDDMM_FFT_STAGE(16)
      LDDMM_FFT_STAGE(8)
      LDDMM_FFT_STAGE(4)
      LDDMM_FFT_STAGE(2)
      LDDMM_FFT_STAGE(3)
      LDDMM_FFT_STAGE(5)
      LDDMM_FFT_STAGE(7)
      LDDMM_FFT_STAGE(9)
      default:
        break;
    }
    __syncthreads();
  }
}

// Rows of H complex pairs at A[r * M + j]: forward transform then split into the
// N2/2 + 1 real-signal frequencies X[k]; X[k] lands in column slot2[k].  Lanes
// walk consecutive rows (stride M = H + 1 complex, an odd number of 8- or
// 16-byte words), which keeps a wavefront's LDS accesses on distinct banks.
template <typename T>
__device__ void rows_r2c(cplx<T>* A, int count, int H, int M, const FftPlan& p2, const cplx<T>* tw2,
                         const cplx<T>* twr, const int* slot2) {
  lds_fft<T, false, true>(A, p2, count, 1, M, tw2);
  const int per = H / 2 + 1;
  for (int idx = threadIdx.x; idx < count * per; idx += blockDim.x) {
    const int k = idx / count, r = idx - k * count;
    cplx<T>* row = A + r * M;
    if (k == 0) {
      const cplx<T> z = row[0];
      row[0] = {z.x + z.y, T(0)};
      row[H] = {z.x - z.y, T(0)};
    } else {
      const int sk = slot2[k], sm = slot2[H - k];
      const cplx<T> a = row[sk], b = row[sm];
      // even part e = (a + conj b) / 2, odd part o = (a - conj b) / 2
      const cplx<T> e = {T(0.5) * (a.x + b.x), T(0.5) * (a.y - b.y)};
      const cplx<T> o = {T(0.5) * (a.x - b.x), T(0.5) * (a.y + b.y)};
      const cplx<T> wo = c_mul(twr[k], o);
      // X[k] = e - i w o ;  X[H-k] = conj(e) - i conj(w o)
      row[sk] = {e.x + wo.y, e.y - wo.x};
      if (sm != sk) row[sm] = {e.x - wo.y, -e.y - wo.x};
    }
  }
  __syncthreads();
}

// Inverse of rows_r2c (times N2): recombine X[k], X[H-k] into the half-length
// spectrum and run the inverse transform; row r then holds pairs (x[2j], x[2j+1]).
template <typename T>
__device__ void rows_c2r(cplx<T>* A, int count, int H, int M, const FftPlan& p2, const cplx<T>* tw2,
                         const cplx<T>* twr, const int* slot2) {
  const int per = H / 2 + 1;
  for (int idx = threadIdx.x; idx < count * per; idx += blockDim.x) {
    const int k = idx / count, r = idx - k * count;
    cplx<T>* row = A + r * M;
    if (k == 0) {
      const cplx<T> a = row[0], b = row[H];
      const cplx<T> p = {a.x + b.x, a.y - b.y};
      const cplx<T> q = {a.x - b.x, a.y + b.y};
      row[0] = {p.x - q.y, p.y + q.x};
    } else {
      const int sk = slot2[k], sm = slot2[H - k];
      const cplx<T> a = row[sk], b = row[sm];
      const cplx<T> p = {a.x + b.x, a.y - b.y};  // X[k] + conj X[H-k]
      const cplx<T> q = {a.x - b.x, a.y + b.y};  // X[k] - conj X[H-k]
      const cplx<T> t = c_mulc(q, twr[k]);       // conj(w) q
      row[sk] = {p.x - t.y, p.y + t.x};          // p + i t
      if (sm != sk) row[sm] = {p.x + t.y, -p.y + t.x};  // conj(p) + i conj(t)
    }
  }
  __syncthreads();
  lds_fft<T, true, true>(A, p2, count, 1, M, tw2);
}

template <typename T>
__device__ void load_table(cplx<T>* dst, const cplx<T>* src, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

// --------------------------------------------------------------------------
// Kernels
// --------------------------------------------------------------------------
template <typename T>
struct PlaneArgs {
  int n0, n1, n2, H, M;
  int planes;  // (x1, x2) planes of the call: components * n0
  long long N;
  FftPlan p1, p2;
  const cplx<T>* tw1;
  const cplx<T>* tw2;
  const cplx<T>* twr;
  const int* slot2;
  const T* add;  // inverse pass with an addend: out = add + add_scale * (transform)
  T add_scale;
  int xcd_run;   // units per XCD run (xcd_grouped); 1: round-robin order
};

// LDS carve-up shared by the plane and row kernels: A | tw1 | tw2 | twr | slot2
template <typename T>
struct PlaneLds {
  cplx<T>* A;
  cplx<T>* tw1;
  cplx<T>* tw2;
  cplx<T>* twr;
  int* slot2;
};

template <typename T>
__device__ PlaneLds<T> carve(unsigned char* smem, int rows, const PlaneArgs<T>& a, bool with_tw1) {
  PlaneLds<T> L;
  L.A = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* p = L.A + rows * a.M;
  L.tw1 = p;
  if (with_tw1) p += a.n1;
  L.tw2 = p;
  p += a.H;
  L.twr = p;
  p += a.H / 2 + 1;
  L.slot2 = reinterpret_cast<int*>(p);
  if (with_tw1) load_table(L.tw1, a.tw1, a.n1);
  load_table(L.tw2, a.tw2, a.H);
  load_table(L.twr, a.twr, a.H / 2 + 1);
  for (int i = threadIdx.x; i <= a.H; i += blockDim.x) L.slot2[i] = a.slot2[i];
  return L;
}

// One (x0, component) plane: real rows -> x2 spectrum -> x1 columns.
template <typename T, int NT>
__global__ void __launch_bounds__(NT) k_plane_fwd(const T* __restrict__ in, cplx<T>* __restrict__ spec,
                                                   PlaneArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int x0 = blockIdx.x, comp = blockIdx.y;
  PlaneLds<T> L = carve(smem, a.n1, a, true);
  const cplx<T>* src = reinterpret_cast<const cplx<T>*>(in + comp * a.N + (long long)x0 * a.n1 * a.n2);
  const int tot = a.n1 * a.H;
  for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
    const int j1 = idx / a.H;
    L.A[j1 * a.M + (idx - j1 * a.H)] = src[idx];
  }
  __syncthreads();
  rows_r2c(L.A, a.n1, a.H, a.M, a.p2, L.tw2, L.twr, L.slot2);
  lds_fft<T, false, true>(L.A, a.p1, a.M, a.M, 1, L.tw1);
  cplx<T>* dst = spec + ((long long)comp * a.n0 + x0) * a.n1 * a.M;
  const int tot2 = a.n1 * a.M;
  for (int idx = threadIdx.x; idx < tot2; idx += blockDim.x) dst[idx] = L.A[idx];
}

// One (x0, component) plane: x1 columns inverse -> x2 rows inverse -> real rows.
template <typename T, int NT>
__global__ void __launch_bounds__(NT) k_plane_inv(const cplx<T>* __restrict__ spec, T* __restrict__ out,
                                                   PlaneArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int x0 = blockIdx.x, comp = blockIdx.y;
  PlaneLds<T> L = carve(smem, a.n1, a, true);
  const cplx<T>* src = spec + ((long long)comp * a.n0 + x0) * a.n1 * a.M;
  const int tot2 = a.n1 * a.M;
  for (int idx = threadIdx.x; idx < tot2; idx += blockDim.x) L.A[idx] = src[idx];
  __syncthreads();
  lds_fft<T, true, true>(L.A, a.p1, a.M, a.M, 1, L.tw1);
  rows_c2r(L.A, a.n1, a.H, a.M, a.p2, L.tw2, L.twr, L.slot2);
  cplx<T>* dst = reinterpret_cast<cplx<T>*>(out + comp * a.N + (long long)x0 * a.n1 * a.n2);
  const int tot = a.n1 * a.H;
  for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
    const int j1 = idx / a.H;
    dst[idx] = L.A[j1 * a.M + (idx - j1 * a.H)];
  }
}

// Split path: `rb` consecutive rows (flat x0 * n1 + x1) per workgroup.
template <typename T>
__global__ void __launch_bounds__(256) k_rows_fwd(const T* __restrict__ in, cplx<T>* __restrict__ spec,
                                                  PlaneArgs<T> a, int rb) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int comp = blockIdx.y;
  const long long rows = (long long)a.n0 * a.n1;
  const long long r0 = (long long)blockIdx.x * rb;
  const int cnt = (int)((rows - r0) < rb ? (rows - r0) : rb);
  PlaneLds<T> L = carve(smem, rb, a, false);
  const cplx<T>* src = reinterpret_cast<const cplx<T>*>(in + comp * a.N) + r0 * a.H;
  for (int idx = threadIdx.x; idx < cnt * a.H; idx += blockDim.x) {
    const int r = idx / a.H;
    L.A[r * a.M + (idx - r * a.H)] = src[idx];
  }
  __syncthreads();
  rows_r2c(L.A, cnt, a.H, a.M, a.p2, L.tw2, L.twr, L.slot2);
  cplx<T>* dst = spec + ((long long)comp * rows + r0) * a.M;
  for (int idx = threadIdx.x; idx < cnt * a.M; idx += blockDim.x) dst[idx] = L.A[idx];
}

template <typename T>
__global__ void __launch_bounds__(256) k_rows_inv(const cplx<T>* __restrict__ spec, T* __restrict__ out,
                                                  PlaneArgs<T> a, int rb) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int comp = blockIdx.y;
  const long long rows = (long long)a.n0 * a.n1;
  const long long r0 = (long long)blockIdx.x * rb;
  const int cnt = (int)((rows - r0) < rb ? (rows - r0) : rb);
  PlaneLds<T> L = carve(smem, rb, a, false);
  const cplx<T>* src = spec + ((long long)comp * rows + r0) * a.M;
  for (int idx = threadIdx.x; idx < cnt * a.M; idx += blockDim.x) L.A[idx] = src[idx];
  __syncthreads();
  rows_c2r(L.A, cnt, a.H, a.M, a.p2, L.tw2, L.twr, L.slot2);
  cplx<T>* dst = reinterpret_cast<cplx<T>*>(out + comp * a.N) + r0 * a.H;
  for (int idx = threadIdx.x; idx < cnt * a.H; idx += blockDim.x) {
    const int r = idx / a.H;
    dst[idx] = L.A[r * a.M + (idx - r * a.H)];
  }
}

template <typename T>
struct PencilArgs {
  FftPlan pl;              // transform along the pencil
  int es;                  // element stride (complex units)
  int nin;                 // sequences per outer index (contiguous)
  long long outer_stride;  // complex units between outer indices
  int tb;                  // sequences per workgroup
  const cplx<T>* tw;
  // symbol (MODE 2, x0 pencils): slot q = k1slot * M + k2slot
  int M;
  T alpha;
  int s;
  int op;
  T scale;
  const T* ksq0;
  const T* ksq1;
  const T* ksq2;
  // MODE 3 (x0 pencils over half planes): sequence q pairs slot q of the even
  // half (at +0) with slot q of the odd half (at +hs); twx[k1 slot] = W_{n1}^{k1}
  // with k1 the half transform's frequency; ksq1 holds |k1|^2 for k1 (first
  // k1half entries) and k1 + n1/2 (next k1half) per slot
  int hs;
  int k1half;
  const cplx<T>* twx;
  int xcd_run;  // tiles per XCD run (xcd_grouped); 1: round-robin order
};

// Runs of consecutive units each XCD takes (xcd_grouped) where neighbouring
// units share cache lines: the two half planes of a plane where a row is not a
// whole number of 128-byte lines (180 FP32 values), and 8 pencil tiles where an
// x0 plane of the spectrum is not (180 x 216 x 180: 9828 complex values).  On
// aligned grids (128^3) the units keep the round-robin order, which measured
// 1 % faster there.
constexpr int kPlaneXcdRun = 2, kPencilXcdRun = 8;

// MODE 0: forward only, 1: inverse only, 2: forward, symbol, inverse.
template <typename T, int MODE, int NT>
__global__ void __launch_bounds__(NT) k_pencil(cplx<T>* __restrict__ spec, PencilArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = a.pl.n, tb = a.tb;
  cplx<T>* A = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* tw = A + n * tb;
  T* ksq0 = reinterpret_cast<T*>(tw + n);
  load_table(tw, a.tw, n);
  if (MODE == 2)
    for (int i = threadIdx.x; i < n; i += blockDim.x) ksq0[i] = a.ksq0[i];
  // runs of neighbouring tiles on one XCD where they share cache lines
  const int lin = a.xcd_run > 1 ? xcd_grouped(int(blockIdx.y * gridDim.x + blockIdx.x), int(gridDim.x * gridDim.y),
                                              a.xcd_run)
                                : int(blockIdx.y * gridDim.x + blockIdx.x);
  const int outer = lin / int(gridDim.x), q0 = (lin - outer * int(gridDim.x)) * tb;
  const int cnt = (a.nin - q0) < tb ? (a.nin - q0) : tb;
  cplx<T>* base = spec + outer * a.outer_stride + q0;
  for (int idx = threadIdx.x; idx < n * tb; idx += blockDim.x) {
    const int j = idx / tb, t = idx - j * tb;
    A[idx] = t < cnt ? base[(long long)j * a.es + t] : cplx<T>{T(0), T(0)};
  }
  __syncthreads();
  if (MODE != 1) lds_fft<T, false, true>(A, a.pl, tb, tb, 1, tw);
  if (MODE == 2) {
    for (int idx = threadIdx.x; idx < n * tb; idx += blockDim.x) {
      const int j = idx / tb, t = idx - j * tb;
      if (t < cnt) {
        const int q = q0 + t;
        const int s1 = q / a.M, s2 = q - s1 * a.M;
        const T base_sym = T(1) + a.alpha * (ksq0[j] + a.ksq1[s1] + a.ksq2[s2]);
        T pw = base_sym;
        for (int i = 1; i < a.s; ++i) pw *= base_sym;
        const T f = a.op == LDDMM_OP_K ? a.scale / pw : a.scale * pw;
        A[idx] = c_scale(A[idx], f);
      }
    }
    __syncthreads();
  }
  if (MODE != 0) lds_fft<T, true, true>(A, a.pl, tb, tb, 1, tw);
  for (int idx = threadIdx.x; idx < n * tb; idx += blockDim.x) {
    const int j = idx / tb, t = idx - j * tb;
    if (t < cnt) base[(long long)j * a.es + t] = A[idx];
  }
}

// --------------------------------------------------------------------------
// Compile-time variants for power-of-two lengths (same algorithm, same LDS
// layout and spectrum layout as the generic kernels above; every index is a
// constant shift and the stage loops unroll).
// --------------------------------------------------------------------------
// Stages I .. END-1 of the transform (in DIF order forward, DIT order inverse).
template <typename T, class P, bool INV, bool SEQ_FAST, int COUNT, int ES, int SS, int NT, int I = 0,
          int END = P::nf>
__device__ __forceinline__ void lds_fft_static(cplx<T>* buf, const cplx<T>* tw) {
  if constexpr (I < END) {
    constexpr int st = INV ? P::nf - 1 - I : I;
    constexpr int total = COUNT * (P::length(0) / P::radix(st));
#pragma unroll
    for (int b0 = 0; b0 < total; b0 += NT) {
      const int b = b0 + int(threadIdx.x);
      if (total % NT == 0 || b < total) fft_stage_item_static<T, P, st, INV, SEQ_FAST, COUNT, ES, SS>(buf, b, tw);
    }
    __syncthreads();
    lds_fft_static<T, P, INV, SEQ_FAST, COUNT, ES, SS, NT, I + 1, END>(buf, tw);
  }
}

template <typename T>
__device__ __forceinline__ T symbol_recip(T x) {
  return T(1) / x;
}
// FP32: the hardware reciprocal (1 ulp; the symbol's argument is >= 1)
template <>
__device__ __forceinline__ float symbol_recip<float>(float x) {
  return __builtin_amdgcn_rcpf(x);
}

// The last DIF stage (stride 1, no twiddles), the K/L symbol and the first DIT
// stage on the same R elements, in registers: between the forward and the
// inverse transform the spectrum does not go back to LDS.  Sequences are
// contiguous (SEQ_FAST, sequence stride 1, element stride ES); the calling
// thread's sequences all have the symbol part k12; ksq0 holds |k0|^2 per slot.
template <typename T, class P, int COUNT, int ES, int NT>
__device__ __forceinline__ void fused_symbol_stage(cplx<T>* buf, const T* ksq0, T k12, T alpha, int s, T scale,
                                                   bool inverse_op) {
  constexpr int st = P::nf - 1;
  constexpr int R = P::radix(st);
  static_assert(P::length(st) == R, "the last stage has stride 1");
  constexpr int total = COUNT * (P::length(0) / R);
#pragma unroll
  for (int b0 = 0; b0 < total; b0 += NT) {
    const int b = b0 + int(threadIdx.x);
    if (total % NT != 0 && b >= total) continue;
    const int u = b / COUNT, sq = b - u * COUNT;
    const int base = sq + u * R * ES;
    cplx<T> a[R];
#pragma unroll
    for (int q = 0; q < R; ++q) a[q] = buf[base + q * ES];
    Dft<T, R, -1>::run(a);
    // (1 + alpha |k|^2)^s with s = 2 (the usual exponent) unrolled; any s by the loop
    const T c12 = T(1) + alpha * k12;
    T pw[R];
#pragma unroll
    for (int q = 0; q < R; ++q) pw[q] = alpha * ksq0[u * R + q] + c12;
    if (s == 2) {
#pragma unroll
      for (int q = 0; q < R; ++q) pw[q] *= pw[q];
    } else {
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const T bq = pw[q];
        for (int i = 1; i < s; ++i) pw[q] *= bq;
      }
    }
#pragma unroll
    for (int q = 0; q < R; ++q) a[q] = c_scale(a[q], inverse_op ? scale * symbol_recip<T>(pw[q]) : scale * pw[q]);
    Dft<T, R, +1>::run(a);
#pragma unroll
    for (int q = 0; q < R; ++q) buf[base + q * ES] = a[q];
  }
  __syncthreads();
}

// Row post-processing: item k in 1..H/2 splits the pair (k, H - k); the last
// item also does k = 0, so a row takes H/2 items (whole rounds of the block
// for the usual sizes).  PACK stores the two real frequencies X[0] and X[H] of
// a row as one complex number X[0] + i X[H] in column 0 (column H is left
// alone): the columns k2 = 0 and k2 = N2/2 are real sequences along x1, and
// one complex transform of the packed column does both.
template <typename T, int H, int COUNT, int NT, bool PACK, int FIRST = 0>
__device__ __forceinline__ void rows_r2c_static(cplx<T>* A, const cplx<T>* tw2, const cplx<T>* twr, const int* slot2) {
  constexpr int M = H + 1;
  constexpr int KI = H / 2;
  lds_fft_static<T, typename PlanOf<H>::type, false, true, COUNT, 1, M, NT, FIRST>(A, tw2);
  constexpr int total = COUNT * KI;
#pragma unroll
  for (int i0 = 0; i0 < total; i0 += NT) {
    const int idx = i0 + int(threadIdx.x);
    if (total % NT != 0 && idx >= total) continue;
    const int k = 1 + idx / COUNT, r = idx - (k - 1) * COUNT;
    cplx<T>* row = A + r * M;
    const int sk = slot2[k], sm = slot2[H - k];
    const cplx<T> a = row[sk], b = row[sm];
    // even part e = (a + conj b) / 2, odd part o = (a - conj b) / 2
    const cplx<T> e = {T(0.5) * (a.x + b.x), T(0.5) * (a.y - b.y)};
    const cplx<T> o = {T(0.5) * (a.x - b.x), T(0.5) * (a.y + b.y)};
    const cplx<T> wo = c_mul(twr[k], o);
    // X[k] = e - i w o ;  X[H-k] = conj(e) - i conj(w o)
    row[sk] = {e.x + wo.y, e.y - wo.x};
    if (sm != sk) row[sm] = {e.x - wo.y, -e.y - wo.x};
    if (k == KI) {
      const cplx<T> z = row[0];
      if (PACK) {
        row[0] = {z.x + z.y, z.x - z.y};
      } else {
        row[0] = {z.x + z.y, T(0)};
        row[H] = {z.x - z.y, T(0)};
      }
    }
  }
  __syncthreads();
}

// Inverse of rows_r2c_static (times N2).  PACK: column 0 holds X[0] + i X[H]
// with X[0], X[H] real.
template <typename T, int H, int COUNT, int NT, bool PACK, int SKIP_LAST = 0>
__device__ __forceinline__ void rows_c2r_static(cplx<T>* A, const cplx<T>* tw2, const cplx<T>* twr, const int* slot2) {
  constexpr int M = H + 1;
  constexpr int KI = H / 2;
  constexpr int total = COUNT * KI;
#pragma unroll
  for (int i0 = 0; i0 < total; i0 += NT) {
    const int idx = i0 + int(threadIdx.x);
    if (total % NT != 0 && idx >= total) continue;
    const int k = 1 + idx / COUNT, r = idx - (k - 1) * COUNT;
    cplx<T>* row = A + r * M;
    const int sk = slot2[k], sm = slot2[H - k];
    const cplx<T> a = row[sk], b = row[sm];
    const cplx<T> p = {a.x + b.x, a.y - b.y};  // X[k] + conj X[H-k]
    const cplx<T> q = {a.x - b.x, a.y + b.y};  // X[k] - conj X[H-k]
    const cplx<T> t = c_mulc(q, twr[k]);       // conj(w) q
    row[sk] = {p.x - t.y, p.y + t.x};          // p + i t
    if (sm != sk) row[sm] = {p.x + t.y, -p.y + t.x};  // conj(p) + i conj(t)
    if (k == KI) {
      if (PACK) {
        const cplx<T> z = row[0];
        row[0] = {z.x + z.y, z.x - z.y};
      } else {
        const cplx<T> a0 = row[0], b0 = row[H];
        const cplx<T> p0 = {a0.x + b0.x, a0.y - b0.y};
        const cplx<T> q0 = {a0.x - b0.x, a0.y + b0.y};
        row[0] = {p0.x - q0.y, p0.y + q0.x};
      }
    }
  }
  __syncthreads();
  using P2 = typename PlanOf<H>::type;
  lds_fft_static<T, P2, true, true, COUNT, 1, M, NT, 0, P2::nf - SKIP_LAST>(A, tw2);
}

// First DIF stage of COUNT rows of length H straight from global memory (row s
// at src + s * RS, RS = H for consecutive rows), in two halves: rows_first_load brings a thread's inputs into
// registers and rows_first_compute transforms them into LDS rows of stride H + 1,
// so the loads of the next plane can be in flight while the current one is
// transformed.  Lanes walk a row's butterflies first, so each load is a
// contiguous run of H / R elements.
template <typename T, int H, int COUNT, int NT>
struct RowStageIn {
  using P2 = typename PlanOf<H>::type;
  static constexpr int R = P2::radix(0), S = H / R, total = COUNT * S, iters = (total + NT - 1) / NT;
  cplx<T> v[iters][R];
};

template <typename T, int H, int COUNT, int NT, int RS = H>
__device__ __forceinline__ void rows_first_load(RowStageIn<T, H, COUNT, NT>& in, const cplx<T>* __restrict__ src) {
  using I = RowStageIn<T, H, COUNT, NT>;
#pragma unroll
  for (int it = 0; it < I::iters; ++it) {
    const int b = it * NT + int(threadIdx.x);
    if (I::total % NT != 0 && b >= I::total) continue;
    const int r = b / I::S, j = b - r * I::S;
#pragma unroll
    for (int q = 0; q < I::R; ++q) in.v[it][q] = src[r * RS + j + q * I::S];
  }
}

template <typename T, int H, int COUNT, int NT>
__device__ __forceinline__ void rows_first_compute(cplx<T>* A, RowStageIn<T, H, COUNT, NT>& in, const cplx<T>* tw) {
  using I = RowStageIn<T, H, COUNT, NT>;
  constexpr int R = I::R, S = I::S, M = H + 1;
#pragma unroll
  for (int it = 0; it < I::iters; ++it) {
    const int b = it * NT + int(threadIdx.x);
    if (I::total % NT != 0 && b >= I::total) continue;
    const int r = b / S, j = b - r * S;
    cplx<T>* v = in.v[it];
    Dft<T, R, -1>::run(v);
    A[r * M + j] = v[0];
    if constexpr (S > 1) {
      cplx<T> w[R];
      twiddle_powers<T, R>(w, j, 1, tw);
#pragma unroll
      for (int q = 1; q < R; ++q) A[r * M + j + q * S] = c_mul(v[q], w[q]);
    } else {
#pragma unroll
      for (int q = 1; q < R; ++q) A[r * M + j + q * S] = v[q];
    }
  }
}

// Store with the non-temporal hint.  The inverse plane pass writes a field that
// only the next kernel reads, so its lines need not stay in the caches; with the
// hint the pass measured 7-10 % faster and the whole Hessian-vector product
// 0.5-2.5 % faster (the other passes' loads and stores measured slower with it).
template <typename T>
__device__ __forceinline__ void store_streaming(cplx<T>* p, const cplx<T>& v) {
  typedef T pair __attribute__((ext_vector_type(2)));
  const pair x = {v.x, v.y};
  __builtin_nontemporal_store(x, reinterpret_cast<pair*>(p));
}

// Last DIT stage of COUNT rows (the inverse of the first row stage) straight to
// global memory (row s at dst + s * RS), with streaming stores.  ADD: dst = add +
// scale * (result), the addend (same layout as dst) loaded before the butterfly
// so its latency overlaps.
template <typename T, int H, int COUNT, int NT, bool ADD = false, int RS = H>
__device__ __forceinline__ void rows_last_stage_global(const cplx<T>* A, cplx<T>* __restrict__ dst,
                                                       const cplx<T>* tw, const cplx<T>* __restrict__ add = nullptr,
                                                       T scale = T(0)) {
  using P2 = typename PlanOf<H>::type;
  constexpr int R = P2::radix(0), S = H / R, M = H + 1;
  constexpr int total = COUNT * S;
#pragma unroll
  for (int b0 = 0; b0 < total; b0 += NT) {
    const int b = b0 + int(threadIdx.x);
    if (total % NT != 0 && b >= total) continue;
    const int r = b / S, j = b - r * S;
    cplx<T> ad[ADD ? R : 1];
    if constexpr (ADD) {
#pragma unroll
      for (int q = 0; q < R; ++q) ad[q] = add[r * RS + j + q * S];
    }
    cplx<T> v[R];
    v[0] = A[r * M + j];
    if constexpr (S > 1) {
      cplx<T> w[R];
      twiddle_powers<T, R>(w, j, 1, tw);
#pragma unroll
      for (int q = 1; q < R; ++q) v[q] = c_mulc(A[r * M + j + q * S], w[q]);
    } else {
#pragma unroll
      for (int q = 1; q < R; ++q) v[q] = A[r * M + j + q * S];
    }
    Dft<T, R, +1>::run(v);
    if constexpr (ADD) {
#pragma unroll
      for (int q = 0; q < R; ++q) v[q] = {ad[q].x + scale * v[q].x, ad[q].y + scale * v[q].y};
    }
#pragma unroll
    for (int q = 0; q < R; ++q) store_streaming(dst + (r * RS + j + q * S), v[q]);
  }
}

template <typename T, int H, int N1>
__device__ __forceinline__ PlaneLds<T> carve_static(unsigned char* smem, int rows, const PlaneArgs<T>& a,
                                                    bool with_tw1) {
  constexpr int M = H + 1;
  PlaneLds<T> L;
  L.A = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* p = L.A + rows * M;
  L.tw1 = p;
  if (with_tw1) p += N1;
  L.tw2 = p;
  p += H;
  L.twr = p;
  p += H / 2 + 1;
  L.slot2 = reinterpret_cast<int*>(p);
  for (int i = threadIdx.x; i < N1 && with_tw1; i += blockDim.x) L.tw1[i] = a.tw1[i];
  for (int i = threadIdx.x; i < H; i += blockDim.x) L.tw2[i] = a.tw2[i];
  for (int i = threadIdx.x; i <= H / 2; i += blockDim.x) L.twr[i] = a.twr[i];
  for (int i = threadIdx.x; i <= H; i += blockDim.x) L.slot2[i] = a.slot2[i];
  return L;
}

// Fused plane kernels.  The k2 = 0 and k2 = N2/2 columns travel packed in
// column 0 through the x1 transform (H columns instead of H + 1) and are split
// apart before the store: with Z the transform of X[0] + i X[N2/2] along x1,
// the two spectra are (Z[k] + conj Z[-k]) / 2 and (Z[k] - conj Z[-k]) / 2i.
//
// Plane p of a call is component p / n0 at x0 = p % n0.  XS = 2 (half planes):
// unit p is the even (h = 0) or odd (h = 1) x1 rows of plane p / 2, N1 of them,
// a transform of length N1 along x1 whose spectrum the x0 pencil pass merges
// with the other half's (the first radix-2 step of the length-2 N1 transform,
// by decimation in x1); units of one plane are consecutive in the spectrum, so
// the layout is [component][x0][h][k1 slot][k2 slot].  With XS = 1 every unit
// is a whole plane.  WALK = false: one unit per workgroup, grid (XS n0,
// components).  WALK = true: a 1D grid of G
// workgroups, workgroup g taking planes g, g + G, g + 2G, ...; the inputs of the
// next plane's first stage are loaded into registers while the current plane
// is transformed and stored, so with fewer workgroups than planes the memory
// phases of consecutive planes overlap inside one workgroup.
template <typename T, int H, int N1, int NT, bool WALK, int XS = 1>
__global__ void __launch_bounds__(NT) k_plane_fwd_s(const T* __restrict__ in, cplx<T>* __restrict__ spec,
                                                    PlaneArgs<T> a) {
  using P1 = typename PlanOf<N1>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int M = H + 1;
  PlaneLds<T> L = carve_static<T, H, N1>(smem, N1, a, true);
  const long long plane_len = (long long)N1 * XS * 2 * H;  // reals of one (x1, x2) plane
  const int per_comp = a.n0 * XS;
  auto plane_src = [&](int q) {
    const int comp = q / per_comp, r = q - comp * per_comp, x0 = r / XS, h = r - x0 * XS;
    return reinterpret_cast<const cplx<T>*>(in + comp * a.N + x0 * plane_len + h * 2 * H);
  };
  // one unit per workgroup; where rows share cache lines, the even and odd rows
  // of a plane on one XCD
  int p = WALK              ? int(blockIdx.x)
          : a.xcd_run > 1 ? xcd_grouped(int(blockIdx.y) * per_comp + int(blockIdx.x), int(gridDim.x * gridDim.y),
                                        a.xcd_run)
                            : int(blockIdx.y) * per_comp + int(blockIdx.x);
  // the first plane's row twiddles come from global memory: the LDS copy is
  // complete only after the first barrier
  const cplx<T>* tw_first = a.tw2;
  RowStageIn<T, H, N1, NT> rin;
  rows_first_load<T, H, N1, NT, XS * H>(rin, plane_src(p));
  for (;;) {
    rows_first_compute<T, H, N1, NT>(L.A, rin, tw_first);
    __syncthreads();
    const int pn = WALK ? p + int(gridDim.x) : a.planes;
    if (WALK && pn < a.planes) rows_first_load<T, H, N1, NT, XS * H>(rin, plane_src(pn));
    rows_r2c_static<T, H, N1, NT, true, 1>(L.A, L.tw2, L.twr, L.slot2);
    lds_fft_static<T, P1, false, true, H, M, 1, NT, 0, P1::nf - 1>(L.A, L.tw1);
    // Last column stage (stride 1, no twiddles) straight to the spectrum:
    // consecutive threads take consecutive columns, so each store is contiguous.
    // The packed column 0 goes back to LDS for the split below.
    cplx<T>* dst = spec + (long long)p * (N1 * M);
    {
      constexpr int R = P1::radix(P1::nf - 1);
      constexpr int total = H * (N1 / R);
#pragma unroll
      for (int b0 = 0; b0 < total; b0 += NT) {
        const int b = b0 + int(threadIdx.x);
        if (total % NT != 0 && b >= total) continue;
        const int u = b / H, col = b - u * H;
        const int base = u * R * M + col;
        cplx<T> v[R];
#pragma unroll
        for (int q = 0; q < R; ++q) v[q] = L.A[base + q * M];
        Dft<T, R, -1>::run(v);
        if (col == 0) {
#pragma unroll
          for (int q = 0; q < R; ++q) L.A[base + q * M] = v[q];
        } else {
#pragma unroll
          for (int q = 0; q < R; ++q) dst[base + q * M] = v[q];
        }
      }
    }
    __syncthreads();
    for (int k = threadIdx.x; k <= N1 / 2; k += NT) {
      const int sk = slot_of<P1>(k), sm = slot_of<P1>(k == 0 ? 0 : N1 - k);
      const cplx<T> zk = L.A[sk * M], zm = L.A[sm * M];
      const cplx<T> lo = {T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y)};
      const cplx<T> hi = {T(0.5) * (zk.y + zm.y), T(0.5) * (zm.x - zk.x)};
      dst[sk * M] = lo;
      dst[sk * M + H] = hi;
      dst[sm * M] = c_conj(lo);
      dst[sm * M + H] = c_conj(hi);
    }
    if (!WALK || pn >= a.planes) break;
    __syncthreads();  // column 0 is read above before the next plane overwrites the LDS
    p = pn;
    tw_first = L.tw2;
  }
}

// Inputs of the first inverse column stage (the last DIF stage of the x1 plan:
// stride 1, no twiddles) in registers; column-0 butterflies also hold column H,
// which is packed into column 0 as X[0] + i X[N2/2].
template <typename T, int H, int N1, int NT>
struct ColStageIn {
  using P1 = typename PlanOf<N1>::type;
  static constexpr int R = P1::radix(P1::nf - 1), total = H * (N1 / R), iters = (total + NT - 1) / NT;
  cplx<T> v[iters][R];
  cplx<T> hi[iters][R];
};

template <typename T, int H, int N1, int NT>
__device__ __forceinline__ void cols_first_load(ColStageIn<T, H, N1, NT>& in, const cplx<T>* __restrict__ src) {
  using I = ColStageIn<T, H, N1, NT>;
  constexpr int R = I::R, M = H + 1;
#pragma unroll
  for (int it = 0; it < I::iters; ++it) {
    const int b = it * NT + int(threadIdx.x);
    if (I::total % NT != 0 && b >= I::total) continue;
    const int u = b / H, col = b - u * H;
    const int base = u * R * M + col;
#pragma unroll
    for (int q = 0; q < R; ++q) in.v[it][q] = src[base + q * M];
    if (col == 0) {
#pragma unroll
      for (int q = 0; q < R; ++q) in.hi[it][q] = src[base + q * M + H];
    }
  }
}

template <typename T, int H, int N1, int NT>
__device__ __forceinline__ void cols_first_compute(cplx<T>* A, ColStageIn<T, H, N1, NT>& in) {
  using I = ColStageIn<T, H, N1, NT>;
  constexpr int R = I::R, M = H + 1;
#pragma unroll
  for (int it = 0; it < I::iters; ++it) {
    const int b = it * NT + int(threadIdx.x);
    if (I::total % NT != 0 && b >= I::total) continue;
    const int u = b / H, col = b - u * H;
    const int base = u * R * M + col;
    cplx<T>* v = in.v[it];
    if (col == 0) {
#pragma unroll
      for (int q = 0; q < R; ++q) v[q] = {v[q].x - in.hi[it][q].y, v[q].y + in.hi[it][q].x};
    }
    Dft<T, R, +1>::run(v);
#pragma unroll
    for (int q = 0; q < R; ++q) A[base + q * M] = v[q];
  }
}

template <typename T, int H, int N1, int NT>
__device__ __forceinline__ void cols_first_stage_global(cplx<T>* A, const cplx<T>* __restrict__ src) {
  using I = ColStageIn<T, H, N1, NT>;
  constexpr int R = I::R, M = H + 1;
#pragma unroll
  for (int it = 0; it < I::iters; ++it) {
    const int b = it * NT + int(threadIdx.x);
    if (I::total % NT != 0 && b >= I::total) continue;
    const int u = b / H, col = b - u * H;
    const int base = u * R * M + col;
    cplx<T> v[R];
#pragma unroll
    for (int q = 0; q < R; ++q) v[q] = src[base + q * M];
    if (col == 0) {
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const cplx<T> hi = src[base + q * M + H];
        v[q] = {v[q].x - hi.y, v[q].y + hi.x};
      }
    }
    Dft<T, R, +1>::run(v);
#pragma unroll
    for (int q = 0; q < R; ++q) A[base + q * M] = v[q];
  }
}

template <typename T, int H, int N1, int NT, bool WALK, bool ADD = false, int XS = 1>
__global__ void __launch_bounds__(NT) k_plane_inv_s(const cplx<T>* __restrict__ spec, T* __restrict__ out,
                                                    PlaneArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int M = H + 1;
  using P1 = typename PlanOf<N1>::type;
  PlaneLds<T> L = carve_static<T, H, N1>(smem, N1, a, true);
  const long long plane_len = (long long)N1 * XS * 2 * H;
  const int per_comp = a.n0 * XS;
  int p = WALK              ? int(blockIdx.x)
          : a.xcd_run > 1 ? xcd_grouped(int(blockIdx.y) * per_comp + int(blockIdx.x), int(gridDim.x * gridDim.y),
                                        a.xcd_run)
                            : int(blockIdx.y) * per_comp + int(blockIdx.x);
  // first column stage straight from the spectrum, consecutive threads on
  // consecutive columns; one plane per workgroup loads and transforms in one go
  // (fewer live registers), the walk keeps the next plane's inputs in registers
  ColStageIn<T, H, N1, NT> cin;
  if (WALK) cols_first_load<T, H, N1, NT>(cin, spec + (long long)p * (N1 * M));
  for (;;) {
    if (WALK)
      cols_first_compute<T, H, N1, NT>(L.A, cin);
    else
      cols_first_stage_global<T, H, N1, NT>(L.A, spec + (long long)p * (N1 * M));
    __syncthreads();
    const int pn = WALK ? p + int(gridDim.x) : a.planes;
    if (WALK && pn < a.planes) cols_first_load<T, H, N1, NT>(cin, spec + (long long)pn * (N1 * M));
    lds_fft_static<T, P1, true, true, H, M, 1, NT, 1>(L.A, L.tw1);
    rows_c2r_static<T, H, N1, NT, true, 1>(L.A, L.tw2, L.twr, L.slot2);
    const int comp = p / per_comp, r = p - comp * per_comp, x0 = r / XS, h = r - x0 * XS;
    const long long off = comp * a.N + x0 * plane_len + h * 2 * H;
    cplx<T>* dst = reinterpret_cast<cplx<T>*>(out + off);
    if constexpr (ADD)
      rows_last_stage_global<T, H, N1, NT, true, XS * H>(L.A, dst, L.tw2,
                                                         reinterpret_cast<const cplx<T>*>(a.add + off), a.add_scale);
    else
      rows_last_stage_global<T, H, N1, NT, false, XS * H>(L.A, dst, L.tw2);
    if (!WALK || pn >= a.planes) break;
    __syncthreads();  // the last row stage reads the LDS the next plane overwrites
    p = pn;
  }
}

template <typename T, int H, int RB, int NT>
__global__ void __launch_bounds__(NT) k_rows_fwd_s(const T* __restrict__ in, cplx<T>* __restrict__ spec,
                                                   PlaneArgs<T> a, int) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int M = H + 1;
  const int comp = blockIdx.y;
  const long long rows = (long long)a.n0 * a.n1;  // a multiple of RB (checked on the host)
  const long long r0 = (long long)blockIdx.x * RB;
  PlaneLds<T> L = carve_static<T, H, 1>(smem, RB, a, false);
  const cplx<T>* src = reinterpret_cast<const cplx<T>*>(in + comp * a.N) + r0 * H;
#pragma unroll
  for (int i0 = 0; i0 < RB * H; i0 += NT) {
    const int idx = i0 + int(threadIdx.x);
    if ((RB * H) % NT != 0 && idx >= RB * H) continue;
    const int r = idx / H;
    L.A[r * M + (idx - r * H)] = src[idx];
  }
  __syncthreads();
  rows_r2c_static<T, H, RB, NT, false>(L.A, L.tw2, L.twr, L.slot2);
  cplx<T>* dst = spec + ((long long)comp * rows + r0) * M;
  for (int idx = threadIdx.x; idx < RB * M; idx += NT) dst[idx] = L.A[idx];
}

template <typename T, int H, int RB, int NT>
__global__ void __launch_bounds__(NT) k_rows_inv_s(const cplx<T>* __restrict__ spec, T* __restrict__ out,
                                                   PlaneArgs<T> a, int) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int M = H + 1;
  const int comp = blockIdx.y;
  const long long rows = (long long)a.n0 * a.n1;
  const long long r0 = (long long)blockIdx.x * RB;
  PlaneLds<T> L = carve_static<T, H, 1>(smem, RB, a, false);
  const cplx<T>* src = spec + ((long long)comp * rows + r0) * M;
  for (int idx = threadIdx.x; idx < RB * M; idx += NT) L.A[idx] = src[idx];
  __syncthreads();
  rows_c2r_static<T, H, RB, NT, false>(L.A, L.tw2, L.twr, L.slot2);
  cplx<T>* dst = reinterpret_cast<cplx<T>*>(out + comp * a.N) + r0 * H;
#pragma unroll
  for (int i0 = 0; i0 < RB * H; i0 += NT) {
    const int idx = i0 + int(threadIdx.x);
    if ((RB * H) % NT != 0 && idx >= RB * H) continue;
    const int r = idx / H;
    dst[idx] = L.A[r * M + (idx - r * H)];
  }
}

// Pencils along an axis of power-of-two length N, TB per workgroup; each thread
// keeps one sequence t = tid % TB, so the symbol's (k1, k2) part is looked up
// once per sequence.  MODE 3 is MODE 2 over half planes: TB pairs per
// workgroup, the pair's two half-plane spectra Y0 (even x1 rows) and Y1 (odd)
// become the pencils of k1 and k1 + n1/2 on load (X = Y0 +- W_{n1}^{k1} Y1), and
// go back to halves on store (Y0 = Xa + Xb, Y1 = conj(W_{n1}^{k1}) (Xa - Xb)), so
// the LDS holds TS = 2 TB sequences.
template <typename T, int MODE, int N, int TB, int NT>
__global__ void __launch_bounds__(NT) k_pencil_s(cplx<T>* __restrict__ spec, PencilArgs<T> a) {
  constexpr bool PAIR = MODE == 3;
  constexpr int TS = PAIR ? 2 * TB : TB;
  static_assert(NT % TS == 0, "threads must cover whole rows of the tile");
  using PN = typename PlanOf<N>::type;
  static_assert(PN::nf >= 2, "first and last stages are fused with different neighbours");
  extern __shared__ __align__(16) unsigned char smem[];
  cplx<T>* A = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* tw = A + N * TS;
  T* ksq0 = reinterpret_cast<T*>(tw + N);
  T* ksq12 = ksq0 + N;
  for (int i = threadIdx.x; i < N; i += NT) tw[i] = a.tw[i];
  // runs of neighbouring tiles on one XCD where they share cache lines
  const int lin = a.xcd_run > 1 ? xcd_grouped(int(blockIdx.y * gridDim.x + blockIdx.x), int(gridDim.x * gridDim.y),
                                              a.xcd_run)
                                : int(blockIdx.y * gridDim.x + blockIdx.x);
  const int comp = lin / int(gridDim.x), q0 = (lin - comp * int(gridDim.x)) * TB;
  const int cnt = (a.nin - q0) < TB ? (a.nin - q0) : TB;
  if (MODE >= 2) {
    for (int i = threadIdx.x; i < N; i += NT) ksq0[i] = a.ksq0[i];
    if (threadIdx.x < TS) {
      const int u = int(threadIdx.x), hb = PAIR ? u / TB : 0;
      const int q = q0 + u - hb * TB;
      const int s1 = q / a.M, s2 = q - s1 * a.M;
      ksq12[u] = q < a.nin ? a.ksq1[hb * a.k1half + s1] + a.ksq2[s2] : T(0);
    }
  }
  const int t = int(threadIdx.x) % TB;
  cplx<T>* base = spec + comp * a.outer_stride + q0;
  const bool live = t < cnt;
  constexpr int R0 = PN::radix(0), S0 = N / R0;  // first DIF / last DIT stage
  constexpr int total0 = TB * S0;
  cplx<T> wx = {T(1), T(0)};  // W_{n1}^{k1} of the thread's pair
  if (PAIR && live) wx = a.twx[(q0 + t) / a.M];
  if (PAIR) {
    // first DIF stage of both pencils of a pair straight from the two halves
#pragma unroll
    for (int b0 = 0; b0 < total0; b0 += NT) {
      const int b = b0 + int(threadIdx.x);
      if (total0 % NT != 0 && b >= total0) continue;
      const int j = b / TB;
      cplx<T> va[R0], vb[R0];
#pragma unroll
      for (int q = 0; q < R0; ++q) {
        const long long o = (long long)(j + q * S0) * a.es + t;
        const cplx<T> y0 = live ? base[o] : cplx<T>{T(0), T(0)};
        const cplx<T> y1 = live ? base[o + a.hs] : cplx<T>{T(0), T(0)};
        const cplx<T> wy = c_mul(wx, y1);
        va[q] = {y0.x + wy.x, y0.y + wy.y};
        vb[q] = {y0.x - wy.x, y0.y - wy.y};
      }
      Dft<T, R0, -1>::run(va);
      Dft<T, R0, -1>::run(vb);
      A[j * TS + t] = va[0];
      A[j * TS + TB + t] = vb[0];
      cplx<T> w[R0];
      twiddle_powers<T, R0>(w, j, 1, a.tw);
#pragma unroll
      for (int q = 1; q < R0; ++q) {
        A[(j + q * S0) * TS + t] = c_mul(va[q], w[q]);
        A[(j + q * S0) * TS + TB + t] = c_mul(vb[q], w[q]);
      }
    }
  } else if (MODE != 1) {
    // first DIF stage straight from the spectrum: consecutive lanes take
    // consecutive pencils (contiguous); twiddles from global memory (the LDS copy
    // is complete only after the barrier)
#pragma unroll
    for (int b0 = 0; b0 < total0; b0 += NT) {
      const int b = b0 + int(threadIdx.x);
      if (total0 % NT != 0 && b >= total0) continue;
      const int j = b / TB;
      cplx<T> v[R0];
#pragma unroll
      for (int q = 0; q < R0; ++q) v[q] = live ? base[(long long)(j + q * S0) * a.es + t] : cplx<T>{T(0), T(0)};
      Dft<T, R0, -1>::run(v);
      A[j * TB + t] = v[0];
      cplx<T> w[R0];
      twiddle_powers<T, R0>(w, j, 1, a.tw);
#pragma unroll
      for (int q = 1; q < R0; ++q) A[(j + q * S0) * TB + t] = c_mul(v[q], w[q]);
    }
  } else {
#pragma unroll
    for (int b0 = 0; b0 < N * TB; b0 += NT) {
      const int idx = b0 + int(threadIdx.x), j = idx / TB;
      if ((N * TB) % NT != 0 && idx >= N * TB) continue;
      A[idx] = live ? base[(long long)j * a.es + t] : cplx<T>{T(0), T(0)};
    }
  }
  __syncthreads();
  if (MODE >= 2) {
    lds_fft_static<T, PN, false, true, TS, TS, 1, NT, 1, PN::nf - 1>(A, tw);
    fused_symbol_stage<T, PN, TS, TS, NT>(A, ksq0, ksq12[int(threadIdx.x) % TS], a.alpha, a.s, a.scale,
                                          a.op == LDDMM_OP_K);
    lds_fft_static<T, PN, true, true, TS, TS, 1, NT, 1, PN::nf - 1>(A, tw);
  } else if (MODE == 0) {
    lds_fft_static<T, PN, false, true, TB, TB, 1, NT, 1>(A, tw);
  } else {
    lds_fft_static<T, PN, true, true, TB, TB, 1, NT, 0, PN::nf - 1>(A, tw);
  }
  if (PAIR) {
    // last DIT stage of both pencils, then back to the two halves
#pragma unroll
    for (int b0 = 0; b0 < total0; b0 += NT) {
      const int b = b0 + int(threadIdx.x);
      if (total0 % NT != 0 && b >= total0) continue;
      const int j = b / TB;
      cplx<T> va[R0], vb[R0], w[R0];
      twiddle_powers<T, R0>(w, j, 1, tw);
      va[0] = A[j * TS + t];
      vb[0] = A[j * TS + TB + t];
#pragma unroll
      for (int q = 1; q < R0; ++q) {
        va[q] = c_mulc(A[(j + q * S0) * TS + t], w[q]);
        vb[q] = c_mulc(A[(j + q * S0) * TS + TB + t], w[q]);
      }
      Dft<T, R0, +1>::run(va);
      Dft<T, R0, +1>::run(vb);
      if (live) {
#pragma unroll
        for (int q = 0; q < R0; ++q) {
          const long long o = (long long)(j + q * S0) * a.es + t;
          base[o] = {va[q].x + vb[q].x, va[q].y + vb[q].y};
          base[o + a.hs] = c_mulc(cplx<T>{va[q].x - vb[q].x, va[q].y - vb[q].y}, wx);
        }
      }
    }
  } else if (MODE != 0) {
    // last DIT stage straight to the spectrum
#pragma unroll
    for (int b0 = 0; b0 < total0; b0 += NT) {
      const int b = b0 + int(threadIdx.x);
      if (total0 % NT != 0 && b >= total0) continue;
      const int j = b / TB;
      cplx<T> v[R0], w[R0];
      twiddle_powers<T, R0>(w, j, 1, tw);
      v[0] = A[j * TB + t];
#pragma unroll
      for (int q = 1; q < R0; ++q) v[q] = c_mulc(A[(j + q * S0) * TB + t], w[q]);
      Dft<T, R0, +1>::run(v);
      if (live) {
#pragma unroll
        for (int q = 0; q < R0; ++q) base[(long long)(j + q * S0) * a.es + t] = v[q];
      }
    }
  } else if (live) {
#pragma unroll
    for (int b0 = 0; b0 < N * TB; b0 += NT) {
      const int idx = b0 + int(threadIdx.x), j = idx / TB;
      if ((N * TB) % NT != 0 && idx >= N * TB) continue;
      base[(long long)j * a.es + t] = A[idx];
    }
  }
}

// --------------------------------------------------------------------------
// Host side
// --------------------------------------------------------------------------
namespace {

template <typename T>
std::vector<cplx<T>> twiddles(int n, int count) {
  std::vector<cplx<T>> t(count);
  for (int m = 0; m < count; ++m) {
    const double ang = -2.0 * M_PI * double(m) / double(n);
    t[m] = {T(std::cos(ang)), T(std::sin(ang))};
  }
  return t;
}

// Host image of the transform tables: each table at a 256-byte aligned offset
// of one blob, uploaded with a single copy (into a context allocation or a
// caller-provided device region).
struct TableBlob {
  std::vector<unsigned char> host;
  template <typename V>
  size_t put(const std::vector<V>& src) {
    const size_t off = (host.size() + 255) & ~size_t(255);
    host.resize(off + src.size() * sizeof(V));
    std::memcpy(host.data() + off, src.data(), src.size() * sizeof(V));
    return off;
  }
};

int fold_sq(int k, int n) {
  const int a = k <= n - k ? k : n - k;
  return a * a;
}

bool allowed_threads(int t) { return t == 256 || t == 512 || t == 1024; }


// Kernel entry points chosen per plan (compile-time variants where instantiated).
template <typename T>
using PlaneFwdFn = void (*)(const T*, cplx<T>*, PlaneArgs<T>);
template <typename T>
using PlaneInvFn = void (*)(const cplx<T>*, T*, PlaneArgs<T>);
template <typename T>
using RowsFwdFn = void (*)(const T*, cplx<T>*, PlaneArgs<T>, int);
template <typename T>
using RowsInvFn = void (*)(const cplx<T>*, T*, PlaneArgs<T>, int);
template <typename T>
using PencilFn = void (*)(cplx<T>*, PencilArgs<T>);

enum { KF_PLANE_FWD, KF_PLANE_INV, KF_ROWS_FWD, KF_ROWS_INV, KF_PENCIL0, KF_PENCIL1F, KF_PENCIL1I, KF_PLANE_INV_ADD };

template <typename T, int NT, bool WALK>
void plane_static(const FftPlan& p2, const FftPlan& p1, void*& f, void*& i, void*& ia) {
  const int H = p2.n, N1 = p1.n;
// The walk keeps a plane's first-stage inputs in registers: not offered for
// planes larger than 64 x 128 complex, where they would spill.
#define LDDMM_PLANE_CASE(h, n1)                                                                   \
  if constexpr (!WALK || (h) * (n1) <= 64 * 128)                                                  \
    if (H == h && N1 == n1 && plan_matches<PlanOf<h>::type>(p2) && plan_matches<PlanOf<n1>::type>(p1)) { \
      f = (void*)(PlaneFwdFn<T>)k_plane_fwd_s<T, h, n1, NT, WALK>;                                \
      i = (void*)(PlaneInvFn<T>)k_plane_inv_s<T, h, n1, NT, WALK, false>;                         \
      ia = (void*)(PlaneInvFn<T>)k_plane_inv_s<T, h, n1, NT, WALK, true>;                         \
      return;                                                                                     \
    }
  LDDMM_PLANE_CASE(8, 16)
  LDDMM_PLANE_CASE(16, 32)
  LDDMM_PLANE_CASE(32, 64)
  LDDMM_PLANE_CASE(64, 128)
  LDDMM_PLANE_CASE(40, 80)
  LDDMM_PLANE_CASE(48, 96)
  LDDMM_PLANE_CASE(56, 112)
  LDDMM_PLANE_CASE(90, 216)
#undef LDDMM_PLANE_CASE
  f = i = ia = nullptr;
}

// Half planes (XS = 2): N1 is half the x1 length; one unit per workgroup.
template <typename T, int NT>
void plane_static_halves(const FftPlan& p2, const FftPlan& p1h, void*& f, void*& i, void*& ia) {
  const int H = p2.n, N1 = p1h.n;
#define LDDMM_HALVES_CASE(h, n1)                                                                   \
  if (H == h && N1 == n1 && plan_matches<PlanOf<h>::type>(p2) && plan_matches<PlanOf<n1>::type>(p1h)) { \
    f = (void*)(PlaneFwdFn<T>)k_plane_fwd_s<T, h, n1, NT, false, 2>;                               \
    i = (void*)(PlaneInvFn<T>)k_plane_inv_s<T, h, n1, NT, false, false, 2>;                        \
    ia = (void*)(PlaneInvFn<T>)k_plane_inv_s<T, h, n1, NT, false, true, 2>;                        \
    return;                                                                                        \
  }
  LDDMM_HALVES_CASE(8, 8)
  LDDMM_HALVES_CASE(16, 16)
  LDDMM_HALVES_CASE(32, 32)
  LDDMM_HALVES_CASE(64, 64)
  LDDMM_HALVES_CASE(128, 128)
  LDDMM_HALVES_CASE(40, 40)
  LDDMM_HALVES_CASE(48, 48)
  LDDMM_HALVES_CASE(56, 56)
  LDDMM_HALVES_CASE(90, 108)
#undef LDDMM_HALVES_CASE
  f = i = ia = nullptr;
}

// x0 pencils with the symbol over half planes, TBP pairs per workgroup
template <typename T>
void* pencil_static_pairs(const FftPlan& pl, int TBP) {
  const int N = pl.n;
#define LDDMM_PAIRS_N(n)                                                                 \
  if (N == n && plan_matches<PlanOf<n>::type>(pl)) {                                     \
    if (TBP == 4) return (void*)(PencilFn<T>)k_pencil_s<T, 3, n, 4, 256>;                \
    if (TBP == 8) return (void*)(PencilFn<T>)k_pencil_s<T, 3, n, 8, 256>;                \
    if (TBP == 16) return (void*)(PencilFn<T>)k_pencil_s<T, 3, n, 16, 256>;              \
  }
  LDDMM_PAIRS_N(16)
  LDDMM_PAIRS_N(32)
  LDDMM_PAIRS_N(64)
  LDDMM_PAIRS_N(128)
  LDDMM_PAIRS_N(256)
  LDDMM_PAIRS_N(80)
  LDDMM_PAIRS_N(96)
  LDDMM_PAIRS_N(112)
  LDDMM_PAIRS_N(180)
#undef LDDMM_PAIRS_N
  return nullptr;
}

template <typename T, int MODE>
void* pencil_static(const FftPlan& pl, int TB) {
  const int N = pl.n;
#define LDDMM_PENCIL_N(n)                                                                \
  if (N == n && plan_matches<PlanOf<n>::type>(pl)) {                                     \
    if (TB == 8) return (void*)(PencilFn<T>)k_pencil_s<T, MODE, n, 8, 256>;              \
    if (TB == 16) return (void*)(PencilFn<T>)k_pencil_s<T, MODE, n, 16, 256>;            \
    if (TB == 32) return (void*)(PencilFn<T>)k_pencil_s<T, MODE, n, 32, 256>;            \
  }
  LDDMM_PENCIL_N(16)
  LDDMM_PENCIL_N(32)
  LDDMM_PENCIL_N(64)
  LDDMM_PENCIL_N(128)
  LDDMM_PENCIL_N(256)
  LDDMM_PENCIL_N(80)
  LDDMM_PENCIL_N(96)
  LDDMM_PENCIL_N(112)
  LDDMM_PENCIL_N(180)
  LDDMM_PENCIL_N(216)
#undef LDDMM_PENCIL_N
  return nullptr;
}

template <typename T>
void rows_static(const FftPlan& p2, int RB, void*& f, void*& i) {
  const int H = p2.n;
#define LDDMM_ROWS_CASE(h, rb)                                         \
  if (H == h && RB == rb && plan_matches<PlanOf<h>::type>(p2)) {       \
    f = (void*)(RowsFwdFn<T>)k_rows_fwd_s<T, h, rb, 256>;              \
    i = (void*)(RowsInvFn<T>)k_rows_inv_s<T, h, rb, 256>;              \
    return;                                                            \
  }
  LDDMM_ROWS_CASE(64, 16)
  LDDMM_ROWS_CASE(64, 32)
  LDDMM_ROWS_CASE(128, 16)
  LDDMM_ROWS_CASE(128, 32)
  LDDMM_ROWS_CASE(90, 16)
  LDDMM_ROWS_CASE(90, 32)
#undef LDDMM_ROWS_CASE
  f = i = nullptr;
}

template <typename T>
void* pencil_generic(int mode, int nt) {
  if (nt == 512) return mode == 0 ? (void*)(PencilFn<T>)k_pencil<T, 0, 512>
                      : mode == 1 ? (void*)(PencilFn<T>)k_pencil<T, 1, 512>
                                  : (void*)(PencilFn<T>)k_pencil<T, 2, 512>;
  return mode == 0 ? (void*)(PencilFn<T>)k_pencil<T, 0, 256>
       : mode == 1 ? (void*)(PencilFn<T>)k_pencil<T, 1, 256>
                   : (void*)(PencilFn<T>)k_pencil<T, 2, 256>;
}

}  // namespace

template <typename T>
int spectral_configure(SpectralPlan<T>& sp, const FftTuning& tune, std::string& err) {
  if (!allowed_threads(tune.plane_threads) || (tune.pencil_threads != 256 && tune.pencil_threads != 512) ||
      tune.pencil_tb < 1 || tune.pencil_tb > 128 || tune.rows_rb < 1 || tune.rows_rb > 64 || tune.plane_grid < 0 ||
      tune.plane_grid > 65535) {
    err = "invalid transform tuning";
    return LDDMM_EINVAL;
  }
  const size_t cb = sizeof(cplx<T>);
  const int n0 = sp.n0, n1 = sp.n1, H = sp.H, M = sp.M;
  const int tb = tune.pencil_tb;
  const size_t tables = size_t(H + H / 2 + 1) * cb + size_t(H + 1) * sizeof(int);
  size_t plane_lds = size_t(n1) * M * cb + size_t(n1) * cb + tables;
  // half planes: compile-time kernels only, one unit per workgroup, pencil
  // tiles of whole pairs
  void* hk[4] = {nullptr, nullptr, nullptr, nullptr};
  const int n1h = n1 / 2;
  const size_t half_lds = size_t(n1h) * M * cb + size_t(n1h) * cb + tables;
  if (tune.plane_halves && !tune.force_split && tune.plane_grid == 0 && tune.use_static && sp.tw1h &&
      tune.pencil_threads == 256 && tb % 2 == 0 && half_lds <= sp.max_lds) {
    if (tune.plane_threads == 512) plane_static_halves<T, 512>(sp.p2, sp.p1h, hk[0], hk[1], hk[2]);
    if (tune.plane_threads == 1024) plane_static_halves<T, 1024>(sp.p2, sp.p1h, hk[0], hk[1], hk[2]);
    hk[3] = pencil_static_pairs<T>(sp.p0, tb / 2);
  }
  const bool halves = hk[0] && hk[3];
  if (halves) plane_lds = half_lds;
  const bool fused = halves || (!tune.force_split && plane_lds <= sp.max_lds);
  // the compile-time pencils also keep TB per-sequence symbol terms
  const size_t p0 = (size_t(n0) * tb + n0) * cb + size_t(n0 + tb) * sizeof(T);
  const size_t p1 = (size_t(n1) * tb + n1) * cb + size_t(n1 + tb) * sizeof(T);
  const size_t rl = size_t(tune.rows_rb) * M * cb + tables;
  if (p0 > sp.max_lds || (!fused && (p1 > sp.max_lds || rl > sp.max_lds))) {
    err = "transform tiles exceed the LDS of a workgroup";
    return LDDMM_EUNSUPPORTED;
  }
  void* k[8] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  int nstatic = 0;
  const bool use_static = tune.use_static != 0;
  // plane walk: compile-time plane kernels only
  const bool walk = tune.plane_grid > 0;
  int plane_grid = 0;
  if (halves) {
    k[KF_PLANE_FWD] = hk[0];
    k[KF_PLANE_INV] = hk[1];
    k[KF_PLANE_INV_ADD] = hk[2];
    k[KF_PENCIL0] = hk[3];
    nstatic += 2;
  } else if (fused) {
    if (use_static) {
      if (tune.plane_threads == 512 && walk) plane_static<T, 512, true>(sp.p2, sp.p1, k[KF_PLANE_FWD], k[KF_PLANE_INV], k[KF_PLANE_INV_ADD]);
      if (tune.plane_threads == 512 && !walk) plane_static<T, 512, false>(sp.p2, sp.p1, k[KF_PLANE_FWD], k[KF_PLANE_INV], k[KF_PLANE_INV_ADD]);
      // the walk's extra registers spill with 1024 threads in FP64: not offered there
      if constexpr (sizeof(T) == 4)
        if (tune.plane_threads == 1024 && walk) plane_static<T, 1024, true>(sp.p2, sp.p1, k[KF_PLANE_FWD], k[KF_PLANE_INV], k[KF_PLANE_INV_ADD]);
      if (tune.plane_threads == 1024 && (!walk || sizeof(T) != 4))
        plane_static<T, 1024, false>(sp.p2, sp.p1, k[KF_PLANE_FWD], k[KF_PLANE_INV], k[KF_PLANE_INV_ADD]);
    }
    if (k[KF_PLANE_FWD]) {
      nstatic++;
      plane_grid = walk && (sizeof(T) == 4 || tune.plane_threads != 1024) ? tune.plane_grid : 0;
    } else {
      k[KF_PLANE_FWD] = tune.plane_threads == 256    ? (void*)(PlaneFwdFn<T>)k_plane_fwd<T, 256>
                        : tune.plane_threads == 1024 ? (void*)(PlaneFwdFn<T>)k_plane_fwd<T, 1024>
                                                     : (void*)(PlaneFwdFn<T>)k_plane_fwd<T, 512>;
      k[KF_PLANE_INV] = tune.plane_threads == 256    ? (void*)(PlaneInvFn<T>)k_plane_inv<T, 256>
                        : tune.plane_threads == 1024 ? (void*)(PlaneInvFn<T>)k_plane_inv<T, 1024>
                                                     : (void*)(PlaneInvFn<T>)k_plane_inv<T, 512>;
    }
  } else {
    const long long rows = (long long)n0 * n1;
    if (use_static && rows % tune.rows_rb == 0) rows_static<T>(sp.p2, tune.rows_rb, k[KF_ROWS_FWD], k[KF_ROWS_INV]);
    if (k[KF_ROWS_FWD]) {
      nstatic++;
    } else {
      k[KF_ROWS_FWD] = (void*)(RowsFwdFn<T>)k_rows_fwd<T>;
      k[KF_ROWS_INV] = (void*)(RowsInvFn<T>)k_rows_inv<T>;
    }
    if (use_static && tune.pencil_threads == 256) {
      k[KF_PENCIL1F] = pencil_static<T, 0>(sp.p1, tb);
      k[KF_PENCIL1I] = pencil_static<T, 1>(sp.p1, tb);
    }
    if (k[KF_PENCIL1F]) {
      nstatic++;
    } else {
      k[KF_PENCIL1F] = pencil_generic<T>(0, tune.pencil_threads);
      k[KF_PENCIL1I] = pencil_generic<T>(1, tune.pencil_threads);
    }
  }
  if (!halves) {
    if (use_static && tune.pencil_threads == 256) k[KF_PENCIL0] = pencil_static<T, 2>(sp.p0, tb);
    if (k[KF_PENCIL0])
      nstatic++;
    else
      k[KF_PENCIL0] = pencil_generic<T>(2, tune.pencil_threads);
  }
  for (void* f : k)
    if (f && hipFuncSetAttribute((const void*)f, hipFuncAttributeMaxDynamicSharedMemorySize, int(sp.max_lds)) !=
                 hipSuccess) {
      err = "hipFuncSetAttribute(MaxDynamicSharedMemorySize) failed";
      return LDDMM_EHIP;
    }
  sp.tune = tune;
  sp.fused = fused;
  sp.halves = halves;
  sp.plane_grid = plane_grid;
  sp.plane_lds = plane_lds;
  sp.pencil0_lds = p0;
  sp.pencil1_lds = p1;
  sp.rows_lds = rl;
  sp.static_kernels = nstatic;
  for (int i = 0; i < 8; ++i) sp.kfn[i] = k[i];
  return 0;
}

template <typename T>
FftTuning default_tuning(const SpectralPlan<T>& sp) {
  FftTuning t;
  const size_t cb = sizeof(cplx<T>);
  // measured best on MI355X at 32^3 .. 256^3 inside the Hessian-vector product:
  // 1024-thread plane workgroups (512 for FP32 half planes), 256-thread pencil
  // workgroups with 256-byte rows (32 FP32 / 16 FP64 pencils); the autotuner
  // keeps this start unless another shape is clearly faster
  t.plane_threads = 1024;
  t.pencil_threads = 256;
  // half planes where compile-time kernels exist (spectral_configure falls back
  // to whole planes otherwise)
  t.plane_halves = 1;
  if (sizeof(T) == 4 && sp.tw1h) {
    // small FP32 half planes (up to 64 x 65 complex) run best with 512 threads
    void *f = nullptr, *i = nullptr, *ia = nullptr;
    plane_static_halves<T, 512>(sp.p2, sp.p1h, f, i, ia);
    if (f && size_t(sp.n1 / 2) * sp.M <= size_t(64) * 65) t.plane_threads = 512;
  }
  int tb = int(256 / cb);
  while (tb > 1 && ((size_t(sp.n0) * tb + sp.n0) * cb + sp.n0 * sizeof(T) > sp.max_lds ||
                    (size_t(sp.n1) * tb + sp.n1) * cb > sp.max_lds))
    tb /= 2;
  t.pencil_tb = tb;
  const size_t tables = size_t(sp.H + sp.H / 2 + 1) * cb + size_t(sp.H + 1) * sizeof(int);
  int rb = 16;
  while (rb > 1 && size_t(rb) * sp.M * cb + tables > sp.max_lds) rb /= 2;
  t.rows_rb = rb;
  t.force_split = 0;
  t.use_static = 1;
  return t;
}

// Plans and the host image of the tables; device pointers are offsets into
// the table block until spectral_place_tables sets its base.
template <typename T>
int spectral_plan_tables(SpectralPlan<T>& sp, const int n[3], size_t max_lds, std::string& err, TableBlob& blob,
                         size_t off[12]) {
  sp = SpectralPlan<T>();
  sp.n0 = n[0];
  sp.n1 = n[1];
  sp.n2 = n[2];
  sp.max_lds = max_lds;
  if (n[0] < 4 || n[1] < 4 || n[2] < 4 || (n[2] & 1)) {
    err = "grid sizes must be >= 4 and N2 even";
    return LDDMM_EUNSUPPORTED;
  }
  sp.H = n[2] / 2;
  sp.M = sp.H + 1;
  if (!make_plan(n[0], sp.p0) || !make_plan(n[1], sp.p1) || !make_plan(sp.H, sp.p2)) {
    err = "grid sizes N0, N1 and N2/2 must factor into 2, 3, 5, 7";
    return LDDMM_EUNSUPPORTED;
  }
  const int H = sp.H, M = sp.M;
  for (int i = 0; i < 12; ++i) off[i] = size_t(-1);
  off[0] = blob.put(twiddles<T>(n[0], n[0]));
  off[1] = blob.put(twiddles<T>(n[1], n[1]));
  off[2] = blob.put(twiddles<T>(H, H));
  off[3] = blob.put(twiddles<T>(n[2], H / 2 + 1));
  std::vector<int> slot(H + 1);
  for (int p = 0; p < H; ++p) slot[digit_reverse(sp.p2, p)] = p;
  slot[H] = H;
  off[4] = blob.put(slot);
  std::vector<T> k0(n[0]), k1(n[1]), k2(M);
  for (int p = 0; p < n[0]; ++p) k0[p] = T(fold_sq(digit_reverse(sp.p0, p), n[0]));
  for (int p = 0; p < n[1]; ++p) k1[p] = T(fold_sq(digit_reverse(sp.p1, p), n[1]));
  for (int p = 0; p < H; ++p) {
    const int k = digit_reverse(sp.p2, p);
    k2[p] = T(k * k);
  }
  k2[H] = T(H * H);
  off[5] = blob.put(k0);
  off[6] = blob.put(k1);
  off[7] = blob.put(k2);
  // half-plane tables: the x1 transform of half length, the merge twiddles
  // W_{n1}^{k1} and |k1|^2, |k1 + n1/2|^2 per slot of the half transform
  if (n[1] % 2 == 0 && n[1] >= 8 && make_plan(n[1] / 2, sp.p1h)) {
    const int h1 = n[1] / 2;
    off[8] = blob.put(twiddles<T>(h1, h1));
    std::vector<cplx<T>> wx(h1);
    std::vector<T> kx(n[1]);
    for (int p = 0; p < h1; ++p) {
      const int k = digit_reverse(sp.p1h, p);
      const double ang = -2.0 * M_PI * double(k) / double(n[1]);
      wx[p] = {T(std::cos(ang)), T(std::sin(ang))};
      kx[p] = T(fold_sq(k, n[1]));
      kx[h1 + p] = T(fold_sq(k + h1, n[1]));
    }
    off[9] = blob.put(wx);
    off[10] = blob.put(kx);
  }
  return 0;
}

// Point the plan's tables into the device copy of the blob at `base`.
template <typename T>
void spectral_place_tables(SpectralPlan<T>& sp, unsigned char* base, const size_t off[12]) {
  auto at = [&](size_t o) { return o == size_t(-1) ? nullptr : static_cast<void*>(base + o); };
  sp.tw0 = static_cast<cplx<T>*>(at(off[0]));
  sp.tw1 = static_cast<cplx<T>*>(at(off[1]));
  sp.tw2 = static_cast<cplx<T>*>(at(off[2]));
  sp.twr = static_cast<cplx<T>*>(at(off[3]));
  sp.slot2 = static_cast<int*>(at(off[4]));
  sp.ksq0 = static_cast<T*>(at(off[5]));
  sp.ksq1 = static_cast<T*>(at(off[6]));
  sp.ksq2 = static_cast<T*>(at(off[7]));
  sp.tw1h = static_cast<cplx<T>*>(at(off[8]));
  sp.twx = static_cast<cplx<T>*>(at(off[9]));
  sp.ksq1x = static_cast<T*>(at(off[10]));
}

template <typename T>
size_t spectrum_bytes(const SpectralPlan<T>& sp, int ncomp) {
  return size_t(ncomp) * sp.n0 * sp.n1 * sp.M * sizeof(cplx<T>);
}

template <typename T>
int spectral_init(SpectralPlan<T>& sp, const int n[3], size_t max_lds, std::string& err) {
  TableBlob blob;
  size_t off[12];
  int rc = spectral_plan_tables(sp, n, max_lds, err, blob, off);
  if (rc) return rc;
  void* tables = nullptr;
  if (hipMalloc(&tables, blob.host.size()) != hipSuccess) {
    err = "out of device memory (transform tables)";
    return LDDMM_ENOMEM;
  }
  sp.table_mem = tables;
  sp.bytes += blob.host.size();
  if (hipMemcpy(tables, blob.host.data(), blob.host.size(), hipMemcpyHostToDevice) != hipSuccess) {
    err = "cannot upload the transform tables";
    return LDDMM_EHIP;
  }
  spectral_place_tables(sp, static_cast<unsigned char*>(tables), off);
  const size_t spec_bytes = spectrum_bytes(sp, 3);
  if (hipMalloc(reinterpret_cast<void**>(&sp.spec), spec_bytes) != hipSuccess) {
    err = "out of device memory (spectrum workspace)";
    return LDDMM_ENOMEM;
  }
  sp.bytes += spec_bytes;
  if ((rc = spectral_configure(sp, default_tuning(sp), err))) return rc;
  return 0;
}

template <typename T>
int spectral_init_in(SpectralPlan<T>& sp, const int n[3], int ncomp, size_t max_lds, unsigned char* region,
                     size_t region_bytes, hipStream_t st, std::vector<unsigned char>& host_tables,
                     std::string& err) {
  TableBlob blob;
  size_t off[12];
  int rc = spectral_plan_tables(sp, n, max_lds, err, blob, off);
  if (rc) return rc;
  const size_t tab = (blob.host.size() + 255) & ~size_t(255);
  const size_t need = tab + spectrum_bytes(sp, ncomp);
  if (need > region_bytes) {
    err = "grid " + std::to_string(n[0]) + "x" + std::to_string(n[1]) + "x" + std::to_string(n[2]) + " with " +
          std::to_string(ncomp) + " component(s) needs " + std::to_string(need) +
          " bytes of static workspace; it holds " + std::to_string(region_bytes);
    sp = SpectralPlan<T>();
    return LDDMM_EUNSUPPORTED;
  }
  host_tables.swap(blob.host);
  // the region may still be read by earlier work on this stream
  if (hipStreamSynchronize(st) != hipSuccess ||
      hipMemcpyAsync(region, host_tables.data(), host_tables.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    err = "cannot upload the transform tables";
    sp = SpectralPlan<T>();
    return LDDMM_EHIP;
  }
  spectral_place_tables(sp, region, off);
  sp.spec = reinterpret_cast<cplx<T>*>(region + tab);
  sp.owns_memory = false;
  if ((rc = spectral_configure(sp, default_tuning(sp), err))) return rc;
  return 0;
}

template <typename T>
void spectral_free(SpectralPlan<T>& sp) {
  if (sp.owns_memory) {
    if (sp.table_mem) (void)hipFree(sp.table_mem);
    if (sp.spec) (void)hipFree(sp.spec);
  }
  sp = SpectralPlan<T>();
}

// Neighbouring pencil tiles share cache lines unless every tile's run starts on
// a 128-byte line: then they take runs of kPencilXcdRun per XCD.
template <typename T>
int pencil_xcd_run(const PencilArgs<T>& k) {
  const long long c = sizeof(cplx<T>);
  return xcd_run_if_split(k.tb * c, k.es * c, k.hs * c, k.outer_stride * c, kPencilXcdRun);
}

template <typename T>
void spectral_apply(const SpectralPlan<T>& sp, const T* in, T* out, int ncomp, double alpha, int s, int op,
                    hipStream_t st, Profiler* prof, const T* add, double add_scale, double out_scale) {
  PlaneArgs<T> pa;
  pa.n0 = sp.n0;
  pa.n1 = sp.n1;
  pa.n2 = sp.n2;
  pa.H = sp.H;
  pa.M = sp.M;
  pa.planes = ncomp * sp.n0;
  pa.N = (long long)sp.n0 * sp.n1 * sp.n2;
  pa.p1 = sp.p1;
  pa.p2 = sp.p2;
  pa.tw1 = sp.tw1;
  pa.tw2 = sp.tw2;
  pa.twr = sp.twr;
  pa.slot2 = sp.slot2;
  pa.add = add;
  pa.add_scale = T(add_scale);
  // half planes share the cache line at a row's end unless rows are whole lines
  pa.xcd_run = sp.halves ? xcd_run_if_split((long long)sp.n2 * sizeof(T), 0, 0, 0, kPlaneXcdRun) : 1;
  const FftTuning& tu = sp.tune;

  const int P = sp.n1 * sp.M;
  PencilArgs<T> k0;
  k0.pl = sp.p0;
  k0.es = P;
  k0.nin = P;
  k0.outer_stride = (long long)sp.n0 * P;
  k0.tb = tu.pencil_tb;
  k0.tw = sp.tw0;
  k0.M = sp.M;
  k0.alpha = T(alpha);
  k0.s = s;
  k0.op = op;
  k0.scale = T(out_scale / (double(sp.n0) * sp.n1 * sp.n2));  // the inverse's 1/N and the caller's factor
  k0.ksq0 = sp.ksq0;
  k0.ksq1 = sp.ksq1;
  k0.ksq2 = sp.ksq2;
  k0.hs = 0;
  k0.k1half = 0;
  k0.twx = nullptr;
  dim3 g0((P + tu.pencil_tb - 1) / tu.pencil_tb, ncomp);
  if (sp.halves) {
    // units (component, x0, h): the x1 transform of half length; pencils in pairs
    pa.planes = 2 * ncomp * sp.n0;
    pa.tw1 = sp.tw1h;
    const int tbp = tu.pencil_tb / 2, pairs = P / 2;
    k0.nin = pairs;
    k0.tb = tbp;
    k0.hs = pairs;
    k0.k1half = sp.n1 / 2;
    k0.ksq1 = sp.ksq1x;
    k0.twx = sp.twx;
    g0 = dim3((pairs + tbp - 1) / tbp, ncomp);
  }
  k0.xcd_run = pencil_xcd_run(k0);
  const PencilFn<T> pencil0 = (PencilFn<T>)sp.kfn[KF_PENCIL0];

  if (sp.fused) {
    // plane walk: at most plane_grid workgroups, never more than there are planes
    const dim3 gp = sp.plane_grid > 0 ? dim3(unsigned(sp.plane_grid < pa.planes ? sp.plane_grid : pa.planes))
                                      : dim3(sp.halves ? 2 * sp.n0 : sp.n0, ncomp);
    {
      KernelTimer t(prof, "fft_plane_fwd");
      LDDMM_LAUNCH(t.start, t.stop, ((PlaneFwdFn<T>)sp.kfn[KF_PLANE_FWD]), gp, tu.plane_threads, sp.plane_lds, st, in, sp.spec, pa);
    }
    {
      KernelTimer t(prof, "fft_pencil_symbol");
      LDDMM_LAUNCH(t.start, t.stop, pencil0, g0, tu.pencil_threads, sp.pencil0_lds, st, sp.spec, k0);
    }
    if (add && sp.kfn[KF_PLANE_INV_ADD]) {
      // the addend rides on the inverse plane pass: out = add + add_scale * K in
      KernelTimer t(prof, "fft_plane_inv_add");
      LDDMM_LAUNCH(t.start, t.stop, ((PlaneInvFn<T>)sp.kfn[KF_PLANE_INV_ADD]), gp, tu.plane_threads, sp.plane_lds, st, sp.spec, out, pa);
      return;
    }
    {
      KernelTimer t(prof, "fft_plane_inv");
      LDDMM_LAUNCH(t.start, t.stop, ((PlaneInvFn<T>)sp.kfn[KF_PLANE_INV]), gp, tu.plane_threads, sp.plane_lds, st, sp.spec, out, pa);
    }
    if (add) launch_axpbyz<T>((long long)ncomp * pa.N, 1.0, add, add_scale, out, out, st, prof);
    return;
  }
  PencilArgs<T> k1 = k0;
  k1.pl = sp.p1;
  k1.es = sp.M;
  k1.nin = sp.M;
  k1.outer_stride = (long long)sp.n1 * sp.M;
  k1.tw = sp.tw1;
  k1.xcd_run = pencil_xcd_run(k1);
  const dim3 g1((sp.M + tu.pencil_tb - 1) / tu.pencil_tb, ncomp * sp.n0);
  const long long rows = (long long)sp.n0 * sp.n1;
  const dim3 gr((unsigned)((rows + tu.rows_rb - 1) / tu.rows_rb), ncomp);
  {
    KernelTimer t(prof, "fft_rows_fwd");
    LDDMM_LAUNCH(t.start, t.stop, ((RowsFwdFn<T>)sp.kfn[KF_ROWS_FWD]), gr, 256, sp.rows_lds, st, in, sp.spec, pa, tu.rows_rb);
  }
  {
    KernelTimer t(prof, "fft_pencil_x1_fwd");
    LDDMM_LAUNCH(t.start, t.stop, ((PencilFn<T>)sp.kfn[KF_PENCIL1F]), g1, tu.pencil_threads, sp.pencil1_lds, st, sp.spec, k1);
  }
  {
    KernelTimer t(prof, "fft_pencil_symbol");
    LDDMM_LAUNCH(t.start, t.stop, pencil0, g0, tu.pencil_threads, sp.pencil0_lds, st, sp.spec, k0);
  }
  {
    KernelTimer t(prof, "fft_pencil_x1_inv");
    LDDMM_LAUNCH(t.start, t.stop, ((PencilFn<T>)sp.kfn[KF_PENCIL1I]), g1, tu.pencil_threads, sp.pencil1_lds, st, sp.spec, k1);
  }
  {
    KernelTimer t(prof, "fft_rows_inv");
    LDDMM_LAUNCH(t.start, t.stop, ((RowsInvFn<T>)sp.kfn[KF_ROWS_INV]), gr, 256, sp.rows_lds, st, sp.spec, out, pa, tu.rows_rb);
  }
  if (add) launch_axpbyz<T>((long long)ncomp * pa.N, 1.0, add, add_scale, out, out, st, prof);
}

#define LDDMM_SINST(T)                                                                                   \
  template int spectral_init<T>(SpectralPlan<T>&, const int[3], size_t, std::string&);                  \
  template int spectral_init_in<T>(SpectralPlan<T>&, const int[3], int, size_t, unsigned char*, size_t,     \
                                   hipStream_t, std::vector<unsigned char>&, std::string&);               \
  template size_t spectrum_bytes<T>(const SpectralPlan<T>&, int);                                        \
  template int spectral_configure<T>(SpectralPlan<T>&, const FftTuning&, std::string&);                 \
  template FftTuning default_tuning<T>(const SpectralPlan<T>&);                                          \
  template void spectral_free<T>(SpectralPlan<T>&);                                                      \
  template void spectral_apply<T>(const SpectralPlan<T>&, const T*, T*, int, double, int, int, hipStream_t, \
                                  Profiler*, const T*, double, double);

LDDMM_SINST(float)
LDDMM_SINST(double)

}  // namespace lddmm
