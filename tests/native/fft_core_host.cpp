// Host-side run of the FFT stage code of fft_core.h (the code the GPU kernels
// execute per butterfly), for CPU tests against numpy.fft.  A stage has no
// intra-stage hazards, so running its butterflies in order on one thread gives
// the same result as the parallel run.
#include <cmath>
#include <vector>

#include "fft_core.h"

using namespace lddmm;

namespace {

template <bool INV>
void run(cplx<double>* buf, const FftPlan& pl, const cplx<double>* tw) {
  const int n = pl.n;
  for (int i = 0; i < pl.nf; ++i) {
    const int st = INV ? pl.nf - 1 - i : i;
    const int r = pl.radix[st];
    const int L = stage_length(pl, st);
    for (int b = 0; b < n / r; ++b) {
      switch (r) {
        case 16: fft_stage_item<double, 16, INV, false>(buf, b, n, L, 1, 1, n, tw); break;
        case 8: fft_stage_item<double, 8, INV, false>(buf, b, n, L, 1, 1, n, tw); break;
        case 4: fft_stage_item<double, 4, INV, false>(buf, b, n, L, 1, 1, n, tw); break;
        case 2: fft_stage_item<double, 2, INV, false>(buf, b, n, L, 1, 1, n, tw); break;
        case 3: fft_stage_item<double, 3, INV, false>(buf, b, n, L, 1, 1, n, tw); break;
        case 5: fft_stage_item<double, 5, INV, false>(buf, b, n, L, 1, 1, n, tw); break;
        case 7: fft_stage_item<double, 7, INV, false>(buf, b, n, L, 1, 1, n, tw); break;
        case 9: fft_stage_item<double, 9, INV, false>(buf, b, n, L, 1, 1, n, tw); break;
        default: break;
      }
    }
  }
}

}  // namespace

extern "C" {

// In-place transform of n complex values (interleaved re, im).  inverse = 0:
// DIF forward (output digit-reversed); 1: DIT inverse (input digit-reversed,
// unnormalised).  Returns the number of stages, or -1 if n does not factor.
int fftcore_transform(int n, double* data, int inverse) {
  FftPlan pl;
  if (!make_plan(n, pl)) return -1;
  std::vector<cplx<double>> tw(n);
  for (int m = 0; m < n; ++m) tw[m] = {std::cos(-2.0 * M_PI * m / n), std::sin(-2.0 * M_PI * m / n)};
  auto* buf = reinterpret_cast<cplx<double>*>(data);
  if (inverse)
    run<true>(buf, pl, tw.data());
  else
    run<false>(buf, pl, tw.data());
  return pl.nf;
}

// perm[p] = frequency held by DIF output slot p.
int fftcore_digit_reverse(int n, int* perm) {
  FftPlan pl;
  if (!make_plan(n, pl)) return -1;
  for (int p = 0; p < n; ++p) perm[p] = digit_reverse(pl, p);
  return 0;
}

}

namespace {

template <class P, bool INV, int I = 0>
void run_static(cplx<double>* buf, const cplx<double>* tw) {
  if constexpr (I < P::nf) {
    constexpr int st = INV ? P::nf - 1 - I : I;
    constexpr int total = P::length(0) / P::radix(st);
    for (int b = 0; b < total; ++b) fft_stage_item_static<double, P, st, INV, false, 1, 1, P::length(0)>(buf, b, tw);
    run_static<P, INV, I + 1>(buf, tw);
  }
}

template <int N>
int static_case(double* data, int inverse) {
  using P = typename PlanOf<N>::type;
  FftPlan rt;
  if (!make_plan(N, rt) || !plan_matches<P>(rt)) return -2;  // compile-time plan must equal make_plan
  for (int p = 0; p < N; ++p)
    if (slot_of<P>(digit_reverse(rt, p)) != p) return -3;  // slot_of inverts digit_reverse
  std::vector<cplx<double>> tw(N);
  for (int m = 0; m < N; ++m) tw[m] = {std::cos(-2.0 * M_PI * m / N), std::sin(-2.0 * M_PI * m / N)};
  auto* buf = reinterpret_cast<cplx<double>*>(data);
  if (inverse)
    run_static<P, true>(buf, tw.data());
  else
    run_static<P, false>(buf, tw.data());
  return P::nf;
}

}  // namespace

extern "C" {

// Same as fftcore_transform through the compile-time plan of length n
// (the lengths instantiated by the GPU kernels); -1 if n has none.
int fftcore_transform_static(int n, double* data, int inverse) {
  switch (n) {
    case 16: return static_case<16>(data, inverse);
    case 32: return static_case<32>(data, inverse);
    case 64: return static_case<64>(data, inverse);
    case 128: return static_case<128>(data, inverse);
    case 256: return static_case<256>(data, inverse);
    case 40: return static_case<40>(data, inverse);
    case 48: return static_case<48>(data, inverse);
    case 56: return static_case<56>(data, inverse);
    case 80: return static_case<80>(data, inverse);
    case 90: return static_case<90>(data, inverse);
    case 96: return static_case<96>(data, inverse);
    case 112: return static_case<112>(data, inverse);
    case 180: return static_case<180>(data, inverse);
    case 216: return static_case<216>(data, inverse);
    default: return -1;
  }
}

}
