// reduce.hip - FP64 reductions (inner products of the CG in V, energies, checks)
// and BLAS-1 updates.
//
// Reductions are deterministic: a fixed grid of kReduceBlocks workgroups, each
// summing a grid-strided share in double, a 64-lane wavefront shuffle tree, a
// per-block slot in `partials`, then one workgroup summing the slots in a fixed
// tree order.  No atomics, so repeated calls give bit-identical results.
#include <cfloat>

#include "lddmm.h"
#include "lddmm_internal.h"

namespace lddmm {

namespace {

constexpr int RT = 256;  // threads per reduction block (4 wavefronts)

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
  return x;
}
__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_down(x, off, 64));
  return x;
}
__device__ __forceinline__ double wave_min(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = fmin(x, __shfl_down(x, off, 64));
  return x;
}

// Block-wide combine of K values per thread; op 0 = sum, 1 = max, 2 = min.
template <int K>
__device__ void block_combine(double (&v)[K], const int (&op)[K], double* out) {
  __shared__ double sh[K][RT / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    v[k] = op[k] == 0 ? wave_sum(v[k]) : op[k] == 1 ? wave_max(v[k]) : wave_min(v[k]);
    if (lane == 0) sh[k][wid] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double a = sh[k][0];
      for (int w = 1; w < RT / 64; ++w)
        a = op[k] == 0 ? a + sh[k][w] : op[k] == 1 ? fmax(a, sh[k][w]) : fmin(a, sh[k][w]);
      out[k] = a;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(RT) k_dot(const T* __restrict__ a, const T* __restrict__ b, long long n,
                                            double* __restrict__ partials) {
  double acc = 0.0;
  for (long long i = blockIdx.x * (long long)RT + threadIdx.x; i < n; i += (long long)gridDim.x * RT)
    acc += double(a[i]) * double(b[i]);
  double v[1] = {acc};
  const int op[1] = {0};
  double out[1];
  block_combine<1>(v, op, out);
  if (threadIdx.x == 0) partials[blockIdx.x] = out[0];
}

template <typename T>
__global__ void __launch_bounds__(RT) k_check(const T* __restrict__ a, long long n, double* __restrict__ partials) {
  double bad = 0.0, mx = 0.0;
  for (long long i = blockIdx.x * (long long)RT + threadIdx.x; i < n; i += (long long)gridDim.x * RT) {
    const double x = double(a[i]);
    if (!isfinite(x))
      bad += 1.0;
    else
      mx = fmax(mx, fabs(x));
  }
  double v[2] = {bad, mx};
  const int op[2] = {0, 1};
  double out[2];
  block_combine<2>(v, op, out);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = out[0];
    partials[2 * blockIdx.x + 1] = out[1];
  }
}

template <typename T>
__global__ void __launch_bounds__(RT) k_minmax(const T* __restrict__ a, long long n, double* __restrict__ partials) {
  double mn = DBL_MAX, mx = -DBL_MAX;
  for (long long i = blockIdx.x * (long long)RT + threadIdx.x; i < n; i += (long long)gridDim.x * RT) {
    const double x = double(a[i]);
    mn = fmin(mn, x);
    mx = fmax(mx, x);
  }
  double v[2] = {mn, mx};
  const int op[2] = {2, 1};
  double out[2];
  block_combine<2>(v, op, out);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = out[0];
    partials[2 * blockIdx.x + 1] = out[1];
  }
}

// Final stage: K interleaved values per partial slot, nparts slots, fixed order.
template <int K>
__global__ void __launch_bounds__(RT) k_finish(const double* __restrict__ partials, int nparts, int op0, int op1,
                                               double* __restrict__ out) {
  double v[K];
  int op[K];
  op[0] = op0;
  if (K > 1) op[K - 1] = op1;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = op[k] == 0 ? 0.0 : op[k] == 1 ? -DBL_MAX : DBL_MAX;
  for (int i = threadIdx.x; i < nparts; i += RT)
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const double x = partials[K * i + k];
      v[k] = op[k] == 0 ? v[k] + x : op[k] == 1 ? fmax(v[k], x) : fmin(v[k], x);
    }
  double r[K];
  block_combine<K>(v, op, r);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) out[k] = r[k];
}

template <typename T>
__global__ void k_axpby(long long n, T alpha, const T* x, T beta, T* y) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    y[i] = alpha * x[i] + beta * y[i];
}

template <typename T>
__global__ void k_axpbyz(long long n, T alpha, const T* x, T beta, const T* y, T* z) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    z[i] = alpha * x[i] + beta * y[i];
}

// CG update with the step length taken on the device: a = rr / (cell * *dsum)
// when that curvature is positive, else 0 (the host sees the curvature at its
// next read and stops); x += a d, r -= a q.
template <typename T>
__global__ void k_cg_step(long long n, double rr, double cell, const double* __restrict__ dsum,
                          const T* __restrict__ d, const T* __restrict__ q, T* __restrict__ x, T* __restrict__ r) {
  const double curv = cell * dsum[0];
  const double a = curv > 0.0 ? rr / curv : 0.0;
  const T ta = T(a), tb = T(-a), one = T(1);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    x[i] = ta * d[i] + one * x[i];
    r[i] = tb * q[i] + one * r[i];
  }
}

// ---- CG scalars kept on the device (one block of kCgSlots doubles per solve) --
// Start: rz = cell * num[0] (the numerator of the first step length), tol = eta *
// sqrt(cell * stop[0]), active, no iterations yet; at most maxit iterations;
// first_d: non-positive curvature on the first direction takes x = d.
__global__ void k_cg_begin(double* __restrict__ s, const double* __restrict__ num, const double* __restrict__ stop,
                           double cell, double eta, int maxit, int first_d) {
  s[CG_MAXIT] = double(maxit);
  s[CG_FIRSTD] = double(first_d);
  s[CG_RZ] = cell * num[0];
  s[CG_TOL] = eta * sqrt(cell * stop[0]);
  s[CG_ACTIVE] = 1.0;
  s[CG_AX] = 0.0;
  s[CG_AR] = 0.0;
  s[CG_BETA] = 0.0;
  s[CG_ITERS] = 0.0;
  s[CG_NEGCURV] = 0.0;
}

// Step length from the curvature cell * curv[0] = <d, H d>: a = rz / curvature
// when it is positive (the iteration counts); otherwise the solve stops without
// counting it, and on its first direction x takes d itself (steepest descent,
// x = 0 + 1 d).  An inactive solve takes no step.
__global__ void k_cg_alpha(double* __restrict__ s, const double* __restrict__ curv, double cell) {
  double ax = 0.0, ar = 0.0;
  if (s[CG_ACTIVE] != 0.0) {
    const double c = cell * curv[0];
    if (c > 0.0) {
      ax = ar = s[CG_RZ] / c;
      s[CG_ITERS] += 1.0;
    } else {
      ax = (s[CG_ITERS] == 0.0 && s[CG_FIRSTD] != 0.0) ? 1.0 : 0.0;
      s[CG_ACTIVE] = 0.0;
      s[CG_NEGCURV] = 1.0;
    }
  }
  s[CG_AX] = ax;
  s[CG_AR] = ar;
}

// After the step: stop once sqrt(cell * stop[0]) <= tol or after maxit
// iterations; else beta =
// rz_new / rz with rz_new = cell * num[0].  beta = 0 when inactive.
__global__ void k_cg_beta(double* __restrict__ s, const double* __restrict__ num, const double* __restrict__ stop,
                          double cell) {
  double beta = 0.0;
  if (s[CG_ACTIVE] != 0.0) {
    if (sqrt(cell * stop[0]) <= s[CG_TOL] || s[CG_ITERS] >= s[CG_MAXIT]) {
      s[CG_ACTIVE] = 0.0;
    } else {
      const double rz_new = cell * num[0];
      beta = rz_new / s[CG_RZ];
      s[CG_RZ] = rz_new;
    }
  }
  s[CG_BETA] = beta;
}

// x += ax d, r -= ar q with the step lengths of the scalar block.
template <typename T>
__global__ void k_cg_step_dev(long long n, const double* __restrict__ s, const T* __restrict__ d,
                              const T* __restrict__ q, T* __restrict__ x, T* __restrict__ r) {
  const T ta = T(s[CG_AX]), tb = T(-s[CG_AR]), one = T(1);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    x[i] = ta * d[i] + one * x[i];
    r[i] = tb * q[i] + one * r[i];
  }
}

// y = x + beta y with beta from the scalar block.
template <typename T>
__global__ void k_cg_direction(long long n, const double* __restrict__ s, const T* __restrict__ x, T* __restrict__ y) {
  const T one = T(1), b = T(s[CG_BETA]);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    y[i] = one * x[i] + b * y[i];
}

template <typename T>
__global__ void k_fill(long long n, T value, T* y) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    y[i] = value;
}

unsigned ew_blocks(long long n) {
  const long long b = (n + 255) / 256;
  return (unsigned)(b < 16384 ? b : 16384);
}

unsigned red_blocks(long long n) {
  const long long b = (n + RT - 1) / RT;
  return (unsigned)(b < kReduceBlocks ? (b > 0 ? b : 1) : kReduceBlocks);
}

}  // namespace

template <typename T>
void launch_dot(const T* a, const T* b, long long n, double* partials, double* out, hipStream_t st,
                Profiler* prof) {
  KernelTimer t(prof, "dot");
  const unsigned nb = red_blocks(n);
  LDDMM_LAUNCH(t.start, nullptr, k_dot<T>, nb, RT, 0, st, a, b, n, partials);
  LDDMM_LAUNCH(nullptr, t.stop, k_finish<1>, 1, RT, 0, st, partials, (int)nb, 0, 0, out);
}

template <typename T>
void launch_check(const T* a, long long n, double* partials, double* out, hipStream_t st, Profiler* prof) {
  KernelTimer t(prof, "check");
  const unsigned nb = red_blocks(n);
  LDDMM_LAUNCH(t.start, nullptr, k_check<T>, nb, RT, 0, st, a, n, partials);
  LDDMM_LAUNCH(nullptr, t.stop, k_finish<2>, 1, RT, 0, st, partials, (int)nb, 0, 1, out);
}

template <typename T>
void launch_minmax(const T* a, long long n, double* partials, double* out, hipStream_t st, Profiler* prof) {
  KernelTimer t(prof, "minmax");
  const unsigned nb = red_blocks(n);
  LDDMM_LAUNCH(t.start, nullptr, k_minmax<T>, nb, RT, 0, st, a, n, partials);
  LDDMM_LAUNCH(nullptr, t.stop, k_finish<2>, 1, RT, 0, st, partials, (int)nb, 2, 1, out);
}

template <typename T>
void launch_axpby(long long n, double alpha, const T* x, double beta, T* y, hipStream_t st, Profiler* prof) {
  KernelTimer t(prof, "axpby");
  LDDMM_LAUNCH(t.start, t.stop, k_axpby<T>, ew_blocks(n), 256, 0, st, n, T(alpha), x, T(beta), y);
}

template <typename T>
void launch_axpbyz(long long n, double alpha, const T* x, double beta, const T* y, T* z, hipStream_t st,
                   Profiler* prof) {
  KernelTimer t(prof, "axpby");
  LDDMM_LAUNCH(t.start, t.stop, k_axpbyz<T>, ew_blocks(n), 256, 0, st, n, T(alpha), x, T(beta), y, z);
}

template <typename T>
void launch_cg_step(long long n, double rr, double cell, const double* dsum, const T* d, const T* q, T* x, T* r,
                    hipStream_t st, Profiler* prof) {
  KernelTimer t(prof, "cg_step");
  LDDMM_LAUNCH(t.start, t.stop, k_cg_step<T>, ew_blocks(n), 256, 0, st, n, rr, cell, dsum, d, q, x, r);
}

void launch_cg_begin(double* s, const double* num, const double* stop, double cell, double eta, int maxit,
                     int first_d, hipStream_t st, Profiler* prof) {
  KernelTimer t(prof, "cg_scalars");
  LDDMM_LAUNCH(t.start, t.stop, k_cg_begin, 1, 1, 0, st, s, num, stop, cell, eta, maxit, first_d);
}

void launch_cg_alpha(double* s, const double* curv, double cell, hipStream_t st, Profiler* prof) {
  KernelTimer t(prof, "cg_scalars");
  LDDMM_LAUNCH(t.start, t.stop, k_cg_alpha, 1, 1, 0, st, s, curv, cell);
}

void launch_cg_beta(double* s, const double* num, const double* stop, double cell, hipStream_t st, Profiler* prof) {
  KernelTimer t(prof, "cg_scalars");
  LDDMM_LAUNCH(t.start, t.stop, k_cg_beta, 1, 1, 0, st, s, num, stop, cell);
}

template <typename T>
void launch_cg_step_dev(long long n, const double* s, const T* d, const T* q, T* x, T* r, hipStream_t st,
                        Profiler* prof) {
  KernelTimer t(prof, "cg_step");
  LDDMM_LAUNCH(t.start, t.stop, k_cg_step_dev<T>, ew_blocks(n), 256, 0, st, n, s, d, q, x, r);
}

template <typename T>
void launch_cg_direction(long long n, const double* s, const T* x, T* y, hipStream_t st, Profiler* prof) {
  KernelTimer t(prof, "axpby");
  LDDMM_LAUNCH(t.start, t.stop, k_cg_direction<T>, ew_blocks(n), 256, 0, st, n, s, x, y);
}

template <typename T>
void launch_fill(long long n, T value, T* y, hipStream_t st, Profiler* prof) {
  KernelTimer t(prof, "fill");
  LDDMM_LAUNCH(t.start, t.stop, k_fill<T>, ew_blocks(n), 256, 0, st, n, value, y);
}

#define LDDMM_RINST(T)                                                                                       \
  template void launch_dot<T>(const T*, const T*, long long, double*, double*, hipStream_t, Profiler*);     \
  template void launch_check<T>(const T*, long long, double*, double*, hipStream_t, Profiler*);             \
  template void launch_minmax<T>(const T*, long long, double*, double*, hipStream_t, Profiler*);            \
  template void launch_axpby<T>(long long, double, const T*, double, T*, hipStream_t, Profiler*);           \
  template void launch_axpbyz<T>(long long, double, const T*, double, const T*, T*, hipStream_t, Profiler*); \
  template void launch_cg_step<T>(long long, double, double, const double*, const T*, const T*, T*, T*,      \
                                  hipStream_t, Profiler*);                                                  \
  template void launch_fill<T>(long long, T, T*, hipStream_t, Profiler*);                                   \
  template void launch_cg_step_dev<T>(long long, const double*, const T*, const T*, T*, T*, hipStream_t,     \
                                      Profiler*);                                                           \
  template void launch_cg_direction<T>(long long, const double*, const T*, T*, hipStream_t, Profiler*);

LDDMM_RINST(float)
LDDMM_RINST(double)

}  // namespace lddmm
