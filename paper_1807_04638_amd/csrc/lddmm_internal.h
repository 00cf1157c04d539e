// lddmm_internal.h - declarations shared by the HIP kernel files and the host engine.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "fft_core.h"
#include "index_math.h"

namespace lddmm {

// ---------------------------------------------------------------------------
// Per-kernel timing (enabled on request).  The events are handed to
// hipExtLaunchKernel, so the dispatch packet itself stamps the start of the
// kernel and its end: the elapsed time is the kernel's execution, without the
// dispatch latency a pair of marker events around the launch would add.
// ---------------------------------------------------------------------------
class Profiler {
 public:
  bool enabled = false;
  void begin(const char* name, hipEvent_t* start, hipEvent_t* stop);
  int read(const char** names, int64_t* counts, double* total_ms, int cap);
  void clear();
  ~Profiler();

 private:
  struct Rec {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<const char*> kinds_;
  std::vector<Rec> recs_;
  std::vector<hipEvent_t> pool_;
  hipEvent_t take();
};

// Timer of one launch (or of a short chain: start from the first, stop from
// the last): KernelTimer t(prof, "name"); LDDMM_LAUNCH(t.start, t.stop, ...).
// Both events are null while the profiler is off.
struct KernelTimer {
  hipEvent_t start = nullptr, stop = nullptr;
  KernelTimer(Profiler* prof, const char* name) {
    if (prof && prof->enabled) prof->begin(name, &start, &stop);
  }
};

#define LDDMM_COMMA ,

// Launch `kern` on stream `st`; with timer events the dispatch records them.
#define LDDMM_LAUNCH(ev0, ev1, kern, grid, block, shmem, st, ...)                             \
  do {                                                                                         \
    if ((ev0) != nullptr || (ev1) != nullptr)                                                  \
      hipExtLaunchKernelGGL((kern), dim3(grid), dim3(block), (shmem), (st), (ev0), (ev1), 0, __VA_ARGS__); \
    else                                                                                       \
      hipLaunchKernelGGL((kern), dim3(grid), dim3(block), (shmem), (st), __VA_ARGS__);          \
  } while (0)

// ---------------------------------------------------------------------------
// Grid geometry passed by value to the field kernels.
// ---------------------------------------------------------------------------
struct Grid {
  int n0, n1, n2;
  long long N;           // n0 * n1 * n2 (3 N < 2^31 is checked at creation)
  double h0, h1, h2;     // 2 pi / N_d
  int rowvec = 0;        // voxels per lane of the row-vectorised stencil kernels (0: one per thread)
  int pair_rows = 1;     // row-vectorised stencils: x1 rows shared by the two halves of a wave
};

FieldTiling make_field_tiling(const Grid& g);

// Voxel (i0, i1, i2) of the calling thread under tiling t; false outside the grid.
__device__ __forceinline__ bool tile_voxel(const FieldTiling& t, int n1, int n2, int& i0, int& i1, int& i2) {
  return tile_voxel_at(t, int(blockIdx.x), int(threadIdx.x), int(threadIdx.y), n1, n2, i0, i1, i2);
}

// ---------------------------------------------------------------------------
// Spectral operator: 3D real FFT, symbol (1 + alpha |k|^2)^(+-s), inverse.
// ---------------------------------------------------------------------------
// Launch shapes of the transform kernels (see fft.hip); chosen per grid and dtype.
struct FftTuning {
  int plane_threads = 512;   // 256, 512 or 1024 threads per (x1, x2) plane workgroup
  int pencil_threads = 256;  // 256 or 512 threads per pencil workgroup
  int pencil_tb = 32;        // contiguous pencils per workgroup
  int rows_rb = 16;          // rows per workgroup on the split path
  int force_split = 0;       // 1: use the split path even where the plane fits the LDS
  int use_static = 1;        // 1: compile-time kernels where instantiated (power-of-two lengths)
  int plane_grid = 0;        // 0: one (x1, x2) plane per workgroup; G > 0: G workgroups walk the planes
  int plane_halves = 0;      // 1: even and odd x1 rows of a plane as two units, merged in the x0 pencil pass
};

template <typename T>
struct SpectralPlan {
  int n0 = 0, n1 = 0, n2 = 0, H = 0, M = 0;  // H = n2 / 2, M = H + 1 spectrum columns
  FftPlan p0{}, p1{}, p2{};                  // lengths n0, n1, H
  cplx<T>* tw0 = nullptr;                    // exp(-2 pi i m / n0), m < n0
  cplx<T>* tw1 = nullptr;                    // exp(-2 pi i m / n1)
  cplx<T>* tw2 = nullptr;                    // exp(-2 pi i m / H)
  cplx<T>* twr = nullptr;                    // exp(-2 pi i k / n2), k <= H / 2
  int* slot2 = nullptr;                      // x2 frequency k (0..H) -> spectrum column
  T* ksq0 = nullptr;                         // squared wavenumber of each slot, per axis
  T* ksq1 = nullptr;
  T* ksq2 = nullptr;
  cplx<T>* spec = nullptr;                   // workspace: 3 * n0 * n1 * M complex
  void* table_mem = nullptr;                 // device block holding the tables above
  bool owns_memory = true;                   // false: tables and spectrum live in a caller's region
  FftPlan p1h{};                             // length n1 / 2 (half planes; n = 0 when n1 is odd)
  cplx<T>* tw1h = nullptr;                   // exp(-2 pi i m / (n1 / 2))
  cplx<T>* twx = nullptr;                    // exp(-2 pi i k1 / n1) per slot of the half transform
  T* ksq1x = nullptr;                        // |k1|^2, then |k1 + n1/2|^2, per slot of the half transform
  bool fused = false;                        // (x2, x1) plane fits one workgroup's LDS
  bool halves = false;                       // half planes in use
  size_t plane_lds = 0, pencil0_lds = 0, pencil1_lds = 0, rows_lds = 0;
  size_t max_lds = 0;                        // LDS bytes available to one workgroup
  FftTuning tune{};
  void* kfn[8] = {};                         // kernel entry points chosen by spectral_configure
  int static_kernels = 0;                    // how many of them are compile-time variants
  int plane_grid = 0;                        // workgroups of the plane walk in use (0: one plane each)
  size_t bytes = 0;                          // device memory held
};

// Returns 0 or a negative LDDMM_E* code.  max_lds = bytes of LDS per workgroup.
template <typename T>
int spectral_init(SpectralPlan<T>& sp, const int n[3], size_t max_lds, std::string& err);
// The same plan with its tables and a spectrum workspace for ncomp components
// placed in a caller-provided device region of region_bytes (nothing is
// allocated): the tables are copied there on stream st, after and before a
// synchronisation of st; host_tables keeps their host image.  LDDMM_EUNSUPPORTED
// (with the bytes needed in err) if the region is too small.
template <typename T>
int spectral_init_in(SpectralPlan<T>& sp, const int n[3], int ncomp, size_t max_lds, unsigned char* region,
                     size_t region_bytes, hipStream_t st, std::vector<unsigned char>& host_tables,
                     std::string& err);
// Bytes of the spectrum workspace for ncomp components.
template <typename T>
size_t spectrum_bytes(const SpectralPlan<T>& sp, int ncomp);
template <typename T>
void spectral_free(SpectralPlan<T>& sp);
// Apply new launch shapes; LDDMM_EINVAL / LDDMM_EUNSUPPORTED if they do not fit.
template <typename T>
int spectral_configure(SpectralPlan<T>& sp, const FftTuning& tune, std::string& err);
template <typename T>
FftTuning default_tuning(const SpectralPlan<T>& sp);
// out = K in (op = 0) or L in (op = 1) for ncomp components, times out_scale;
// in == out allowed.  With add != nullptr: out = add + add_scale * out_scale *
// (K or L) in, add == out allowed.
template <typename T>
void spectral_apply(const SpectralPlan<T>& sp, const T* in, T* out, int ncomp, double alpha, int s, int op,
                    hipStream_t st, Profiler* prof, const T* add = nullptr, double add_scale = 0.0,
                    double out_scale = 1.0);

// ---------------------------------------------------------------------------
// Field kernels (stencils, Heun stages, final conditions) - stencil.hip
// ---------------------------------------------------------------------------
// mu_out = a0 * mu0 + a1 * (mu - dt ad*_v mu)      (EPDiff stage, momentum form)
template <typename T>
void launch_epdiff_stage(const Grid& g, const T* v, const T* mu, const T* mu0, T* mu_out, double dt, double a0,
                         double a1, hipStream_t st, Profiler* prof);
// Tangent stage at coefficients (v, mu) with W = K dmu:
//   X_out   = a0 X0   + a1 (X   + dt (W + ad_v X))
//   dmu_out = a0 dmu0 + a1 (dmu + dt (-ad*_W mu - ad*_v dmu))
// With Gfin: X_out receives cfin (Gfin . X_new) Gfin instead and dmu_out is not
// written (the last stage of the sweep feeding the GN final condition).
// zero (row-vectorised kernels only, see stencil_zero_start): 1, X is zero and
// not read; 2, X0 is zero and not read.
template <typename T>
void launch_tangent_stage(const Grid& g, const T* X, const T* dmu, const T* W, const T* v, const T* mu,
                          const T* X0, const T* dmu0, T* X_out, T* dmu_out, double dt, double a0, double a1,
                          hipStream_t st, Profiler* prof, const T* Gfin = nullptr, double cfin = 0.0, int zero = 0);
// Full Newton sweep (first-order adjoint terms kept).
// Fused Newton stage with the K application left out (W = K dmu):
//   Z = dU + ad*_dw mu + ad*_w1 dmu;  Q = a0 dw0 + a1 (dw - dt (ad_v dw + ad_W w1));
//   dU_out = a0 dU0 + a1 (dU + dt (ad*_v dU + ad*_W U1));  then dw_out = Q + a1 dt K Z
template <typename T>
void launch_newton_stage(const Grid& g, const T* dU, const T* dw, const T* mu, const T* w1, const T* dmu, const T* v,
                         const T* Wv, const T* U1, const T* dU0, const T* dw0, T* Z, T* Q, T* dU_out, double dt,
                         double a0, double a1, hipStream_t st, Profiler* prof);
// Newton final condition: s = -G.X, U = c s G + c r grad_h s
template <typename T>
void launch_newton_final(const Grid& g, const T* G, const T* X, const T* r, double c, T* s, T* U, hipStream_t st,
                         Profiler* prof);
// Adjoint stage at (v, mu) with the K application left out:
//   Z     = U + ad*_w mu                        (argument of K)
//   Q     = a0 w0 + a1 (w - dt ad_v w)          (then w_out = Q + a1 dt K Z)
//   U_out = a0 U0 + a1 (U + dt ad*_v U)
// With qadd: Q += qs qadd (the last stage adds 2 v of the V-gradient 2 v + w_0).
// zero (row-vectorised kernels only): 2, w0 is zero and not read.
template <typename T>
void launch_adjoint_stage(const Grid& g, const T* U, const T* w, const T* mu, const T* v, const T* U0, const T* w0,
                          T* Z, T* Q, T* U_out, double dt, double a0, double a1, hipStream_t st, Profiler* prof,
                          const T* qadd = nullptr, double qs = 0.0, int zero = 0);
// True when the stage launchers honour `zero` (the row-vectorised kernels run);
// otherwise the caller provides the zero fields.
bool stencil_zero_start(const Grid& g);
// r = J1 - I1, G = grad_h J1
template <typename T>
void launch_residual_grad(const Grid& g, const T* J1, const T* I1, T* r, T* G, hipStream_t st, Profiler* prof);
// U = c * s * G  (pointwise scalar s times the vector G)
template <typename T>
void launch_scalar_times_vec(const Grid& g, const T* s, const T* G, double c, T* U, hipStream_t st,
                             Profiler* prof);
// U = c * (G . X) G
template <typename T>
void launch_gn_final(const Grid& g, const T* G, const T* X, double c, T* U, hipStream_t st, Profiler* prof);
// det = det(I + D_h u)
template <typename T>
void launch_jacobian_det(const Grid& g, const T* u, T* det, hipStream_t st, Profiler* prof);

// ---------------------------------------------------------------------------
// Semi-Lagrangian transport - sl.hip
// ---------------------------------------------------------------------------
// u_new(x) = u_old(X) + (X - x), X = x - dt/2 (v_new(x) + v_old(x - dt v_new(x)))
template <typename T>
void launch_sl_step(const Grid& g, const T* u_old, const T* v_old, const T* v_new, T* u_new, double dt,
                    hipStream_t st, Profiler* prof);
// J(x) = I(x + u(x))
template <typename T>
void launch_compose(const Grid& g, const T* I, const T* u, T* J, hipStream_t st, Profiler* prof);

// PDE-LDDMM (Section 2.3, the comparison method): the image transported by the
// state equation, the adjoint (continuity) equation, the incremental state.
// m_new(x) = m_old(X), X the Heun foot of launch_sl_step
template <typename T>
void launch_pde_state(const Grid& g, const T* m_old, const T* v_old, const T* v_new, T* m_new, double dt,
                      hipStream_t st, Profiler* prof);
// dm_new(x) = dm_old(X) + dt/2 (s_old(X) + s_new(x))
template <typename T>
void launch_pde_incr(const Grid& g, const T* dm_old, const T* s_old, const T* s_new, const T* v_old, const T* v_new,
                     T* dm_new, double dt, hipStream_t st, Profiler* prof);
// lam_old(x) = lam_new(Y) exp(dt/2 (D_old(x) + D_new(Y))), Y = x + dt/2 (v_old(x) + v_new(x + dt v_old(x)))
template <typename T>
void launch_pde_adjoint(const Grid& g, const T* lam_new, const T* D_old, const T* D_new, const T* v_old,
                        const T* v_new, T* lam_old, double dt, hipStream_t st, Profiler* prof);
// D = div_h v
template <typename T>
void launch_div(const Grid& g, const T* v, T* D, hipStream_t st, Profiler* prof);
// out += w lam grad_h m
template <typename T>
void launch_pde_lambda_grad(const Grid& g, const T* m, const T* lam, double w, T* out, hipStream_t st,
                            Profiler* prof);
// s = -grad_h m . dv
template <typename T>
void launch_pde_source(const Grid& g, const T* m, const T* dv, T* s, hipStream_t st, Profiler* prof);

// ---------------------------------------------------------------------------
// Reductions and BLAS-1 - reduce.hip.  Reductions are deterministic two-stage
// (fixed grid, fixed summation order, no atomics) and accumulate in double.
// ---------------------------------------------------------------------------
constexpr int kReduceBlocks = 1024;
// out[0] = sum_i a[i] * b[i] over n elements (partials: kReduceBlocks doubles)
template <typename T>
void launch_dot(const T* a, const T* b, long long n, double* partials, double* out, hipStream_t st,
                Profiler* prof);
// out[0] = number of non-finite entries, out[1] = max |a|
template <typename T>
void launch_check(const T* a, long long n, double* partials, double* out, hipStream_t st, Profiler* prof);
// out[0] = min a, out[1] = max a
template <typename T>
void launch_minmax(const T* a, long long n, double* partials, double* out, hipStream_t st, Profiler* prof);
// y = alpha x + beta y
template <typename T>
void launch_axpby(long long n, double alpha, const T* x, double beta, T* y, hipStream_t st, Profiler* prof);
// z = alpha x + beta y
// CG step on the device: a = rr / (cell * dsum[0]) if that is positive, else 0;
// x += a d, r -= a q.
template <typename T>
void launch_cg_step(long long n, double rr, double cell, const double* dsum, const T* d, const T* q, T* x, T* r,
                    hipStream_t st, Profiler* prof);
template <typename T>
void launch_axpbyz(long long n, double alpha, const T* x, double beta, const T* y, T* z, hipStream_t st,
                   Profiler* prof);
template <typename T>
void launch_fill(long long n, T value, T* y, hipStream_t st, Profiler* prof);

// CG with its scalars on the device: a block of kCgSlots doubles per solve.
// num / stop / curv point at FP64 sums (cell factor not applied) left by
// launch_dot.  V-CG: num = stop = <L r, r>; PCG in L2: num = <r, K r>, stop =
// <r, r>.  The host reads CG_ACTIVE / CG_ITERS to end early; nothing else needs it.
enum { CG_RZ = 0, CG_TOL, CG_ACTIVE, CG_AX, CG_AR, CG_BETA, CG_ITERS, CG_NEGCURV, CG_MAXIT, CG_FIRSTD, kCgSlots };
// first_d: non-positive curvature on the first direction returns x = d (CG in V)
void launch_cg_begin(double* s, const double* num, const double* stop, double cell, double eta, int maxit,
                     int first_d, hipStream_t st, Profiler* prof);
// step lengths from <d, H d>; counts the iteration or stops on non-positive curvature
void launch_cg_alpha(double* s, const double* curv, double cell, hipStream_t st, Profiler* prof);
// stop test on the new residual (or at maxit iterations), else beta and the next numerator
void launch_cg_beta(double* s, const double* num, const double* stop, double cell, hipStream_t st, Profiler* prof);
template <typename T>
void launch_cg_step_dev(long long n, const double* s, const T* d, const T* q, T* x, T* r, hipStream_t st,
                        Profiler* prof);
// y = x + beta y
template <typename T>
void launch_cg_direction(long long n, const double* s, const T* x, T* y, hipStream_t st, Profiler* prof);

}  // namespace lddmm
