// sl.hip - semi-Lagrangian transport of the state equation (Section 2.3:
// d_t J + grad J . v = 0, J(0) = I_0) through the inverse-map displacement
// u = phi^-1 - id, and the final composition J_1 = I_0 o (id + u_1).
//
// One step, with grid-time velocities v_old = v_n and v_new = v_{n+1}:
//   foot point  X = x - dt/2 (v_new(x) + v_old(x - dt v_new(x)))   (Heun backtrace)
//   u_new(x)    = u_old(X) + (X - x)
// Interpolation is periodic trilinear.  Each voxel's query point is handled as
// its integer index plus a small offset in voxels, so the fractional weights
// keep full precision in FP32 at any grid index.
#include "lddmm.h"
#include "lddmm_internal.h"

namespace lddmm {

namespace {

template <typename T>
struct SlGeo {
  int n0, n1, n2;
  int N;
  T invh[3];
  FieldTiling ft;
};

template <typename T>
SlGeo<T> make_sl_geo(const Grid& g) {
  SlGeo<T> o;
  o.n0 = g.n0;
  o.n1 = g.n1;
  o.n2 = g.n2;
  o.N = g.N;
  o.invh[0] = T(1.0 / g.h0);
  o.invh[1] = T(1.0 / g.h1);
  o.invh[2] = T(1.0 / g.h2);
  o.ft = make_field_tiling(g);
  return o;
}

// Corners and weights of the trilinear stencil at voxel (i0, i1, i2) displaced by
// (d0, d1, d2) voxels.  The two x2 corners of each (x0, x1) pair are adjacent in
// memory unless the lower one is the last of its row (periodic wrap), so a pair
// is one two-element load: o[k] is the lower corner of pair k = 2 c0 + c1, wrap
// says the upper corner is the first of the row (o[k] - (N2 - 1)).
template <typename T>
struct Tri {
  int o[4];
  int n2m1;
  bool wrap;
  T w01[4];   // (x0, x1) weight of pair k
  T t2;       // x2 fraction: weights 1 - t2, t2 of the lower and upper corner
};

template <typename T>
__device__ __forceinline__ Tri<T> tri_setup(const SlGeo<T>& g, int i0, int i1, int i2, T d0, T d1, T d2) {
  // cells and weights per axis (offsets clamped, indices wrapped: sl_axis)
  int a0, b0, a1, b1, a2, b2;
  T t0, t1, t2;
  sl_axis(i0, d0, g.n0, a0, b0, t0);
  sl_axis(i1, d1, g.n1, a1, b1, t1);
  sl_axis(i2, d2, g.n2, a2, b2, t2);
  (void)b2;
  const int s0 = g.n1 * g.n2;
  const int r0[2] = {a0 * s0, b0 * s0};
  const int r1[2] = {a1 * g.n2, b1 * g.n2};
  const T w0[2] = {T(1) - t0, t0}, w1[2] = {T(1) - t1, t1};
  Tri<T> tr;
  // offsets fit in int: 3 N < 2^31
#pragma unroll
  for (int c0 = 0; c0 < 2; ++c0)
#pragma unroll
    for (int c1 = 0; c1 < 2; ++c1) {
      const int k = c0 * 2 + c1;
      tr.o[k] = r0[c0] + r1[c1] + a2;
      tr.w01[k] = w0[c0] * w1[c1];
    }
  tr.n2m1 = g.n2 - 1;
  tr.wrap = a2 == g.n2 - 1;
  tr.t2 = t2;
  return tr;
}

// Two consecutive elements f[o], f[o + 1] as one 8-byte load (4-byte aligned:
// the hardware takes element-aligned vector loads from global memory).
__device__ __forceinline__ void load_pair(const float* __restrict__ f, int o, float& lo, float& hi) {
  typedef float vec2 __attribute__((ext_vector_type(2)));
  vec2 v;
  __builtin_memcpy(&v, f + o, sizeof(vec2));
  lo = v.x;
  hi = v.y;
}

// FP32 reads each x2 pair with one load (half the gathers); FP64 reads the
// corners one by one (its 16-byte pairs measured slower than two loads).
template <typename T>
__device__ __forceinline__ T tri_eval(const Tri<T>& tr, const T* __restrict__ f) {
  T acc = T(0);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    T lo, hi;
    if constexpr (sizeof(T) == 4) {
      if (!tr.wrap) {
        load_pair(f, tr.o[k], lo, hi);
      } else {
        lo = f[tr.o[k]];
        hi = f[tr.o[k] - tr.n2m1];
      }
    } else {
      lo = f[tr.o[k]];
      hi = f[tr.wrap ? tr.o[k] - tr.n2m1 : tr.o[k] + 1];
    }
    acc += tr.w01[k] * (lo + tr.t2 * (hi - lo));
  }
  return acc;
}

template <typename T>
__global__ void __launch_bounds__(256)
    k_sl_step(SlGeo<T> g, const T* __restrict__ u_old, const T* __restrict__ v_old, const T* __restrict__ v_new,
              T* __restrict__ u_new, T dt) {
  int i0, i1, i2;
  if (!tile_voxel(g.ft, g.n1, g.n2, i0, i1, i2)) return;
  const int o = (i0 * g.n1 + i1) * g.n2 + i2;
  T vn[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) vn[c] = v_new[c * g.N + o];
  const Tri<T> tp = tri_setup(g, i0, i1, i2, -dt * vn[0] * g.invh[0], -dt * vn[1] * g.invh[1], -dt * vn[2] * g.invh[2]);
  T disp[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) disp[c] = T(-0.5) * dt * (vn[c] + tri_eval(tp, v_old + c * g.N));
  const Tri<T> tx = tri_setup(g, i0, i1, i2, disp[0] * g.invh[0], disp[1] * g.invh[1], disp[2] * g.invh[2]);
#pragma unroll
  for (int c = 0; c < 3; ++c) u_new[c * g.N + o] = tri_eval(tx, u_old + c * g.N) + disp[c];
}

template <typename T>
__global__ void __launch_bounds__(256)
    k_compose(SlGeo<T> g, const T* __restrict__ I, const T* __restrict__ u, T* __restrict__ J) {
  int i0, i1, i2;
  if (!tile_voxel(g.ft, g.n1, g.n2, i0, i1, i2)) return;
  const int o = (i0 * g.n1 + i1) * g.n2 + i2;
  const Tri<T> t = tri_setup(g, i0, i1, i2, u[o] * g.invh[0], u[g.N + o] * g.invh[1], u[2 * g.N + o] * g.invh[2]);
  J[o] = tri_eval(t, I);
}

// ---------------------------------------------------------------------------
// PDE-LDDMM (Section 2.3): the image itself transported by the state equation,
// the adjoint (continuity) equation along forward characteristics, the
// incremental state with its source term.
// ---------------------------------------------------------------------------
// m_new(x) = m_old(X), X = x - dt/2 (v_new(x) + v_old(x - dt v_new(x)))
template <typename T>
__global__ void __launch_bounds__(256)
    k_pde_state(SlGeo<T> g, const T* __restrict__ m_old, const T* __restrict__ v_old, const T* __restrict__ v_new,
                T* __restrict__ m_new, T dt) {
  int i0, i1, i2;
  if (!tile_voxel(g.ft, g.n1, g.n2, i0, i1, i2)) return;
  const int o = (i0 * g.n1 + i1) * g.n2 + i2;
  T vn[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) vn[c] = v_new[c * g.N + o];
  const Tri<T> tp = tri_setup(g, i0, i1, i2, -dt * vn[0] * g.invh[0], -dt * vn[1] * g.invh[1], -dt * vn[2] * g.invh[2]);
  T disp[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) disp[c] = T(-0.5) * dt * (vn[c] + tri_eval(tp, v_old + c * g.N));
  const Tri<T> tx = tri_setup(g, i0, i1, i2, disp[0] * g.invh[0], disp[1] * g.invh[1], disp[2] * g.invh[2]);
  m_new[o] = tri_eval(tx, m_old);
}

// dm_new(x) = dm_old(X) + dt/2 (s_old(X) + s_new(x)), X as in k_pde_state
template <typename T>
__global__ void __launch_bounds__(256)
    k_pde_incr(SlGeo<T> g, const T* __restrict__ dm_old, const T* __restrict__ s_old, const T* __restrict__ s_new,
               const T* __restrict__ v_old, const T* __restrict__ v_new, T* __restrict__ dm_new, T dt) {
  int i0, i1, i2;
  if (!tile_voxel(g.ft, g.n1, g.n2, i0, i1, i2)) return;
  const int o = (i0 * g.n1 + i1) * g.n2 + i2;
  T vn[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) vn[c] = v_new[c * g.N + o];
  const Tri<T> tp = tri_setup(g, i0, i1, i2, -dt * vn[0] * g.invh[0], -dt * vn[1] * g.invh[1], -dt * vn[2] * g.invh[2]);
  T disp[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) disp[c] = T(-0.5) * dt * (vn[c] + tri_eval(tp, v_old + c * g.N));
  const Tri<T> tx = tri_setup(g, i0, i1, i2, disp[0] * g.invh[0], disp[1] * g.invh[1], disp[2] * g.invh[2]);
  dm_new[o] = tri_eval(tx, dm_old) + T(0.5) * dt * (tri_eval(tx, s_old) + s_new[o]);
}

// lam_old(x) = lam_new(Y) exp(dt/2 (D_old(x) + D_new(Y))),
// Y = x + dt/2 (v_old(x) + v_new(x + dt v_old(x))), D = div v
template <typename T>
__global__ void __launch_bounds__(256)
    k_pde_adjoint(SlGeo<T> g, const T* __restrict__ lam_new, const T* __restrict__ D_old, const T* __restrict__ D_new,
                  const T* __restrict__ v_old, const T* __restrict__ v_new, T* __restrict__ lam_old, T dt) {
  int i0, i1, i2;
  if (!tile_voxel(g.ft, g.n1, g.n2, i0, i1, i2)) return;
  const int o = (i0 * g.n1 + i1) * g.n2 + i2;
  T vo[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) vo[c] = v_old[c * g.N + o];
  const Tri<T> tp = tri_setup(g, i0, i1, i2, dt * vo[0] * g.invh[0], dt * vo[1] * g.invh[1], dt * vo[2] * g.invh[2]);
  T disp[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) disp[c] = T(0.5) * dt * (vo[c] + tri_eval(tp, v_new + c * g.N));
  const Tri<T> ty = tri_setup(g, i0, i1, i2, disp[0] * g.invh[0], disp[1] * g.invh[1], disp[2] * g.invh[2]);
  lam_old[o] = tri_eval(ty, lam_new) * exp(T(0.5) * dt * (D_old[o] + tri_eval(ty, D_new)));
}

// D = div_h v (central differences)
template <typename T>
__global__ void __launch_bounds__(256) k_div(SlGeo<T> g, const T* __restrict__ v, T* __restrict__ D) {
  int i0, i1, i2;
  if (!tile_voxel(g.ft, g.n1, g.n2, i0, i1, i2)) return;
  const int s0 = g.n1 * g.n2;
  const int o = i0 * s0 + i1 * g.n2 + i2;
  const int p0 = periodic_next(i0, g.n0) * s0 + i1 * g.n2 + i2, m0 = periodic_prev(i0, g.n0) * s0 + i1 * g.n2 + i2;
  const int p1 = i0 * s0 + periodic_next(i1, g.n1) * g.n2 + i2, m1 = i0 * s0 + periodic_prev(i1, g.n1) * g.n2 + i2;
  const int p2 = i0 * s0 + i1 * g.n2 + periodic_next(i2, g.n2), m2 = i0 * s0 + i1 * g.n2 + periodic_prev(i2, g.n2);
  D[o] = T(0.5) * (g.invh[0] * (v[p0] - v[m0]) + g.invh[1] * (v[g.N + p1] - v[g.N + m1]) +
                   g.invh[2] * (v[2 * g.N + p2] - v[2 * g.N + m2]));
}

// With ssrc: s = -grad_h m . dv (the incremental state's source) into ssrc.
// Else out += w lam grad_h m (a time point's term of the gradient or Hessian).
template <typename T>
__global__ void __launch_bounds__(256)
    k_pde_grad_m(SlGeo<T> g, const T* __restrict__ m, const T* __restrict__ lam, const T* __restrict__ dv, T w,
                 T* __restrict__ out, T* __restrict__ ssrc) {
  int i0, i1, i2;
  if (!tile_voxel(g.ft, g.n1, g.n2, i0, i1, i2)) return;
  const int s0 = g.n1 * g.n2;
  const int o = i0 * s0 + i1 * g.n2 + i2;
  T gm[3];
  gm[0] = T(0.5) * g.invh[0] * (m[periodic_next(i0, g.n0) * s0 + i1 * g.n2 + i2] - m[periodic_prev(i0, g.n0) * s0 + i1 * g.n2 + i2]);
  gm[1] = T(0.5) * g.invh[1] * (m[i0 * s0 + periodic_next(i1, g.n1) * g.n2 + i2] - m[i0 * s0 + periodic_prev(i1, g.n1) * g.n2 + i2]);
  gm[2] = T(0.5) * g.invh[2] * (m[i0 * s0 + i1 * g.n2 + periodic_next(i2, g.n2)] - m[i0 * s0 + i1 * g.n2 + periodic_prev(i2, g.n2)]);
  if (ssrc) {
    ssrc[o] = -(gm[0] * dv[o] + gm[1] * dv[g.N + o] + gm[2] * dv[2 * g.N + o]);
    return;
  }
  const T a = w * lam[o];
#pragma unroll
  for (int c = 0; c < 3; ++c) out[c * g.N + o] += a * gm[c];
}

}  // namespace

template <typename T>
void launch_pde_state(const Grid& g, const T* m_old, const T* v_old, const T* v_new, T* m_new, double dt,
                      hipStream_t st, Profiler* prof) {
  KernelTimer t(prof, "pde_state");
  const FieldTiling ft = make_field_tiling(g);
  LDDMM_LAUNCH(t.start, t.stop, k_pde_state<T>, ft.blocks, dim3(ft.BX, ft.BY), 0, st, make_sl_geo<T>(g), m_old, v_old, v_new, m_new, T(dt));
}

template <typename T>
void launch_pde_incr(const Grid& g, const T* dm_old, const T* s_old, const T* s_new, const T* v_old, const T* v_new,
                     T* dm_new, double dt, hipStream_t st, Profiler* prof) {
  KernelTimer t(prof, "pde_incremental_state");
  const FieldTiling ft = make_field_tiling(g);
  LDDMM_LAUNCH(t.start, t.stop, k_pde_incr<T>, ft.blocks, dim3(ft.BX, ft.BY), 0, st, make_sl_geo<T>(g), dm_old, s_old, s_new, v_old, v_new, dm_new, T(dt));
}

template <typename T>
void launch_pde_adjoint(const Grid& g, const T* lam_new, const T* D_old, const T* D_new, const T* v_old,
                        const T* v_new, T* lam_old, double dt, hipStream_t st, Profiler* prof) {
  KernelTimer t(prof, "pde_adjoint");
  const FieldTiling ft = make_field_tiling(g);
  LDDMM_LAUNCH(t.start, t.stop, k_pde_adjoint<T>, ft.blocks, dim3(ft.BX, ft.BY), 0, st, make_sl_geo<T>(g), lam_new, D_old, D_new, v_old, v_new, lam_old, T(dt));
}

template <typename T>
void launch_div(const Grid& g, const T* v, T* D, hipStream_t st, Profiler* prof) {
  KernelTimer t(prof, "divergence");
  const FieldTiling ft = make_field_tiling(g);
  LDDMM_LAUNCH(t.start, t.stop, k_div<T>, ft.blocks, dim3(ft.BX, ft.BY), 0, st, make_sl_geo<T>(g), v, D);
}

template <typename T>
void launch_pde_lambda_grad(const Grid& g, const T* m, const T* lam, double w, T* out, hipStream_t st,
                            Profiler* prof) {
  KernelTimer t(prof, "pde_lambda_grad_m");
  const FieldTiling ft = make_field_tiling(g);
  LDDMM_LAUNCH(t.start, t.stop, k_pde_grad_m<T>, ft.blocks, dim3(ft.BX, ft.BY), 0, st, make_sl_geo<T>(g), m, lam, static_cast<const T*>(nullptr), T(w), out, static_cast<T*>(nullptr));
}

template <typename T>
void launch_pde_source(const Grid& g, const T* m, const T* dv, T* s, hipStream_t st, Profiler* prof) {
  KernelTimer t(prof, "pde_source");
  const FieldTiling ft = make_field_tiling(g);
  LDDMM_LAUNCH(t.start, t.stop, k_pde_grad_m<T>, ft.blocks, dim3(ft.BX, ft.BY), 0, st, make_sl_geo<T>(g), m, static_cast<const T*>(nullptr), dv, T(0), static_cast<T*>(nullptr), s);
}

template <typename T>
void launch_sl_step(const Grid& g, const T* u_old, const T* v_old, const T* v_new, T* u_new, double dt,
                    hipStream_t st, Profiler* prof) {
  KernelTimer t(prof, "sl_step");
  const FieldTiling ft = make_field_tiling(g);
  LDDMM_LAUNCH(t.start, t.stop, k_sl_step<T>, ft.blocks, dim3(ft.BX, ft.BY), 0, st, make_sl_geo<T>(g), u_old, v_old, v_new, u_new, T(dt));
}

template <typename T>
void launch_compose(const Grid& g, const T* I, const T* u, T* J, hipStream_t st, Profiler* prof) {
  KernelTimer t(prof, "compose");
  const FieldTiling ft = make_field_tiling(g);
  LDDMM_LAUNCH(t.start, t.stop, k_compose<T>, ft.blocks, dim3(ft.BX, ft.BY), 0, st, make_sl_geo<T>(g), I, u, J);
}

template void launch_sl_step<float>(const Grid&, const float*, const float*, const float*, float*, double,
                                    hipStream_t, Profiler*);
template void launch_sl_step<double>(const Grid&, const double*, const double*, const double*, double*, double,
                                     hipStream_t, Profiler*);
template void launch_compose<float>(const Grid&, const float*, const float*, float*, hipStream_t, Profiler*);
template void launch_compose<double>(const Grid&, const double*, const double*, double*, hipStream_t, Profiler*);

#define LDDMM_PDE_INST(T)                                                                                       \
  template void launch_pde_state<T>(const Grid&, const T*, const T*, const T*, T*, double, hipStream_t, Profiler*); \
  template void launch_pde_incr<T>(const Grid&, const T*, const T*, const T*, const T*, const T*, T*, double,      \
                                   hipStream_t, Profiler*);                                                     \
  template void launch_pde_adjoint<T>(const Grid&, const T*, const T*, const T*, const T*, const T*, T*, double,   \
                                      hipStream_t, Profiler*);                                                  \
  template void launch_div<T>(const Grid&, const T*, T*, hipStream_t, Profiler*);                               \
  template void launch_pde_lambda_grad<T>(const Grid&, const T*, const T*, double, T*, hipStream_t, Profiler*);  \
  template void launch_pde_source<T>(const Grid&, const T*, const T*, T*, hipStream_t, Profiler*);
LDDMM_PDE_INST(float)
LDDMM_PDE_INST(double)

}  // namespace lddmm
