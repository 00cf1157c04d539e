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

}  // namespace

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

}  // namespace lddmm
