// stencil.hip - pointwise and 7-point-stencil kernels of the EPDiff shooting and
// of the tangent / adjoint Jacobi sweeps.
//
// Operators (periodic grid, second-order central differences delta_d):
//   (Dv)_{cd}      = delta_d v_c
//   ad_v w         = (Dv) w - (Dw) v                          (Jacobi field, Section 3)
//   ad*_v mu       = (Dv)^T mu + sum_d delta_d(mu v_d)        (EPDiff, Section 2.2)
// ad* is the conservative form of the paper's (Dv)^T Lv + D(Lv) v + Lv div v; on
// the grid it is the exact transpose of ad_v, which keeps the adjoint sweep the
// exact transpose of the tangent sweep.
//
// Two forms of each stage kernel: one voxel per thread, and row-vectorised (a
// lane owns VW consecutive voxels of an x2 row, x2 neighbours come from the
// adjacent lanes, x1 rows may be shared by the two halves of a wave).  Blocks are
// laid out XCD-aware (FieldTiling); neighbours come through the cache hierarchy.
// The adjoint and Newton stages leave their K application out: they write K's
// argument and the rest of the w update, and the inverse transform adds the K
// term on its way out.
#include "lddmm.h"
#include "lddmm_internal.h"

namespace lddmm {

bool stencil_zero_start(const Grid& g) { return row_vector_valid(g.n2, g.rowvec); }

FieldTiling make_field_tiling(const Grid& g) { return field_tiling(g.n0, g.n1, g.n2); }

namespace {

template <typename T>
struct Geo {
  int n0, n1, n2;
  int N;  // voxels per component
  T inv2h[3];
  FieldTiling ft;
  int pair;  // launch the PAIR row-vectorised kernels: a wave holds two x1 rows (see VNbr)
};

template <typename T>
Geo<T> make_geo(const Grid& g) {
  Geo<T> o;
  o.n0 = g.n0;
  o.n1 = g.n1;
  o.n2 = g.n2;
  o.N = int(g.N);
  o.inv2h[0] = T(0.5 / g.h0);
  o.inv2h[1] = T(0.5 / g.h1);
  o.inv2h[2] = T(0.5 / g.h2);
  o.ft = make_field_tiling(g);
  o.pair = 0;
  return o;
}

// Linear offsets of the voxel and its six periodic neighbours:
// 0 centre, 1 +x0, 2 -x0, 3 +x1, 4 -x1, 5 +x2, 6 -x2.
struct Nbr {
  int o[7];
};

template <typename T>
__device__ __forceinline__ bool voxel(const Geo<T>& g, int& i0, int& i1, int& i2) {
  return tile_voxel(g.ft, g.n1, g.n2, i0, i1, i2);
}

template <typename T>
__device__ __forceinline__ Nbr neighbours(const Geo<T>& g, int i0, int i1, int i2) {
  const int p0 = periodic_next(i0, g.n0), m0 = periodic_prev(i0, g.n0);
  const int p1 = periodic_next(i1, g.n1), m1 = periodic_prev(i1, g.n1);
  const int p2 = periodic_next(i2, g.n2), m2 = periodic_prev(i2, g.n2);
  const int s0 = g.n1 * g.n2;
  const int r0 = i0 * s0, rp0 = p0 * s0, rm0 = m0 * s0;
  const int r1 = i1 * g.n2;
  Nbr n;
  n.o[0] = r0 + r1 + i2;
  n.o[1] = rp0 + r1 + i2;
  n.o[2] = rm0 + r1 + i2;
  n.o[3] = r0 + p1 * g.n2 + i2;
  n.o[4] = r0 + m1 * g.n2 + i2;
  n.o[5] = r0 + r1 + p2;
  n.o[6] = r0 + r1 + m2;
  return n;
}

// Three components of a vector field at the 7 stencil points.
template <typename T>
struct St7 {
  T f[7][3];
};

template <typename T>
__device__ __forceinline__ void load7(St7<T>& s, const T* __restrict__ p, const Nbr& nb, int N) {
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int k = 0; k < 7; ++k) s.f[k][c] = p[c * N + nb.o[k]];
}

template <typename T>
__device__ __forceinline__ void load1(T out[3], const T* __restrict__ p, int o, int N) {
#pragma unroll
  for (int c = 0; c < 3; ++c) out[c] = p[c * N + o];
}

template <typename T>
__device__ __forceinline__ void store1(T* __restrict__ p, const T v[3], int o, int N) {
#pragma unroll
  for (int c = 0; c < 3; ++c) p[c * N + o] = v[c];
}

// delta_d of component c
template <typename T>
__device__ __forceinline__ T dd(const St7<T>& s, int c, int d, const Geo<T>& g) {
  return (s.f[1 + 2 * d][c] - s.f[2 + 2 * d][c]) * g.inv2h[d];
}

// ad_v w = (Dv) w - (Dw) v at the centre
template <typename T>
__device__ __forceinline__ void ad(const St7<T>& v, const St7<T>& w, const Geo<T>& g, T out[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    T acc = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) acc += dd(v, c, d, g) * w.f[0][d] - dd(w, c, d, g) * v.f[0][d];
    out[c] = acc;
  }
}

// ad*_v mu = (Dv)^T mu + sum_d delta_d(mu v_d) at the centre
template <typename T>
__device__ __forceinline__ void adstar(const St7<T>& v, const St7<T>& mu, const Geo<T>& g, T out[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    T acc = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      acc += dd(v, d, c, g) * mu.f[0][d];
      acc += (mu.f[1 + 2 * d][c] * v.f[1 + 2 * d][d] - mu.f[2 + 2 * d][c] * v.f[2 + 2 * d][d]) * g.inv2h[d];
    }
    out[c] = acc;
  }
}

// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
    k_epdiff_stage(Geo<T> g, const T* __restrict__ v, const T* __restrict__ mu, const T* mu0, T* mu_out, T dt,
                   T a0, T a1) {
  int i0, i1, i2;
  if (!voxel(g, i0, i1, i2)) return;
  const Nbr nb = neighbours(g, i0, i1, i2);
  St7<T> V, Mu;
  load7(V, v, nb, g.N);
  load7(Mu, mu, nb, g.N);
  T a[3];
  adstar(V, Mu, g, a);
  T out[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) out[c] = a1 * (Mu.f[0][c] - dt * a[c]);
  if (a0 != T(0)) {
    T m0[3];
    load1(m0, mu0, nb.o[0], g.N);
#pragma unroll
    for (int c = 0; c < 3; ++c) out[c] += a0 * m0[c];
  }
  store1(mu_out, out, nb.o[0], g.N);
}

template <typename T>
__global__ void __launch_bounds__(256)
    k_tangent_stage(Geo<T> g, const T* __restrict__ X, const T* __restrict__ dmu, const T* __restrict__ W,
                    const T* __restrict__ v, const T* __restrict__ mu, const T* X0, const T* dmu0, T* X_out,
                    T* dmu_out, T dt, T a0, T a1, const T* __restrict__ Gf, T cf) {
  int i0, i1, i2;
  if (!voxel(g, i0, i1, i2)) return;
  const Nbr nb = neighbours(g, i0, i1, i2);
  St7<T> Xs, Ws, Vs;
  load7(Xs, X, nb, g.N);
  load7(Ws, W, nb, g.N);
  load7(Vs, v, nb, g.N);
  T aX[3];
  ad(Vs, Xs, g, aX);
  T xo[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) xo[c] = a1 * (Xs.f[0][c] + dt * (Ws.f[0][c] + aX[c]));
  St7<T> Ms, Ds;
  load7(Ms, mu, nb, g.N);
  load7(Ds, dmu, nb, g.N);
  T t1[3], t2[3];
  adstar(Ws, Ms, g, t1);
  adstar(Vs, Ds, g, t2);
  T mo[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) mo[c] = a1 * (Ds.f[0][c] - dt * (t1[c] + t2[c]));
  if (a0 != T(0)) {
    T x0v[3], m0v[3];
    load1(x0v, X0, nb.o[0], g.N);
    load1(m0v, dmu0, nb.o[0], g.N);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      xo[c] += a0 * x0v[c];
      mo[c] += a0 * m0v[c];
    }
  }
  if (Gf) {  // last stage of the sweep: X_out receives cf (G . X) G, dmu is not kept
    T gv[3];
    load1(gv, Gf, nb.o[0], g.N);
    const T sg = cf * (gv[0] * xo[0] + gv[1] * xo[1] + gv[2] * xo[2]);
#pragma unroll
    for (int c = 0; c < 3; ++c) xo[c] = sg * gv[c];
    store1(X_out, xo, nb.o[0], g.N);
    return;
  }
  store1(X_out, xo, nb.o[0], g.N);
  store1(dmu_out, mo, nb.o[0], g.N);
}

// Adjoint stage at (v, mu) except for K: Z = U + ad*_w mu is K's argument, and the
// w update is split as w_out = Q + a1 dt K Z with Q = a0 w0 + a1 (w - dt ad_v w),
// so the K pass adds a1 dt K Z to Q on its way out (the w stencil is read once).
template <typename T>
__global__ void __launch_bounds__(256)
    k_adjoint_stage(Geo<T> g, const T* __restrict__ U, const T* __restrict__ w, const T* __restrict__ mu,
                    const T* __restrict__ v, const T* U0, const T* w0, T* __restrict__ Z, T* __restrict__ Q,
                    T* U_out, T dt, T a0, T a1, const T* __restrict__ qadd, T qs) {
  int i0, i1, i2;
  if (!voxel(g, i0, i1, i2)) return;
  const Nbr nb = neighbours(g, i0, i1, i2);
  St7<T> Ws, Vs;
  load7(Ws, w, nb, g.N);
  load7(Vs, v, nb, g.N);
  T z[3], aw[3], aU[3];
  {
    St7<T> Ms;
    load7(Ms, mu, nb, g.N);
    adstar(Ws, Ms, g, z);  // ad*_w mu
  }
  ad(Vs, Ws, g, aw);  // ad_v w
  T u[3];
  {
    St7<T> Us;
    load7(Us, U, nb, g.N);
    adstar(Vs, Us, g, aU);  // ad*_v U
#pragma unroll
    for (int c = 0; c < 3; ++c) u[c] = Us.f[0][c];
  }
  T q[3], uo[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    z[c] += u[c];
    q[c] = a1 * (Ws.f[0][c] - dt * aw[c]);
    uo[c] = a1 * (u[c] + dt * aU[c]);
  }
  if (a0 != T(0)) {
    T u0[3], ww0[3];
    load1(u0, U0, nb.o[0], g.N);
    load1(ww0, w0, nb.o[0], g.N);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      uo[c] += a0 * u0[c];
      q[c] += a0 * ww0[c];
    }
  }
  if (qadd) {
    T qa[3];
    load1(qa, qadd, nb.o[0], g.N);
#pragma unroll
    for (int c = 0; c < 3; ++c) q[c] += qs * qa[c];
  }
  store1(Z, z, nb.o[0], g.N);
  store1(Q, q, nb.o[0], g.N);
  store1(U_out, uo, nb.o[0], g.N);
}

// ---------------------------------------------------------------------------
// Full Newton Hessian (Section 3 incremental adjoint Jacobi system with the
// first-order adjoint terms kept).  The sweep carries (dU, dw); (U1, w1) is the
// first-order adjoint at the same stage and (W, dmu) = (K dmu, dmu) the
// variation of the trajectory point.
// ---------------------------------------------------------------------------
// Fused Newton stage (the same split as the adjoint stage): with W = K dmu,
//   Z     = dU + ad*_dw mu + ad*_w1 dmu                        (argument of K)
//   Q     = a0 dw0 + a1 (dw - dt (ad_v dw + ad_W w1))          (dw_out = Q + a1 dt K Z)
//   dU_out = a0 dU0 + a1 (dU + dt (ad*_v dU + ad*_W U1))
template <typename T>
__global__ void __launch_bounds__(256)
    k_newton_stage(Geo<T> g, const T* __restrict__ dU, const T* __restrict__ dw, const T* __restrict__ mu,
                   const T* __restrict__ w1, const T* __restrict__ dmu, const T* __restrict__ v,
                   const T* __restrict__ Wv, const T* __restrict__ U1, const T* dU0, const T* dw0,
                   T* __restrict__ Z, T* __restrict__ Q, T* dU_out, T dt, T a0, T a1) {
  int i0, i1, i2;
  if (!voxel(g, i0, i1, i2)) return;
  const Nbr nb = neighbours(g, i0, i1, i2);
  T z[3], aU[3], aw[3], t[3], du[3], dwc[3];
  {
    St7<T> Dw, Vs;
    load7(Dw, dw, nb, g.N);
    load7(Vs, v, nb, g.N);
    {
      St7<T> M;
      load7(M, mu, nb, g.N);
      adstar(Dw, M, g, z);  // ad*_dw mu
    }
    ad(Vs, Dw, g, aw);  // ad_v dw
    St7<T> D;
    load7(D, dU, nb, g.N);
    adstar(Vs, D, g, aU);  // ad*_v dU
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      du[c] = D.f[0][c];
      dwc[c] = Dw.f[0][c];
    }
  }
  {
    St7<T> W1, Wk;
    load7(W1, w1, nb, g.N);
    {
      St7<T> Dm;
      load7(Dm, dmu, nb, g.N);
      adstar(W1, Dm, g, t);  // ad*_w1 dmu
#pragma unroll
      for (int c = 0; c < 3; ++c) z[c] += t[c];
    }
    load7(Wk, Wv, nb, g.N);
    ad(Wk, W1, g, t);  // ad_W w1
#pragma unroll
    for (int c = 0; c < 3; ++c) aw[c] += t[c];
    St7<T> A;
    load7(A, U1, nb, g.N);
    adstar(Wk, A, g, t);  // ad*_W U1
#pragma unroll
    for (int c = 0; c < 3; ++c) aU[c] += t[c];
  }
  T q[3], uo[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    z[c] += du[c];
    uo[c] = a1 * (du[c] + dt * aU[c]);
    q[c] = a1 * (dwc[c] - dt * aw[c]);
  }
  if (a0 != T(0)) {
    T u0[3], ww0[3];
    load1(u0, dU0, nb.o[0], g.N);
    load1(ww0, dw0, nb.o[0], g.N);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      uo[c] += a0 * u0[c];
      q[c] += a0 * ww0[c];
    }
  }
  store1(Z, z, nb.o[0], g.N);
  store1(Q, q, nb.o[0], g.N);
  store1(dU_out, uo, nb.o[0], g.N);
}

// delta m_1 = -grad J_1 . X (pointwise)
template <typename T>
__global__ void k_dm1(long long N, const T* __restrict__ G, const T* __restrict__ X, T* __restrict__ s) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x)
    s[i] = -(G[i] * X[i] + G[N + i] * X[N + i] + G[2 * N + i] * X[2 * N + i]);
}

// Newton final condition: U = c s grad J_1 + c r grad_h s  (c = -2/sigma^2:
// delta lambda_1 grad J_1 + lambda_1 grad(delta m_1) with lambda_1 = c r)
template <typename T>
__global__ void __launch_bounds__(256)
    k_newton_final(Geo<T> g, const T* __restrict__ s, const T* __restrict__ r, const T* __restrict__ G, T c,
                   T* __restrict__ U) {
  int i0, i1, i2;
  if (!voxel(g, i0, i1, i2)) return;
  const Nbr nb = neighbours(g, i0, i1, i2);
  const T s0 = s[nb.o[0]], r0 = r[nb.o[0]];
#pragma unroll
  for (int d = 0; d < 3; ++d)
    U[d * g.N + nb.o[0]] =
        c * s0 * G[d * g.N + nb.o[0]] + c * r0 * (s[nb.o[1 + 2 * d]] - s[nb.o[2 + 2 * d]]) * g.inv2h[d];
}

template <typename T>
__global__ void __launch_bounds__(256)
    k_residual_grad(Geo<T> g, const T* __restrict__ J1, const T* __restrict__ I1, T* __restrict__ r,
                    T* __restrict__ G) {
  int i0, i1, i2;
  if (!voxel(g, i0, i1, i2)) return;
  const Nbr nb = neighbours(g, i0, i1, i2);
  r[nb.o[0]] = J1[nb.o[0]] - I1[nb.o[0]];
#pragma unroll
  for (int d = 0; d < 3; ++d) G[d * g.N + nb.o[0]] = (J1[nb.o[1 + 2 * d]] - J1[nb.o[2 + 2 * d]]) * g.inv2h[d];
}

template <typename T>
__global__ void k_scalar_times_vec(long long N, const T* __restrict__ s, const T* __restrict__ G, T c,
                                   T* __restrict__ U) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x) {
    const T f = c * s[i];
#pragma unroll
    for (int d = 0; d < 3; ++d) U[d * N + i] = f * G[d * N + i];
  }
}

template <typename T>
__global__ void k_gn_final(long long N, const T* __restrict__ G, const T* __restrict__ X, T c, T* __restrict__ U) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x) {
    const T g0 = G[i], g1 = G[N + i], g2 = G[2 * N + i];
    const T f = c * (g0 * X[i] + g1 * X[N + i] + g2 * X[2 * N + i]);
    U[i] = f * g0;
    U[N + i] = f * g1;
    U[2 * N + i] = f * g2;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_jacobian_det(Geo<T> g, const T* __restrict__ u, T* __restrict__ det) {
  int i0, i1, i2;
  if (!voxel(g, i0, i1, i2)) return;
  const Nbr nb = neighbours(g, i0, i1, i2);
  T J[3][3];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int d = 0; d < 3; ++d)
      J[c][d] = (u[c * g.N + nb.o[1 + 2 * d]] - u[c * g.N + nb.o[2 + 2 * d]]) * g.inv2h[d] + (c == d ? T(1) : T(0));
  det[nb.o[0]] = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                 J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

// ---------------------------------------------------------------------------
// Row-vectorised variants for N2 = VW * RW with 32 <= RW <= 64 lanes.  A lane
// owns VW consecutive voxels of an x2 row and a row is RW consecutive lanes of
// one wavefront (rows of 32 lanes fill a half wave each, longer rows a whole
// wave with lanes RW..63 idle), so every x0 or x1 neighbour is one VW-wide load and the x2
// neighbours come from the two adjacent lanes (periodic inside the row).  Same
// operators as the kernels above, accumulated one direction at a time; about a
// third of their load instructions, which is what limits those kernels (the
// texture address and data units, not HBM, saturate first).
// ---------------------------------------------------------------------------
// Row-vectorised neighbourhoods.  In the PAIR kernels the 64 lanes of a wave hold
// two adjacent x1 rows: lanes 0-31 row i1 (i1 even), lanes 32-63 row i1 + 1.
// The row each half needs from the other comes by a lane swap, and only the
// outer row (i1 - 1 below, i1 + 2 above) is loaded: the x1 pair of a lane is
// then (other half's row, outer row), which is (+x1, -x1) in the lower half and
// (-x1, +x1) in the upper half, so the upper half takes -1/2h as its x1 factor.
template <int VW>
struct VNbr {
  int o;            // first voxel of the lane
  int ox[4];        // the same voxel at +x0, -x0, +x1, -x1
  int left, right;  // lanes holding the x2 neighbours
  bool upper;       // lanes 32-63 of a paired wave
};

template <typename T, int VW>
__device__ __forceinline__ bool vvoxel(const Geo<T>& g, int RW, VNbr<VW>& nb) {
  int i0, i1, j;
  if (!tile_voxel(g.ft, g.n1, g.n2 / VW, i0, i1, j)) return false;
  const int i2 = j * VW;
  const int p0 = periodic_next(i0, g.n0), m0 = periodic_prev(i0, g.n0);
  const int p1 = periodic_next(i1, g.n1), m1 = periodic_prev(i1, g.n1);
  const int s0 = g.n1 * g.n2;
  const int r1 = i1 * g.n2 + i2;
  nb.o = i0 * s0 + r1;
  nb.ox[0] = p0 * s0 + r1;
  nb.ox[1] = m0 * s0 + r1;
  nb.ox[2] = i0 * s0 + p1 * g.n2 + i2;
  nb.ox[3] = i0 * s0 + m1 * g.n2 + i2;
  const int lane = int(threadIdx.x + threadIdx.y * blockDim.x) & 63;
  row_lanes(lane, RW, nb.left, nb.right);
  nb.upper = lane >= 32;
  return true;
}

// Factor 1/2h of direction e for the lane (sign-flipped for x1 in the upper
// half of a paired wave).
template <typename T, int VW, bool PAIR>
__device__ __forceinline__ T vinv2h(const Geo<T>& g, const VNbr<VW>& nb, int e) {
  return (PAIR && e == 1 && nb.upper) ? -g.inv2h[1] : g.inv2h[e];
}

// Three voxels per lane: a run of three values aligned only to one element (one
// 12-byte or 24-byte access); widths 1, 2 and 4 use naturally aligned vectors.
template <typename T, int VW>
struct alignas(sizeof(T)) VRun {
  T v[VW];
};

template <typename T, int VW>
__device__ __forceinline__ void vld(T out[VW], const T* __restrict__ p) {
  if constexpr (VW == 3) {
    const VRun<T, 3> x = *reinterpret_cast<const VRun<T, 3>*>(p);
#pragma unroll
    for (int k = 0; k < 3; ++k) out[k] = x.v[k];
  } else {
    typedef T vec __attribute__((ext_vector_type(VW)));
    const vec x = *reinterpret_cast<const vec*>(p);
#pragma unroll
    for (int k = 0; k < VW; ++k) out[k] = x[k];
  }
}

template <typename T, int VW>
__device__ __forceinline__ void vload3(T out[3][VW], const T* __restrict__ f, int o, int N) {
#pragma unroll
  for (int c = 0; c < 3; ++c) vld<T, VW>(out[c], f + c * N + o);
}

template <typename T, int VW>
__device__ __forceinline__ void vstore3(T* __restrict__ f, const T in[3][VW], int o, int N) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if constexpr (VW == 3) {
      VRun<T, 3> x;
#pragma unroll
      for (int k = 0; k < 3; ++k) x.v[k] = in[c][k];
      *reinterpret_cast<VRun<T, 3>*>(f + c * N + o) = x;
    } else {
      typedef T vec __attribute__((ext_vector_type(VW)));
      vec x;
#pragma unroll
      for (int k = 0; k < VW; ++k) x[k] = in[c][k];
      *reinterpret_cast<vec*>(f + c * N + o) = x;
    }
  }
}

// A vector field at the +e and -e neighbours of the lane's VW voxels.
template <typename T, int VW>
struct VPair {
  T p[3][VW], m[3][VW];
};

template <typename T, int VW>
__device__ __forceinline__ void vpair_load(VPair<T, VW>& s, const T* __restrict__ f, const VNbr<VW>& nb, int e,
                                           int N) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    vld<T, VW>(s.p[c], f + c * N + nb.ox[2 * e]);
    vld<T, VW>(s.m[c], f + c * N + nb.ox[2 * e + 1]);
  }
}

// x2 neighbours: the lane's own values shifted by one, the ends from the
// adjacent lanes of the row.
template <typename T, int VW>
__device__ __forceinline__ void vpair_shift(VPair<T, VW>& s, const T c0[3][VW], const VNbr<VW>& nb) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const T from_right = __shfl(c0[c][0], nb.right);
    const T from_left = __shfl(c0[c][VW - 1], nb.left);
#pragma unroll
    for (int k = 0; k < VW; ++k) {
      s.p[c][k] = k + 1 < VW ? c0[c][k + 1] : from_right;
      s.m[c][k] = k > 0 ? c0[c][k - 1] : from_left;
    }
  }
}

// x1 pair of a paired wave: (other half's row by lane swap, outer row loaded).
template <typename T, int VW>
__device__ __forceinline__ void vpair_swap(VPair<T, VW>& s, const T* __restrict__ f, const T c0[3][VW],
                                           const VNbr<VW>& nb, int N) {
  const int outer = nb.upper ? nb.ox[2] : nb.ox[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    vld<T, VW>(s.m[c], f + c * N + outer);
#pragma unroll
    for (int k = 0; k < VW; ++k) s.p[c][k] = __shfl_xor(c0[c][k], 32);
  }
}

template <typename T, int VW, bool PAIR>
__device__ __forceinline__ void vpair(VPair<T, VW>& s, const T* __restrict__ f, const T c0[3][VW],
                                      const VNbr<VW>& nb, int e, int N) {
  if (PAIR && e == 1)
    vpair_swap<T, VW>(s, f, c0, nb, N);
  else if (e < 2)
    vpair_load<T, VW>(s, f, nb, e, N);
  else
    vpair_shift<T, VW>(s, c0, nb);
}

// Direction-e share of ad_v w and of ad*_v mu at each of the lane's voxels.
template <typename T, int VW>
__device__ __forceinline__ void vad_dir(T out[3][VW], const VPair<T, VW>& v, const VPair<T, VW>& w,
                                        const T v0[3][VW], const T w0[3][VW], int e, T inv2h) {
#pragma unroll
  for (int k = 0; k < VW; ++k)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      out[c][k] += ((v.p[c][k] - v.m[c][k]) * w0[e][k] - (w.p[c][k] - w.m[c][k]) * v0[e][k]) * inv2h;
}

template <typename T, int VW>
__device__ __forceinline__ void vadstar_dir(T out[3][VW], const VPair<T, VW>& v, const VPair<T, VW>& mu,
                                            const T mu0[3][VW], int e, T inv2h) {
#pragma unroll
  for (int k = 0; k < VW; ++k) {
    T s = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) s += (v.p[d][k] - v.m[d][k]) * mu0[d][k];
    out[e][k] += s * inv2h;
#pragma unroll
    for (int c = 0; c < 3; ++c) out[c][k] += (mu.p[c][k] * v.p[e][k] - mu.m[c][k] * v.m[e][k]) * inv2h;
  }
}

template <typename T, int VW>
__device__ __forceinline__ void vheun(T out[3][VW], const T* y0, T a0, int o, int N) {
  if (a0 != T(0)) {
    T z[3][VW];
    vload3<T, VW>(z, y0, o, N);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int k = 0; k < VW; ++k) out[c][k] += a0 * z[c][k];
  }
}

template <typename T, int VW, bool PAIR>
__global__ void __launch_bounds__(256)
    k_epdiff_stage_v(Geo<T> g, int RW, const T* __restrict__ v, const T* __restrict__ mu, const T* mu0,
                     T* mu_out, T dt, T a0, T a1) {
  VNbr<VW> nb;
  if (!vvoxel<T, VW>(g, RW, nb)) return;
  T m[3][VW], vc[3][VW], a[3][VW] = {};
  vload3<T, VW>(m, mu, nb.o, g.N);
  vload3<T, VW>(vc, v, nb.o, g.N);
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    VPair<T, VW> Vp, Mp;
    vpair<T, VW, PAIR>(Vp, v, vc, nb, e, g.N);
    vpair<T, VW, PAIR>(Mp, mu, m, nb, e, g.N);
    vadstar_dir<T, VW>(a, Vp, Mp, m, e, vinv2h<T, VW, PAIR>(g, nb, e));
  }
  T out[3][VW];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int k = 0; k < VW; ++k) out[c][k] = a1 * (m[c][k] - dt * a[c][k]);
  vheun<T, VW>(out, mu0, a0, nb.o, g.N);
  vstore3<T, VW>(mu_out, out, nb.o, g.N);
}

// ZS (the sweep's first step starts from X = 0): bit 1, the stage's X is zero
// and not read (no ad_v X); bit 2, its start value X0 is zero and not read.
template <typename T, int VW, bool PAIR, int ZS = 0>
__global__ void __launch_bounds__(256)
    k_tangent_stage_v(Geo<T> g, int RW, const T* __restrict__ X, const T* __restrict__ dmu, const T* __restrict__ W,
                      const T* __restrict__ v, const T* __restrict__ mu, const T* X0, const T* dmu0, T* X_out,
                      T* dmu_out, T dt, T a0, T a1, const T* __restrict__ Gf, T cf) {
  VNbr<VW> nb;
  if (!vvoxel<T, VW>(g, RW, nb)) return;
  T x[3][VW] = {}, vc[3][VW], dm[3][VW];
  if constexpr (!(ZS & 1)) vload3<T, VW>(x, X, nb.o, g.N);
  vload3<T, VW>(vc, v, nb.o, g.N);
  vload3<T, VW>(dm, dmu, nb.o, g.N);
  T aX[3][VW] = {}, t1[3][VW] = {}, t2[3][VW] = {};
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    VPair<T, VW> Vp, Dp;
    vpair<T, VW, PAIR>(Vp, v, vc, nb, e, g.N);
    if constexpr (!(ZS & 1)) {
      VPair<T, VW> Xp;
      vpair<T, VW, PAIR>(Xp, X, x, nb, e, g.N);
      vad_dir<T, VW>(aX, Vp, Xp, vc, x, e, vinv2h<T, VW, PAIR>(g, nb, e));  // ad_v X
    }
    vpair<T, VW, PAIR>(Dp, dmu, dm, nb, e, g.N);
    vadstar_dir<T, VW>(t2, Vp, Dp, dm, e, vinv2h<T, VW, PAIR>(g, nb, e));  // ad*_v dmu
  }
  T w[3][VW], m[3][VW];
  vload3<T, VW>(w, W, nb.o, g.N);
  vload3<T, VW>(m, mu, nb.o, g.N);
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    VPair<T, VW> Wp, Mp;
    vpair<T, VW, PAIR>(Wp, W, w, nb, e, g.N);
    vpair<T, VW, PAIR>(Mp, mu, m, nb, e, g.N);
    vadstar_dir<T, VW>(t1, Wp, Mp, m, e, vinv2h<T, VW, PAIR>(g, nb, e));  // ad*_W mu
  }
  T xo[3][VW], mo[3][VW];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int k = 0; k < VW; ++k) {
      xo[c][k] = a1 * (x[c][k] + dt * (w[c][k] + aX[c][k]));
      mo[c][k] = a1 * (dm[c][k] - dt * (t1[c][k] + t2[c][k]));
    }
  if constexpr (!(ZS & 2)) vheun<T, VW>(xo, X0, a0, nb.o, g.N);
  vheun<T, VW>(mo, dmu0, a0, nb.o, g.N);
  if (Gf) {  // last stage of the sweep: X_out receives cf (G . X) G, dmu is not kept
    T gv[3][VW];
    vload3<T, VW>(gv, Gf, nb.o, g.N);
#pragma unroll
    for (int k = 0; k < VW; ++k) {
      const T sg = cf * (gv[0][k] * xo[0][k] + gv[1][k] * xo[1][k] + gv[2][k] * xo[2][k]);
#pragma unroll
      for (int c = 0; c < 3; ++c) xo[c][k] = sg * gv[c][k];
    }
    vstore3<T, VW>(X_out, xo, nb.o, g.N);
    return;
  }
  vstore3<T, VW>(X_out, xo, nb.o, g.N);
  vstore3<T, VW>(dmu_out, mo, nb.o, g.N);
}

// ZS bit 2: the start value w0 is zero and not read (the sweep's first corrector).
template <typename T, int VW, bool PAIR, int ZS = 0>
__global__ void __launch_bounds__(256)
    k_adjoint_stage_v(Geo<T> g, int RW, const T* __restrict__ U, const T* __restrict__ w, const T* __restrict__ mu,
                      const T* __restrict__ v, const T* U0, const T* w0, T* __restrict__ Z, T* __restrict__ Q,
                      T* U_out, T dt, T a0, T a1, const T* __restrict__ qadd, T qs) {
  VNbr<VW> nb;
  if (!vvoxel<T, VW>(g, RW, nb)) return;
  T u[3][VW], vc[3][VW], wc[3][VW], m[3][VW];
  vload3<T, VW>(u, U, nb.o, g.N);
  vload3<T, VW>(vc, v, nb.o, g.N);
  vload3<T, VW>(wc, w, nb.o, g.N);
  vload3<T, VW>(m, mu, nb.o, g.N);
  T z[3][VW] = {}, aU[3][VW] = {}, aw[3][VW] = {};
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const T h = vinv2h<T, VW, PAIR>(g, nb, e);
    VPair<T, VW> Wp, Vp;
    vpair<T, VW, PAIR>(Wp, w, wc, nb, e, g.N);
    {
      VPair<T, VW> Mp;
      vpair<T, VW, PAIR>(Mp, mu, m, nb, e, g.N);
      vadstar_dir<T, VW>(z, Wp, Mp, m, e, h);  // ad*_w mu
    }
    vpair<T, VW, PAIR>(Vp, v, vc, nb, e, g.N);
    vad_dir<T, VW>(aw, Vp, Wp, vc, wc, e, h);  // ad_v w
    {
      VPair<T, VW> Up;
      vpair<T, VW, PAIR>(Up, U, u, nb, e, g.N);
      vadstar_dir<T, VW>(aU, Vp, Up, u, e, h);  // ad*_v U
    }
  }
  T q[3][VW], uo[3][VW];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int k = 0; k < VW; ++k) {
      z[c][k] += u[c][k];
      q[c][k] = a1 * (wc[c][k] - dt * aw[c][k]);
      uo[c][k] = a1 * (u[c][k] + dt * aU[c][k]);
    }
  if constexpr (!(ZS & 2)) vheun<T, VW>(q, w0, a0, nb.o, g.N);
  vheun<T, VW>(uo, U0, a0, nb.o, g.N);
  if (qadd) vheun<T, VW>(q, qadd, qs, nb.o, g.N);
  vstore3<T, VW>(Z, z, nb.o, g.N);
  vstore3<T, VW>(Q, q, nb.o, g.N);
  vstore3<T, VW>(U_out, uo, nb.o, g.N);
}

template <typename T, int VW, bool PAIR>
__global__ void __launch_bounds__(256)
    k_newton_stage_v(Geo<T> g, int RW, const T* __restrict__ dU, const T* __restrict__ dw, const T* __restrict__ mu,
                     const T* __restrict__ w1, const T* __restrict__ dmu, const T* __restrict__ v,
                     const T* __restrict__ Wv, const T* __restrict__ U1, const T* dU0, const T* dw0,
                     T* __restrict__ Z, T* __restrict__ Q, T* dU_out, T dt, T a0, T a1) {
  VNbr<VW> nb;
  if (!vvoxel<T, VW>(g, RW, nb)) return;
  T du[3][VW], dwc[3][VW], m[3][VW], w1c[3][VW], dm[3][VW], vc[3][VW], wk[3][VW], u1[3][VW];
  vload3<T, VW>(du, dU, nb.o, g.N);
  vload3<T, VW>(dwc, dw, nb.o, g.N);
  vload3<T, VW>(m, mu, nb.o, g.N);
  vload3<T, VW>(w1c, w1, nb.o, g.N);
  vload3<T, VW>(dm, dmu, nb.o, g.N);
  vload3<T, VW>(vc, v, nb.o, g.N);
  vload3<T, VW>(wk, Wv, nb.o, g.N);
  vload3<T, VW>(u1, U1, nb.o, g.N);
  T z[3][VW] = {}, aU[3][VW] = {}, aw[3][VW] = {};
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const T h = vinv2h<T, VW, PAIR>(g, nb, e);
    VPair<T, VW> Dwp, Vp, W1p, Wkp;
    vpair<T, VW, PAIR>(Dwp, dw, dwc, nb, e, g.N);
    {
      VPair<T, VW> Mp;
      vpair<T, VW, PAIR>(Mp, mu, m, nb, e, g.N);
      vadstar_dir<T, VW>(z, Dwp, Mp, m, e, h);  // ad*_dw mu
    }
    vpair<T, VW, PAIR>(Vp, v, vc, nb, e, g.N);
    vad_dir<T, VW>(aw, Vp, Dwp, vc, dwc, e, h);  // ad_v dw
    {
      VPair<T, VW> Dp;
      vpair<T, VW, PAIR>(Dp, dU, du, nb, e, g.N);
      vadstar_dir<T, VW>(aU, Vp, Dp, du, e, h);  // ad*_v dU
    }
    vpair<T, VW, PAIR>(W1p, w1, w1c, nb, e, g.N);
    {
      VPair<T, VW> Dmp;
      vpair<T, VW, PAIR>(Dmp, dmu, dm, nb, e, g.N);
      vadstar_dir<T, VW>(z, W1p, Dmp, dm, e, h);  // ad*_w1 dmu
    }
    vpair<T, VW, PAIR>(Wkp, Wv, wk, nb, e, g.N);
    vad_dir<T, VW>(aw, Wkp, W1p, wk, w1c, e, h);  // ad_W w1
    {
      VPair<T, VW> Ap;
      vpair<T, VW, PAIR>(Ap, U1, u1, nb, e, g.N);
      vadstar_dir<T, VW>(aU, Wkp, Ap, u1, e, h);  // ad*_W U1
    }
  }
  T q[3][VW], uo[3][VW];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int k = 0; k < VW; ++k) {
      z[c][k] += du[c][k];
      uo[c][k] = a1 * (du[c][k] + dt * aU[c][k]);
      q[c][k] = a1 * (dwc[c][k] - dt * aw[c][k]);
    }
  vheun<T, VW>(uo, dU0, a0, nb.o, g.N);
  vheun<T, VW>(q, dw0, a0, nb.o, g.N);
  vstore3<T, VW>(Z, z, nb.o, g.N);
  vstore3<T, VW>(Q, q, nb.o, g.N);
  vstore3<T, VW>(dU_out, uo, nb.o, g.N);
}

// Lane width VW of the row-vectorised kernels for this grid (0: one voxel per thread).
int row_vector_width(const Grid& g) { return row_vector_valid(g.n2, g.rowvec) ? g.rowvec : 0; }

template <typename T>
Geo<T> make_vgeo(const Grid& g, int VW) {
  Geo<T> o = make_geo<T>(g);
  Grid gv = g;
  gv.n2 = g.n2 / VW;
  o.ft = make_field_tiling(gv);
  // 32 lanes per row: a wave holds rows (i1, i1 + 1) with i1 even; with N1 even
  // both rows of every wave exist
  o.pair = (g.n2 / VW == 32 && o.ft.BX == 32 && o.ft.BY % 2 == 0 && g.n1 % 2 == 0 && g.pair_rows) ? 1 : 0;
  return o;
}

#define LDDMM_ROWVEC_AT(kern, vw, pr, ...) \
  LDDMM_LAUNCH(t.start, t.stop, kern<T LDDMM_COMMA vw LDDMM_COMMA pr>, grid_, block_, 0, st, gv, RW, __VA_ARGS__)
// The same for kernels instantiated for VW = 1, 2 only.
#define LDDMM_ROWVEC12(kern, ...)                                      \
  do {                                                                 \
    const Geo<T> gv = make_vgeo<T>(g, VW);                             \
    const dim3 grid_(gv.ft.blocks), block_(gv.ft.BX, gv.ft.BY);        \
    const int RW = g.n2 / VW;                                          \
    if (VW == 1 && gv.pair)                                            \
      LDDMM_ROWVEC_AT(kern, 1, true, __VA_ARGS__);                     \
    else if (VW == 1)                                                  \
      LDDMM_ROWVEC_AT(kern, 1, false, __VA_ARGS__);                    \
    else if (gv.pair)                                                  \
      LDDMM_ROWVEC_AT(kern, 2, true, __VA_ARGS__);                     \
    else                                                               \
      LDDMM_ROWVEC_AT(kern, 2, false, __VA_ARGS__);                    \
  } while (0)
#define LDDMM_ROWVEC(kern, ...)                                        \
  do {                                                                 \
    const Geo<T> gv = make_vgeo<T>(g, VW);                             \
    const dim3 grid_(gv.ft.blocks), block_(gv.ft.BX, gv.ft.BY);        \
    const int RW = g.n2 / VW;                                          \
    if (VW == 1 && gv.pair)                                            \
      LDDMM_ROWVEC_AT(kern, 1, true, __VA_ARGS__);                     \
    else if (VW == 1)                                                  \
      LDDMM_ROWVEC_AT(kern, 1, false, __VA_ARGS__);                    \
    else if (VW == 2 && gv.pair)                                       \
      LDDMM_ROWVEC_AT(kern, 2, true, __VA_ARGS__);                     \
    else if (VW == 2)                                                  \
      LDDMM_ROWVEC_AT(kern, 2, false, __VA_ARGS__);                    \
    else if (VW == 3 && gv.pair)                                       \
      LDDMM_ROWVEC_AT(kern, 3, true, __VA_ARGS__);                     \
    else if (VW == 3)                                                  \
      LDDMM_ROWVEC_AT(kern, 3, false, __VA_ARGS__);                    \
    else if (gv.pair)                                                  \
      LDDMM_ROWVEC_AT(kern, 4, true, __VA_ARGS__);                     \
    else                                                               \
      LDDMM_ROWVEC_AT(kern, 4, false, __VA_ARGS__);                    \
  } while (0)

// The same for the tangent and adjoint kernels with their zero-start variant ZS.
#define LDDMM_ROWVEC_Z_AT(kern, vw, pr, z, ...)                                                       \
  LDDMM_LAUNCH(t.start, t.stop, kern<T LDDMM_COMMA vw LDDMM_COMMA pr LDDMM_COMMA z>, grid_, block_, 0, st, gv, RW, \
               __VA_ARGS__)
#define LDDMM_ROWVEC_Z(kern, z, ...)                                   \
  do {                                                                 \
    const Geo<T> gv = make_vgeo<T>(g, VW);                             \
    const dim3 grid_(gv.ft.blocks), block_(gv.ft.BX, gv.ft.BY);        \
    const int RW = g.n2 / VW;                                          \
    if (VW == 1 && gv.pair)                                            \
      LDDMM_ROWVEC_Z_AT(kern, 1, true, z, __VA_ARGS__);                \
    else if (VW == 1)                                                  \
      LDDMM_ROWVEC_Z_AT(kern, 1, false, z, __VA_ARGS__);               \
    else if (VW == 2 && gv.pair)                                       \
      LDDMM_ROWVEC_Z_AT(kern, 2, true, z, __VA_ARGS__);                \
    else if (VW == 2)                                                  \
      LDDMM_ROWVEC_Z_AT(kern, 2, false, z, __VA_ARGS__);               \
    else if (VW == 3 && gv.pair)                                       \
      LDDMM_ROWVEC_Z_AT(kern, 3, true, z, __VA_ARGS__);                \
    else if (VW == 3)                                                  \
      LDDMM_ROWVEC_Z_AT(kern, 3, false, z, __VA_ARGS__);               \
    else if (gv.pair)                                                  \
      LDDMM_ROWVEC_Z_AT(kern, 4, true, z, __VA_ARGS__);                \
    else                                                               \
      LDDMM_ROWVEC_Z_AT(kern, 4, false, z, __VA_ARGS__);               \
  } while (0)

dim3 ft_grid(const Grid& g) { return dim3(make_field_tiling(g).blocks); }
dim3 ft_block(const Grid& g) {
  const FieldTiling t = make_field_tiling(g);
  return dim3(t.BX, t.BY);
}

unsigned flat_blocks(long long N) {
  long long b = (N + 255) / 256;
  return (unsigned)(b < 8192 ? b : 8192);
}

}  // namespace

template <typename T>
void launch_epdiff_stage(const Grid& g, const T* v, const T* mu, const T* mu0, T* mu_out, double dt, double a0,
                         double a1, hipStream_t st, Profiler* prof) {
  KernelTimer t(prof, a0 != 0.0 ? "epdiff_stage_corr" : "epdiff_stage_pred");
  if (const int VW = row_vector_width(g)) {
    LDDMM_ROWVEC(k_epdiff_stage_v, v, mu, mu0 ? mu0 : mu, mu_out, T(dt), T(a0), T(a1));
    return;
  }
  LDDMM_LAUNCH(t.start, t.stop, k_epdiff_stage<T>, ft_grid(g), ft_block(g), 0, st, make_geo<T>(g), v, mu, mu0 ? mu0 : mu, mu_out, T(dt), T(a0), T(a1));
}

template <typename T>
void launch_tangent_stage(const Grid& g, const T* X, const T* dmu, const T* W, const T* v, const T* mu,
                          const T* X0, const T* dmu0, T* X_out, T* dmu_out, double dt, double a0, double a1,
                          hipStream_t st, Profiler* prof, const T* Gfin, double cfin, int zero) {
  const bool zs = zero != 0 && row_vector_width(g) != 0;  // the zero-start variant runs
  KernelTimer t(prof, a0 != 0.0 ? (zs ? "tangent_stage_corr_first" : "tangent_stage_corr")
                                : (zs ? "tangent_stage_pred_first" : "tangent_stage_pred"));
  if (const int VW = row_vector_width(g)) {
    if (zero == 1)
      LDDMM_ROWVEC_Z(k_tangent_stage_v, 1, X, dmu, W, v, mu, X0 ? X0 : X, dmu0 ? dmu0 : dmu, X_out, dmu_out, T(dt),
                     T(a0), T(a1), Gfin, T(cfin));
    else if (zero == 2)
      LDDMM_ROWVEC_Z(k_tangent_stage_v, 2, X, dmu, W, v, mu, X0 ? X0 : X, dmu0 ? dmu0 : dmu, X_out, dmu_out, T(dt),
                     T(a0), T(a1), Gfin, T(cfin));
    else
      LDDMM_ROWVEC_Z(k_tangent_stage_v, 0, X, dmu, W, v, mu, X0 ? X0 : X, dmu0 ? dmu0 : dmu, X_out, dmu_out, T(dt),
                     T(a0), T(a1), Gfin, T(cfin));
    return;
  }
  LDDMM_LAUNCH(t.start, t.stop, k_tangent_stage<T>, ft_grid(g), ft_block(g), 0, st, make_geo<T>(g), X, dmu, W, v, mu, X0 ? X0 : X, dmu0 ? dmu0 : dmu, X_out, dmu_out, T(dt), T(a0), T(a1), Gfin, T(cfin));
}

template <typename T>
void launch_adjoint_stage(const Grid& g, const T* U, const T* w, const T* mu, const T* v, const T* U0, const T* w0,
                          T* Z, T* Q, T* U_out, double dt, double a0, double a1, hipStream_t st, Profiler* prof,
                          const T* qadd, double qs, int zero) {
  const bool zs = zero != 0 && row_vector_width(g) != 0;  // the zero-start variant runs
  KernelTimer t(prof, a0 != 0.0 ? (zs ? "adjoint_stage_corr_first" : "adjoint_stage_corr") : "adjoint_stage_pred");
  if (const int VW = row_vector_width(g)) {
    if (zero == 2)
      LDDMM_ROWVEC_Z(k_adjoint_stage_v, 2, U, w, mu, v, U0 ? U0 : U, w0 ? w0 : w, Z, Q, U_out, T(dt), T(a0), T(a1),
                     qadd, T(qs));
    else
      LDDMM_ROWVEC_Z(k_adjoint_stage_v, 0, U, w, mu, v, U0 ? U0 : U, w0 ? w0 : w, Z, Q, U_out, T(dt), T(a0), T(a1),
                     qadd, T(qs));
    return;
  }
  LDDMM_LAUNCH(t.start, t.stop, k_adjoint_stage<T>, ft_grid(g), ft_block(g), 0, st, make_geo<T>(g), U, w, mu, v, U0 ? U0 : U, w0 ? w0 : w, Z, Q, U_out, T(dt), T(a0), T(a1), qadd, T(qs));
}

template <typename T>
void launch_residual_grad(const Grid& g, const T* J1, const T* I1, T* r, T* G, hipStream_t st, Profiler* prof) {
  KernelTimer t(prof, "residual_grad");
  LDDMM_LAUNCH(t.start, t.stop, k_residual_grad<T>, ft_grid(g), ft_block(g), 0, st, make_geo<T>(g), J1, I1, r, G);
}

template <typename T>
void launch_scalar_times_vec(const Grid& g, const T* s, const T* G, double c, T* U, hipStream_t st,
                             Profiler* prof) {
  KernelTimer t(prof, "final_condition");
  LDDMM_LAUNCH(t.start, t.stop, k_scalar_times_vec<T>, flat_blocks(g.N), 256, 0, st, g.N, s, G, T(c), U);
}

template <typename T>
void launch_gn_final(const Grid& g, const T* G, const T* X, double c, T* U, hipStream_t st, Profiler* prof) {
  KernelTimer t(prof, "gn_final_condition");
  LDDMM_LAUNCH(t.start, t.stop, k_gn_final<T>, flat_blocks(g.N), 256, 0, st, g.N, G, X, T(c), U);
}

template <typename T>
void launch_newton_stage(const Grid& g, const T* dU, const T* dw, const T* mu, const T* w1, const T* dmu, const T* v,
                         const T* Wv, const T* U1, const T* dU0, const T* dw0, T* Z, T* Q, T* dU_out, double dt,
                         double a0, double a1, hipStream_t st, Profiler* prof) {
  KernelTimer t(prof, a0 != 0.0 ? "newton_stage_corr" : "newton_stage_pred");
  // eight stencil fields: at most two voxels per lane keeps the registers in bounds
  int VW = row_vector_width(g);
  if (VW > 2) VW = row_vector_valid(g.n2, 2) ? 2 : 0;
  if (VW) {
    LDDMM_ROWVEC12(k_newton_stage_v, dU, dw, mu, w1, dmu, v, Wv, U1, dU0 ? dU0 : dU, dw0 ? dw0 : dw, Z, Q, dU_out,
                   T(dt), T(a0), T(a1));
    return;
  }
  LDDMM_LAUNCH(t.start, t.stop, k_newton_stage<T>, ft_grid(g), ft_block(g), 0, st, make_geo<T>(g), dU, dw, mu, w1, dmu, v, Wv, U1, dU0 ? dU0 : dU, dw0 ? dw0 : dw, Z, Q, dU_out, T(dt), T(a0), T(a1));
}

template <typename T>
void launch_newton_final(const Grid& g, const T* G, const T* X, const T* r, double c, T* s, T* U, hipStream_t st,
                         Profiler* prof) {
  KernelTimer t(prof, "newton_final_condition");
  LDDMM_LAUNCH(t.start, nullptr, k_dm1<T>, flat_blocks(g.N), 256, 0, st, g.N, G, X, s);
  LDDMM_LAUNCH(nullptr, t.stop, k_newton_final<T>, ft_grid(g), ft_block(g), 0, st, make_geo<T>(g), s, r, G, T(c), U);
}

template <typename T>
void launch_jacobian_det(const Grid& g, const T* u, T* det, hipStream_t st, Profiler* prof) {
  KernelTimer t(prof, "jacobian_det");
  LDDMM_LAUNCH(t.start, t.stop, k_jacobian_det<T>, ft_grid(g), ft_block(g), 0, st, make_geo<T>(g), u, det);
}

#define LDDMM_INST(T)                                                                                            \
  template void launch_epdiff_stage<T>(const Grid&, const T*, const T*, const T*, T*, double, double, double,    \
                                       hipStream_t, Profiler*);                                                  \
  template void launch_tangent_stage<T>(const Grid&, const T*, const T*, const T*, const T*, const T*, const T*, \
                                        const T*, T*, T*, double, double, double, hipStream_t, Profiler*,        \
                                        const T*, double, int);                                                  \
  template void launch_adjoint_stage<T>(const Grid&, const T*, const T*, const T*, const T*, const T*, const T*, \
                                        T*, T*, T*, double, double, double, hipStream_t, Profiler*, const T*,    \
                                        double, int);                                                            \
  template void launch_residual_grad<T>(const Grid&, const T*, const T*, T*, T*, hipStream_t, Profiler*);       \
  template void launch_scalar_times_vec<T>(const Grid&, const T*, const T*, double, T*, hipStream_t, Profiler*); \
  template void launch_gn_final<T>(const Grid&, const T*, const T*, double, T*, hipStream_t, Profiler*);        \
  template void launch_jacobian_det<T>(const Grid&, const T*, T*, hipStream_t, Profiler*);                      \
  template void launch_newton_stage<T>(const Grid&, const T*, const T*, const T*, const T*, const T*, const T*,  \
                                       const T*, const T*, const T*, const T*, T*, T*, T*, double, double, double, \
                                       hipStream_t, Profiler*);                                                  \
  template void launch_newton_final<T>(const Grid&, const T*, const T*, const T*, double, T*, T*, hipStream_t,    \
                                       Profiler*);

LDDMM_INST(float)
LDDMM_INST(double)

}  // namespace lddmm
