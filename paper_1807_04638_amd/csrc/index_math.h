// index_math.h - index arithmetic of the field kernels, shared by the GPU code
// and host checks.
//
//   field_tiling / tile_voxel_at   voxel tiling of the stencil and SL kernels
//                                  (XCD-aware order of the x1 tiles)
//   periodic_next / periodic_prev  neighbours on the periodic grid
//   xcd_grouped, xcd_run_if_split  unit of a block so that each XCD takes runs
//                                  of consecutive units that share cache lines
//   row_lanes                      x2 neighbours inside a row of lanes of the
//                                  row-vectorised stencils
//   sl_axis                        cell and weight of a displaced point along one
//                                  axis for the semi-Lagrangian gathers
//
// Every function is __host__ __device__ (or host-only where marked) so that a host
// program can run the exact code the kernels run over every block and thread of a
// launch, with bounds checks, address and undefined-behaviour sanitizers.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>

namespace lddmm {

#define LDI_HD __host__ __device__ __forceinline__

// Voxel tiling of the field kernels: a block covers BX x BY voxels of one x0
// plane (BX spans a whole x2 row when N2 <= 256, so x2 halos stay inside the
// tile).  With XCD-aware mapping the 8 XCDs (which take blocks round-robin)
// each own a contiguous slab of x1 rows for every x0, so x1 halos and the
// neighbouring x0 planes a block needs were loaded into the same L2.  XCD x
// owns tile rows [x TY / 8, (x + 1) TY / 8) (rounded down), so where 8 does not
// divide TY the slabs differ by one row; the grid then holds 8 slab blocks per
// (x2 tile, x0 plane) and the blocks past an XCD's own rows do nothing.
struct FieldTiling {
  int BX, BY;      // block shape (threads)
  int TX, TY;      // tiles along x2 and x1
  int slab;        // most tile rows of x1 one XCD owns (0: plain linear order)
  unsigned blocks; // TX * N0 * (8 slab, or TY in linear order)
};

// Host: the tiling of an n0 x n1 x n2 grid (n2 = row length in lanes for the
// row-vectorised kernels).
inline FieldTiling field_tiling(int n0, int n1, int n2) {
  FieldTiling t;
  int bx = (n2 + 31) / 32 * 32;
  if (bx > 256) bx = 256;
  t.BX = bx;
  t.BY = 256 / bx > 0 ? 256 / bx : 1;
  t.TX = (n2 + t.BX - 1) / t.BX;
  t.TY = (n1 + t.BY - 1) / t.BY;
  // XCD-aware order where the largest slab is at most 15 % above the mean
  // (uneven slabs make the XCDs with one more row finish last)
  const int s = (t.TY + 7) / 8;
  t.slab = (t.TY >= 8 && 800 * s <= 115 * t.TY) ? s : 0;
  t.blocks = unsigned(t.TX) * unsigned(t.slab ? 8 * t.slab : t.TY) * unsigned(n0);
  return t;
}

// Voxel (i0, i1, i2) of thread (tx, ty) of block b under tiling t; false for the
// threads of an edge tile that fall outside the grid and for every thread of a
// block past its XCD's own slab.
LDI_HD bool tile_voxel_at(const FieldTiling& t, int b, int tx, int ty, int n1, int n2, int& i0, int& i1, int& i2) {
  int bx, by;
  bool own = true;
  if (t.slab) {
    const int x = b & 7, k = b >> 3;
    const int r = k / t.TX;
    bx = k - r * t.TX;
    const int rz = r / t.slab;
    const int ry = r - rz * t.slab;
    const int lo = (x * t.TY) >> 3, rows = (((x + 1) * t.TY) >> 3) - lo;
    own = ry < rows;
    by = lo + ry;
    i0 = rz;
  } else {
    const int r = b / t.TX;
    bx = b - r * t.TX;
    i0 = r / t.TY;
    by = r - i0 * t.TY;
  }
  i2 = bx * t.BX + tx;
  i1 = by * t.BY + ty;
  return own && i2 < n2 && i1 < n1;
}

// Unit of block b (of B) such that each XCD takes runs of g consecutive units:
// blocks go to the 8 XCDs round-robin (block b to XCD b mod 8), so within each
// span of 8 g blocks XCD x gets units [x g, x g + g) of the span, in order; a
// last span of fewer than 8 g blocks keeps unit = block.  Units next to each
// other in memory then share an L2 (a cache line split between two of them is
// fetched once), while the units in flight stay as close together as in
// round-robin order.
LDI_HD int xcd_grouped(int b, int B, int g) {
  const int span = 8 * g, s = b / span;
  if ((s + 1) * span > B) return b;
  const int r = b - s * span;
  return s * span + (r & 7) * g + (r >> 3);
}

// Host: run length for xcd_grouped.  Units share a 128-byte cache line with
// their neighbours unless every byte offset and stride that places them (a row,
// a tile, a plane of the spectrum) is a whole number of lines: then `run`, else
// 1 (round-robin order).
inline int xcd_run_if_split(long long a, long long b, long long c, long long d, int run) {
  return (a % 128 == 0 && b % 128 == 0 && c % 128 == 0 && d % 128 == 0) ? 1 : run;
}

LDI_HD int periodic_next(int i, int n) { return i + 1 == n ? 0 : i + 1; }
LDI_HD int periodic_prev(int i, int n) { return i == 0 ? n - 1 : i - 1; }

// Row-vectorised stencils: a row of RW lanes (32 <= RW <= 64) starts a 32-lane
// half of a wave (RW = 32: two rows per wave) or a whole wave (RW > 32; lanes
// RW..63 hold no voxel).  The lanes holding the x2 neighbours of `lane`,
// periodic inside its row.
LDI_HD void row_lanes(int lane, int RW, int& left, int& right) {
  const int seg = RW <= 32 ? 32 : 64;
  const int base = lane & ~(seg - 1);
  const int pos = lane - base;
  left = base + (pos == 0 ? RW - 1 : (pos - 1) % RW);
  right = base + (pos + 1) % RW;
}

// Host: a row-vectorised width vw (voxels per lane: 1, 2, 3 or 4) is valid when
// a row of n2 voxels is 32 to 64 lanes.
inline bool row_vector_valid(int n2, int vw) {
  if (vw < 1 || vw > 4) return false;
  return n2 % vw == 0 && n2 / vw >= 32 && n2 / vw <= 64;
}

// Semi-Lagrangian gather along one axis: grid index i displaced by d voxels.
// Offsets beyond a million voxels (or NaN) are clamped first, so the integer
// conversion cannot overflow and the periodic wrap keeps every index in
// [0, n).  a = lower cell index, b = the next one (periodic), t in [0, 1] the
// weight of b.
constexpr double kSlMaxVoxels = 1.0e6;
template <typename T>
LDI_HD void sl_axis(int i, T d, int n, int& a, int& b, T& t) {
  constexpr T lim = T(kSlMaxVoxels);
  d = fmin(fmax(d, -lim), lim);
  const T f = floor(d);
  t = d - f;
  int j = (i + int(f)) % n;
  a = j < 0 ? j + n : j;
  b = a + 1 == n ? 0 : a + 1;
}

// ---------------------------------------------------------------------------
// Host: trajectory storage policy (vector fields held per policy, c = interval)
//   store-all   4 nt + 2             (mu_n, v_n for n <= nt; mu*_n, v*_n for n < nt)
//   checkpoint  ceil(nt/c) + 4 c + 1 (mu every c steps; one segment: mu, v, mu*, v*)
//   recompute   7                    (mu_0; rolling mu, v pairs; mu*, v*)
// ---------------------------------------------------------------------------
enum { TRAJ_STORE_ALL = 0, TRAJ_CHECKPOINT = 1, TRAJ_RECOMPUTE = 2 };

inline size_t traj_fields(int policy, int nt, int c) {
  if (policy == TRAJ_STORE_ALL) return size_t(4) * nt + 2;
  if (policy == TRAJ_CHECKPOINT) return size_t((nt + c - 1) / c) + size_t(4) * c + 1;
  return 7;
}

struct TrajChoice {
  int policy;
  int every;  // checkpoint interval (0 unless TRAJ_CHECKPOINT)
};

// checkpoint_every > 0: checkpoint every min(c, nt) steps; < 0: recompute; 0:
// store-all, unless budget > 0 and fixed + store-all would exceed it: then the
// largest interval whose total fits, else recompute.  fixed = bytes held besides
// the trajectory, vbytes = bytes of one vector field.
inline TrajChoice choose_trajectory(int nt, int checkpoint_every, long long budget, size_t fixed, size_t vbytes) {
  if (checkpoint_every > 0) return {TRAJ_CHECKPOINT, checkpoint_every < nt ? checkpoint_every : nt};
  if (checkpoint_every < 0) return {TRAJ_RECOMPUTE, 0};
  if (budget <= 0 || fixed + traj_fields(TRAJ_STORE_ALL, nt, 0) * vbytes <= size_t(budget))
    return {TRAJ_STORE_ALL, 0};
  for (int c = nt; c >= 1; --c)
    if (fixed + traj_fields(TRAJ_CHECKPOINT, nt, c) * vbytes <= size_t(budget)) return {TRAJ_CHECKPOINT, c};
  return {TRAJ_RECOMPUTE, 0};
}

}  // namespace lddmm
