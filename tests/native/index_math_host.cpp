// Host run of the field kernels' index arithmetic (index_math.h) and of the FFT
// plan code (fft_core.h) over every block and thread of real launch shapes,
// built with address and undefined-behaviour sanitizers.  Every index a kernel
// would form is checked against the bounds of the array it addresses; coverage
// maps are std::vector with checked access, so an out-of-range index is a
// reported failure and any wild access a sanitizer abort.  Exit status 0 = all
// checks passed; the last line names the number of checks.
#include <cmath>
#include <cstdint>
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <limits>
#include <random>
#include <vector>

#include "fft_core.h"
#include "index_math.h"

using namespace lddmm;

namespace {

long long g_checks = 0;
int g_failures = 0;

void expect(bool ok, const char* what, long long a = 0, long long b = 0, long long c = 0) {
  ++g_checks;
  if (!ok) {
    if (g_failures < 20) std::fprintf(stderr, "FAIL %s (%lld, %lld, %lld)\n", what, a, b, c);
    ++g_failures;
  }
}

// Every voxel of an n0 x n1 x n2 grid is visited exactly once by the launch
// (blocks x BX x BY threads), and only in-range indices are produced.
void check_tiling(int n0, int n1, int n2) {
  const FieldTiling t = field_tiling(n0, n1, n2);
  expect(t.BX % 32 == 0 && t.BX >= 32 && t.BX <= 256 && t.BX * t.BY <= 256, "block shape", t.BX, t.BY);
  expect(t.blocks == unsigned(t.TX) * unsigned(t.slab ? 8 * t.slab : t.TY) * unsigned(n0), "block count", t.blocks);
  if (t.slab) {
    expect(t.slab == (t.TY + 7) / 8 && 8 * t.slab <= 1.15 * t.TY, "slab balance", t.slab, t.TY);
  } else {
    expect(t.TY < 8 || 8 * ((t.TY + 7) / 8) > 1.15 * t.TY, "linear order only where slabs would be uneven", t.TY);
  }
  std::vector<uint8_t> seen(size_t(n0) * n1 * n2, 0);
  for (unsigned b = 0; b < t.blocks; ++b) {
    for (int ty = 0; ty < t.BY; ++ty)
      for (int tx = 0; tx < t.BX; ++tx) {
        int i0 = -1, i1 = -1, i2 = -1;
        if (!tile_voxel_at(t, int(b), tx, ty, n1, n2, i0, i1, i2)) continue;
        const bool in = i0 >= 0 && i0 < n0 && i1 >= 0 && i1 < n1 && i2 >= 0 && i2 < n2;
        expect(in, "voxel in range", i0, i1, i2);
        if (!in) continue;
        seen.at((size_t(i0) * n1 + i1) * n2 + i2) += 1;
      }
    if (t.slab) {
      // XCD-aware order: block b runs on XCD x = b mod 8, which owns x1 tiles
      // [x TY / 8, (x + 1) TY / 8) of every x0 plane
      int i0, i1, i2;
      if (tile_voxel_at(t, int(b), 0, 0, n1, n2, i0, i1, i2)) {
        const int x = int(b & 7), by = i1 / t.BY;
        expect(by >= x * t.TY / 8 && by < (x + 1) * t.TY / 8, "XCD slab ownership", b, i1);
      }
    }
  }
  long long once = 0;
  for (uint8_t s : seen) once += s == 1;
  expect(once == (long long)seen.size(), "each voxel exactly once", n0, n1, n2);
}

// Paired-row kernels: with rows of 32 lanes and N1 even, the two halves of every
// wave hold rows i1 (even) and i1 + 1 of the same x0 plane and the same x2
// columns, so each half's x1 neighbour is in the other half (lane ^ 32).
void check_pairs(int n0, int n1, int lanes) {
  const FieldTiling t = field_tiling(n0, n1, lanes);
  const int threads = t.BX * t.BY;
  expect(threads % 64 == 0, "whole waves", threads);
  for (unsigned b = 0; b < t.blocks; ++b)
    for (int tid = 0; tid < threads; ++tid) {
      const int lane = tid & 63;
      if (lane >= 32) continue;
      const int up = tid + 32;
      int a0, a1, a2, c0, c1, c2;
      const bool va = tile_voxel_at(t, int(b), tid % t.BX, tid / t.BX, n1, lanes, a0, a1, a2);
      const bool vc = tile_voxel_at(t, int(b), up % t.BX, up / t.BX, n1, lanes, c0, c1, c2);
      expect(va == vc, "both halves valid or neither", int(b), tid);
      if (!va || !vc) continue;
      expect(a1 % 2 == 0 && c1 == a1 + 1 && a0 == c0 && a2 == c2, "paired rows", a1, c1, a2 - c2);
    }
}

// Row-vectorised rows of RW lanes (32 to 64): every voxel lane's x2 neighbour
// lanes lie inside its own row, periodically; a launch over (N0, N1, RW) lanes
// puts each row at the start of a 32-lane half (RW = 32) or of a wave (RW > 32)
// with the lane's position in the row equal to its x2 index.
void check_row_lanes(int n0, int n1, int RW) {
  const int seg = RW <= 32 ? 32 : 64;
  for (int lane = 0; lane < 64; ++lane) {
    const int base = lane / seg * seg, pos = lane - base;
    int l, r;
    row_lanes(lane, RW, l, r);
    expect(l >= 0 && l < 64 && r >= 0 && r < 64, "row lanes in the wave", lane, l, r);
    if (pos >= RW) continue;  // no voxel on this lane
    expect(l >= base && l < base + RW && r >= base && r < base + RW, "row lanes inside the row", lane, l, r);
    expect(l == base + (pos + RW - 1) % RW && r == base + (pos + 1) % RW, "row lanes periodic", lane, l, r);
  }
  const FieldTiling t = field_tiling(n0, n1, RW);
  const int threads = t.BX * t.BY;
  for (unsigned b = 0; b < t.blocks; ++b)
    for (int tid = 0; tid < threads; ++tid) {
      int i0, i1, j;
      if (!tile_voxel_at(t, int(b), tid % t.BX, tid / t.BX, n1, RW, i0, i1, j)) continue;
      const int lane = tid & 63, pos = lane - lane / seg * seg;
      expect(pos == j, "lane position = x2 lane index", lane, j);
    }
}

// XCD-grouped units: a bijection of [0, B); in every whole span of 8 g blocks
// each XCD (block b mod 8) takes g consecutive units in the order of its
// blocks; a last partial span keeps unit = block.
void check_xcd_grouped(int B, int g) {
  std::vector<int> seen(B, 0), xcd(B, -1);
  for (int b = 0; b < B; ++b) {
    const int u = xcd_grouped(b, B, g);
    expect(u >= 0 && u < B, "unit in range", 100LL * B + g, b, u);
    if (u < 0 || u >= B) continue;
    ++seen[u];
    xcd[u] = b & 7;
    if (b >= 8 && u >= 1 && (b / (8 * g) + 1) * 8 * g <= B && (b / 8) % g != 0)
      expect(xcd_grouped(b - 8, B, g) == u - 1, "an XCD's units consecutive in block order", 100LL * B + g, b, u);
  }
  for (int u = 0; u < B; ++u) expect(seen[u] == 1, "every unit exactly once", B, g, u);
  const int whole = B / (8 * g) * 8 * g;
  for (int u = 0; u + 1 < whole; ++u)
    if ((u + 1) % g != 0) expect(xcd[u] == xcd[u + 1], "units of a run on one XCD", B, g, u);
}

// Run lengths of the transform passes from their alignment: rows of N2 reals
// (plane passes), and the pencil pass's tile, x0-plane, half and component
// strides in complex values (half planes: tiles of TB pairs, x0 stride N1 M,
// halves N1 M / 2 apart, components N0 N1 M apart, M = N2 / 2 + 1).
void check_xcd_runs() {
  struct Case {
    int n0, n1, n2, esize, tb, plane_run, pencil_run;
  };
  const Case cases[] = {
      {128, 128, 128, 4, 16, 1, 1},  // 512-byte rows, 4160-value halves: aligned
      {128, 128, 128, 8, 8, 1, 1},
      {256, 256, 256, 4, 16, 1, 1},
      {180, 216, 180, 4, 16, 2, 8},  // 720-byte rows, 9828-value halves
      {180, 216, 180, 8, 8, 2, 8},
      {96, 96, 96, 4, 16, 1, 1},     // 384-byte rows, 2352-value halves
      {80, 80, 80, 4, 16, 2, 8},     // 320-byte rows, 1640-value halves
      {112, 112, 112, 4, 16, 2, 8},
      {128, 128, 128, 4, 4, 1, 8},   // tiles of 4 pairs: 32-byte runs share lines
  };
  for (const Case& c : cases) {
    const long long M = c.n2 / 2 + 1, cs = 2LL * c.esize, P = (long long)c.n1 * M;
    const int plane = xcd_run_if_split((long long)c.n2 * c.esize, 0, 0, 0, 2);
    const int pencil = xcd_run_if_split(c.tb * cs, P * cs, P / 2 * cs, (long long)c.n0 * P * cs, 8);
    expect(plane == c.plane_run, "plane pass run length", c.n2, c.esize, plane);
    expect(pencil == c.pencil_run, "pencil pass run length", c.n1 * 1000LL + c.n2, c.tb, pencil);
  }
}

void check_periodic(int n) {
  for (int i = 0; i < n; ++i) {
    const int p = periodic_next(i, n), m = periodic_prev(i, n);
    expect(p >= 0 && p < n && m >= 0 && m < n, "periodic neighbour in range", i, p, m);
    expect(p == (i + 1) % n && m == (i + n - 1) % n, "periodic neighbour", i, p, m);
  }
}

// Semi-Lagrangian cells: indices in range for any displacement (NaN, infinities,
// huge values clamped), the upper cell the periodic successor, and, where the
// displacement is moderate, the cell and weight of floor(i + d).
template <typename T>
void check_sl_axis(int n, std::mt19937_64& rng) {
  std::vector<double> ds = {0.0, 0.25, -0.25, 0.5, -0.5, 1.0, -1.0, 1.0 - 1e-7, -1e-7, double(n), -double(n),
                            n + 0.25, -n - 0.25, 3.5 * n, -3.5 * n, 1e6, -1e6, 1e6 + 0.5, 1e7, -1e7, 1e30, -1e30,
                            std::numeric_limits<double>::infinity(), -std::numeric_limits<double>::infinity(),
                            std::numeric_limits<double>::quiet_NaN()};
  std::uniform_real_distribution<double> u(-4.0 * n, 4.0 * n);
  for (int k = 0; k < 200; ++k) ds.push_back(u(rng));
  const int is[] = {0, 1, n / 2, n - 2, n - 1};
  for (int i : is)
    for (double dd : ds) {
      const T d = T(dd);
      int a = -1, b = -1;
      T t = T(-1);
      sl_axis<T>(i, d, n, a, b, t);
      expect(a >= 0 && a < n && b >= 0 && b < n && b == (a + 1) % n, "sl cell in range", i, a, b);
      expect(t >= T(0) && t <= T(1), "sl weight in [0, 1]", i, (long long)(t * 1000));
      if (std::isfinite(dd) && std::fabs(dd) < 1e5) {
        const double f = std::floor(double(d));
        const long long want = (((long long)i + (long long)f) % n + n) % n;
        expect(a == want, "sl cell = floor(i + d) mod n", i, a, want);
      }
      // trilinear pair offsets in a row of n voxels: the lower corner, and the
      // upper one adjacent unless the lower ends the row (then the row's first)
      const int hi = a == n - 1 ? a - (n - 1) : a + 1;
      expect(hi >= 0 && hi < n && hi == b, "sl pair upper corner", a, hi, b);
    }
}

void check_trajectory_policy() {
  const size_t V = 1000;
  for (int nt = 1; nt <= 40; ++nt)
    for (int ce : {0, 1, 3, 4, 7, 100, -1}) {
      for (long long budget : {0LL, 5000LL, 9000LL, 12000LL, 20000LL, 40000LL, 80000LL, 200000LL}) {
        const size_t fixed = 3000;
        const TrajChoice ch = choose_trajectory(nt, ce, budget, fixed, V);
        expect(ch.policy >= TRAJ_STORE_ALL && ch.policy <= TRAJ_RECOMPUTE, "policy value", ch.policy);
        if (ce > 0) {
          expect(ch.policy == TRAJ_CHECKPOINT && ch.every == (ce < nt ? ce : nt), "explicit interval", nt, ce,
                 ch.every);
          continue;
        }
        if (ce < 0) {
          expect(ch.policy == TRAJ_RECOMPUTE, "explicit recompute", nt);
          continue;
        }
        const size_t all = fixed + traj_fields(TRAJ_STORE_ALL, nt, 0) * V;
        if (budget <= 0 || all <= size_t(budget)) {
          expect(ch.policy == TRAJ_STORE_ALL, "store-all when it fits", nt, budget);
          continue;
        }
        if (ch.policy == TRAJ_CHECKPOINT) {
          expect(ch.every >= 1 && ch.every <= nt, "interval range", nt, ch.every);
          expect(fixed + traj_fields(TRAJ_CHECKPOINT, nt, ch.every) * V <= size_t(budget), "interval fits", nt,
                 ch.every, budget);
          for (int c = ch.every + 1; c <= nt; ++c)
            expect(fixed + traj_fields(TRAJ_CHECKPOINT, nt, c) * V > size_t(budget), "largest interval", nt, c);
        } else {
          expect(ch.policy == TRAJ_RECOMPUTE, "recompute only as the last resort", nt, budget);
          for (int c = 1; c <= nt; ++c)
            expect(fixed + traj_fields(TRAJ_CHECKPOINT, nt, c) * V > size_t(budget), "no interval fits", nt, c);
        }
      }
    }
}

// Plans: every length whose prime factors are 2, 3, 5, 7 gets a plan whose
// digit reversal is a permutation and whose stage loops stay inside the
// sequence when run on the host (forward DIF then inverse DIT = n x identity).
template <bool INV>
void run_stages(cplx<double>* buf, const FftPlan& pl, const cplx<double>* tw) {
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
        default: expect(false, "radix", r); break;
      }
    }
  }
}

void check_plans(std::mt19937_64& rng) {
  std::normal_distribution<double> g;
  for (int n = 2; n <= 1024; ++n) {
    int m = n;
    for (int p : {2, 3, 5, 7})
      while (m % p == 0) m /= p;
    FftPlan pl{};
    const bool ok = make_plan(n, pl);
    expect(ok == (m == 1), "plan exists iff factors <= 7", n);
    if (!ok) continue;
    std::vector<int> hit(n, 0);
    for (int p = 0; p < n; ++p) hit.at(digit_reverse(pl, p)) += 1;
    bool perm = true;
    for (int h : hit) perm = perm && h == 1;
    expect(perm, "digit reversal is a permutation", n);
    std::vector<cplx<double>> tw(n), x(n), y(n);
    for (int k = 0; k < n; ++k) tw[k] = {std::cos(-2.0 * M_PI * k / n), std::sin(-2.0 * M_PI * k / n)};
    for (int k = 0; k < n; ++k) x[k] = {g(rng), g(rng)};
    y = x;
    run_stages<false>(y.data(), pl, tw.data());
    run_stages<true>(y.data(), pl, tw.data());
    double err = 0, ref = 0;
    for (int k = 0; k < n; ++k) {
      err = std::fmax(err, std::fabs(y[k].x / n - x[k].x) + std::fabs(y[k].y / n - x[k].y));
      ref = std::fmax(ref, std::fabs(x[k].x) + std::fabs(x[k].y));
    }
    expect(err <= 1e-12 * ref * n, "round trip", n);
  }
}

}  // namespace

int main() {
  std::mt19937_64 rng(12345);
  const int grids[][3] = {{4, 4, 4},      {5, 7, 6},      {4, 12, 20},   {6, 64, 64},    {4, 72, 96},
                          {4, 216, 180}, {8, 128, 128}, {4, 256, 256}, {128, 128, 128}, {16, 24, 30},
                          {180, 216, 180}, {7, 10, 8},    {4, 80, 80},   {4, 96, 112}};
  for (const auto& n : grids) check_tiling(n[0], n[1], n[2]);
  // rows of 33 to 64 lanes take 4 x1 rows per block: tile-row counts that 8 divides,
  // that it does not (uneven slabs, padded grid: 216 / 4 = 54, 100 / 4 = 25) and
  // where slabs would be too uneven (linear order)
  for (int n1 : {12, 20, 28, 32, 54, 60, 100, 112, 216, 217})
    for (int lanes : {40, 45, 54, 56, 64}) check_tiling(3, n1, lanes);
  // row-vectorised launches tile (N0, N1, N2 / VW) lanes
  for (int n1 : {4, 8, 64, 128, 216, 256}) {
    check_tiling(4, n1, 32);
    check_tiling(4, n1, 64);
    check_pairs(4, n1, 32);
  }
  check_pairs(128, 128, 32);
  for (int RW : {32, 33, 40, 45, 48, 54, 56, 60, 63, 64})
    for (int n1 : {4, 7, 12, 216}) check_row_lanes(4, n1, RW);
  for (int n2 : {64, 80, 96, 112, 128, 180, 192, 216, 256}) {
    // the widths the engine may take for a row of n2 voxels
    for (int vw : {0, 1, 2, 3, 4, 5}) {
      const bool ok = row_vector_valid(n2, vw);
      expect(ok == (vw >= 1 && vw <= 4 && n2 % vw == 0 && n2 / vw >= 32 && n2 / vw <= 64), "row width validity",
             n2, vw);
      if (ok) check_tiling(4, 12, n2 / vw);
    }
  }
  for (int n : {4, 5, 6, 7, 8, 12, 64, 128, 180, 216, 256, 512}) check_periodic(n);
  // unit counts of the transform launches: planes and half planes, pencil tiles
  for (int B : {1, 3, 7, 8, 9, 15, 16, 17, 384, 768, 780, 1080, 1083, 1536, 2457, 4096, 4113})
    for (int g : {1, 2, 4, 8}) check_xcd_grouped(B, g);
  check_xcd_runs();
  for (int n : {4, 5, 7, 20, 64, 128, 180, 216, 256}) {
    check_sl_axis<float>(n, rng);
    check_sl_axis<double>(n, rng);
  }
  check_trajectory_policy();
  check_plans(rng);
  std::printf("index math: %lld checks, %d failures\n", g_checks, g_failures);
  return g_failures == 0 ? 0 : 1;
}
