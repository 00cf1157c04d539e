// lddmm_api.cpp - host engine and C ABI of the LDDMM hot path.
//
// The engine owns the device workspace of one registration problem and drives
// the kernels of fft.hip / stencil.hip / sl.hip / reduce.hip on one stream:
//   shoot      EPDiff in momentum form with Heun steps (Section 2.2), optional
//              trajectory store and semi-Lagrangian state transport (Section 2.3)
//   gradient   final condition lambda(1) grad J_1 (Section 3) carried back by the
//              adjoint Jacobi sweep (the transposed Heun step of the tangent sweep)
//   hessvec    forward tangent sweep (incremental EPDiff + Jacobi field), the
//              Gauss-Newton final condition, the same adjoint sweep (Section 3)
//   cg / gn    CG in the V inner product and the inexact Gauss-Newton loop with
//              Armijo backtracking (Section 2.3 reduced KKT system, Section 3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <thread>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "lddmm.h"
#include "lddmm_internal.h"

namespace lddmm {

// Message of the calling thread's last failed context-free call (noalloc.hip).
const char* noalloc_last_error();

// ---------------------------------------------------------------------------
// Profiler
// ---------------------------------------------------------------------------
hipEvent_t Profiler::take() {
  if (!pool_.empty()) {
    hipEvent_t e = pool_.back();
    pool_.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

void Profiler::begin(const char* name, hipEvent_t* start, hipEvent_t* stop) {
  int kind = -1;
  for (size_t i = 0; i < kinds_.size(); ++i)
    if (kinds_[i] == name || std::strcmp(kinds_[i], name) == 0) {
      kind = int(i);
      break;
    }
  if (kind < 0) {
    kinds_.push_back(name);
    kind = int(kinds_.size()) - 1;
  }
  Rec r{kind, take(), take()};
  recs_.push_back(r);
  *start = r.a;
  *stop = r.b;
}

int Profiler::read(const char** names, int64_t* counts, double* total_ms, int cap) {
  std::vector<int64_t> c(kinds_.size(), 0);
  std::vector<double> ms(kinds_.size(), 0.0);
  for (auto& r : recs_) {
    (void)hipEventSynchronize(r.b);
    float t = 0.f;
    if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
      c[r.kind] += 1;
      ms[r.kind] += t;
    }
  }
  const int n = int(kinds_.size());
  for (int i = 0; i < n && i < cap; ++i) {
    if (names) names[i] = kinds_[i];
    if (counts) counts[i] = c[i];
    if (total_ms) total_ms[i] = ms[i];
  }
  return n;
}

void Profiler::clear() {
  for (auto& r : recs_) {
    pool_.push_back(r.a);
    pool_.push_back(r.b);
  }
  recs_.clear();
  kinds_.clear();
}

Profiler::~Profiler() {
  clear();
  for (hipEvent_t e : pool_) (void)hipEventDestroy(e);
}

// ---------------------------------------------------------------------------
// Engine
// ---------------------------------------------------------------------------
template <typename T>
class Engine {
 public:
  lddmm_params P{};
  Grid g{};
  long long N = 0;
  double cell = 0.0, dt = 0.0;
  hipStream_t st = nullptr;
  bool own_stream = false;  // created by a batch; destroyed with the engine
  std::string* err = nullptr;
  // Hessian-vector product replayed from a captured hipGraph (exec.graph = 1)
  bool use_graph = false;
  int cus = 0;  // compute units of the device (plane-walk candidates of the autotuner)
  hipGraphExec_t hv_exec = nullptr;
  const T* graph_dv = nullptr;
  const T* graph_ldv = nullptr;
  T* graph_hv = nullptr;
  Profiler prof;
  SpectralPlan<T> sp;
  std::vector<void*> allocs;
  size_t bytes = 0;

  // images and final conditions
  T *I0 = nullptr, *I1 = nullptr, *J1 = nullptr, *Jtmp = nullptr, *res = nullptr, *G = nullptr, *lin_v0 = nullptr;
  // trajectory store: mu_n, v_n (n <= nt), Heun predictors mu*_n, v*_n (n < nt)
  std::vector<T*> tmu, tv, tmus, tvs;
  // trajectory memory policy: store every step, keep mu every c steps and
  // re-materialise one segment at a time, or keep mu_0 only and replay
  int traj_policy = TRAJ_STORE_ALL, traj_every = 0;
  size_t traj_bytes = 0;
  std::vector<T*> ck;                                 // mu_{k c} (checkpoint) or mu_0 (recompute)
  std::vector<T*> seg_mu_buf, seg_v_buf, seg_mus, seg_vs;  // one materialised segment
  std::vector<const T*> seg_mu, seg_v;                // views into ck / lin_v0 / seg_*_buf
  int seg_loaded = -1;
  T *rb_mu[2] = {nullptr, nullptr}, *rb_v[2] = {nullptr, nullptr}, *rb_mus = nullptr, *rb_vs = nullptr;
  const T *rc_mu = nullptr, *rc_v = nullptr;
  int rc_m = -1;
  bool rc_star = false;
  // shooting scratch (no store) and displacement ping-pong
  T *sm[2] = {nullptr, nullptr}, *sv[2] = {nullptr, nullptr}, *sms = nullptr, *svs = nullptr;
  T *u[2] = {nullptr, nullptr};
  // tangent (X, dmu) and adjoint (U^, w) states, predictors, K-argument and the
  // adjoint stage's w-update part Qw (w_out = Qw + a1 dt K Z)
  T *X = nullptr, *Mu = nullptr, *Xs = nullptr, *Mus = nullptr, *W = nullptr;
  T *U = nullptr, *Wh = nullptr, *Us = nullptr, *Whs = nullptr, *Z = nullptr, *Qw = nullptr;
  // CG and Gauss-Newton vectors
  T *cr = nullptr, *cd = nullptr, *cHd = nullptr, *cLr = nullptr, *cLd = nullptr, *cx = nullptr;
  T *gv = nullptr, *Lg = nullptr, *trial = nullptr, *tmpS = nullptr;
  double* partials = nullptr;
  // FP64 results on the device and their pinned host mirror.  Slots: 0 dot
  // scratch; 2, 3 energy sums; 4-7 CG sums; 8, 9 check (non-finite count, max
  // |x|); 10 gradient norm sum; 11 <g, p> sum.  cgs: CG scalar block.
  static constexpr int kResSlots = 16;
  double* dres = nullptr;
  double* hres = nullptr;
  double* cgs = nullptr;
  double* hcg = nullptr;  // pinned host mirror of cgs

  // full Newton Hessian: first-order adjoint (U^, w) at the two stage inputs of
  // every backward step, and the tangent's trajectory variations (dmu, K dmu) at
  // the two stage points of every forward step (allocated on first use)
  std::vector<T*> nU1, nW1, nU2, nW2, tdmu, tdmuK, tdmus, tdmusK;
  int64_t newton_epoch = -1;
  bool use_newton = false;  // CG applies the Newton Hessian (solve method LDDMM_NEWTON_V)

  bool have_images = false, linearized = false;
  int64_t lin_epoch = 0;
  double E = 0, Ereg = 0, Edata = 0, base_sq = 0;

  ~Engine() {
    if (st) (void)hipStreamSynchronize(st);
    drop_graph();
    for (int c = 0; c < 3; ++c) {
      if (bst_c[c]) (void)hipStreamSynchronize(bst_c[c]);
      if (bst_c[c]) (void)hipStreamDestroy(bst_c[c]);
      if (bev_c[c]) (void)hipEventDestroy(bev_c[c]);
    }
    if (bev_fork) (void)hipEventDestroy(bev_fork);
    if (own_stream && st) (void)hipStreamDestroy(st);
    spectral_free(sp);
    for (void* p : allocs) (void)hipFree(p);
    if (hres) (void)hipHostFree(hres);
  }

  int fail(int code, const std::string& msg) {
    if (err) *err = msg;
    return code;
  }

  int alloc(T** p, long long count) {
    void* q = nullptr;
    if (hipMalloc(&q, size_t(count) * sizeof(T)) != hipSuccess) return LDDMM_ENOMEM;
    allocs.push_back(q);
    bytes += size_t(count) * sizeof(T);
    *p = static_cast<T*>(q);
    return 0;
  }

  int init(const lddmm_params& p, hipStream_t stream, std::string* e) {
    P = p;
    st = stream;
    err = e;
    g.n0 = p.n[0];
    g.n1 = p.n[1];
    g.n2 = p.n[2];
    g.N = (long long)p.n[0] * p.n[1] * p.n[2];
    g.h0 = 2.0 * M_PI / p.n[0];
    g.h1 = 2.0 * M_PI / p.n[1];
    g.h2 = 2.0 * M_PI / p.n[2];
    // stencil kernels: rows of 32-256 voxels go row-vectorised by default, the
    // smallest valid width in FP64 and the widest in FP32 (32-lane rows, paired
    // where N1 is even), the widths the autotuner keeps on MI355X; other rows
    // take one voxel per thread.  The autotuner times them all.
    g.rowvec = 0;
    for (int vw : {1, 2, 3, 4})
      if (row_vector_valid(g.n2, vw)) {
        g.rowvec = vw;
        if (sizeof(T) == 8) break;
      }
    N = g.N;
    cell = g.h0 * g.h1 * g.h2;
    dt = 1.0 / p.nt;
    int dev = 0, lds = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return fail(LDDMM_EHIP, "cannot query the device");
    std::string msg;
    int rc = spectral_init(sp, p.n, size_t(lds), msg);
    if (rc) return fail(rc, msg);
    bytes += sp.bytes;
    const long long V = 3 * N;
    T** vecs[] = {&G, &lin_v0, &sm[0], &sm[1], &sv[0], &sv[1], &sms, &svs, &u[0], &u[1], &X, &Mu, &Xs, &Mus, &W,
                  &U, &Wh, &Us, &Whs, &Z, &Qw, &cr, &cd, &cHd, &cLr, &cLd, &cx, &gv, &Lg, &trial};
    for (T** q : vecs)
      if (alloc(q, V)) return fail(LDDMM_ENOMEM, "out of device memory (workspace)");
    T** scal[] = {&I0, &I1, &J1, &Jtmp, &res, &tmpS};
    for (T** q : scal)
      if (alloc(q, N)) return fail(LDDMM_ENOMEM, "out of device memory (images)");
    if (int rc2 = alloc_trajectory(p, size_t(V) * sizeof(T))) return rc2;
    void* q = nullptr;
    if (hipMalloc(&q, sizeof(double) * 2 * kReduceBlocks) != hipSuccess) return fail(LDDMM_ENOMEM, "partials");
    allocs.push_back(q);
    partials = static_cast<double*>(q);
    if (hipMalloc(&q, sizeof(double) * (kResSlots + kCgSlots)) != hipSuccess) return fail(LDDMM_ENOMEM, "results");
    allocs.push_back(q);
    dres = static_cast<double*>(q);
    cgs = dres + kResSlots;
    if (hipHostMalloc(reinterpret_cast<void**>(&hres), sizeof(double) * (kResSlots + kCgSlots),
                      hipHostMallocDefault) != hipSuccess)
      return fail(LDDMM_ENOMEM, "pinned results");
    hcg = hres + kResSlots;
    return 0;
  }


  // ---- trajectory memory (policy: choose_trajectory) -------------------------
  int alloc_trajectory(const lddmm_params& p, size_t vbytes) {
    const int nt = p.nt;
    const TrajChoice ch = choose_trajectory(nt, p.checkpoint_every, (long long)p.mem_budget_bytes, bytes, vbytes);
    const int policy = ch.policy, c = ch.every;
    traj_policy = policy;
    traj_every = c;
    const size_t before = bytes;
    const long long V = 3 * N;
    auto grab = [&](std::vector<T*>& vec, size_t n) {
      vec.assign(n, nullptr);
      for (T*& q : vec)
        if (alloc(&q, V)) return false;
      return true;
    };
    bool ok = true;
    if (policy == TRAJ_STORE_ALL) {
      ok = grab(tmu, nt + 1) && grab(tv, nt + 1) && grab(tmus, nt) && grab(tvs, nt);
    } else if (policy == TRAJ_CHECKPOINT) {
      ok = grab(ck, (nt + c - 1) / c) && grab(seg_mu_buf, c) && grab(seg_v_buf, c) && grab(seg_mus, c) &&
           grab(seg_vs, c);
      seg_mu.assign(c, nullptr);
      seg_v.assign(c, nullptr);
    } else {
      ok = grab(ck, 1) && alloc(&rb_mu[0], V) == 0 && alloc(&rb_mu[1], V) == 0 && alloc(&rb_v[0], V) == 0 &&
           alloc(&rb_v[1], V) == 0 && alloc(&rb_mus, V) == 0 && alloc(&rb_vs, V) == 0;
    }
    if (!ok) return fail(LDDMM_ENOMEM, "out of device memory (trajectory)");
    traj_bytes = bytes - before;
    return 0;
  }

  // Where shoot_core puts mu_{n} (n >= 1) when storing: the trajectory for
  // store-all, a checkpoint slot at multiples of c, else scratch (nullptr).
  T* store_slot_mu(int n) {
    if (traj_policy == TRAJ_STORE_ALL) return tmu[n];
    if (traj_policy == TRAJ_CHECKPOINT && n < P.nt && n % traj_every == 0) return ck[n / traj_every];
    return nullptr;
  }
  T* store_slot_mu0() { return traj_policy == TRAJ_STORE_ALL ? tmu[0] : ck[0]; }

  struct Step {
    const T *mu, *v, *mus, *vs;
  };

  // One Heun step of the shooting from (mu, v): mus, vs always; next mu/v if asked.
  void heun_step(const T* mu, const T* v, T* mus, T* vs, T* mu_next, T* v_next) {
    launch_epdiff_stage<T>(g, v, mu, nullptr, mus, dt, 0.0, 1.0, st, &prof);
    applyK(mus, vs);
    if (mu_next) {
      launch_epdiff_stage<T>(g, vs, mus, mu, mu_next, dt, 0.5, 0.5, st, &prof);
      applyK(mu_next, v_next);
    }
  }

  // Segment k of the checkpointed trajectory: steps [k c, min((k+1) c, nt)),
  // recomputed from mu_{k c} with the shooting kernels (bitwise the stored run).
  void materialize(int k) {
    const int c = traj_every;
    const int n0 = k * c;
    const int len = std::min(c, P.nt - n0);
    seg_mu[0] = ck[k];
    if (k == 0) {
      seg_v[0] = lin_v0;
    } else {
      applyK(ck[k], seg_v_buf[0]);
      seg_v[0] = seg_v_buf[0];
    }
    for (int i = 0; i < len; ++i) {
      const bool more = i + 1 < len;
      heun_step(seg_mu[i], seg_v[i], seg_mus[i], seg_vs[i], more ? seg_mu_buf[i + 1] : nullptr,
                more ? seg_v_buf[i + 1] : nullptr);
      if (more) {
        seg_mu[i + 1] = seg_mu_buf[i + 1];
        seg_v[i + 1] = seg_v_buf[i + 1];
      }
    }
    seg_loaded = k;
  }

  // Coefficients of step n for the sweeps (valid until the next call).
  Step traj_view(int n) {
    if (traj_policy == TRAJ_STORE_ALL) return {tmu[n], tv[n], tmus[n], tvs[n]};
    if (traj_policy == TRAJ_CHECKPOINT) {
      const int k = n / traj_every;
      if (k != seg_loaded) materialize(k);
      const int i = n - k * traj_every;
      return {seg_mu[i], seg_v[i], seg_mus[i], seg_vs[i]};
    }
    // recompute: advance the rolling state, restarting from mu_0 when going back
    if (rc_m < 0 || rc_m > n) {
      rc_m = 0;
      rc_mu = ck[0];
      rc_v = lin_v0;
      rc_star = false;
    }
    while (true) {
      if (!rc_star) {
        heun_step(rc_mu, rc_v, rb_mus, rb_vs, nullptr, nullptr);
        rc_star = true;
      }
      if (rc_m == n) break;
      const int nx = (rc_mu == rb_mu[0]) ? 1 : 0;
      launch_epdiff_stage<T>(g, rb_vs, rb_mus, rc_mu, rb_mu[nx], dt, 0.5, 0.5, st, &prof);
      applyK(rb_mu[nx], rb_v[nx]);
      rc_mu = rb_mu[nx];
      rc_v = rb_v[nx];
      ++rc_m;
      rc_star = false;
    }
    return {rc_mu, rc_v, rb_mus, rb_vs};
  }

  void traj_invalidate() {
    seg_loaded = -1;
    rc_m = -1;
    rc_star = false;
  }

  int hip_status(const char* where) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(LDDMM_EHIP, std::string(where) + ": " + hipGetErrorString(e));
    return 0;
  }

  // ---- primitives -------------------------------------------------------
  // While a graph is captured with exec.branch_k = 1, a vector field's transform
  // is recorded as three independent per-component chains (forked from st onto
  // the branch streams and joined back), so the passes of one component can
  // overlap those of another.
  bool branch_k = false;   // option
  bool capturing = false;  // a graph capture on st is in progress
  hipStream_t bst_c[3] = {nullptr, nullptr, nullptr};
  hipEvent_t bev_fork = nullptr, bev_c[3] = {nullptr, nullptr, nullptr};
  int ensure_branch_streams() {
    if (bst_c[0]) return 0;
    if (hipEventCreateWithFlags(&bev_fork, hipEventDisableTiming) != hipSuccess) return LDDMM_EHIP;
    for (int c = 0; c < 3; ++c)
      if (hipStreamCreateWithFlags(&bst_c[c], hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&bev_c[c], hipEventDisableTiming) != hipSuccess)
        return LDDMM_EHIP;
    return 0;
  }
  void spectral(const T* in, T* out, int ncomp, int op, const T* add = nullptr, double add_scale = 0.0,
                double out_scale = 1.0) {
    if (ncomp != 3 || !capturing || !branch_k || !bst_c[0]) {
      spectral_apply(sp, in, out, ncomp, P.alpha, P.s, op, st, &prof, add, add_scale, out_scale);
      return;
    }
    (void)hipEventRecord(bev_fork, st);
    const size_t cstride = size_t(sp.n0) * sp.n1 * sp.M;
    for (int c = 0; c < 3; ++c) {
      (void)hipStreamWaitEvent(bst_c[c], bev_fork, 0);
      SpectralPlan<T> spc = sp;
      spc.spec = sp.spec + c * cstride;
      spectral_apply(spc, in + c * N, out + c * N, 1, P.alpha, P.s, op, bst_c[c], &prof, add ? add + c * N : nullptr,
                     add_scale, out_scale);
      (void)hipEventRecord(bev_c[c], bst_c[c]);
    }
    for (int c = 0; c < 3; ++c) (void)hipStreamWaitEvent(st, bev_c[c], 0);
  }
  void applyK(const T* in, T* out, int ncomp = 3) { spectral(in, out, ncomp, LDDMM_OP_K); }
  void applyL(const T* in, T* out, int ncomp = 3) { spectral(in, out, ncomp, LDDMM_OP_L); }
  // out = add + scale K in (vector fields): the adjoint stage's w update
  void applyK_add(const T* in, const T* add, double scale, T* out) { spectral(in, out, 3, LDDMM_OP_K, add, scale); }
  // out = scale K in (vector fields)
  void applyK_scaled(const T* in, double scale, T* out) {
    spectral(in, out, 3, LDDMM_OP_K, nullptr, 0.0, scale);
  }
  void copy(T* dst, const T* src, long long count) {
    (void)hipMemcpyAsync(dst, src, size_t(count) * sizeof(T), hipMemcpyDeviceToDevice, st);
  }
  // copy dres[0 .. k) to the pinned host mirror and wait
  void fetch(int k) {
    (void)hipMemcpyAsync(hres, dres, sizeof(double) * k, hipMemcpyDeviceToHost, st);
    (void)hipStreamSynchronize(st);
  }
  // enqueue a copy of every result slot and the CG scalars to the host mirror;
  // readable after wait()
  void post_fetch() {
    (void)hipMemcpyAsync(hres, dres, sizeof(double) * (kResSlots + kCgSlots), hipMemcpyDeviceToHost, st);
  }
  void wait() { (void)hipStreamSynchronize(st); }
  // dres[slot] = sum a.b over ncomp components (FP64), enqueued only
  void dot_dev(const T* a, const T* b, int ncomp, int slot) {
    launch_dot(a, b, ncomp * N, partials, dres + slot, st, &prof);
  }
  // h0 h1 h2 sum a.b over ncomp components (FP64), synchronising
  double dot(const T* a, const T* b, int ncomp = 3) {
    dot_dev(a, b, ncomp, 0);
    fetch(1);
    return cell * hres[0];
  }
  int check_finite(const T* a, long long count, const char* what) {
    launch_check(a, count, partials, dres, st, &prof);
    fetch(2);
    if (hres[0] != 0.0) return fail(LDDMM_ENONFINITE, std::string(what) + " holds NaN or Inf");
    return 0;
  }
  double maxabs(const T* a, long long count) {
    launch_check(a, count, partials, dres, st, &prof);
    fetch(2);
    return hres[1];
  }

  // ---- forward shooting ---------------------------------------------------
  // EPDiff (momentum form, Heun) from v0; store => trajectory arrays; with_sl =>
  // u transported and J composed into Jout; want_energy => dres[2] = <L v0, v0>
  // and dres[3] = ||Jout - I1||^2 (sums without the cell factor).  Returns the
  // final (mu, v).
  void shoot_core(const T* v0, bool store, bool with_sl, T* Jout, T** mu_last, T** v_last,
                  bool want_energy = false) {
    const bool all = store && traj_policy == TRAJ_STORE_ALL;
    T* mu_cur = store ? store_slot_mu0() : sm[0];
    T* v_cur = all ? tv[0] : sv[0];
    applyL(v0, mu_cur);
    copy(v_cur, v0, 3 * N);
    if (store) traj_invalidate();
    if (want_energy) dot_dev(mu_cur, v0, 3, 2);
    if (with_sl) launch_fill<T>(3 * N, T(0), u[0], st, &prof);
    for (int n = 0; n < P.nt; ++n) {
      T* ms = all ? tmus[n] : sms;
      T* vs = all ? tvs[n] : svs;
      T* mu_next = store ? store_slot_mu(n + 1) : nullptr;
      if (!mu_next) mu_next = (mu_cur == sm[0]) ? sm[1] : sm[0];
      T* v_next = all ? tv[n + 1] : ((v_cur == sv[0]) ? sv[1] : sv[0]);
      heun_step(mu_cur, v_cur, ms, vs, mu_next, v_next);
      if (with_sl) launch_sl_step<T>(g, u[n & 1], v_cur, v_next, u[(n + 1) & 1], dt, st, &prof);
      mu_cur = mu_next;
      v_cur = v_next;
    }
    if (with_sl) launch_compose<T>(g, I0, u[P.nt & 1], Jout, st, &prof);
    if (want_energy) {
      launch_axpbyz<T>(N, 1.0, Jout, -1.0, I1, tmpS, st, &prof);
      dot_dev(tmpS, tmpS, 1, 3);
    }
    if (mu_last) *mu_last = mu_cur;
    if (v_last) *v_last = v_cur;
  }

  T* final_u() { return u[P.nt & 1]; }

  // Energy terms left in dres[2], dres[3] by shoot_core(want_energy).
  double fetch_energy() {
    (void)hipMemcpyAsync(hres, dres + 2, sizeof(double) * 2, hipMemcpyDeviceToHost, st);
    (void)hipStreamSynchronize(st);
    return cell * hres[0] + cell * hres[1] / P.sigma2;
  }

  int shoot(const T* v0, T* Jo, T* uo, T* vo, double* energy_out) {
    if (int rc = check_finite(v0, 3 * N, "v0")) return rc;
    const bool need_img = Jo || uo || energy_out;
    if (need_img && !have_images) return fail(LDDMM_ESTATE, "images not set");
    T *ml = nullptr, *vl = nullptr;
    shoot_core(v0, false, need_img, Jtmp, &ml, &vl, energy_out != nullptr);
    if (Jo) copy(Jo, Jtmp, N);
    if (uo) copy(uo, final_u(), 3 * N);
    if (vo) copy(vo, vl, 3 * N);
    if (energy_out) *energy_out = fetch_energy();
    return hip_status("shoot");
  }

  int linearize(const T* v0, T* J1out, double* energy_out) {
    if (!have_images) return fail(LDDMM_ESTATE, "images not set");
    if (int rc = check_finite(v0, 3 * N, "v0")) return rc;
    linearize_nocheck(v0);
    if (J1out) copy(J1out, J1, N);
    if (energy_out) *energy_out = E;
    return hip_status("linearize");
  }

  // Linearization in two halves: the device work (trajectory store, residual,
  // G = grad J_1 and the sums of both energy terms in dres[2], dres[3]), then,
  // once those sums are on the host, the energy.
  void linearize_enqueue(const T* v0) {
    if (v0 != lin_v0) copy(lin_v0, v0, 3 * N);
    shoot_core(lin_v0, true, true, J1, nullptr, nullptr);
    launch_residual_grad<T>(g, J1, I1, res, G, st, &prof);
    dot_dev(store_slot_mu0(), lin_v0, 3, 2);
    dot_dev(res, res, 1, 3);
  }
  void linearize_finish() {
    Ereg = cell * hres[2];
    Edata = cell * hres[3] / P.sigma2;
    E = Ereg + Edata;
    linearized = true;
    ++lin_epoch;
  }
  void linearize_nocheck(const T* v0) {
    linearize_enqueue(v0);
    post_fetch();
    wait();
    linearize_finish();
  }

  // ---- adjoint Jacobi sweep (transposed Heun) ------------------------------
  // Input: U holds U^(1).  Output: Wh holds w_0 (U holds U^_0).
  // Each stage is one stencil kernel (Z = U + ad*_w mu, the U update and the
  // part Q of the w update) and one K application that adds a1 dt K Z to Q.
  void adjoint_pred(const Step& c) {
    launch_adjoint_stage<T>(g, U, Wh, c.mus, c.vs, nullptr, nullptr, Z, Qw, Us, dt, 0.0, 1.0, st, &prof);
    applyK_add(Z, Qw, dt, Whs);
  }
  // The sweep's first stage starts from w = 0: ad*_w mu and ad_v w vanish, so
  // Z = U and Q = 0.  The U update U + dt ad*_v U is the EPDiff stage's operator
  // taken with -dt, and the predictor of w is dt K U.
  void adjoint_pred_first(const Step& c) {
    launch_epdiff_stage<T>(g, c.vs, U, nullptr, Us, -dt, 0.0, 1.0, st, &prof);
    applyK_scaled(U, dt, Whs);
  }
  // out = w (default Wh) + 2 vadd when vadd is given; zero: launcher flag for a
  // zero start value of w (not read)
  void adjoint_corr(const Step& c, T* out = nullptr, const T* vadd = nullptr, int zero = 0) {
    launch_adjoint_stage<T>(g, Us, Whs, c.mu, c.v, U, Wh, Z, Qw, U, dt, 0.5, 0.5, st, &prof, vadd, 2.0, zero);
    applyK_add(Z, Qw, 0.5 * dt, out ? out : Wh);
  }
  // With out: the last stage writes 2 vadd + w_0 (the V-gradient form) to out
  // instead of w_0 to Wh.  The sweep starts from w = 0: the row-vectorised
  // first corrector does not read it, the one-voxel kernels read a zero fill.
  void backward(T* out = nullptr, const T* vadd = nullptr) {
    const bool zs = stencil_zero_start(g);
    if (!zs) launch_fill<T>(3 * N, T(0), Wh, st, &prof);
    for (int n = P.nt - 1; n >= 0; --n) {
      const Step c = traj_view(n);
      const bool first = n == P.nt - 1;
      if (first)
        adjoint_pred_first(c);
      else
        adjoint_pred(c);
      const bool last = n == 0 && out;
      adjoint_corr(c, last ? out : nullptr, last ? vadd : nullptr, first && zs ? 2 : 0);
    }
  }

  // ---- tangent sweep: X_nt from X_0 = 0, dmu_0 = L dv ------------------------
  // The first stage's K dmu_0 = K L dv is dv itself (K = L^-1 symbol by symbol),
  // so it takes dv without a transform.  With Ufin the last stage writes the GN
  // final condition (2 / sigma^2) (G . X_nt) G to Ufin instead of X_nt.  With
  // Ldv (= L dv, read only) the first step reads dmu_0 from there instead of
  // applying L.
  void tangent(const T* dv, T* Ufin = nullptr, const T* Ldv = nullptr) {
    if (!Ldv) applyL(dv, Mu);
    const T* Mu0 = Ldv ? Ldv : Mu;
    // X_0 = 0: the row-vectorised first stages do not read it, the one-voxel
    // kernels read a zero fill
    const bool zs = stencil_zero_start(g);
    if (!zs) launch_fill<T>(3 * N, T(0), X, st, &prof);
    for (int n = 0; n < P.nt; ++n) {
      const Step c = traj_view(n);
      const T* Min = n > 0 ? Mu : Mu0;  // dmu at the step's start
      const bool z0 = n == 0 && zs;
      if (n > 0) applyK(Mu, W);
      launch_tangent_stage<T>(g, X, Min, n > 0 ? W : dv, c.v, c.mu, nullptr, nullptr, Xs, Mus, dt, 0.0, 1.0, st,
                              &prof, nullptr, 0.0, z0 ? 1 : 0);
      applyK(Mus, W);
      if (Ufin && n == P.nt - 1)
        launch_tangent_stage<T>(g, Xs, Mus, W, c.vs, c.mus, X, Min, Ufin, nullptr, dt, 0.5, 0.5, st, &prof, G,
                                2.0 / P.sigma2, z0 ? 2 : 0);
      else
        launch_tangent_stage<T>(g, Xs, Mus, W, c.vs, c.mus, X, Min, X, Mu, dt, 0.5, 0.5, st, &prof, nullptr, 0.0,
                                z0 ? 2 : 0);
    }
  }

  void gradient_core(T* gout) {
    launch_scalar_times_vec<T>(g, res, G, -2.0 / P.sigma2, U, st, &prof);
    backward(gout, lin_v0);  // gout = 2 v0 + w_0
  }

  int gradient(const T* v0, T* gout, double* energy_out) {
    if (int rc = linearize(v0, nullptr, energy_out)) return rc;
    gradient_core(gout);
    return hip_status("gradient");
  }

  // Ldv: L dv when the caller already has it (CG keeps the L-image of its
  // direction); else the tangent sweep applies L itself.
  void hessvec_kernels(const T* dv, T* hv, const T* Ldv = nullptr) {
    tangent(dv, U, Ldv);  // U = (2 / sigma^2) (G . X_nt) G
    backward(hv, dv);     // hv = 2 dv + w_0
  }

  void drop_hv_graph() {
    if (hv_exec) (void)hipGraphExecDestroy(hv_exec);
    hv_exec = nullptr;
    graph_dv = nullptr;
    graph_ldv = nullptr;
    graph_hv = nullptr;
  }
  // every captured graph (launch shapes or options changed); graph_gen tells
  // batches that graphs they captured from this context are stale
  int graph_gen = 0;
  void drop_graph() {
    drop_hv_graph();
    drop_cg_graph();
    ++graph_gen;
  }

  // The Hv at a fixed linearization is a fixed sequence of launches on fixed
  // buffers (the trajectory, G and the work fields), so it is captured once per
  // (dv, hv) pair and replayed; the linearization's data change, not its
  // addresses.  Store-all trajectories only (the segment bookkeeping of the
  // other policies lives on the host), and never while profiling.
  void hessvec_core(const T* dv, T* hv, const T* Ldv = nullptr) {
    if (!use_graph || traj_policy != TRAJ_STORE_ALL || prof.enabled || !st) {
      hessvec_kernels(dv, hv, Ldv);
      return;
    }
    if (!hv_exec || graph_dv != dv || graph_hv != hv || graph_ldv != Ldv) {
      drop_hv_graph();
      hipGraph_t graph = nullptr;
      if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        hessvec_kernels(dv, hv, Ldv);
        return;
      }
      capturing = true;
      hessvec_kernels(dv, hv, Ldv);
      capturing = false;
      if (hipStreamEndCapture(st, &graph) != hipSuccess || !graph) {
        (void)hipGetLastError();
        hessvec_kernels(dv, hv, Ldv);
        return;
      }
      const hipError_t e = hipGraphInstantiate(&hv_exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) {
        hv_exec = nullptr;
        (void)hipGetLastError();
        hessvec_kernels(dv, hv, Ldv);
        return;
      }
      graph_dv = dv;
      graph_ldv = Ldv;
      graph_hv = hv;
    }
    (void)hipGraphLaunch(hv_exec, st);
  }

  // ---- full Newton Hessian-vector product -----------------------------------
  int ensure_newton() {
    if (!nU1.empty()) return 0;
    const long long V = 3 * N;
    for (auto* vec : {&nU1, &nW1, &nU2, &nW2, &tdmu, &tdmuK, &tdmus, &tdmusK}) {
      vec->assign(P.nt, nullptr);
      for (int n = 0; n < P.nt; ++n)
        if (alloc(&(*vec)[n], V)) {
          for (auto* w : {&nU1, &nW1, &nU2, &nW2, &tdmu, &tdmuK, &tdmus, &tdmusK}) w->clear();
          return fail(LDDMM_ENOMEM, "cannot allocate the Newton stage histories");
        }
    }
    return 0;
  }

  // The gradient's adjoint sweep, keeping its state at each stage input.
  void backward_record() {
    const long long V = 3 * N;
    launch_scalar_times_vec<T>(g, res, G, -2.0 / P.sigma2, U, st, &prof);
    launch_fill<T>(V, T(0), Wh, st, &prof);
    for (int n = P.nt - 1; n >= 0; --n) {
      const Step c = traj_view(n);
      copy(nU1[n], U, V);
      copy(nW1[n], Wh, V);
      adjoint_pred(c);
      copy(nU2[n], Us, V);
      copy(nW2[n], Whs, V);
      adjoint_corr(c);
    }
  }

  // The tangent sweep, keeping the trajectory variation at each stage point.
  void tangent_record(const T* dv) {
    const long long V = 3 * N;
    applyL(dv, Mu);
    launch_fill<T>(V, T(0), X, st, &prof);
    for (int n = 0; n < P.nt; ++n) {
      const Step c = traj_view(n);
      copy(tdmu[n], Mu, V);
      if (n > 0)
        applyK(Mu, tdmuK[n]);
      else
        copy(tdmuK[0], dv, V);  // K L dv = dv
      launch_tangent_stage<T>(g, X, Mu, tdmuK[n], c.v, c.mu, nullptr, nullptr, Xs, Mus, dt, 0.0, 1.0, st, &prof);
      copy(tdmus[n], Mus, V);
      applyK(Mus, tdmusK[n]);
      launch_tangent_stage<T>(g, Xs, Mus, tdmusK[n], c.vs, c.mus, X, Mu, X, Mu, dt, 0.5, 0.5, st, &prof);
    }
  }

  // 2 dv + dw_0 of the linearised adjoint sweep (dU, dw in U, Wh; stage in Us, Whs).
  void newton_core(const T* dv, T* hv) {
    if (newton_epoch != lin_epoch) {
      backward_record();
      newton_epoch = lin_epoch;
    }
    tangent_record(dv);
    launch_newton_final<T>(g, G, X, res, -2.0 / P.sigma2, tmpS, U, st, &prof);
    launch_fill<T>(3 * N, T(0), Wh, st, &prof);
    for (int n = P.nt - 1; n >= 0; --n) {
      const Step c = traj_view(n);
      launch_newton_stage<T>(g, U, Wh, c.mus, nW1[n], tdmus[n], c.vs, tdmusK[n], nU1[n], nullptr, nullptr, Z, Qw,
                             Us, dt, 0.0, 1.0, st, &prof);
      applyK_add(Z, Qw, dt, Whs);
      launch_newton_stage<T>(g, Us, Whs, c.mu, nW2[n], tdmu[n], c.v, tdmuK[n], nU2[n], U, Wh, Z, Qw, U, dt, 0.5, 0.5,
                             st, &prof);
      applyK_add(Z, Qw, 0.5 * dt, Wh);
    }
    launch_axpbyz<T>(3 * N, 2.0, dv, 1.0, Wh, hv, st, &prof);
  }

  int hessvec_newton(const T* v0, const T* dv, T* hv) {
    if (v0) {
      if (int rc = linearize(v0, nullptr, nullptr)) return rc;
    } else if (!linearized) {
      return fail(LDDMM_ESTATE, "hessvec_newton without a linearization");
    }
    if (int rc = ensure_newton()) return rc;
    newton_core(dv, hv);
    return hip_status("hessvec_newton");
  }

  // Hessian applied inside CG; Ldv = L dv (the GN product takes it instead of
  // applying L to dv).
  void apply_hessian(const T* dv, T* hv, const T* Ldv) {
    if (use_newton)
      newton_core(dv, hv);
    else
      hessvec_core(dv, hv, Ldv);
  }

  // ---- autotuner: time the transform variants on this grid, keep the fastest
  int autotune(int reps, int* tried) {
    if (reps <= 0) reps = 5;
    (void)hipStreamSynchronize(st);
    const FftTuning start = sp.tune;
    const bool start_halves = sp.halves;  // in use, not only requested
    FftTuning best = start;
    float best_ms = -1.f, start_ms = -1.f;
    int count = 0;
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return fail(LDDMM_EHIP, "events");
    const bool was = prof.enabled;
    prof.enabled = false;
    // operand: any vector work field (contents do not matter for timing)
    // plane walk candidates: one plane per workgroup, one workgroup per compute
    // unit, two planes per workgroup (vector fields: 3 n0 planes)
    const int planes = 3 * g.n0;
    const int grids[3] = {0, cus < planes ? cus : 0, planes > 1 ? (planes + 1) / 2 : 0};
    for (int pt : {512, 1024})
      for (int tb : {8, 16, 32})
        for (int stc : {1, 0})
          for (int gi = 0; gi < 4; ++gi) {
          // gi = 0: half planes; 1: whole planes, one per workgroup; 2, 3: plane walks
          if (gi > 1 && (grids[gi - 1] == 0 || stc == 0 || grids[gi - 1] == grids[gi - 2])) continue;
          if (gi == 0 && stc == 0) continue;
          FftTuning t = start;
          t.plane_threads = pt;
          t.pencil_tb = tb;
          t.pencil_threads = 256;
          t.use_static = stc;
          t.plane_grid = gi > 0 ? grids[gi - 1] : 0;
          t.plane_halves = gi == 0 ? 1 : 0;
          std::string msg;
          if (spectral_configure(sp, t, msg) != 0) continue;
          if (gi == 0 && !sp.halves) continue;  // no half-plane kernels for this shape
          // each K application is followed by a tangent stage, as in the sweeps:
          // timed alone, back to back, the shapes rank differently than in use
          applyK(W, Z);
          (void)hipEventRecord(a, st);
          for (int r = 0; r < reps; ++r) {
            applyK(W, Z);
            launch_tangent_stage<T>(g, X, Mu, Z, Xs, Mus, X, Mu, Us, Whs, dt, 0.0, 1.0, st, nullptr);
          }
          (void)hipEventRecord(b, st);
          (void)hipEventSynchronize(b);
          float ms = 0.f;
          (void)hipEventElapsedTime(&ms, a, b);
          ++count;
          if (best_ms < 0.f || ms < best_ms) {
            best_ms = ms;
            best = t;
          }
          if (t.plane_threads == start.plane_threads && t.pencil_tb == start.pencil_tb &&
              t.pencil_threads == start.pencil_threads && t.use_static == start.use_static &&
              t.plane_grid == start.plane_grid && (t.plane_halves != 0) == start_halves)
            start_ms = ms;
        }
    // Keep the starting shape unless another one is clearly faster: variants
    // within timing noise of each other would otherwise trade places between runs.
    if (start_ms > 0.f && start_ms <= 1.03f * best_ms) {
      best = start;
      best_ms = start_ms;
    }
    // Stencil kernels: one voxel per thread or VW voxels per lane, timed on the
    // tangent stage (the largest of them); work fields only, contents irrelevant.
    {
      const int start_vw = g.rowvec, start_pair = g.pair_rows;
      int best_vw = start_vw, best_pair = start_pair;
      float best_t = -1.f, start_t = -1.f;
      for (int vp : {0, 1, 2, 3, 4, 0x11, 0x12, 0x13, 0x14}) {
        const int vw = vp & 0xf, pr = vp >> 4;
        if (vw != 0 && !row_vector_valid(g.n2, vw)) continue;
        if (pr && (vw == 0 || g.n2 / vw != 32 || g.n1 % 2 != 0)) continue;  // pairing needs 32-lane rows
        g.rowvec = vw;
        g.pair_rows = pr;
        launch_tangent_stage<T>(g, X, Mu, W, Xs, Mus, X, Mu, Us, Whs, dt, 0.0, 1.0, st, nullptr);
        (void)hipEventRecord(a, st);
        for (int r = 0; r < reps; ++r)
          launch_tangent_stage<T>(g, X, Mu, W, Xs, Mus, X, Mu, Us, Whs, dt, 0.0, 1.0, st, nullptr);
        (void)hipEventRecord(b, st);
        (void)hipEventSynchronize(b);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, a, b);
        ++count;
        if (best_t < 0.f || ms < best_t) {
          best_t = ms;
          best_vw = vw;
          best_pair = pr;
        }
        if (vw == start_vw && (pr == start_pair || vw == 0 || g.n2 / vw != 32)) start_t = ms;
      }
      const bool keep = start_t > 0.f && start_t <= 1.03f * best_t;
      g.rowvec = keep ? start_vw : best_vw;
      g.pair_rows = keep ? start_pair : best_pair;
    }
    std::string msg;
    if (int rc = spectral_configure(sp, best, msg)) {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
      prof.enabled = was;
      return fail(rc, msg);
    }
    // Transforms of a vector field as one chain or as three per-component chains
    // (exec.branch_k, graphs only): a graph of at least 8 K applications, each
    // followed by a tangent stage, is captured for each setting and the two are
    // replayed in turn three times; the start setting is kept unless the other's
    // fastest replay is more than 0.5 % faster (both give bitwise the same
    // results; the Hv gains more than this proxy shows).
    if (st && ensure_branch_streams() == 0) {
      const bool start_bk = branch_k;
      hipGraph_t graphs[2] = {nullptr, nullptr};
      hipGraphExec_t execs[2] = {nullptr, nullptr};
      for (int bk = 0; bk < 2; ++bk) {
        branch_k = bk != 0;
        if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
          (void)hipGetLastError();
          break;
        }
        capturing = true;
        for (int r = 0; r < (reps > 8 ? reps : 8); ++r) {
          applyK(W, Z);
          launch_tangent_stage<T>(g, X, Mu, Z, Xs, Mus, X, Mu, Us, Whs, dt, 0.0, 1.0, st, nullptr);
        }
        capturing = false;
        if (hipStreamEndCapture(st, &graphs[bk]) != hipSuccess || !graphs[bk] ||
            hipGraphInstantiate(&execs[bk], graphs[bk], nullptr, nullptr, 0) != hipSuccess) {
          (void)hipGetLastError();
          execs[bk] = nullptr;
          break;
        }
      }
      branch_k = start_bk;
      if (execs[0] && execs[1]) {
        float tb[2] = {-1.f, -1.f};
        for (int bk = 0; bk < 2; ++bk) (void)hipGraphLaunch(execs[bk], st);  // warm-up
        for (int round = 0; round < 3; ++round)
          for (int bk = 0; bk < 2; ++bk) {
            (void)hipEventRecord(a, st);
            (void)hipGraphLaunch(execs[bk], st);
            (void)hipEventRecord(b, st);
            (void)hipEventSynchronize(b);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, a, b);
            if (tb[bk] < 0.f || ms < tb[bk]) tb[bk] = ms;
            ++count;
          }
        const int other = start_bk ? 0 : 1;
        if (tb[0] > 0.f && tb[1] > 0.f && tb[other] * 1.005f < tb[start_bk ? 1 : 0]) branch_k = other != 0;
      }
      for (int bk = 0; bk < 2; ++bk) {
        if (execs[bk]) (void)hipGraphExecDestroy(execs[bk]);
        if (graphs[bk]) (void)hipGraphDestroy(graphs[bk]);
      }
    }
    // reported: one K application of the chosen shape, timed alone
    applyK(W, Z);
    (void)hipEventRecord(a, st);
    for (int r = 0; r < reps; ++r) applyK(W, Z);
    (void)hipEventRecord(b, st);
    (void)hipEventSynchronize(b);
    float kms = 0.f;
    (void)hipEventElapsedTime(&kms, a, b);
    prof.enabled = was;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    drop_graph();
    autotune_ms = kms / reps;
    if (tried) *tried = count;
    return hip_status("autotune");
  }
  float autotune_ms = 0.f;

  int hessvec(const T* v0, const T* dv, T* hv) {
    if (v0) {
      if (int rc = linearize(v0, nullptr, nullptr)) return rc;
    } else if (!linearized) {
      return fail(LDDMM_ESTATE, "hessvec without a linearization");
    }
    hessvec_core(dv, hv);
    return hip_status("hessvec");
  }

  int vjp(const T* gbar, T* out) {
    if (!linearized) return fail(LDDMM_ESTATE, "vjp without a linearization");
    launch_scalar_times_vec<T>(g, gbar, G, -1.0, U, st, &prof);
    backward();
    applyL(Wh, out);
    return hip_status("vjp");
  }

  // ---- CG in V and PCG in L2, scalars on the device ---------------------------
  // CG in V for H x = -g (||r||_V <= eta ||g||_V or maxit): r, d, H d, L r, L d in
  // cr, cd, cHd, cLr, cLd.  The CG in V tracks the L-image of its direction
  // linearly (L d = L r + beta L d) for its inner products, and the GN product
  // takes it as its start value.
  // PCG in L2 for (L H) x = -g_L2 with preconditioner K (the "GN, L2" variant):
  // r, z = K r, d, q = L H d in cr, cLr, cd, cHd; H d itself in cLd; stops at
  // ||r||_L2 <= eta ||g_L2||_L2.
  // Every decision (step length, stop, beta) is taken on the device from the
  // FP64 sums; the host only reads whether the solve is still active.
  bool cg_l2 = false;  // the solve in progress is the PCG in L2
  int cg_maxit = 0;
  void cg_begin(const T* gin, T* x, double eta, int maxit, bool l2) {
    const long long V = 3 * N;
    cg_l2 = l2;
    cg_maxit = maxit;
    launch_axpbyz<T>(V, -1.0, gin, 0.0, gin, cr, st, &prof);
    launch_fill<T>(V, T(0), x, st, &prof);
    if (!l2) {
      copy(cd, cr, V);
      applyL(cr, cLr);
      copy(cLd, cLr, V);
      dot_dev(cLr, cr, 3, 4);
      launch_cg_begin(cgs, dres + 4, dres + 4, cell, eta, maxit, 1, st, &prof);
    } else {
      applyK(cr, cLr);
      copy(cd, cLr, V);
      dot_dev(cr, cLr, 3, 4);
      dot_dev(gin, gin, 3, 7);
      launch_cg_begin(cgs, dres + 4, dres + 7, cell, eta, maxit, 0, st, &prof);
    }
  }
  // One iteration (enqueue only; a no-op in effect once the solve has stopped).
  // hess_kernels: launch the Hessian kernel by kernel (inside a capture).
  void cg_iteration(T* x, bool hess_kernels = false) {
    const long long V = 3 * N;
    if (!cg_l2) {
      if (hess_kernels && !use_newton)
        hessvec_kernels(cd, cHd, cLd);
      else
        apply_hessian(cd, cHd, cLd);
      dot_dev(cLd, cHd, 3, 5);
      launch_cg_alpha(cgs, dres + 5, cell, st, &prof);
      launch_cg_step_dev<T>(V, cgs, cd, cHd, x, cr, st, &prof);
      applyL(cr, cLr);
      dot_dev(cLr, cr, 3, 6);
      launch_cg_beta(cgs, dres + 6, dres + 6, cell, st, &prof);
      launch_cg_direction<T>(V, cgs, cr, cd, st, &prof);
      launch_cg_direction<T>(V, cgs, cLr, cLd, st, &prof);
    } else {
      if (hess_kernels)
        hessvec_kernels(cd, cLd);
      else
        hessvec_core(cd, cLd);
      applyL(cLd, cHd);
      dot_dev(cd, cHd, 3, 5);
      launch_cg_alpha(cgs, dres + 5, cell, st, &prof);
      launch_cg_step_dev<T>(V, cgs, cd, cHd, x, cr, st, &prof);
      dot_dev(cr, cr, 3, 6);
      applyK(cr, cLr);
      dot_dev(cr, cLr, 3, 4);
      launch_cg_beta(cgs, dres + 4, dres + 6, cell, st, &prof);
      launch_cg_direction<T>(V, cgs, cLr, cd, st, &prof);
    }
  }
  bool cg_active() const { return hcg[CG_ACTIVE] != 0.0; }
  int cg_iters_done() const { return int(hcg[CG_ITERS]); }

  // The CG iteration replayed from a captured graph (exec.graph, store-all, Gauss-
  // Newton Hessian, not profiling): its launches and buffers are fixed for the
  // context, only the data change.  cgi_graph is kept for batches, which nest it.
  hipGraph_t cgi_graph = nullptr;
  hipGraphExec_t cgi_exec = nullptr;
  T* cgi_x = nullptr;
  bool cgi_l2 = false;
  bool cg_graph_ok() const { return use_graph && traj_policy == TRAJ_STORE_ALL && !prof.enabled && st && !use_newton; }
  void drop_cg_graph() {
    if (cgi_exec) (void)hipGraphExecDestroy(cgi_exec);
    if (cgi_graph) (void)hipGraphDestroy(cgi_graph);
    cgi_exec = nullptr;
    cgi_graph = nullptr;
    cgi_x = nullptr;
  }
  // Capture one iteration for (x, method) unless already captured; false if
  // capture is not possible (the caller then runs the iteration eagerly).
  bool ensure_cg_graph(T* x) {
    if (!cg_graph_ok()) return false;
    if (cgi_graph && cgi_x == x && cgi_l2 == cg_l2) return true;
    drop_cg_graph();
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    capturing = true;
    cg_iteration(x, true);
    capturing = false;
    hipGraph_t graph = nullptr;
    if (hipStreamEndCapture(st, &graph) != hipSuccess || !graph) {
      (void)hipGetLastError();
      return false;
    }
    if (hipGraphInstantiate(&cgi_exec, graph, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipGraphDestroy(graph);
      cgi_exec = nullptr;
      return false;
    }
    cgi_graph = graph;
    cgi_x = x;
    cgi_l2 = cg_l2;
    return true;
  }
  void cg_step_enqueue(T* x) {
    if (ensure_cg_graph(x))
      (void)hipGraphLaunch(cgi_exec, st);
    else
      cg_iteration(x);
  }
  // Whole solve on this context: one host read per iteration to stop early.
  int krylov(const T* gin, T* x, double eta, int maxit, bool l2, int* iters) {
    cg_begin(gin, x, eta, maxit, l2);
    for (int it = 1; it <= maxit; ++it) {
      cg_step_enqueue(x);
      post_fetch();
      wait();
      if (!cg_active()) break;
    }
    if (maxit < 1) {
      post_fetch();
      wait();
    }
    if (iters) *iters = cg_iters_done();
    return 0;
  }
  int cg(const T* gin, T* x, double eta, int maxit, int* iters) { return krylov(gin, x, eta, maxit, false, iters); }
  int pcg_l2(const T* gl2, T* x, double eta, int maxit, int* iters) { return krylov(gl2, x, eta, maxit, true, iters); }

  int cg_solve(const T* gin, T* x, double eta, int maxit, int* iters) {
    if (!linearized) return fail(LDDMM_ESTATE, "cg_solve without a linearization");
    if (maxit < 0 || !(eta >= 0.0)) return fail(LDDMM_EINVAL, "bad CG settings");
    cg(gin, x, eta, maxit, iters);
    return hip_status("cg_solve");
  }

  // ---- inexact Gauss-Newton-Krylov -----------------------------------------
  // The solve is a sequence of phases, each an enqueue followed (after the host
  // has the results) by a decision: the gradient at the current iterate, the
  // Krylov solve for the step, <g, p>, the Armijo trials, the bookkeeping of the
  // iteration.  gn_solve runs the phases of one context in order; a batch runs
  // each phase for all of its contexts before waiting once (gn_* below).
  struct Gn {
    lddmm_solve_opts op{};
    int method = LDDMM_GN_V;
    int k = 0;
    bool done = false;
    bool at_v = false;  // the current linearization is at v
    bool lin_pending = false;
    bool needs_krylov = false;
    bool searching = false;
    bool accepted = false;
    double g0 = 0, ginf0 = 0, gn = 0, ginf = 0, eta = 0, gp = 0, tau = 1, sign = 1;
    double E0 = 0, Er0 = 0, Ed0 = 0;
    const T* dir = nullptr;
    int its = 0, trials = 0, h = 0;
    T* v = nullptr;
    lddmm_solve_report R{};
    lddmm_iter_log* log = nullptr;
    int log_cap = 0;
  };
  Gn gs;
  struct NewtonScope {  // CG applies the Newton Hessian for this solve only
    bool& flag;
    NewtonScope(bool& f, bool on) : flag(f) { flag = on; }
    ~NewtonScope() { flag = false; }
  };

  int gn_setup(T* v, const lddmm_solve_opts* o, lddmm_iter_log* log, int log_cap) {
    if (!have_images) return fail(LDDMM_ESTATE, "images not set");
    if (int rc = check_finite(v, 3 * N, "v0")) return rc;
    Gn s;
    if (o) s.op = *o;
    s.method = s.op.method;
    if (s.method != LDDMM_GN_V && s.method != LDDMM_GN_L2 && s.method != LDDMM_GD_V && s.method != LDDMM_NEWTON_V)
      return fail(LDDMM_EINVAL, "unknown optimisation method");
    if (s.method == LDDMM_NEWTON_V)
      if (int rc = ensure_newton()) return rc;
    if (s.op.gn_iters <= 0) s.op.gn_iters = s.method == LDDMM_GD_V ? 50 : 10;
    if (s.op.cg_iters <= 0) s.op.cg_iters = 20;
    if (s.op.max_halvings <= 0) s.op.max_halvings = 10;
    if (s.op.c1 <= 0) s.op.c1 = 1e-4;
    if (s.op.gtol <= 0) s.op.gtol = 1e-3;
    if (s.op.eta_max <= 0) s.op.eta_max = 0.5;
    s.v = v;
    s.log = log;
    s.log_cap = log_cap;
    gs = s;
    return 0;
  }

  // Gradient phase: linearize at v unless an accepted trial already did (each
  // line-search trial is a full linearization: the trajectory store costs the same
  // writes as a plain shoot's scratch), the gradient, its L-image, and the sums of
  // the method's gradient norm and max |g|.
  void gn_grad_enqueue() {
    Gn& s = gs;
    const long long V = 3 * N;
    s.lin_pending = !s.at_v;
    if (s.lin_pending) linearize_enqueue(s.v);
    gradient_core(gv);
    applyL(gv, Lg);
    // the method's gradient and norm: g_V with ||g||_V, or g_L2 = L g_V with ||.||_L2
    if (s.method == LDDMM_GN_L2)
      dot_dev(Lg, Lg, 3, 10);
    else
      dot_dev(Lg, gv, 3, 10);
    launch_check(s.method == LDDMM_GN_L2 ? Lg : gv, V, partials, dres + 8, st, &prof);
    post_fetch();
  }
  void gn_grad_finish() {
    Gn& s = gs;
    if (s.lin_pending) linearize_finish();
    s.lin_pending = false;
    s.at_v = true;
    s.R.gradients++;
    if (s.k == 0) s.R.E_first = E;
    s.gn = s.method == LDDMM_GN_L2 ? std::sqrt(cell * hres[10]) : std::sqrt(std::max(0.0, cell * hres[10]));
    s.ginf = hres[9];
    if (s.k == 0) {
      s.g0 = s.gn;
      s.ginf0 = s.ginf;
    }
    s.R.g_rel_final = s.g0 > 0 ? s.gn / s.g0 : 0.0;
    if (s.g0 == 0.0 || s.gn / s.g0 <= s.op.gtol) {
      s.R.stop_reason = 1;
      s.done = true;
      return;
    }
    // search direction p and the slope <g, p> of E along it (same value in V and L2)
    s.eta = 0.0;
    s.gp = 0.0;
    s.tau = 1.0;
    s.sign = 1.0;
    s.its = 0;
    s.dir = cx;
    s.needs_krylov = s.method != LDDMM_GD_V;
    if (!s.needs_krylov) {
      s.dir = gv;
      s.sign = -1.0;
      s.gp = -s.gn * s.gn;
      s.tau = 0.5;
    } else {
      s.eta = std::min(s.op.eta_max, std::sqrt(s.gn / s.g0));
    }
  }
  // Krylov phase (CG in V or PCG in L2), begun here and stepped by the caller.
  void gn_krylov_begin() {
    Gn& s = gs;
    cg_begin(s.method == LDDMM_GN_L2 ? Lg : gv, cx, s.eta, s.op.cg_iters, s.method == LDDMM_GN_L2);
  }
  // <g, p> after the Krylov solve
  void gn_slope_enqueue() {
    Gn& s = gs;
    s.its = cg_iters_done();
    s.R.cg_total += s.its;
    s.R.hessvecs += s.its;
    dot_dev(Lg, cx, 3, 11);
    post_fetch();
  }
  void gn_slope_finish() { gs.gp = cell * hres[11]; }
  void gn_search_begin() {
    Gn& s = gs;
    s.E0 = E;
    s.Er0 = Ereg;
    s.Ed0 = Edata;
    s.accepted = false;
    s.trials = 0;
    s.h = 0;
    s.searching = true;
  }
  void gn_trial_enqueue() {
    Gn& s = gs;
    launch_axpbyz<T>(3 * N, 1.0, s.v, s.sign * s.tau, s.dir, trial, st, &prof);
    linearize_enqueue(trial);
    s.at_v = false;
    post_fetch();
  }
  void gn_trial_finish() {
    Gn& s = gs;
    linearize_finish();
    s.R.shoots++;
    s.trials++;
    if (E <= s.E0 + s.op.c1 * s.tau * s.gp) {
      s.accepted = true;
      s.searching = false;
      return;
    }
    s.tau *= 0.5;
    if (++s.h > s.op.max_halvings) s.searching = false;
  }
  // end of an outer iteration: log, accept the step or stop
  void gn_iteration_end() {
    Gn& s = gs;
    if (s.log && s.k < s.log_cap) {
      lddmm_iter_log& L = s.log[s.k];
      L.E = s.E0;
      L.E_reg = s.Er0;
      L.E_data = s.Ed0;
      L.mse_rel = base_sq > 0 ? 100.0 * s.Ed0 * P.sigma2 / base_sq : 0.0;
      L.g_norm = s.gn;
      L.g_inf_rel = s.ginf0 > 0 ? s.ginf / s.ginf0 : 0.0;
      L.eta = s.eta;
      L.tau = s.accepted ? s.tau : 0.0;
      L.cg_iters = s.its;
      L.ls_trials = s.trials;
    }
    s.R.iters = s.k + 1;
    if (!s.accepted) {
      s.R.stop_reason = 2;
      s.done = true;
      return;
    }
    copy(s.v, trial, 3 * N);
    s.at_v = true;  // the accepted trial's linearization is the one at the new v
    if (++s.k >= s.op.gn_iters) s.done = true;
  }
  // after the last iteration: the linearization at the returned v and the report
  void gn_final_enqueue() {
    if (!gs.at_v) linearize_enqueue(gs.v);
    post_fetch();
  }
  void gn_final_finish(lddmm_solve_report* rep) {
    Gn& s = gs;
    if (!s.at_v) linearize_finish();
    s.at_v = true;
    s.R.E_final = E;
    s.R.mse_rel_final = base_sq > 0 ? 100.0 * Edata * P.sigma2 / base_sq : 0.0;
    if (rep) *rep = s.R;
  }

  int gn_solve(T* v, const lddmm_solve_opts* o, lddmm_solve_report* rep, lddmm_iter_log* log, int log_cap) {
    if (int rc = gn_setup(v, o, log, log_cap)) return rc;
    NewtonScope newton_scope(use_newton, gs.method == LDDMM_NEWTON_V);
    Gn& s = gs;
    while (!s.done) {
      gn_grad_enqueue();
      wait();
      gn_grad_finish();
      if (s.done) break;
      if (s.needs_krylov) {
        gn_krylov_begin();
        for (int it = 1; it <= s.op.cg_iters; ++it) {
          cg_step_enqueue(cx);
          post_fetch();
          wait();
          if (!cg_active()) break;
        }
        gn_slope_enqueue();
        wait();
        gn_slope_finish();
      }
      gn_search_begin();
      while (s.searching) {
        gn_trial_enqueue();
        wait();
        gn_trial_finish();
      }
      gn_iteration_end();
    }
    gn_final_enqueue();
    wait();
    gn_final_finish(rep);
    return hip_status("gn_solve");
  }

  int set_images(const T* a, const T* b) {
    if (int rc = check_finite(a, N, "I0")) return rc;
    if (int rc = check_finite(b, N, "I1")) return rc;
    copy(I0, a, N);
    copy(I1, b, N);
    launch_axpbyz<T>(N, 1.0, I0, -1.0, I1, tmpS, st, &prof);
    base_sq = dot(tmpS, tmpS, 1);
    have_images = true;
    linearized = false;
    return hip_status("set_images");
  }

  int set_option(const char* key, int64_t value) {
    FftTuning t = sp.tune;
    const std::string k(key);
    if (k == "fft.plane_threads")
      t.plane_threads = int(value);
    else if (k == "fft.pencil_threads")
      t.pencil_threads = int(value);
    else if (k == "fft.pencil_tb")
      t.pencil_tb = int(value);
    else if (k == "fft.rows_rb")
      t.rows_rb = int(value);
    else if (k == "fft.force_split")
      t.force_split = value != 0;
    else if (k == "fft.static")
      t.use_static = value != 0;
    else if (k == "fft.plane_grid")
      t.plane_grid = int(value);
    else if (k == "fft.plane_halves")
      t.plane_halves = value != 0;
    else if (k == "exec.graph") {
      if (value != 0 && !st) return fail(LDDMM_EINVAL, "exec.graph needs a non-default stream");
      (void)hipStreamSynchronize(st);
      use_graph = value != 0;
      drop_graph();
      return 0;
    } else if (k == "stencil.rowvec") {
      if (value != 0 && !row_vector_valid(g.n2, int(value)))
        return fail(LDDMM_EINVAL, "stencil.rowvec: N2 / value must be 32 to 64 with value 1, 2, 3 or 4");
      (void)hipStreamSynchronize(st);
      g.rowvec = int(value);
      drop_graph();
      return 0;
    } else if (k == "exec.branch_k") {
      if (value != 0 && value != 1) return fail(LDDMM_EINVAL, "exec.branch_k: 0 or 1");
      (void)hipStreamSynchronize(st);
      if (value && ensure_branch_streams()) return fail(LDDMM_EHIP, "cannot create the branch streams");
      branch_k = value != 0;
      drop_graph();
      return 0;
    } else if (k == "stencil.pair_rows") {
      if (value != 0 && value != 1) return fail(LDDMM_EINVAL, "stencil.pair_rows: 0 or 1");
      (void)hipStreamSynchronize(st);
      g.pair_rows = int(value);
      drop_graph();
      return 0;
    } else
      return fail(LDDMM_EINVAL, "unknown or read-only option " + k);
    if (value < 0 || value > (1 << 20)) return fail(LDDMM_EINVAL, "option value out of range");
    (void)hipStreamSynchronize(st);
    std::string msg;
    if (int rc = spectral_configure(sp, t, msg)) return fail(rc, msg);
    drop_graph();
    return 0;
  }

  int get_option(const char* key, int64_t* value) {
    const std::string k(key);
    const FftTuning& t = sp.tune;
    if (k == "fft.plane_threads")
      *value = t.plane_threads;
    else if (k == "fft.pencil_threads")
      *value = t.pencil_threads;
    else if (k == "fft.pencil_tb")
      *value = t.pencil_tb;
    else if (k == "fft.rows_rb")
      *value = t.rows_rb;
    else if (k == "fft.force_split")
      *value = t.force_split;
    else if (k == "fft.fused")
      *value = sp.fused ? 1 : 0;
    else if (k == "fft.static")
      *value = t.use_static;
    else if (k == "fft.static_kernels")
      *value = sp.static_kernels;
    else if (k == "fft.plane_grid")
      *value = t.plane_grid;
    else if (k == "stencil.pair_rows")
      *value = g.pair_rows;
    else if (k == "fft.plane_walk")
      *value = sp.plane_grid;
    else if (k == "fft.plane_halves")
      *value = t.plane_halves;
    else if (k == "fft.plane_halves_used")
      *value = sp.halves ? 1 : 0;
    else if (k == "traj.policy")
      *value = traj_policy;
    else if (k == "traj.every")
      *value = traj_every;
    else if (k == "traj.bytes")
      *value = int64_t(traj_bytes);
    else if (k == "lin.epoch")
      *value = lin_epoch;
    else if (k == "exec.graph")
      *value = use_graph ? 1 : 0;
    else if (k == "exec.branch_k")
      *value = branch_k ? 1 : 0;
    else if (k == "stencil.rowvec")
      *value = g.rowvec;
    else
      return fail(LDDMM_EINVAL, "unknown option " + k);
    return 0;
  }

  // ---- PDE-LDDMM (Section 2.3), the comparison method ----------------------
  // Velocities over time: stationary, one vector field; non-stationary, nt + 1
  // vector fields v_0..v_nt at t_n = n dt, stacked ([nt+1][3][N0][N1][N2]).  The
  // state m_n is the image transported by SL, the adjoint lambda the continuity
  // equation along forward characteristics; gradient and Gauss-Newton Hessian in
  // the space-time L2 product (trapezoid weights in time), solved by PCG with K
  // per time point.  Workspace allocated on first use.
  bool pde_ready = false, pde_lin = false, pde_stat = false;
  T *pv = nullptr, *pg = nullptr, *ptrial = nullptr, *px = nullptr, *pr = nullptr, *pz = nullptr, *pd = nullptr,
    *pq = nullptr, *pacc = nullptr;
  std::vector<T*> pm, pD;              // m_n and div v_n, n = 0..nt
  T *plam[2] = {nullptr, nullptr}, *pdm[2] = {nullptr, nullptr}, *psrc[2] = {nullptr, nullptr};
  double pE = 0, pEreg = 0, pEdata = 0;

  int pde_slices(bool stationary) const { return stationary ? 1 : P.nt + 1; }
  // quadrature weight of time point n (trapezoid, dt)
  double pde_w(int n) const { return (n == 0 || n == P.nt) ? 0.5 * dt : dt; }
  int ensure_pde() {
    if (pde_ready) return 0;
    const long long V = 3 * N, S = (long long)(P.nt + 1) * V;
    for (T** q : {&pv, &pg, &ptrial, &px, &pr, &pz, &pd, &pq})
      if (alloc(q, S)) return fail(LDDMM_ENOMEM, "out of device memory (PDE-LDDMM workspace)");
    if (alloc(&pacc, V)) return fail(LDDMM_ENOMEM, "out of device memory (PDE-LDDMM workspace)");
    pm.assign(P.nt + 1, nullptr);
    pD.assign(P.nt + 1, nullptr);
    for (auto* vec : {&pm, &pD})
      for (T*& q : *vec)
        if (alloc(&q, N)) return fail(LDDMM_ENOMEM, "out of device memory (PDE-LDDMM workspace)");
    for (T** q : {&plam[0], &plam[1], &pdm[0], &pdm[1], &psrc[0], &psrc[1]})
      if (alloc(q, N)) return fail(LDDMM_ENOMEM, "out of device memory (PDE-LDDMM workspace)");
    pde_ready = true;
    return 0;
  }
  // time point n of a stack (every point is the single field when stationary)
  const T* slice(const T* stack, int n, bool stationary) const {
    return stationary ? stack : stack + (long long)n * 3 * N;
  }
  T* slice(T* stack, int n, bool stationary) const { return stationary ? stack : stack + (long long)n * 3 * N; }

  // FP64 space-time L2 product sum_n w_n <a_n, b_n> of two stacks (synchronising)
  double pde_dot(const T* a, const T* b, bool stationary) {
    const long long V = 3 * N;
    if (stationary) return dot(a, b);
    dot_dev(a, b, 3 * (P.nt + 1), 12);                                  // all time points
    launch_dot(a, b, V, partials, dres + 13, st, &prof);                  // t = 0
    launch_dot(a + P.nt * V, b + P.nt * V, V, partials, dres + 14, st, &prof);  // t = 1
    post_fetch();
    wait();
    return cell * dt * (hres[12] - 0.5 * hres[13] - 0.5 * hres[14]);
  }
  // state sweep, divergences and both energy terms at the stack v (copied)
  void pde_linearize(const T* v, bool stationary) {
    const long long V = 3 * N;
    const int ns = pde_slices(stationary);
    if (v != pv) copy(pv, v, ns * V);
    copy(pm[0], I0, N);
    for (int n = 0; n < P.nt; ++n)
      launch_pde_state<T>(g, pm[n], slice(pv, n, stationary), slice(pv, n + 1, stationary), pm[n + 1], dt, st, &prof);
    for (int n = 0; n < ns; ++n) launch_div<T>(g, slice(pv, n, stationary), pD[n], st, &prof);
    // regulariser: <L v, v> (stationary) or sum_n w_n <L v_n, v_n>
    double ereg = 0;
    for (int n = 0; n < ns; ++n) {
      applyL(slice(pv, n, stationary), pacc);
      const double d = dot(pacc, slice(pv, n, stationary));
      ereg += stationary ? d : pde_w(n) * d;
    }
    launch_axpbyz<T>(N, 1.0, pm[P.nt], -1.0, I1, tmpS, st, &prof);
    pEreg = ereg;
    pEdata = dot(tmpS, tmpS, 1) / P.sigma2;
    pE = pEreg + pEdata;
    pde_lin = true;
    pde_stat = stationary;
  }
  // Backward sweep of a final lambda in plam[nt & 1]: out = 2 L base + sum over
  // time of lambda_n grad m_n (per time point, or its time integral when stationary).
  void pde_backward(const T* base, T* out, bool stationary) {
    const long long V = 3 * N;
    if (stationary) launch_fill<T>(V, T(0), pacc, st, &prof);
    for (int n = P.nt; n >= 0; --n) {
      const T* lam = plam[n & 1];
      if (n < P.nt)
        launch_pde_adjoint<T>(g, plam[(n + 1) & 1], pD[stationary ? 0 : n], pD[stationary ? 0 : n + 1],
                              slice(pv, n, stationary), slice(pv, n + 1, stationary), plam[n & 1], dt, st, &prof);
      if (stationary) {
        launch_pde_lambda_grad<T>(g, pm[n], lam, pde_w(n), pacc, st, &prof);
      } else {
        T* o = slice(out, n, false);
        spectral(slice(base, n, false), o, 3, LDDMM_OP_L, nullptr, 0.0, 2.0);  // 2 L base_n
        launch_pde_lambda_grad<T>(g, pm[n], lam, 1.0, o, st, &prof);
      }
    }
    if (stationary) spectral(base, out, 3, LDDMM_OP_L, pacc, 2.0);  // pacc + 2 L base
  }
  int pde_check(bool stationary) {
    if (!have_images) return fail(LDDMM_ESTATE, "images not set");
    (void)stationary;
    return ensure_pde();
  }
  int pde_energy(bool stationary, const T* v, T* m1, double* energy) {
    if (int rc = pde_check(stationary)) return rc;
    if (int rc = check_finite(v, (long long)pde_slices(stationary) * 3 * N, "v")) return rc;
    pde_linearize(v, stationary);
    if (m1) copy(m1, pm[P.nt], N);
    if (energy) *energy = pE;
    return hip_status("pde_energy");
  }
  void pde_gradient_core(T* gout) {
    launch_axpbyz<T>(N, -2.0 / P.sigma2, pm[P.nt], 2.0 / P.sigma2, I1, plam[P.nt & 1], st, &prof);
    pde_backward(pv, gout, pde_stat);
  }
  int pde_gradient(bool stationary, const T* v, T* gout, double* energy) {
    if (int rc = pde_energy(stationary, v, nullptr, energy)) return rc;
    pde_gradient_core(gout);
    return hip_status("pde_gradient");
  }
  // Gauss-Newton Hessian at the current PDE linearization
  void pde_hessvec_core(const T* dv, T* hv) {
    const bool stationary = pde_stat;
    launch_fill<T>(N, T(0), pdm[0], st, &prof);
    launch_pde_source<T>(g, pm[0], slice(dv, 0, stationary), psrc[0], st, &prof);
    for (int n = 0; n < P.nt; ++n) {
      launch_pde_source<T>(g, pm[n + 1], slice(dv, n + 1, stationary), psrc[(n + 1) & 1], st, &prof);
      launch_pde_incr<T>(g, pdm[n & 1], psrc[n & 1], psrc[(n + 1) & 1], slice(pv, n, stationary),
                         slice(pv, n + 1, stationary), pdm[(n + 1) & 1], dt, st, &prof);
    }
    launch_axpbyz<T>(N, -2.0 / P.sigma2, pdm[P.nt & 1], 0.0, pdm[P.nt & 1], plam[P.nt & 1], st, &prof);
    pde_backward(dv, hv, stationary);
  }
  int pde_hessvec(bool stationary, const T* v, const T* dv, T* hv) {
    if (int rc = pde_check(stationary)) return rc;
    if (v) {
      if (int rc = pde_energy(stationary, v, nullptr, nullptr)) return rc;
    } else if (!pde_lin || pde_stat != stationary) {
      return fail(LDDMM_ESTATE, "pde_hessvec without a PDE linearization of this parameterisation");
    }
    pde_hessvec_core(dv, hv);
    return hip_status("pde_hessvec");
  }
  // K per time point
  void pde_precondition(const T* r, T* z, bool stationary) {
    for (int n = 0; n < pde_slices(stationary); ++n) applyK(slice(r, n, stationary), slice(z, n, stationary));
  }
  // PCG in the space-time L2 product for H x = -g, preconditioner K
  int pde_pcg(const T* gin, T* x, double eta, int maxit) {
    const bool stn = pde_stat;
    const long long S = (long long)pde_slices(stn) * 3 * N;
    launch_axpbyz<T>(S, -1.0, gin, 0.0, gin, pr, st, &prof);
    launch_fill<T>(S, T(0), x, st, &prof);
    pde_precondition(pr, pz, stn);
    copy(pd, pz, S);
    double rz = pde_dot(pr, pz, stn);
    const double tol = eta * std::sqrt(pde_dot(gin, gin, stn));
    int it = 0;
    for (it = 1; it <= maxit; ++it) {
      pde_hessvec_core(pd, pq);
      const double dq = pde_dot(pd, pq, stn);
      if (!(dq > 0.0)) {
        --it;
        break;
      }
      const double a = rz / dq;
      launch_axpby<T>(S, a, pd, 1.0, x, st, &prof);
      launch_axpby<T>(S, -a, pq, 1.0, pr, st, &prof);
      if (std::sqrt(pde_dot(pr, pr, stn)) <= tol) break;
      pde_precondition(pr, pz, stn);
      const double rz_new = pde_dot(pr, pz, stn);
      launch_axpby<T>(S, 1.0, pz, rz_new / rz, pd, st, &prof);
      rz = rz_new;
    }
    if (it > maxit) it = maxit;
    return it;
  }
  int pde_gn_solve(bool stationary, T* v, const lddmm_solve_opts* o, lddmm_solve_report* rep, lddmm_iter_log* log,
                   int log_cap) {
    if (int rc = pde_check(stationary)) return rc;
    const long long S = (long long)pde_slices(stationary) * 3 * N;
    if (int rc = check_finite(v, S, "v")) return rc;
    lddmm_solve_opts op{};
    if (o) op = *o;
    if (op.gn_iters <= 0) op.gn_iters = 10;
    if (op.cg_iters <= 0) op.cg_iters = 20;
    if (op.max_halvings <= 0) op.max_halvings = 10;
    if (op.c1 <= 0) op.c1 = 1e-4;
    if (op.gtol <= 0) op.gtol = 1e-3;
    if (op.eta_max <= 0) op.eta_max = 0.5;
    lddmm_solve_report R{};
    double g0 = 0, ginf0 = 0;
    bool at_v = false;
    for (int k = 0; k < op.gn_iters; ++k) {
      if (!at_v) pde_linearize(v, stationary);
      at_v = true;
      pde_gradient_core(pg);
      R.gradients++;
      if (k == 0) R.E_first = pE;
      const double gn = std::sqrt(pde_dot(pg, pg, stationary));
      const double ginf = maxabs(pg, S);
      if (k == 0) {
        g0 = gn;
        ginf0 = ginf;
      }
      R.g_rel_final = g0 > 0 ? gn / g0 : 0.0;
      if (g0 == 0.0 || gn / g0 <= op.gtol) {
        R.stop_reason = 1;
        break;
      }
      const double eta = std::min(op.eta_max, std::sqrt(gn / g0));
      const int its = pde_pcg(pg, px, eta, op.cg_iters);
      R.cg_total += its;
      R.hessvecs += its;
      const double gp = pde_dot(pg, px, stationary);
      const double E0 = pE, Er0 = pEreg, Ed0 = pEdata;
      double tau = 1.0;
      bool accepted = false;
      int trials = 0;
      for (int h = 0; h <= op.max_halvings; ++h) {
        launch_axpbyz<T>(S, 1.0, v, tau, px, ptrial, st, &prof);
        pde_linearize(ptrial, stationary);
        at_v = false;
        R.shoots++;
        trials++;
        if (pE <= E0 + op.c1 * tau * gp) {
          accepted = true;
          break;
        }
        tau *= 0.5;
      }
      if (log && k < log_cap) {
        lddmm_iter_log& L = log[k];
        L.E = E0;
        L.E_reg = Er0;
        L.E_data = Ed0;
        L.mse_rel = base_sq > 0 ? 100.0 * Ed0 * P.sigma2 / base_sq : 0.0;
        L.g_norm = gn;
        L.g_inf_rel = ginf0 > 0 ? ginf / ginf0 : 0.0;
        L.eta = eta;
        L.tau = accepted ? tau : 0.0;
        L.cg_iters = its;
        L.ls_trials = trials;
      }
      R.iters = k + 1;
      if (!accepted) {
        R.stop_reason = 2;
        break;
      }
      copy(v, ptrial, S);
      at_v = true;  // the accepted trial's linearization is the one at the new v
    }
    if (!at_v) pde_linearize(v, stationary);
    R.E_final = pE;
    R.mse_rel_final = base_sq > 0 ? 100.0 * pEdata * P.sigma2 / base_sq : 0.0;
    if (rep) *rep = R;
    return hip_status("pde_gn_solve");
  }

  // inverse-map displacement of the PDE-LDDMM flow: ping-pong between u1 and
  // pacc so that the last step writes u1
  int pde_displacement(bool stationary, const T* v, T* u1) {
    if (int rc = ensure_pde()) return rc;
    if (int rc = check_finite(v, (long long)pde_slices(stationary) * 3 * N, "v")) return rc;
    T* buf[2] = {P.nt % 2 == 0 ? u1 : pacc, P.nt % 2 == 0 ? pacc : u1};
    launch_fill<T>(3 * N, T(0), buf[0], st, &prof);
    for (int n = 0; n < P.nt; ++n)
      launch_sl_step<T>(g, buf[n & 1], slice(v, n, stationary), slice(v, n + 1, stationary), buf[(n + 1) & 1], dt,
                        st, &prof);
    return hip_status("pde_displacement");
  }

  int jacobian(const T* uin, T* det, double* mn, double* mx) {
    T* out = det ? det : tmpS;
    launch_jacobian_det<T>(g, uin, out, st, &prof);
    if (mn || mx) {
      launch_minmax<T>(out, N, partials, dres, st, &prof);
      fetch(2);
      if (mn) *mn = hres[0];
      if (mx) *mx = hres[1];
    }
    return hip_status("jacobian_det");
  }
};

}  // namespace lddmm

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
struct lddmm_ctx {
  int dtype = LDDMM_F32;
  std::unique_ptr<lddmm::Engine<float>> f;
  std::unique_ptr<lddmm::Engine<double>> d;
  std::string err;
};

#define LDDMM_DISPATCH(ctx, call)                                                  \
  do {                                                                             \
    if (!(ctx)) return LDDMM_EINVAL;                                               \
    (ctx)->err.clear();                                                            \
    if ((ctx)->dtype == LDDMM_F32) {                                               \
      auto& E = *(ctx)->f;                                                         \
      using T = float;                                                             \
      return call;                                                                 \
    } else {                                                                       \
      auto& E = *(ctx)->d;                                                         \
      using T = double;                                                            \
      return call;                                                                 \
    }                                                                              \
  } while (0)

static bool good_size(int n) {
  if (n < 4) return false;
  for (int p : {2, 3, 5, 7})
    while (n % p == 0) n /= p;
  return n == 1;
}

extern "C" {

int lddmm_create(const lddmm_params* params, void* hip_stream, lddmm_ctx** out) {
  if (!params || !out) return LDDMM_EINVAL;
  *out = nullptr;
  const lddmm_params& p = *params;
  if (p.dtype != LDDMM_F32 && p.dtype != LDDMM_F64) return LDDMM_EINVAL;
  if (p.nt < 1 || p.s < 1 || !(p.alpha > 0) || !(p.sigma2 > 0)) return LDDMM_EINVAL;
  for (int d = 0; d < 3; ++d)
    if (!good_size(p.n[d])) return LDDMM_EUNSUPPORTED;
  if (p.n[2] & 1) return LDDMM_EUNSUPPORTED;
  // field kernels index the three components of a vector field with 32-bit offsets
  if (3LL * p.n[0] * p.n[1] * p.n[2] >= (1LL << 31)) return LDDMM_EUNSUPPORTED;
  auto* c = new lddmm_ctx();
  c->dtype = p.dtype;
  int rc;
  if (p.dtype == LDDMM_F32) {
    c->f.reset(new lddmm::Engine<float>());
    rc = c->f->init(p, static_cast<hipStream_t>(hip_stream), &c->err);
  } else {
    c->d.reset(new lddmm::Engine<double>());
    rc = c->d->init(p, static_cast<hipStream_t>(hip_stream), &c->err);
  }
  if (rc) {
    delete c;
    return rc;
  }
  *out = c;
  return LDDMM_OK;
}

int lddmm_destroy(lddmm_ctx* ctx) {
  if (!ctx) return LDDMM_EINVAL;
  if (ctx->f) (void)hipStreamSynchronize(ctx->f->st);
  if (ctx->d) (void)hipStreamSynchronize(ctx->d->st);
  delete ctx;
  return LDDMM_OK;
}

int lddmm_set_images(lddmm_ctx* ctx, const void* I0, const void* I1) {
  if (!I0 || !I1) return LDDMM_EINVAL;
  LDDMM_DISPATCH(ctx, E.set_images(static_cast<const T*>(I0), static_cast<const T*>(I1)));
}

int lddmm_apply_operator(lddmm_ctx* ctx, int op, int ncomp, const void* in, void* out) {
  if (!in || !out || (op != LDDMM_OP_K && op != LDDMM_OP_L) || (ncomp != 1 && ncomp != 3)) return LDDMM_EINVAL;
  LDDMM_DISPATCH(ctx, ((op == LDDMM_OP_K ? E.applyK(static_cast<const T*>(in), static_cast<T*>(out), ncomp)
                                         : E.applyL(static_cast<const T*>(in), static_cast<T*>(out), ncomp)),
                        E.hip_status("apply_operator")));
}

int lddmm_dot(lddmm_ctx* ctx, int ncomp, const void* a, const void* b, double* out) {
  if (!a || !b || !out || (ncomp != 1 && ncomp != 3)) return LDDMM_EINVAL;
  LDDMM_DISPATCH(ctx, (*out = E.dot(static_cast<const T*>(a), static_cast<const T*>(b), ncomp),
                       E.hip_status("dot")));
}

int lddmm_shoot(lddmm_ctx* ctx, const void* v0, void* J1, void* u1, void* v1, double* energy) {
  if (!v0) return LDDMM_EINVAL;
  LDDMM_DISPATCH(ctx, E.shoot(static_cast<const T*>(v0), static_cast<T*>(J1), static_cast<T*>(u1),
                              static_cast<T*>(v1), energy));
}

int lddmm_linearize(lddmm_ctx* ctx, const void* v0, void* J1, double* energy) {
  if (!v0) return LDDMM_EINVAL;
  LDDMM_DISPATCH(ctx, E.linearize(static_cast<const T*>(v0), static_cast<T*>(J1), energy));
}

int lddmm_gradient(lddmm_ctx* ctx, const void* v0, void* g, double* energy) {
  if (!v0 || !g) return LDDMM_EINVAL;
  LDDMM_DISPATCH(ctx, E.gradient(static_cast<const T*>(v0), static_cast<T*>(g), energy));
}

int lddmm_hessvec(lddmm_ctx* ctx, const void* v0, const void* dv, void* hv) {
  if (!dv || !hv) return LDDMM_EINVAL;
  LDDMM_DISPATCH(ctx, E.hessvec(static_cast<const T*>(v0), static_cast<const T*>(dv), static_cast<T*>(hv)));
}

int lddmm_hessvec_newton(lddmm_ctx* ctx, const void* v0, const void* dv, void* hv) {
  if (!dv || !hv) return LDDMM_EINVAL;
  LDDMM_DISPATCH(ctx, E.hessvec_newton(static_cast<const T*>(v0), static_cast<const T*>(dv), static_cast<T*>(hv)));
}

int lddmm_vjp(lddmm_ctx* ctx, const void* gbar_J1, void* gbar_v0) {
  if (!gbar_J1 || !gbar_v0) return LDDMM_EINVAL;
  LDDMM_DISPATCH(ctx, E.vjp(static_cast<const T*>(gbar_J1), static_cast<T*>(gbar_v0)));
}

int lddmm_cg_solve(lddmm_ctx* ctx, const void* g, void* x, double eta, int maxit, int* iters) {
  if (!g || !x) return LDDMM_EINVAL;
  LDDMM_DISPATCH(ctx, E.cg_solve(static_cast<const T*>(g), static_cast<T*>(x), eta, maxit, iters));
}

int lddmm_gn_solve(lddmm_ctx* ctx, void* v0_inout, const lddmm_solve_opts* opts, lddmm_solve_report* report,
                   lddmm_iter_log* log, int log_cap) {
  if (!v0_inout || log_cap < 0) return LDDMM_EINVAL;
  LDDMM_DISPATCH(ctx, E.gn_solve(static_cast<T*>(v0_inout), opts, report, log, log_cap));
}

int lddmm_pde_energy(lddmm_ctx* ctx, int stationary, const void* v, void* m1, double* energy) {
  if (!v) return LDDMM_EINVAL;
  LDDMM_DISPATCH(ctx, E.pde_energy(stationary != 0, static_cast<const T*>(v), static_cast<T*>(m1), energy));
}

int lddmm_pde_gradient(lddmm_ctx* ctx, int stationary, const void* v, void* g, double* energy) {
  if (!v || !g) return LDDMM_EINVAL;
  LDDMM_DISPATCH(ctx, E.pde_gradient(stationary != 0, static_cast<const T*>(v), static_cast<T*>(g), energy));
}

int lddmm_pde_hessvec(lddmm_ctx* ctx, int stationary, const void* v, const void* dv, void* hv) {
  if (!dv || !hv) return LDDMM_EINVAL;
  LDDMM_DISPATCH(ctx, E.pde_hessvec(stationary != 0, static_cast<const T*>(v), static_cast<const T*>(dv),
                                    static_cast<T*>(hv)));
}

int lddmm_pde_gn_solve(lddmm_ctx* ctx, int stationary, void* v_inout, const lddmm_solve_opts* opts,
                       lddmm_solve_report* report, lddmm_iter_log* log, int log_cap) {
  if (!v_inout || log_cap < 0) return LDDMM_EINVAL;
  LDDMM_DISPATCH(ctx, E.pde_gn_solve(stationary != 0, static_cast<T*>(v_inout), opts, report, log, log_cap));
}

int lddmm_pde_displacement(lddmm_ctx* ctx, int stationary, const void* v, void* u1) {
  if (!v || !u1) return LDDMM_EINVAL;
  LDDMM_DISPATCH(ctx, E.pde_displacement(stationary != 0, static_cast<const T*>(v), static_cast<T*>(u1)));
}

int lddmm_jacobian_det(lddmm_ctx* ctx, const void* u, void* det, double* det_min, double* det_max) {
  if (!u) return LDDMM_EINVAL;
  LDDMM_DISPATCH(ctx, E.jacobian(static_cast<const T*>(u), static_cast<T*>(det), det_min, det_max));
}

int lddmm_profile_enable(lddmm_ctx* ctx, int enable) {
  LDDMM_DISPATCH(ctx, ((void)hipStreamSynchronize(E.st), E.prof.clear(), E.prof.enabled = enable != 0, 0));
}

int lddmm_profile_read(lddmm_ctx* ctx, const char** names, int64_t* counts, double* total_ms, int cap) {
  if (cap < 0) return LDDMM_EINVAL;
  LDDMM_DISPATCH(ctx, E.prof.read(names, counts, total_ms, cap));
}

int lddmm_set_option(lddmm_ctx* ctx, const char* key, int64_t value) {
  if (!key) return LDDMM_EINVAL;
  LDDMM_DISPATCH(ctx, E.set_option(key, value));
}

int lddmm_get_option(lddmm_ctx* ctx, const char* key, int64_t* value) {
  if (!key || !value) return LDDMM_EINVAL;
  LDDMM_DISPATCH(ctx, E.get_option(key, value));
}

int lddmm_autotune(lddmm_ctx* ctx, int reps, int* tried, double* ms_per_apply) {
  LDDMM_DISPATCH(ctx, ([&]() {
                   const int rc = E.autotune(reps, tried);
                   if (ms_per_apply) *ms_per_apply = E.autotune_ms;
                   return rc;
                 }()));
}

int lddmm_sync(lddmm_ctx* ctx) {
  LDDMM_DISPATCH(ctx, (hipStreamSynchronize(E.st) == hipSuccess ? LDDMM_OK : LDDMM_EHIP));
}

int lddmm_memory_bytes(lddmm_ctx* ctx, int64_t* bytes) {
  if (!bytes) return LDDMM_EINVAL;
  LDDMM_DISPATCH(ctx, (*bytes = int64_t(E.bytes), 0));
}

const char* lddmm_strerror(int status) {
  switch (status) {
    case LDDMM_OK: return "ok";
    case LDDMM_EINVAL: return "invalid argument";
    case LDDMM_EUNSUPPORTED: return "unsupported grid size";
    case LDDMM_ENOMEM: return "out of device memory";
    case LDDMM_EHIP: return "HIP runtime error";
    case LDDMM_ENONFINITE: return "non-finite input";
    case LDDMM_ESTATE: return "invalid call order";
    case LDDMM_ELINESEARCH: return "line search failed";
    default: return "unknown status";
  }
}

const char* lddmm_last_error(lddmm_ctx* ctx) {
  if (ctx) return ctx->err.c_str();
  const char* m = lddmm::noalloc_last_error();
  return m[0] ? m : "null context";
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------
// Persistent host workers of a batch: run(set, fn) calls fn(i) for every pair i of
// set, pair i on worker i, and returns when all are done.  The lockstep solve
// uses them to enqueue a phase's launches for all pairs in parallel.
class PairWorkers {
 public:
  void start(int n, int device) {
    stop_ = false;
    gen_.assign(n, 0);
    for (int i = 0; i < n; ++i)
      th_.emplace_back([this, i, device]() {
        (void)hipSetDevice(device);
        uint64_t seen = 0;
        while (true) {
          std::function<void(int)> job;
          {
            std::unique_lock<std::mutex> lk(mu_);
            cv_.wait(lk, [&] { return stop_ || gen_[i] != seen; });
            if (stop_) return;
            seen = gen_[i];
            job = job_;
          }
          job(i);
          {
            std::lock_guard<std::mutex> lk(mu_);
            if (--pending_ == 0) done_.notify_all();
          }
        }
      });
  }
  void run(const std::vector<int>& set, const std::function<void(int)>& fn) {
    if (set.empty()) return;
    if (set.size() == 1 || th_.empty()) {
      for (int i : set) fn(i);
      return;
    }
    std::unique_lock<std::mutex> lk(mu_);
    job_ = fn;
    pending_ = int(set.size());
    for (int i : set) ++gen_[i];
    cv_.notify_all();
    done_.wait(lk, [&] { return pending_ == 0; });
  }
  ~PairWorkers() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto& t : th_) t.join();
  }

 private:
  std::mutex mu_;
  std::condition_variable cv_, done_;
  std::vector<std::thread> th_;
  std::vector<uint64_t> gen_;
  std::function<void(int)> job_;
  int pending_ = 0;
  bool stop_ = false;
};

struct lddmm_batch {
  std::vector<lddmm_ctx*> ctx;
  int device = 0;
  PairWorkers workers;
  // Graphs spanning every pair: captured on the batch stream, forked to and
  // joined from the pairs' streams with events.
  hipStream_t bst = nullptr;
  hipEvent_t ev_b = nullptr;
  std::vector<hipEvent_t> ev;
  // one CG iteration of a set of pairs (bit i = pair i; bit 63: PCG in L2), valid
  // for the pairs' graph generations it was captured with
  std::vector<std::pair<uint64_t, hipGraphExec_t>> cg_all;
  std::vector<int> cg_gens;
  // one Gauss-Newton Hv of every pair for the dv / hv pointers it was captured with
  hipGraphExec_t hv_all = nullptr;
  std::vector<const void*> hv_ptrs;
  std::vector<int> hv_gens;
  void drop_graphs() {
    for (auto& e : cg_all) (void)hipGraphExecDestroy(e.second);
    cg_all.clear();
    if (hv_all) (void)hipGraphExecDestroy(hv_all);
    hv_all = nullptr;
    hv_ptrs.clear();
  }
};

namespace {

hipStream_t ctx_stream(lddmm_ctx* c) { return c->dtype == LDDMM_F32 ? c->f->st : c->d->st; }

// Run fn(i) for every pair, on one host thread per pair (concurrent) or in order.
template <class F>
int for_pairs(lddmm_batch* b, int concurrent, F fn) {
  const int n = int(b->ctx.size());
  std::vector<int> rc(n, 0);
  if (concurrent) {
    std::vector<std::thread> th;
    th.reserve(n);
    for (int i = 0; i < n; ++i)
      th.emplace_back([&, i]() {
        (void)hipSetDevice(b->device);
        rc[i] = fn(i);
      });
    for (auto& t : th) t.join();
  } else {
    for (int i = 0; i < n; ++i) rc[i] = fn(i);
  }
  for (int i = 0; i < n; ++i)
    if (rc[i]) return rc[i];
  return LDDMM_OK;
}

template <typename T>
lddmm::Engine<T>* engine_of(lddmm_ctx* c);
template <>
lddmm::Engine<float>* engine_of<float>(lddmm_ctx* c) {
  return c->f.get();
}
template <>
lddmm::Engine<double>* engine_of<double>(lddmm_ctx* c) {
  return c->d.get();
}

// Capture fn(i) for the pairs of `set` into one graph on the batch stream (each
// pair's work on its own stream, forked and joined with events).
template <class F>
hipGraphExec_t capture_across(lddmm_batch* b, const std::vector<int>& set, F fn) {
  if (hipStreamBeginCapture(b->bst, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  (void)hipEventRecord(b->ev_b, b->bst);
  for (int i : set) {
    const hipStream_t s = ctx_stream(b->ctx[i]);
    (void)hipStreamWaitEvent(s, b->ev_b, 0);
    fn(i);
    (void)hipEventRecord(b->ev[i], s);
    (void)hipStreamWaitEvent(b->bst, b->ev[i], 0);
  }
  hipGraph_t g = nullptr;
  if (hipStreamEndCapture(b->bst, &g) != hipSuccess || !g) {
    (void)hipGetLastError();
    return nullptr;
  }
  hipGraphExec_t ex = nullptr;
  if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGetLastError();
    ex = nullptr;
  }
  (void)hipGraphDestroy(g);
  return ex;
}

// Launch a graph spanning the pairs of `set`, ordered after their streams' work
// and before anything enqueued on them afterwards.
void launch_across(lddmm_batch* b, const std::vector<int>& set, hipGraphExec_t ex) {
  for (int i : set) {
    (void)hipEventRecord(b->ev[i], ctx_stream(b->ctx[i]));
    (void)hipStreamWaitEvent(b->bst, b->ev[i], 0);
  }
  (void)hipGraphLaunch(ex, b->bst);
  (void)hipEventRecord(b->ev_b, b->bst);
  for (int i : set) (void)hipStreamWaitEvent(ctx_stream(b->ctx[i]), b->ev_b, 0);
}

template <typename T>
std::vector<int> graph_gens(lddmm_batch* b) {
  std::vector<int> g;
  for (lddmm_ctx* c : b->ctx) g.push_back(engine_of<T>(c)->graph_gen);
  return g;
}

// One CG iteration of the pairs in `live` (a subset of the solve's Krylov set):
// one graph spanning them where every pair can be captured, else each pair's
// own iteration graph (or kernels).
template <typename T>
void batch_cg_step(lddmm_batch* b, const std::vector<int>& live) {
  bool all_graph = live.size() > 1 && b->ctx.size() <= 63;
  for (int i : live) all_graph = all_graph && engine_of<T>(b->ctx[i])->cg_graph_ok();
  if (all_graph) {
    if (graph_gens<T>(b) != b->cg_gens) {
      b->drop_graphs();
      b->cg_gens = graph_gens<T>(b);
    }
    // key: the pairs, and bit 63 for the PCG in L2 (the method of the solve)
    uint64_t mask = engine_of<T>(b->ctx[live[0]])->cg_l2 ? uint64_t(1) << 63 : 0;
    for (int i : live) mask |= uint64_t(1) << i;
    hipGraphExec_t ex = nullptr;
    for (auto& e : b->cg_all)
      if (e.first == mask) ex = e.second;
    if (!ex) {
      ex = capture_across(b, live, [&](int i) {
        auto* E = engine_of<T>(b->ctx[i]);
        E->capturing = true;
        E->cg_iteration(E->cx, true);
        E->capturing = false;
      });
      if (ex) b->cg_all.emplace_back(mask, ex);
    }
    if (ex) {
      launch_across(b, live, ex);
      return;
    }
  }
  for (int i : live) {
    auto* E = engine_of<T>(b->ctx[i]);
    E->cg_step_enqueue(E->cx);
  }
}

// Gauss-Newton solves of every pair in lockstep: each phase (gradient, Krylov
// iteration, <g, p>, line-search trial, final linearization) is enqueued for all
// pairs that need it (by the batch's per-pair workers, or as one graph spanning
// the pairs for a CG iteration) before the host waits once for them.
// Per pair, the same kernels run in the same order with the same decisions as
// lddmm_gn_solve on that pair alone.
template <typename T>
int batch_gn_lockstep(lddmm_batch* b, void* const* v0, const lddmm_solve_opts* opts, lddmm_solve_report* reps) {
  using E_t = lddmm::Engine<T>;
  const int n = int(b->ctx.size());
  std::vector<E_t*> E(n);
  for (int i = 0; i < n; ++i) {
    E[i] = engine_of<T>(b->ctx[i]);
    b->ctx[i]->err.clear();
    if (int rc = E[i]->gn_setup(static_cast<T*>(v0[i]), opts, nullptr, 0)) return rc;
  }
  std::vector<std::unique_ptr<typename E_t::NewtonScope>> scopes;
  for (int i = 0; i < n; ++i)
    scopes.emplace_back(new typename E_t::NewtonScope(E[i]->use_newton, E[i]->gs.method == LDDMM_NEWTON_V));
  auto pick = [&](auto pred) {
    std::vector<int> out;
    for (int i = 0; i < n; ++i)
      if (pred(i)) out.push_back(i);
    return out;
  };
  while (true) {
    const std::vector<int> act = pick([&](int i) { return !E[i]->gs.done; });
    if (act.empty()) break;
    b->workers.run(act, [&](int i) { E[i]->gn_grad_enqueue(); });
    for (int i : act) {
      E[i]->wait();
      E[i]->gn_grad_finish();
    }
    const std::vector<int> kr = pick([&](int i) { return !E[i]->gs.done && E[i]->gs.needs_krylov; });
    b->workers.run(kr, [&](int i) { E[i]->gn_krylov_begin(); });
    std::vector<int> live = kr;
    const int maxit = kr.empty() ? 0 : E[kr[0]]->gs.op.cg_iters;
    for (int it = 1; it <= maxit && !live.empty(); ++it) {
      batch_cg_step<T>(b, live);
      for (int i : live) E[i]->post_fetch();
      std::vector<int> next;
      for (int i : live) {
        E[i]->wait();
        if (E[i]->cg_active()) next.push_back(i);
      }
      live.swap(next);
    }
    for (int i : kr) E[i]->gn_slope_enqueue();
    for (int i : kr) {
      E[i]->wait();
      E[i]->gn_slope_finish();
    }
    const std::vector<int> srch = pick([&](int i) { return !E[i]->gs.done; });
    for (int i : srch) E[i]->gn_search_begin();
    while (true) {
      const std::vector<int> tr = pick([&](int i) { return !E[i]->gs.done && E[i]->gs.searching; });
      if (tr.empty()) break;
      b->workers.run(tr, [&](int i) { E[i]->gn_trial_enqueue(); });
      for (int i : tr) {
        E[i]->wait();
        E[i]->gn_trial_finish();
      }
    }
    for (int i : srch) E[i]->gn_iteration_end();
  }
  b->workers.run(pick([](int) { return true; }), [&](int i) { E[i]->gn_final_enqueue(); });
  int rc = 0;
  for (int i = 0; i < n; ++i) {
    E[i]->wait();
    E[i]->gn_final_finish(reps ? &reps[i] : nullptr);
    if (!rc) rc = E[i]->hip_status("batch_gn_solve");
  }
  return rc;
}

// reps Gauss-Newton Hessian-vector products of every pair at its current
// linearization, each round one graph spanning all pairs where they can be
// captured (store-all trajectories, graph replay on), else pair by pair.
template <typename T>
int batch_hessvec_lockstep(lddmm_batch* b, void* const* dv, void* const* hv, int reps) {
  const int n = int(b->ctx.size());
  std::vector<int> all(n);
  bool graph = n > 1;
  for (int i = 0; i < n; ++i) {
    all[i] = i;
    auto* E = engine_of<T>(b->ctx[i]);
    if (!E->linearized) {
      b->ctx[i]->err = "hessvec without a linearization";
      return LDDMM_ESTATE;
    }
    graph = graph && E->use_graph && E->traj_policy == lddmm::TRAJ_STORE_ALL && !E->prof.enabled;
  }
  if (graph) {
    std::vector<const void*> ptrs;
    for (int i = 0; i < n; ++i) {
      ptrs.push_back(dv[i]);
      ptrs.push_back(hv[i]);
    }
    if (!b->hv_all || ptrs != b->hv_ptrs || graph_gens<T>(b) != b->hv_gens) {
      if (b->hv_all) (void)hipGraphExecDestroy(b->hv_all);
      b->hv_all = capture_across(b, all, [&](int i) {
        auto* E = engine_of<T>(b->ctx[i]);
        E->capturing = true;
        E->hessvec_kernels(static_cast<const T*>(dv[i]), static_cast<T*>(hv[i]));
        E->capturing = false;
      });
      b->hv_ptrs = ptrs;
      b->hv_gens = graph_gens<T>(b);
    }
    graph = b->hv_all != nullptr;
  }
  for (int r = 0; r < reps; ++r) {
    if (graph) {
      launch_across(b, all, b->hv_all);
    } else {
      for (int i = 0; i < n; ++i)
        engine_of<T>(b->ctx[i])->hessvec_core(static_cast<const T*>(dv[i]), static_cast<T*>(hv[i]));
    }
  }
  int rc = 0;
  for (int i = 0; i < n; ++i) {
    if (hipStreamSynchronize(ctx_stream(b->ctx[i])) != hipSuccess && !rc) rc = LDDMM_EHIP;
    if (!rc) rc = engine_of<T>(b->ctx[i])->hip_status("batch_hessvec");
  }
  return rc;
}

bool same_dtype(lddmm_batch* b) {
  for (lddmm_ctx* c : b->ctx)
    if (c->dtype != b->ctx[0]->dtype) return false;
  return true;
}

}  // namespace

extern "C" {

int lddmm_batch_create(const lddmm_params* per_pair, int npairs, lddmm_batch** out) {
  if (!per_pair || npairs < 1 || !out) return LDDMM_EINVAL;
  *out = nullptr;
  auto* b = new lddmm_batch();
  if (hipGetDevice(&b->device) != hipSuccess) {
    delete b;
    return LDDMM_EHIP;
  }
  if (hipStreamCreateWithFlags(&b->bst, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_b, hipEventDisableTiming) != hipSuccess) {
    lddmm_batch_destroy(b);
    return LDDMM_EHIP;
  }
  for (int i = 0; i < npairs; ++i) {
    hipStream_t s = nullptr;
    hipEvent_t e = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      lddmm_batch_destroy(b);
      return LDDMM_EHIP;
    }
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      (void)hipStreamDestroy(s);
      lddmm_batch_destroy(b);
      return LDDMM_EHIP;
    }
    b->ev.push_back(e);
    lddmm_ctx* c = nullptr;
    const int rc = lddmm_create(&per_pair[i], s, &c);
    if (rc) {
      (void)hipStreamDestroy(s);
      lddmm_batch_destroy(b);
      return rc;
    }
    if (c->dtype == LDDMM_F32) {
      c->f->own_stream = true;
      c->f->use_graph = true;
    } else {
      c->d->own_stream = true;
      c->d->use_graph = true;
    }
    b->ctx.push_back(c);
  }
  b->workers.start(npairs, b->device);
  *out = b;
  return LDDMM_OK;
}

int lddmm_batch_destroy(lddmm_batch* b) {
  if (!b) return LDDMM_EINVAL;
  if (b->bst) (void)hipStreamSynchronize(b->bst);
  b->drop_graphs();
  for (lddmm_ctx* c : b->ctx) lddmm_destroy(c);
  for (hipEvent_t e : b->ev) (void)hipEventDestroy(e);
  if (b->ev_b) (void)hipEventDestroy(b->ev_b);
  if (b->bst) (void)hipStreamDestroy(b->bst);
  delete b;
  return LDDMM_OK;
}

int lddmm_batch_get(lddmm_batch* b, int i, lddmm_ctx** out) {
  if (!b || !out || i < 0 || i >= int(b->ctx.size())) return LDDMM_EINVAL;
  *out = b->ctx[i];
  return LDDMM_OK;
}

int lddmm_batch_sync(lddmm_batch* b) {
  if (!b) return LDDMM_EINVAL;
  for (lddmm_ctx* c : b->ctx)
    if (hipStreamSynchronize(ctx_stream(c)) != hipSuccess) return LDDMM_EHIP;
  return LDDMM_OK;
}

int lddmm_batch_gn_solve(lddmm_batch* b, void* const* v0_inout, const lddmm_solve_opts* opts,
                         lddmm_solve_report* reports, int concurrent) {
  if (!b || !v0_inout) return LDDMM_EINVAL;
  for (size_t i = 0; i < b->ctx.size(); ++i)
    if (!v0_inout[i]) return LDDMM_EINVAL;
  if (concurrent == LDDMM_BATCH_LOCKSTEP && same_dtype(b))
    return b->ctx[0]->dtype == LDDMM_F32 ? batch_gn_lockstep<float>(b, v0_inout, opts, reports)
                                         : batch_gn_lockstep<double>(b, v0_inout, opts, reports);
  return for_pairs(b, concurrent, [&](int i) {
    const int rc = lddmm_gn_solve(b->ctx[i], v0_inout[i], opts, reports ? &reports[i] : nullptr, nullptr, 0);
    // the solve's last copy into v0 may still be in flight on the pair's stream
    const bool synced = hipStreamSynchronize(ctx_stream(b->ctx[i])) == hipSuccess;
    return rc ? rc : (synced ? LDDMM_OK : LDDMM_EHIP);
  });
}

int lddmm_batch_hessvec(lddmm_batch* b, void* const* dv, void* const* hv, int reps, int concurrent) {
  if (!b || !dv || !hv || reps < 1) return LDDMM_EINVAL;
  for (size_t i = 0; i < b->ctx.size(); ++i)
    if (!dv[i] || !hv[i]) return LDDMM_EINVAL;
  if (concurrent == LDDMM_BATCH_LOCKSTEP && same_dtype(b))
    return b->ctx[0]->dtype == LDDMM_F32 ? batch_hessvec_lockstep<float>(b, dv, hv, reps)
                                         : batch_hessvec_lockstep<double>(b, dv, hv, reps);
  return for_pairs(b, concurrent, [&](int i) {
    for (int r = 0; r < reps; ++r) {
      const int rc = lddmm_hessvec(b->ctx[i], nullptr, dv[i], hv[i]);
      if (rc) return rc;
    }
    return hipStreamSynchronize(ctx_stream(b->ctx[i])) == hipSuccess ? LDDMM_OK : LDDMM_EHIP;
  });
}

int lddmm_batch_autotune(lddmm_batch* b, int reps) {
  if (!b) return LDDMM_EINVAL;
  return for_pairs(b, 0, [&](int i) { return lddmm_autotune(b->ctx[i], reps, nullptr, nullptr); });
}

}  // extern "C"
