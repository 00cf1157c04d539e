// noalloc.hip - the K / L application for callers that cannot allocate device
// memory (code under HIP graph capture, serving loops, harnesses that forbid
// hipMalloc).
//
// The transform needs a spectrum workspace between its passes and small tables
// of twiddles and squared wavenumbers.  Here both live in one file-scope device
// array: the tables at its head, the spectrum after them.  Each device holds
// its own copy of the array (at its own address) from the first use until the
// process ends; host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device, never through the
// array's name.
#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "lddmm.h"
#include "lddmm_internal.h"

static __device__ __align__(256) unsigned char scratch[LDDMM_NOALLOC_WORKSPACE_BYTES];

namespace lddmm {
namespace {

// Per-device state: the device address of `scratch` and the plan whose tables
// sit at its head (the last grid and dtype used on that device).
struct NoallocDevice {
  std::mutex mu;
  unsigned char* ws = nullptr;
  int n[3] = {0, 0, 0};
  int dtype = -1;
  SpectralPlan<float> pf;
  SpectralPlan<double> pd;
  std::vector<unsigned char> host_tables;
};

std::mutex g_devices_mu;
std::map<int, std::unique_ptr<NoallocDevice>> g_devices;
thread_local std::string t_error;

int fail(int code, const std::string& msg) {
  t_error = msg;
  return code;
}

bool good_length(int n) {
  if (n < 4) return false;
  for (int p : {2, 3, 5, 7})
    while (n % p == 0) n /= p;
  return n == 1;
}

NoallocDevice* device_state(int dev) {
  std::lock_guard<std::mutex> lk(g_devices_mu);
  auto& slot = g_devices[dev];
  if (!slot) slot.reset(new NoallocDevice());
  return slot.get();
}

template <typename T>
SpectralPlan<T>& plan_of(NoallocDevice& d);
template <>
SpectralPlan<float>& plan_of<float>(NoallocDevice& d) {
  return d.pf;
}
template <>
SpectralPlan<double>& plan_of<double>(NoallocDevice& d) {
  return d.pd;
}

template <typename T>
int apply(NoallocDevice& d, const int32_t n[3], int dtype, double alpha, int s, int op, int ncomp, const T* in,
          T* out, hipStream_t st) {
  SpectralPlan<T>& sp = plan_of<T>(d);
  const bool same = d.dtype == dtype && d.n[0] == n[0] && d.n[1] == n[1] && d.n[2] == n[2];
  if (!same) {
    // new grid or dtype: its tables replace the previous ones at the head of
    // the workspace (a copy and two synchronisations of st, so not while st is
    // being captured)
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess)
      return fail(LDDMM_EHIP, "apply_operator_noalloc: cannot query the stream's capture status");
    if (cs != hipStreamCaptureStatusNone)
      return fail(LDDMM_ESTATE,
                  "apply_operator_noalloc: the first call for a grid and dtype uploads the transform tables; make it "
                  "before capturing the stream");
    int dev = 0, lds = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      return fail(LDDMM_EHIP, "apply_operator_noalloc: cannot query the device");
    d.dtype = -1;  // the head of the workspace is rewritten below
    spectral_free(d.pf);
    spectral_free(d.pd);
    const int nn[3] = {n[0], n[1], n[2]};
    std::string msg;
    const int rc = spectral_init_in(sp, nn, ncomp, size_t(lds), d.ws, size_t(LDDMM_NOALLOC_WORKSPACE_BYTES), st,
                                    d.host_tables, msg);
    if (rc) return fail(rc, "apply_operator_noalloc: " + msg);
    d.dtype = dtype;
    d.n[0] = n[0];
    d.n[1] = n[1];
    d.n[2] = n[2];
  }
  // the plan was built for some component count; this call's spectrum must fit too
  const size_t head = size_t(reinterpret_cast<unsigned char*>(sp.spec) - d.ws);
  const size_t need = head + spectrum_bytes(sp, ncomp);
  if (need > size_t(LDDMM_NOALLOC_WORKSPACE_BYTES))
    return fail(LDDMM_EUNSUPPORTED, "apply_operator_noalloc: " + std::to_string(ncomp) + " component(s) of grid " +
                                        std::to_string(n[0]) + "x" + std::to_string(n[1]) + "x" +
                                        std::to_string(n[2]) + " need " + std::to_string(need) +
                                        " bytes of static workspace; it holds " +
                                        std::to_string(size_t(LDDMM_NOALLOC_WORKSPACE_BYTES)));
  spectral_apply(sp, in, out, ncomp, alpha, s, op, st, nullptr);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(LDDMM_EHIP, std::string("apply_operator_noalloc: ") + hipGetErrorString(e));
  return LDDMM_OK;
}

}  // namespace

const char* noalloc_last_error() { return t_error.c_str(); }

}  // namespace lddmm

extern "C" int lddmm_apply_operator_noalloc(const int32_t n[3], int dtype, double alpha, int s, int op, int ncomp,
                                            const void* in, void* out, void* hip_stream) {
  using namespace lddmm;
  t_error.clear();
  if (!n || !in || !out || (op != LDDMM_OP_K && op != LDDMM_OP_L) || (ncomp != 1 && ncomp != 3) ||
      (dtype != LDDMM_F32 && dtype != LDDMM_F64) || !(alpha > 0) || s < 1)
    return fail(LDDMM_EINVAL, "apply_operator_noalloc: invalid argument");
  for (int k = 0; k < 3; ++k)
    if (!good_length(n[k])) return fail(LDDMM_EUNSUPPORTED, "apply_operator_noalloc: grid sizes must be products of 2, 3, 5, 7 and at least 4");
  if (n[2] & 1) return fail(LDDMM_EUNSUPPORTED, "apply_operator_noalloc: N2 must be even");
  if (3LL * n[0] * n[1] * n[2] >= (1LL << 31)) return fail(LDDMM_EUNSUPPORTED, "apply_operator_noalloc: grid too large");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(LDDMM_EHIP, "apply_operator_noalloc: no current device");
  NoallocDevice* d = device_state(dev);
  std::lock_guard<std::mutex> lk(d->mu);
  if (!d->ws) {
    // once per device, with that device current: this device's copy of the array
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(LDDMM_EHIP, std::string("apply_operator_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
    d->ws = static_cast<unsigned char*>(p);
  }
  const hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (dtype == LDDMM_F32)
    return apply<float>(*d, n, dtype, alpha, s, op, ncomp, static_cast<const float*>(in), static_cast<float*>(out), st);
  return apply<double>(*d, n, dtype, alpha, s, op, ncomp, static_cast<const double*>(in), static_cast<double*>(out),
                       st);
}
