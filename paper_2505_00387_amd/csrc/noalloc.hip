// The adjoint entry point that allocates nothing (aahrt_adjoint_noalloc).
//
// aahrt_adjoint keeps the trace spectra, the per-trace spreading bounds, the per-slice
// fixed-point scales and the model spectra in the plan's workspace.  This variant runs the
// same kernels with those intermediates in one file-scope device array instead, so that a
// call makes no allocation of any kind: for callers that cannot allocate (code under stream
// capture, serving loops, harnesses that forbid hipMalloc).
//
// The array lives in the library's code object: each GPU the library runs on holds its own
// copy, at its own address, until the process ends.  Host code never uses the array's name
// as a device address (on the host it is only a stand-in): the address is looked up once per
// device with hipGetSymbolAddress, with that device current, and that pointer is what the
// kernels are given.  Every call on one GPU shares the array and leaves its contents behind;
// all of it is overwritten by each call before it is read (the bounds and scales are
// recomputed, the spectra fully rewritten), so nothing needs clearing, and calls that
// overlap in time on one GPU race on it.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "aahrt_internal.hpp"

namespace aahrt {

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

thread_local std::string g_msg;

int set_error(int code, const std::string& m) {
  g_msg = m;
  return code;
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Device address of this GPU's copy of the array (the caller has made the device current).
int scratch_of(int device, unsigned char** out) {
  if (device < 0 || device >= kMaxDevices) return set_error(AAHRT_E_UNSUPPORTED, "device ordinal above 63");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return set_error(AAHRT_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[device] = ptr;
  }
  *out = static_cast<unsigned char*>(g_scratch[device]);
  return AAHRT_OK;
}

}  // namespace

size_t noalloc_scratch_limit() { return kScratchBytes; }

const char* noalloc_last_message() { return g_msg.c_str(); }

// Scratch bytes the adjoint of a plan needs: trace spectra, model spectra, one bound per
// trace and one scale per (gather, azimuth slice), each 256-byte aligned.
size_t noalloc_adjoint_bytes(const Dims& dm) {
  const size_t rows = (size_t)dm.batch * dm.ntheta * dm.nq;
  return align256((size_t)dm.ntr * dm.nf * sizeof(float2)) + align256(rows * dm.nf * sizeof(float2)) +
         align256((size_t)dm.ntr * sizeof(float)) + align256((size_t)dm.batch * dm.ntheta * sizeof(float));
}

// m = L^T d with every intermediate in the static array.  The plan is already current on
// its device; arguments were checked by the caller.
int adjoint_noalloc(Plan& P, const float* d, float* m, hipStream_t s) {
  const Dims& dm = P.dm;
  const size_t need = noalloc_adjoint_bytes(dm);
  if (need > kScratchBytes)
    return set_error(AAHRT_E_UNSUPPORTED, "the adjoint of this plan needs " + std::to_string(need) +
                                              " scratch bytes; the static scratch holds " +
                                              std::to_string(kScratchBytes));
  unsigned char* base = nullptr;
  int rc = scratch_of(P.device, &base);
  if (rc != AAHRT_OK) return rc;
  const size_t rows = (size_t)dm.batch * dm.ntheta * dm.nq;
  float2* dhat = reinterpret_cast<float2*>(base);
  base += align256((size_t)dm.ntr * dm.nf * sizeof(float2));
  float2* mhat = reinterpret_cast<float2*>(base);
  base += align256(rows * dm.nf * sizeof(float2));
  float* tr_bound = reinterpret_cast<float*>(base);
  base += align256((size_t)dm.ntr * sizeof(float));
  float* slice_scale = reinterpret_cast<float*>(base);
  hipError_t e = launch_data_r2c(P, d, dhat, tr_bound, s);
  if (e == hipSuccess) e = launch_nufft_spread(P, dhat, tr_bound, slice_scale, mhat, s);
  if (e == hipSuccess) e = launch_model_c2r(P, mhat, m, s);
  if (e != hipSuccess) return set_error(AAHRT_E_HIP, std::string("adjoint kernels: ") + hipGetErrorString(e));
  return AAHRT_OK;
}

}  // namespace aahrt
