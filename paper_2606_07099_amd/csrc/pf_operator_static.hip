// pf_operator_values_static (declared in sable_pf.h): the operator value
// refresh of pf_operator_values for callers that cannot allocate device
// memory, e.g. code under HIP graph capture.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "pf_operators.h"
#include "sable_pf.h"

// Operator refresh without allocation: the per-bus state (e, f, P, Q) that
// the value kernel reads lives in a fixed device array instead of the
// template's growable buffer.  Each device holds its own copy of the array
// until the process ends; host code reaches it only through the address
// hipGetSymbolAddress returns for the current device, taken once per device
// on the first call there.  Batches whose state does not fit are processed
// in consecutive pieces on the caller's stream.

namespace {

constexpr size_t kStaticStateDoubles = size_t(4) << 20;   // 32 MiB: 2^20 (scenario, bus) pairs
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kStaticStateDoubles];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// the array's address on `dev` (which must be current), or null on failure
void* scratch_on(int dev, hipError_t& err) {
  err = hipSuccess;
  if (dev < 0 || dev >= kMaxDevices) { err = hipErrorInvalidDevice; return nullptr; }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (err != hipSuccess || !ptr) {
      if (err == hipSuccess) err = hipErrorInvalidSymbol;
      return nullptr;
    }
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" int pf_operator_values_static(pf_template* t, int32_t which, int32_t count, const double* vm,
                                         const double* va, double* values, void* hip_stream) {
  sable::OpParams p{};
  int dev = 0;
  int rc = sable::operator_params(t, which, count, vm, va, values, "pf_operator_values_static", p, dev);
  if (rc != PF_OK) return rc;
  const size_t per = 4 * (size_t)p.n_bus;   // doubles of state per scenario
  if (per > kStaticStateDoubles) {
    sable::set_error("pf_operator_values_static: " + std::to_string(p.n_bus) +
                     " buses exceed the fixed state array (at most " + std::to_string(kStaticStateDoubles / 4) +
                     " buses)");
    return PF_EINVAL;
  }
  if (count == 0 || p.nnz == 0) return PF_OK;
  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess) prev = -1;
  if (prev != dev && hipSetDevice(dev) != hipSuccess) {
    sable::set_error("pf_operator_values_static: cannot select the template's device");
    return PF_EHIP;
  }
  hipError_t he = hipSuccess;
  void* ptr = scratch_on(dev, he);
  if (ptr) {
    const int piece = (int)std::min<size_t>((size_t)count, kStaticStateDoubles / per);
    for (int b0 = 0; b0 < count && he == hipSuccess; b0 += piece) {
      sable::OpParams q = p;
      q.count = std::min(piece, count - b0);
      q.vm = p.vm + (size_t)b0 * p.n_bus;
      q.va = p.va + (size_t)b0 * p.n_bus;
      q.values = p.values + (size_t)b0 * p.nnz;
      q.ef = static_cast<double*>(ptr);
      he = sable::launch_operator_values(q, static_cast<hipStream_t>(hip_stream));
    }
  }
  if (prev >= 0 && prev != dev) (void)hipSetDevice(prev);
  if (he != hipSuccess) {
    sable::set_error(std::string("pf_operator_values_static: ") + (ptr ? "launch: " : "fixed state array: ") +
                     hipGetErrorString(he));
    return PF_EHIP;
  }
  return PF_OK;
}
