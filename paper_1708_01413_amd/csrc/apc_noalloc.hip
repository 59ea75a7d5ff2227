// Allocation-free adjoint: apc_backward_noalloc runs apc_backward with its
// checkpoint scratch in a fixed device array of this library instead of a
// caller-provided workspace, for callers that cannot allocate device memory
// (code under stream capture, tight serving loops, harnesses that forbid it).
//
// The array below is a file-scope device variable: every GPU the library
// runs on holds its own copy until the process ends.  In host code its name
// stands for a host-side shadow, not a device address, so host code never
// passes it to a kernel or a copy: the device address of each GPU's copy is
// looked up once per device (with that device current) when a plan is set up
// on it, and only that address is used afterwards.

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "apc.h"
#include "apc_internal.h"

namespace {

constexpr size_t kNoAllocBytes = size_t(64) << 20;  // 64 MiB per GPU
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};  // device address of each GPU's copy

}  // namespace

namespace apc {

size_t noalloc_scratch_bytes() { return kNoAllocBytes; }

// Called by apc_setup with the plan's device current.
hipError_t noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  g_scratch[device] = ptr;
  return hipSuccess;
}

void* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  return g_scratch[device];
}

}  // namespace apc

extern "C" apc_status apc_backward_noalloc(apc_plan p, const double* dXbar, int64_t ldd, int32_t T,
                                           int32_t ckpt_every, double* dB, int64_t lddb,
                                           double* dgamma, double* deta) {
  if (!p) return apc::report(APC_EINVAL, "plan is NULL");
  const size_t need = apc_backward_workspace_bytes(p, T, ckpt_every);
  if (need > kNoAllocBytes)
    return apc::report(APC_EINVAL,
                       "this adjoint needs %zu bytes of scratch; the allocation-free variant holds "
                       "%zu (use apc_backward with a workspace)",
                       need, kNoAllocBytes);
  void* ws = apc::noalloc_scratch(apc::plan_device(p));
  if (!ws) return apc::report(APC_EHIP, "the static scratch of device %d is not initialised",
                              apc::plan_device(p));
  // apc_backward validates every other argument, clears what must start at
  // zero with fill kernels, and writes everything else before reading it.
  return apc_backward(p, dXbar, ldd, T, ckpt_every, dB, lddb, dgamma, deta, ws, kNoAllocBytes);
}
