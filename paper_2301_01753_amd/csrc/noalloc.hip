// gym_solve_noalloc: the FP64 solve of gym_solve without any device
// allocation, for callers that cannot allocate (code under HIP graph capture
// set-up, tight serving loops, harnesses that forbid hipMalloc).
//
// Its Krylov workspace lives in `scratch`, a file-scope device array of
// kNoallocBytes that every GPU the library runs on holds until the process
// ends.  In host code the array's name is only a host-side stand-in: its
// device address on each GPU is asked once, at gym_create with that device
// current, and only that address is ever handed to kernels.  All calls on one
// GPU share the array (and a host array of Krylov states), so calls that
// overlap on one GPU race; the caller serialises them.
#include <hip/hip_runtime.h>

#include "gym_internal.hpp"

namespace gym {

constexpr size_t kNoallocBytes = size_t(128) << 20;  // 128 MiB per GPU
constexpr int kNoallocMaxRhs = 64;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

namespace {
void* g_scratch[kMaxDevices] = {};
MinresState g_states[kMaxDevices][2 * kNoallocMaxRhs];
}  // namespace

int solve_f64_on(gym_op* op, const gym_solve_opts* opts, int nrhs, const double* b, double* x, gym_solve_info* info,
                 hipStream_t s, void* base, size_t bytes, MinresState* host_states, int max_rhs);

// Called by gym_create with `device` current.
int noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(GYM_E_ARG, "device index beyond the scratch table");
  if (g_scratch[device]) return 0;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
  g_scratch[device] = p;
  return 0;
}

}  // namespace gym

extern "C" int gym_solve_noalloc(gym_op* op, const gym_solve_opts* opts, int nrhs, const double* b, double* x,
                                 gym_solve_info* info, void* stream) {
  if (!op) return gym::fail(GYM_E_ARG, "bad argument");
  const int dev = op->ctx->device;
  if (dev < 0 || dev >= gym::kMaxDevices) return gym::fail(GYM_E_ARG, "device index beyond the scratch table");
  return gym::solve_f64_on(op, opts, nrhs, b, x, info, (hipStream_t)stream, gym::g_scratch[dev],
                           gym::kNoallocBytes, gym::g_states[dev], gym::kNoallocMaxRhs);
}
