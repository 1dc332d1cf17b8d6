// Allocation-free lowest eigenvalue of H_eff: the Lanczos basis lives in a fixed device array
// of this library instead of memory allocated per call.
//
// `scratch` is one file-scope device array per GPU (each device that loads the library holds
// its own copy until the process ends).  Host code never uses its name as an address: the
// device address is looked up once per device with hipGetSymbolAddress, while that device is
// current, when a context is created on it, and kept in `g_scratch`.  Every call on one GPU
// shares that GPU's array, which keeps the last call's contents; the library runs one call
// at a time (a lock held for the whole call, which returns only after its device work has
// finished), since overlapping calls on one GPU would race on the array.
#include <mutex>

#include "state.h"

namespace lcc {

constexpr size_t kScratchBytes = (size_t)64 << 20;  // 64 MiB per device
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

namespace {
constexpr int kMaxDevices = 64;
constexpr int kMaxSteps = 128;
std::mutex g_scratch_mu;                 // held for the whole of a call: one call at a time
double* g_scratch[kMaxDevices] = {};
double g_host_ws[2 * kMaxSteps * kMaxSteps + 3 * kMaxSteps];  // Lanczos bookkeeping
}  // namespace

// Once per device, with that device current (called from lcc_context_create).
void scratch_register_current_device() {
  int dev = -1;
  check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) throw Error{LCC_ERR_NODEV, "device index beyond the scratch table"};
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[dev]) return;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    throw Error{LCC_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
  }
  g_scratch[dev] = static_cast<double*>(ptr);
}

void lowest_eigenvalue_noalloc(Env& env, int steps, uint64_t seed, double* theta, double* residual) {
  const int dev = env.ctx->device;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  double* ws = (dev >= 0 && dev < kMaxDevices) ? g_scratch[dev] : nullptr;
  if (!ws) throw Error{LCC_ERR_STATE, "the scratch array of this device was not registered"};
  if (steps < 1 || steps > kMaxSteps) throw Error{LCC_ERR_ARG, "steps must be in [1, 128]"};
  const int64_t need = lanczos_workspace_elems(env, steps);
  if ((size_t)need * sizeof(double) > kScratchBytes)
    throw Error{LCC_ERR_ARG, "Lanczos workspace of " + std::to_string((size_t)need * sizeof(double)) +
                                 " bytes ((steps + 2) x vector length x 8) exceeds the " +
                                 std::to_string(kScratchBytes) + "-byte scratch array"};
  // every Krylov vector is written before it is read (start vector filled, later vectors
  // written with a zero coefficient on their old contents, w by the product), so nothing
  // left in the array by an earlier call enters the result
  (void)lowest_eigenpair_in(env, steps, 1, 0.0, seed, nullptr, theta, residual, ws, g_host_ws, true);
}

}  // namespace lcc
