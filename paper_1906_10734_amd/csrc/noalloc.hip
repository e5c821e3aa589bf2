// The solve entry point that allocates nothing: every device buffer of the solve is carved from a
// fixed device array of this library instead of hipMalloc, for callers that cannot allocate.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "hpm_internal.h"

namespace hpm {

constexpr size_t kNoAllocBytes = size_t(64) << 20;  // 64 MiB per device, held until exit
constexpr int kNoAllocDevices = 64;

// The scratch region. In host code this name is only a stand-in for the device symbol: its
// device address comes from hipGetSymbolAddress, once per device (each device holds its own
// copy), and only that address is ever handed to kernels or copies.
static __device__ __align__(256) char scratch[kNoAllocBytes];

static std::mutex g_noalloc_mx;               // one no-allocation solve at a time per process
static char* g_scratch[kNoAllocDevices] = {};  // device address of scratch, per device

// caller holds g_noalloc_mx; "dev" is the current device
static char* scratch_on(int dev) {
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      fail(HPM_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[dev] = static_cast<char*>(ptr);
  }
  return g_scratch[dev];
}

}  // namespace hpm

using namespace hpm;

extern "C" hpm_status hpm_solve_noalloc(const hpm_problem* problem, int64_t n, const void* x,
                                        const void* y, const void* z, const void* m, void* phi,
                                        void* ax, void* ay, void* az, void* stream) {
  return guarded([&] {
    check_problem(problem);
    check_size(problem, n);
    if (!x || !y || !z || !m || !phi || !ax || !ay || !az)
      fail(HPM_ERR_INVALID_ARG, "array pointer is NULL");
    const size_t need = plan_bytes_estimate(*problem, n);
    if (need > kNoAllocBytes)
      fail(HPM_ERR_NO_MEMORY, "this problem needs about " + std::to_string(need >> 20) +
                                  " MiB; the no-allocation scratch region holds " +
                                  std::to_string(kNoAllocBytes >> 20) + " MiB");
    int dev = 0;
    HPM_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoAllocDevices) fail(HPM_ERR_DEVICE, "device index out of range");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lk(g_noalloc_mx);
    Arena arena{scratch_on(dev), kNoAllocBytes, 0};
    ArenaScope scope(&arena);
    Plan p;
    p.noalloc = true;
    create_plan(p, problem, n, x, y, z, s);
    execute_plan(p, m, phi, ax, ay, az, s);
    HPM_HIP(hipStreamSynchronize(s));
  });
}
