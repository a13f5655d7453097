// deflate_project for callers that cannot allocate device memory (code under
// HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
// the same kernels as deflate_project, with their scratch in a file-scope
// device array instead of a caller workspace.
#include "krylov_ws.h"

#include <mutex>

namespace sk {
namespace {

// Scratch of the projection kernels: partial sums, counters, F L^H v and
// the state struct.  7 MiB holds deflate_project_workspace_bytes(m, n) for
// every m <= 128 and n <= 12 * 16^4 (a 16^4 lattice); each GPU the library
// runs on keeps its own copy until the process ends.
constexpr size_t kNoAllocBytes = size_t(7) << 20;
constexpr int64_t kNoAllocMaxN = int64_t(12) * 16 * 16 * 16 * 16;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kNoAllocBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's scratch array, looked up once per device
// with that device current (the array's name is only a host-side handle).
int scratch_of_current_device(void** out) {
  int dev = -1;
  SK_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device %d outside the %d the workspace-free entry points support", dev, kMaxDevices);
    return SK_ERR_ARG;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    SK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) {
      set_error("hipGetSymbolAddress returned a null scratch address");
      return SK_ERR_HIP;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SK_OK;
}

}  // namespace
}  // namespace sk

using namespace sk;

extern "C" {

int deflate_project_noalloc(int m, int64_t n, const double* R, const double* L, const double* F,
                            const double* in, double* r_out, double* xp_out, double* coeff,
                            hipStream_t stream) {
  SK_TRY(deflate_project_check(m, n, R, L, F, in, r_out, xp_out, coeff));
  SK_CHECK(n <= kNoAllocMaxN, "n = %lld exceeds the workspace-free limit %lld (a 16^4 lattice)",
           (long long)n, (long long)kNoAllocMaxN);
  const size_t need = deflate_project_workspace_bytes(m, n);
  SK_CHECK(need <= kNoAllocBytes, "m = %d, n = %lld need %zu scratch bytes, more than the %zu held",
           m, (long long)n, need, kNoAllocBytes);
  void* ptr = nullptr;
  SK_TRY(scratch_of_current_device(&ptr));
  return deflate_project_run(m, n, R, L, F, in, r_out, xp_out, coeff, ptr, stream);
}

}  // extern "C"
