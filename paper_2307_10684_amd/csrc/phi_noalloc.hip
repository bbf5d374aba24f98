// adr_precompute_phi_noalloc: the matrix functions of adr_precompute_phi for
// callers that cannot allocate device memory.  The work area is a fixed array
// in each GPU's memory (held until the process ends) instead of a block the
// library allocates on the first call and grows for larger n.
#include "adr.h"

#include <cmath>
#include <mutex>

#include "common.h"
#include "host_common.h"

namespace {

constexpr size_t kScratchDoubles = adr::host::phi_scratch_doubles(ADR_PHI_NOALLOC_MAX_N);

// The work area.  In host code this name is a stand-in, not a device address:
// kernels receive the address that hipGetSymbolAddress returns for the
// current device (g_scratch below), never the name itself.
static __device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_mu;
constexpr int kMaxDevices = 64;
double* g_scratch[kMaxDevices] = {};   // the array's address on each device

}  // namespace

extern "C" int adr_precompute_phi_noalloc(int n, const double* A_dev, double tau, double* E_dev,
                                          double* P1_dev, double* P2_dev, void* stream) {
  if (n < 1 || !A_dev || !std::isfinite(tau) || tau == 0.0) return ADR_EINVAL;
  if (!E_dev && !P1_dev && !P2_dev) return ADR_EINVAL;
  if (n > ADR_PHI_NOALLOC_MAX_N) return ADR_ENOMEM;   // beyond the fixed work area
  // one call at a time: each waits for its own work before returning, so no two
  // calls use the array at once (nothing in it has to start at zero)
  std::lock_guard<std::mutex> lock(g_mu);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return ADR_EDEVICE;
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return ADR_EDEVICE;
    g_scratch[dev] = static_cast<double*>(ptr);
  }
  double* outs[3] = {E_dev, P1_dev, P2_dev};
  return adr::host::precompute_phi_in(n, A_dev, tau, outs, g_scratch[dev],
                                      static_cast<hipStream_t>(stream));
}
