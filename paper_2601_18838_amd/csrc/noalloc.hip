// Allocation-free energy reduction: the scratch of the FP64 energy sums lives
// in a file-scope device array instead of the plan's workspace, so the entry
// point that uses it never allocates (for callers that cannot: code under
// stream capture, tight serving loops, harnesses that forbid allocation).
#include <mutex>

#include "kernels.hpp"
#include "noalloc.hpp"

namespace kpme {

namespace {

// The per-block (sum q pot, sum q, sum q^2) partials of the energy reduction:
// kSumBlocks triples.  Each GPU the library runs on holds its own copy until
// the process ends; every call on a GPU shares that GPU's copy.
static __device__ __align__(256) double scratch[kNoallocScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};   // device address of `scratch`, per device

}  // namespace

hipError_t noalloc_scratch(int device, double** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[device]) {
    // the array's name is a host-side stand-in: its device address comes from
    // the runtime, once per device, with that device current
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return e;
    g_ptr[device] = static_cast<double*>(p);
  }
  *out = g_ptr[device];
  return hipSuccess;
}

hipError_t launch_energy_noalloc(int device, int prec, int64_t n, const void* q,
                                 const void* pot, double beta, double volume,
                                 double* energy4, hipStream_t st) {
  double* s = nullptr;
  const hipError_t e = noalloc_scratch(device, &s);
  if (e != hipSuccess) return e;
  // the reduction writes every partial it reads: nothing to clear
  return launch_energy(prec, n, q, pot, beta, volume, s, energy4, st);
}

}  // namespace kpme
