// Exact sums at sampled targets without any allocation: the variant of
// fmm_direct_sampled for callers that cannot allocate device memory (code
// under stream capture, tight serving loops).  The partial sums of the
// source chunks live in a file-scope device array instead of a buffer from
// the allocator; the kernels, the chunking and so the results are those of
// fmm_direct_sampled.
#include <hip/hip_runtime.h>

#include <array>
#include <mutex>
#include <string>

#include "fmm_internal.h"

namespace fmm {
namespace {

// kDirectPartialMax doubles (8 MiB), held by each device the library runs on
// until the process ends.
static __device__ __align__(256) double scratch[kDirectPartialMax];

// Device address of `scratch` on each device.  In host code the array's name
// is only a stand-in: the address comes from hipGetSymbolAddress, taken once
// per device with that device current (every device has its own copy).
std::mutex g_scratch_mu;
std::array<double*, 64> g_scratch{};

double* scratch_ptr() {
  int dev = 0;
  FMM_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) throw FmmError{FMM_ERR_HIP, "device index out of range"};
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    FMM_HIP_CHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_scratch[dev] = static_cast<double*>(ptr);
  }
  return g_scratch[dev];
}

}  // namespace
}  // namespace fmm

extern "C" int fmm_direct_sampled_noalloc(const double* positions, const double* charges,
                                          int64_t n, const int64_t* targets, int64_t nt,
                                          int kernel, double* potential, double* forces,
                                          hipStream_t stream) {
  using namespace fmm;
  const int rc = direct_check_args(positions, charges, n, targets, nt, kernel, potential, forces);
  if (rc != FMM_OK) return rc;
  const int chunks = direct_chunks(n, nt);
  if (direct_partial_doubles(nt, chunks) > size_t(kDirectPartialMax)) {
    set_error("nt above " + std::to_string(kDirectPartialMax / 4) +
              ": the partial sums would not fit the static scratch");
    set_error_code(FMM_ERR_ARG);
    return FMM_ERR_ARG;
  }
  try {
    launch_direct(positions, charges, n, targets, nt, kernel, potential, forces, scratch_ptr(),
                  chunks, stream);
  } catch (const FmmError& e) {
    set_error(e.msg);
    set_error_code(e.code);
    return e.code;
  }
  return FMM_OK;
}
