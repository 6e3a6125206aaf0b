// Exact pairwise sums at chosen targets: the direct summation of Eq. (1)
// with the kernels of Eq. (2) that the FMM approximates, for checking an FMM
// result against it at a sample of particles.
//
//   phi_k = sum_{j: r > 0} q_j / r^p,   F_k = q_i sum_{j: r > 0} q_j p (x_i - x_j) / r^(p+2)
//
// with i = targets[k], r = |x_i - x_j| and p = 1 (1/r) or 2 (1/r^2).
//
// Layout of the work: the sources are cut into S equal chunks; workgroup
// (g, c) takes targets 64 g .. 64 g + 63 (one per lane) against chunk c,
// its four wavefronts each a quarter of every 256-source block staged in
// LDS, and writes the chunk's four partial sums per target to a scratch
// buffer [S][nt64][4].  A second kernel adds the S partials of each target
// in chunk order.  The split depends only on (n, nt), so the summation order
// and the bits are the same on every call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "device_util.h"
#include "fmm_internal.h"

namespace fmm {
namespace {

constexpr int kDirTargets = 64;    // targets per workgroup, one per lane
constexpr int kDirThreads = 256;   // four wavefronts share a chunk
constexpr int kDirStage = 256;     // sources staged in LDS per step
constexpr int64_t kDirMinChunk = 16384;  // sources per chunk at least
constexpr int kDirMaxChunks = 256;

__host__ __device__ inline int64_t pad64(int64_t nt) {
  return (nt + kDirTargets - 1) / kDirTargets * kDirTargets;
}

__global__ __launch_bounds__(kDirThreads) void direct_partial_kernel(
    const double* __restrict__ pos, const double* __restrict__ q, int64_t n,
    const int64_t* __restrict__ targets, int64_t nt, int p, int chunks,
    double* __restrict__ part) {
  __shared__ double sx[kDirStage], sy[kDirStage], sz[kDirStage], sq[kDirStage];
  __shared__ double red[4][kDirTargets][4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t k = int64_t(blockIdx.x) * kDirTargets + lane;
  const int c = blockIdx.y;
  int64_t i = k < nt ? targets[k] : 0;
  const bool valid = k < nt && i >= 0 && i < n;
  if (!valid) i = 0;
  const double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
  const int64_t j0 = n * c / chunks, j1 = n * (c + 1) / chunks;
  double ph = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
  for (int64_t b = j0; b < j1; b += kDirStage) {
    const int cnt = j1 - b < kDirStage ? int(j1 - b) : kDirStage;
    __syncthreads();
    for (int e = threadIdx.x; e < cnt; e += kDirThreads) {
      const int64_t j = b + e;
      sx[e] = pos[3 * j];
      sy[e] = pos[3 * j + 1];
      sz[e] = pos[3 * j + 2];
      sq[e] = q[j];
    }
    __syncthreads();
    for (int e = w; e < cnt; e += 4) {
      const double dx = xi - sx[e], dy = yi - sy[e], dz = zi - sz[e];
      const double r2 = (dx * dx + dy * dy) + dz * dz;
      if (r2 > 0.0) {
        const double ir2 = 1.0 / r2;
        double pot, g;
        if (p == 2) {
          pot = sq[e] * ir2;
          g = 2.0 * pot * ir2;
        } else {
          const double ir = 1.0 / sqrt(r2);
          pot = sq[e] * ir;
          g = pot * ir2;
        }
        ph += pot;
        fx += g * dx;
        fy += g * dy;
        fz += g * dz;
      }
    }
  }
  // the four wavefronts' sums, added in wavefront order
  red[w][lane][0] = ph;
  red[w][lane][1] = fx;
  red[w][lane][2] = fy;
  red[w][lane][3] = fz;
  __syncthreads();
  if (w == 0) {
    double acc[4];
    for (int v = 0; v < 4; ++v) acc[v] = red[0][lane][v];
    for (int u = 1; u < 4; ++u)
      for (int v = 0; v < 4; ++v) acc[v] += red[u][lane][v];
    double* out = part + ((int64_t(c) * pad64(nt)) + k) * 4;
    for (int v = 0; v < 4; ++v) out[v] = valid ? acc[v] : NAN;
  }
}

__global__ __launch_bounds__(256) void direct_sum_kernel(
    const double* __restrict__ q, int64_t n, const int64_t* __restrict__ targets, int64_t nt,
    int chunks, const double* __restrict__ part, double* __restrict__ phi,
    double* __restrict__ f) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= nt) return;
  const int64_t stride = pad64(nt) * 4;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int c = 0; c < chunks; ++c)
    for (int v = 0; v < 4; ++v) acc[v] += part[c * stride + 4 * k + v];
  const int64_t i = targets[k];
  const double qi = (i >= 0 && i < n) ? q[i] : NAN;
  phi[k] = acc[0];
  f[3 * k] = qi * acc[1];
  f[3 * k + 1] = qi * acc[2];
  f[3 * k + 2] = qi * acc[3];
}

int fail(int code, const std::string& msg) {
  set_error(msg);
  return code;
}

template <typename F>
int guarded(F&& fn) {
  try {
    return fn();
  } catch (const FmmError& e) {
    return fail(e.code, e.msg);
  } catch (const std::exception& e) {
    return fail(FMM_ERR_HIP, e.what());
  }
}

}  // namespace

// Source chunks for n sources and nt targets: about n / 16384, at most 256,
// and few enough that the partial sums stay within kDirectPartialMax values.
int direct_chunks(int64_t n, int64_t nt) {
  int64_t s = (n + kDirMinChunk - 1) / kDirMinChunk;
  s = std::min<int64_t>(s, kDirMaxChunks);
  s = std::min<int64_t>(s, kDirectPartialMax / (4 * pad64(nt)));
  return int(std::max<int64_t>(s, 1));
}

size_t direct_partial_doubles(int64_t nt, int chunks) { return size_t(4) * chunks * pad64(nt); }

void launch_direct(const double* pos, const double* q, int64_t n, const int64_t* targets,
                   int64_t nt, int p, double* phi, double* f, double* part, int chunks,
                   hipStream_t s) {
  const dim3 grid(unsigned(pad64(nt) / kDirTargets), unsigned(chunks));
  direct_partial_kernel<<<grid, kDirThreads, 0, s>>>(pos, q, n, targets, nt, p, chunks, part);
  FMM_HIP_CHECK(hipGetLastError());
  direct_sum_kernel<<<unsigned((nt + 255) / 256), 256, 0, s>>>(q, n, targets, nt, chunks, part,
                                                              phi, f);
  FMM_HIP_CHECK(hipGetLastError());
}

int direct_check_args(const double* pos, const double* q, int64_t n, const int64_t* targets,
                      int64_t nt, int kernel, const double* phi, const double* f) {
  if (!pos || !q || !targets || !phi || !f) return fail(FMM_ERR_ARG, "NULL pointer argument");
  if (n < 1 || n > int64_t(2147483646)) return fail(FMM_ERR_ARG, "n outside 1 .. 2^31-2");
  if (nt < 1 || nt > int64_t(1) << 30) return fail(FMM_ERR_ARG, "nt outside 1 .. 2^30");
  if (kernel != FMM_KERNEL_INV_R && kernel != FMM_KERNEL_INV_R2)
    return fail(FMM_ERR_ARG, "unknown kernel " + std::to_string(kernel));
  return FMM_OK;
}

}  // namespace fmm

extern "C" int fmm_direct_sampled(const double* positions, const double* charges, int64_t n,
                                  const int64_t* targets, int64_t nt, int kernel,
                                  double* potential, double* forces, hipStream_t stream) {
  using namespace fmm;
  const int rc = direct_check_args(positions, charges, n, targets, nt, kernel, potential, forces);
  if (rc != FMM_OK) return rc;
  return guarded([&]() -> int {
    const int chunks = direct_chunks(n, nt);
    const size_t bytes = sizeof(double) * direct_partial_doubles(nt, chunks);
    double* part = static_cast<double*>(dev_alloc(bytes));
    try {
      launch_direct(positions, charges, n, targets, nt, kernel, potential, forces, part, chunks,
                    stream);
      FMM_HIP_CHECK(hipStreamSynchronize(stream));
    } catch (...) {
      (void)hipStreamSynchronize(stream);
      dev_free(part);
      throw;
    }
    dev_free(part);
    return FMM_OK;
  });
}
