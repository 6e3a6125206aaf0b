// Operator tables and the M2L kernel.
//
// M2L (Sec. 2.1.2, Eq. 3): for a target cell C and a far source cell B at
// level l, with centres differing by w_l t (t in [-3,3]^3, |t|_inf >= 2), the
// local expansion gains K_{l,t} W_B where
//     K_{l,t}[m][n] = 1 / |x_m - y_n| = 1 / |a_l (xb_m - xb_n - 2t)|,
// a_l = L / 2^(l+1) the half-width.  1/r is homogeneous, so every level uses
// the unit operators Kh_t[m][n] = 1 / |xb_m - xb_n - 2t| and one scalar
// 1/a_l per level (Sec. 2.1.2: the 316 operators are computed once).
// The 316 unit operators are signed permutations of 16 canonical ones
// (Sec. 2.1.2): with t = G tc, (G v)_d = s_d v_{pi(d)},
//     Kh_t[m][n] = Kh_tc[g(m)][g(n)],  g(m)_{pi(d)} = s_d > 0 ? m_d : l-1-m_d,
// because the mirrored Chebyshev nodes satisfy xb_{l-1-k} = -xb_k.
//
// FP32 operators (mixed modes) have their rows in the Chebyshev-coefficient
// basis instead of node values: Kh'_t = T3 Kh_t with T3 = T1 (x) T1 (x) T1,
// T1[n][m] = C[m][n] = (n == 0 ? 1 : 2 T_n(xb_m)) / l, which maps the values
// of a degree < l polynomial at the nodes to its Chebyshev coefficients
// (Eq. 5).  A local expansion then accumulates in FP32 as coefficients,
// whose magnitudes fall with the degree like those of the smooth far field
// they describe, so each rounding error is relative to its own coefficient;
// summed as node values, the rounding errors are alike at every node and the
// force, the gradient of the interpolant (L2P), multiplies their
// high-degree part by up to l^2.  The loc-sum pass turns the coefficients
// back into node values in FP64 (T3^-1: T_n(xb_m) along each dimension).
// Mirroring a dimension maps T_n to (-1)^n T_n, so the signed permutations
// act on coefficient rows as permutations with the sign (-1)^(sum of the
// mirrored dimensions' degrees).
//
// The contraction is organised target-stationary: a work tile holds 64
// target cells of one level and one child parity, which share the same 189
// offsets; for each offset the tile computes Y(l^3 x 64) += Kh_t (l^3 x l^3)
// X(l^3 x 64) on MFMA, X the gathered source multipoles, and writes its local
// expansions once (no atomics, deterministic).
#include <hip/hip_runtime.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <vector>

#include "device_util.h"
#include "fmm_internal.h"
#include "jobs.h"

namespace fmm {

thread_local hipEvent_t g_time_ev[kTimedSteps][2] = {{nullptr, nullptr}};

// ------------------------------------------------------------ tables
namespace {

struct OffsetInfo {
  int t[3];
  int canon;   // index into the 16 canonical offsets
  int pi[3];   // t_d = s_d * tc[pi[d]]
  int sg[3];
};

struct StaticTables {
  std::vector<OffsetInfo> offs;        // the 316 far offsets (packed order)
  std::vector<std::array<int, 3>> canon;  // 16 canonical offsets, tc0 >= tc1 >= tc2 >= 0
  int id_to_kid[343];
  std::vector<int> slot_kid;           // [8][189]
  std::vector<signed char> slot_t;     // [8][189][3]
};

const StaticTables& tables() {
  static StaticTables T = [] {
    StaticTables S;
    for (int i = 0; i < 343; ++i) S.id_to_kid[i] = -1;
    std::map<std::array<int, 3>, int> cidx;
    for (int tx = -3; tx <= 3; ++tx)
      for (int ty = -3; ty <= 3; ++ty)
        for (int tz = -3; tz <= 3; ++tz) {
          const int t[3] = {tx, ty, tz};
          int mx = 0;
          for (int d = 0; d < 3; ++d) mx = std::max(mx, std::abs(t[d]));
          if (mx < 2) continue;
          OffsetInfo o;
          int ord[3] = {0, 1, 2};
          std::stable_sort(ord, ord + 3, [&](int a, int b) { return std::abs(t[a]) > std::abs(t[b]); });
          std::array<int, 3> tc;
          for (int j = 0; j < 3; ++j) {
            tc[j] = std::abs(t[ord[j]]);
            o.pi[ord[j]] = j;
          }
          for (int d = 0; d < 3; ++d) {
            o.t[d] = t[d];
            o.sg[d] = t[d] < 0 ? -1 : 1;
          }
          auto it = cidx.find(tc);
          if (it == cidx.end()) {
            it = cidx.emplace(tc, int(S.canon.size())).first;
            S.canon.push_back(tc);
          }
          o.canon = it->second;
          S.id_to_kid[(tx + 3) * 49 + (ty + 3) * 7 + (tz + 3)] = int(S.offs.size());
          S.offs.push_back(o);
        }
    // per child parity p (bit d = parity of the cell coordinate along d):
    // offsets with t_d in [-2-p_d, 3-p_d], in the order the M2L kernels take
    // them: z outermost, x innermost, each axis in steps of two cells (-3,
    // -1, 1, 3, 2, 0, -2) and rows in alternate directions.  The targets of
    // a work item are same-parity cells two apart (4 x 4 x 2 of them), so an
    // offset two cells from the last one reads mostly the same source
    // multipoles, which are then still in L2 (30M-particle order-10 cube:
    // M2L 4327 -> 4222 ms against the lexicographic order)
    static const int zig[7] = {-3, -1, 1, 3, 2, 0, -2};
    for (int p = 0; p < 8; ++p) {
      int cnt = 0;
      for (int i0 = 0; i0 < 7; ++i0)
        for (int i1 = 0; i1 < 7; ++i1)
          for (int i2 = 0; i2 < 7; ++i2) {
            const int tz = zig[i0], ty = zig[i0 % 2 ? 6 - i1 : i1];
            const int tx = zig[(i0 * 7 + i1) % 2 ? 6 - i2 : i2];
            const int t[3] = {tx, ty, tz};
            bool ok = std::max({std::abs(tx), std::abs(ty), std::abs(tz)}) >= 2;
            for (int d = 0; d < 3; ++d) {
              const int pd = (p >> d) & 1;
              ok = ok && t[d] >= -2 - pd && t[d] <= 3 - pd;
            }
            if (!ok) continue;
            S.slot_kid.push_back(S.id_to_kid[(tx + 3) * 49 + (ty + 3) * 7 + (tz + 3)]);
            for (int d = 0; d < 3; ++d) S.slot_t.push_back((signed char)t[d]);
            ++cnt;
          }
      if (cnt != kSlots) throw FmmError{FMM_ERR_HIP, "internal: parity offset count"};
    }
    if (int(S.offs.size()) != kOffsets || S.canon.size() != 16)
      throw FmmError{FMM_ERR_HIP, "internal: offset tables"};
    return S;
  }();
  return T;
}

// Chebyshev roots of T_l, mirrored exactly (xb_{l-1-k} = -xb_k, 0 in the
// middle for odd l).
void cheb_nodes(int l, double* xi) {
  for (int m = 0; m < l; ++m) xi[m] = std::cos((2.0 * m + 1.0) * M_PI / (2.0 * l));
  for (int m = 0; m < l / 2; ++m) xi[l - 1 - m] = -xi[m];
  if (l & 1) xi[l / 2] = 0.0;
}

void cheb_T(int l, double x, double* T) {
  T[0] = 1.0;
  if (l > 1) T[1] = x;
  for (int n = 2; n < l; ++n) T[n] = 2.0 * x * T[n - 1] - T[n - 2];
}

// Canonical unit operators: Kc[c][m][n] = |xb_m - xb_n - 2 tc|^-p for the
// kernel |x - y|^-p (p = 1 or 2)
__global__ void canon_kernel(const double* __restrict__ xi, const int* __restrict__ tc,
                             int l, int ncanon, int p, double* __restrict__ Kc) {
  const int l3 = l * l * l;
  const int64_t total = int64_t(ncanon) * l3 * l3;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int c = int(e / (int64_t(l3) * l3));
    const int r = int(e % (int64_t(l3) * l3));
    const int m = r / l3, n = r % l3;
    const int m1 = m / (l * l), m2 = (m / l) % l, m3 = m % l;
    const int n1 = n / (l * l), n2 = (n / l) % l, n3 = n % l;
    const double dx = xi[m1] - xi[n1] - 2.0 * tc[3 * c];
    const double dy = xi[m2] - xi[n2] - 2.0 * tc[3 * c + 1];
    const double dz = xi[m3] - xi[n3] - 2.0 * tc[3 * c + 2];
    const double r2 = dx * dx + dy * dy + dz * dz;
    Kc[e] = p == 2 ? 1.0 / r2 : 1.0 / sqrt(r2);
  }
}

// Rows to Chebyshev coefficients:
//   out[c][u][col] = sum_a T3[u][a] in[c][a][col],  T3[u][a] = prod_d C[a_d][u_d]
// for nmat row-major l^3 x ncol matrices (a and u are node and degree triples).
__global__ void modal_rows_kernel(const double* __restrict__ in, const double* __restrict__ cheb,
                                  int l, int ncol, int nmat, double* __restrict__ out) {
  const int l3 = l * l * l;
  const int64_t total = int64_t(nmat) * l3 * ncol;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int col = int(e % ncol);
    const int64_t r = e / ncol;
    const int u = int(r % l3), c = int(r / l3);
    const int u1 = u / (l * l), u2 = (u / l) % l, u3 = u % l;
    const double* src = in + int64_t(c) * l3 * ncol + col;
    double v = 0.0;
    for (int a1 = 0; a1 < l; ++a1) {
      const double c1 = cheb[a1 * l + u1];
      for (int a2 = 0; a2 < l; ++a2) {
        const double c12 = c1 * cheb[a2 * l + u2];
        const double* s3 = src + int64_t((a1 * l + a2) * l) * ncol;
        for (int a3 = 0; a3 < l; ++a3) v += c12 * cheb[a3 * l + u3] * s3[int64_t(a3) * ncol];
      }
    }
    out[e] = v;
  }
}

// Row index and sign of a coefficient row u of offset kid in its canonical
// class's coefficient rows: the dimension permutation without the mirroring,
// which flips the sign of odd degrees.
__device__ inline int modal_row(const int* in, int l, int u, double& sgn) {
  const int uu[3] = {u / (l * l), (u / l) % l, u % l};
  int gu[3];
  sgn = 1.0;
  for (int d = 0; d < 3; ++d) {
    gu[in[1 + d]] = uu[d];
    if (in[4 + d] < 0 && (uu[d] & 1)) sgn = -sgn;
  }
  return (gu[0] * l + gu[1]) * l + gu[2];
}

// Pack the 316 operators in MFMA fragment order:
//   kp[((kid*mt + i)*kc + c)*256 + lane*4 + s] = Kh_t[16 i + lane%16][16 c + 4 (lane/16) + s]
// (zero outside l^3), gathering from the canonical operator through g; the
// FP32 pack from the coefficient rows KcM = T3 Kc through modal_row.
__global__ void pack_kernel(const double* __restrict__ Kc, const double* __restrict__ KcM,
                            const int* __restrict__ info, int l, int mt, int kc,
                            double* __restrict__ kp64, float* __restrict__ kp32) {
  const int l3 = l * l * l;
  const int64_t total = int64_t(kOffsets) * mt * kc * 256;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int s = int(e & 3), lane = int((e >> 2) & 63);
    int64_t r = e >> 8;
    const int c = int(r % kc);
    r /= kc;
    const int i = int(r % mt);
    const int kid = int(r / mt);
    const int row = 16 * i + (lane & 15);
    const int col = 16 * c + 4 * (lane >> 4) + s;
    double v = 0.0, vm = 0.0;
    if (row < l3 && col < l3) {
      const int* in = info + 7 * kid;  // canon, pi[3], sg[3]
      int mm[3] = {row / (l * l), (row / l) % l, row % l};
      int nn[3] = {col / (l * l), (col / l) % l, col % l};
      int gm[3], gn[3];
      for (int d = 0; d < 3; ++d) {
        gm[in[1 + d]] = in[4 + d] > 0 ? mm[d] : l - 1 - mm[d];
        gn[in[1 + d]] = in[4 + d] > 0 ? nn[d] : l - 1 - nn[d];
      }
      const int gmi = (gm[0] * l + gm[1]) * l + gm[2];
      const int gni = (gn[0] * l + gn[1]) * l + gn[2];
      v = Kc[(int64_t(in[0]) * l3 + gmi) * l3 + gni];
      double sgn;
      const int gu = modal_row(in, l, row, sgn);
      vm = sgn * KcM[(int64_t(in[0]) * l3 + gu) * l3 + gni];
    }
    kp64[e] = v;
    kp32[e] = float(vm);
  }
}

std::mutex g_ops_mu;
// (device, order, kernel exponent)
std::map<std::tuple<int, int, int>, std::unique_ptr<OpSet>> g_ops;

}  // namespace

const OpSet* get_opset(int l, int kernel, hipStream_t s) {
  int dev = 0;
  FMM_HIP_CHECK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_ops_mu);
  auto it = g_ops.find(std::make_tuple(dev, l, kernel));
  if (it != g_ops.end()) return it->second.get();
  const StaticTables& T = tables();
  auto op = std::make_unique<OpSet>();
  op->order = l;
  op->l3 = l * l * l;
  op->mt = (op->l3 + 15) / 16;
  op->kc = op->mt;
  op->ld = 16 * op->mt;

  double xi[kMaxOrder], Tm[kMaxOrder];
  cheb_nodes(l, xi);
  std::vector<double> cheb(l * l), child(2 * l * l), child_modal(2 * l * l, 0.0);
  for (int m = 0; m < l; ++m) {
    cheb_T(l, xi[m], Tm);
    for (int n = 0; n < l; ++n) {
      cheb[m * l + n] = (n == 0 ? 1.0 : 2.0 * Tm[n]) / l;
    }
  }
  // child-to-parent interpolation S(xb_m; (sigma + xb_m')/2), sigma = -1, +1
  for (int sg = 0; sg < 2; ++sg)
    for (int mp = 0; mp < l; ++mp) {
      double Tu[kMaxOrder];
      cheb_T(l, ((sg ? 1.0 : -1.0) + xi[mp]) / 2.0, Tu);
      for (int m = 0; m < l; ++m) {
        double v = 0.0;
        for (int n = 0; n < l; ++n) v += cheb[m * l + n] * Tu[n];
        child[(sg * l + m) * l + mp] = v;
      }
    }
  // the same re-expansion on Chebyshev coefficients: T_k((sigma + x)/2) is a
  // polynomial of degree k < l, so its coefficients are its values at the l
  // nodes transformed with C (exact): R[n][k] = sum_m C[m][n] T_k((sigma + xb_m)/2)
  for (int sg = 0; sg < 2; ++sg)
    for (int m = 0; m < l; ++m) {
      double Tu[kMaxOrder];
      cheb_T(l, ((sg ? 1.0 : -1.0) + xi[m]) / 2.0, Tu);
      for (int n = 0; n < l; ++n)
        for (int k = 0; k < l; ++k) child_modal[(sg * l + n) * l + k] += cheb[m * l + n] * Tu[k];
    }

  std::vector<int> tc(3 * 16), info(7 * kOffsets);
  for (int c = 0; c < 16; ++c)
    for (int d = 0; d < 3; ++d) tc[3 * c + d] = T.canon[c][d];
  for (int k = 0; k < kOffsets; ++k) {
    const OffsetInfo& o = T.offs[k];
    info[7 * k] = o.canon;
    for (int d = 0; d < 3; ++d) {
      info[7 * k + 1 + d] = o.pi[d];
      info[7 * k + 4 + d] = o.sg[d];
    }
  }

  std::vector<void*> tmp;
  auto up = [&](const void* h, size_t b, bool keep) {
    void* d = dev_alloc(b);
    if (!keep) tmp.push_back(d);
    FMM_HIP_CHECK(hipMemcpyAsync(d, h, b, hipMemcpyHostToDevice, s));
    return d;
  };
  try {
    op->cheb = static_cast<double*>(up(cheb.data(), sizeof(double) * cheb.size(), true));
    op->child_modal =
        static_cast<double*>(up(child_modal.data(), sizeof(double) * child_modal.size(), true));
    op->child = static_cast<double*>(up(child.data(), sizeof(double) * child.size(), true));
    op->slot_kid = static_cast<int*>(up(T.slot_kid.data(), sizeof(int) * T.slot_kid.size(), true));
    op->slot_t = static_cast<signed char*>(up(T.slot_t.data(), T.slot_t.size(), true));
    double* xi_d = static_cast<double*>(up(xi, sizeof(double) * l, false));
    int* tc_d = static_cast<int*>(up(tc.data(), sizeof(int) * tc.size(), false));
    int* info_d = static_cast<int*>(up(info.data(), sizeof(int) * info.size(), false));
    double* kc_d = static_cast<double*>(dev_alloc(sizeof(double) * 16 * size_t(op->l3) * op->l3));
    tmp.push_back(kc_d);
    double* kcm_d = static_cast<double*>(dev_alloc(sizeof(double) * 16 * size_t(op->l3) * op->l3));
    tmp.push_back(kcm_d);
    const size_t npack = size_t(kOffsets) * op->mt * op->kc * 256;
    op->kpack64 = static_cast<double*>(dev_alloc(sizeof(double) * npack));
    op->kpack32 = static_cast<float*>(dev_alloc(sizeof(float) * npack));
    canon_kernel<<<1024, 256, 0, s>>>(xi_d, tc_d, l, 16, kernel, kc_d);
    FMM_HIP_CHECK(hipGetLastError());
    modal_rows_kernel<<<4096, 256, 0, s>>>(kc_d, op->cheb, l, op->l3, 16, kcm_d);
    FMM_HIP_CHECK(hipGetLastError());
    pack_kernel<<<4096, 256, 0, s>>>(kc_d, kcm_d, info_d, l, op->mt, op->kc, op->kpack64,
                                     op->kpack32);
    FMM_HIP_CHECK(hipGetLastError());
    FMM_HIP_CHECK(hipStreamSynchronize(s));
  } catch (...) {
    (void)hipStreamSynchronize(s);
    for (void* q : tmp) dev_free(q);
    throw;
  }
  for (void* q : tmp) dev_free(q);
  const OpSet* r = op.get();
  g_ops[std::make_tuple(dev, l, kernel)] = std::move(op);
  return r;
}

// ------------------------------------------------------------- M2L kernel
typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Vec4;
template <>
struct Vec4<double> {
  typedef d4 type;
};
template <>
struct Vec4<float> {
  typedef f4 type;
};

__device__ inline d4 mfma16x16x4(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f4 mfma16x16x4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// One workgroup = 4 wavefronts = one (tile, M-block) item.  Wavefront w owns
// the M-tiles [mt0, mt0 + MTW) of the output rows and all 64 target columns
// (four 16-column N-tiles).  K-chunks of 16 coefficients = 4 MFMA k-steps;
// lane group g = lane/16 holds k = 16c + 4g + s at step s, so both operands
// are fetched as 4 consecutive values per lane.  FOLD: FP32 partial sums are
// added into FP64 accumulators after every far offset.
// Build-time tuning of the dense kernel: wavefronts per SIMD the register
// allocation must allow, and whether FP64 double-buffers the B fragments.
#ifndef FMM_M2L_WAVES_PER_SIMD
#define FMM_M2L_WAVES_PER_SIMD 2
#endif
#ifndef FMM_M2L_F64_PREFETCH_B
#define FMM_M2L_F64_PREFETCH_B 1
#endif

template <typename T, int MTW, bool FOLD>
__global__ __launch_bounds__(256, FMM_M2L_WAVES_PER_SIMD) void m2l_kernel(
    const JobDev* __restrict__ jobs, const StepTab* __restrict__ tab) {
  typedef typename Vec4<T>::type T4;
  const int total = step_total(*tab);
  const int wave = wuni(int(threadIdx.x >> 6)), lane = threadIdx.x & 63;
  const int g = lane >> 4, c16 = lane & 15;
  for (int it = blockIdx.x; it < total; it += gridDim.x) {
    // with one block per item, blocks are dealt round-robin to the 8 XCDs:
    // give each XCD a contiguous run of tiles so neighbouring tiles share
    // source multipoles in its L2
    int b = it;
    if (int(gridDim.x) == total) {
      const int n8 = (total / 8) * 8;
      if (b < n8) b = (b % 8) * (n8 / 8) + b / 8;
    }
    const int k = step_find(*tab, b);
    const JobDev& J = jobs[tab->job[k]];
    const int local = b - tab->start[k] + tab->first[k];
    const int tile = local / J.nmb, mb = local % J.nmb;
    const int MT = J.mt, KC = J.kc, ld = J.ld;
    const int mt0 = (mb * 4 + wave) * MTW;
    if (mt0 >= MT) continue;
    const int nmt = min(MTW, MT - mt0);
    const M2LTile tl = J.tiles[tile];
    const T* __restrict__ Wp = FOLD ? reinterpret_cast<const T*>(J.W32)
                                    : reinterpret_cast<const T*>(J.W);
    const T* __restrict__ Kp = FOLD ? reinterpret_cast<const T*>(J.kp32)
                                    : reinterpret_cast<const T*>(J.kp64);

    T4 acc[MTW][4];
    d4 acc64[FOLD ? MTW : 1][4];
    for (int i = 0; i < MTW; ++i)
      for (int j = 0; j < 4; ++j) {
        acc[i][j] = T4{0, 0, 0, 0};
        if (FOLD) acc64[FOLD ? i : 0][j] = d4{0, 0, 0, 0};
      }

    const int nact = wuni(gld(J.tile_nact + tile));
    const unsigned char* act = J.tile_act + int64_t(tile) * kSlots;
    const int* srcb = J.tile_src + int64_t(tile) * kSlots * kTileN;
    const int* kidp = J.slot_kid + tl.parity * kSlots;

    for (int ia = 0; ia < nact; ++ia) {
      const int s = wuni(int(gld(act + ia)));
      const int kid = wuni(gld(kidp + s));
      const T* bptr[4];
      for (int j = 0; j < 4; ++j)
        bptr[j] = Wp + int64_t(gld(srcb + s * kTileN + 16 * j + c16)) * ld + 4 * g;
      const T* aptr = Kp + (int64_t(kid) * MT + mt0) * KC * 256 + lane * 4;

      // The A and B fragments are double-buffered one chunk ahead.  In FP64
      // the B buffer costs a few spilled registers at MTW = 3 and still wins
      // (36.8 vs 42.7 ms for the 1M-particle order-7 M2L on gfx950).
      constexpr bool kPrefetchB = sizeof(T) == 4 || FMM_M2L_F64_PREFETCH_B;
      T4 bv[4], av[MTW];
      for (int j = 0; j < 4; ++j) bv[j] = gld(reinterpret_cast<const T4*>(bptr[j]));
      for (int i = 0; i < MTW; ++i)
        av[i] = i < nmt ? gld(reinterpret_cast<const T4*>(aptr + int64_t(i) * KC * 256))
                        : T4{0, 0, 0, 0};
      for (int c = 0; c < KC; ++c) {
        T4 bn[kPrefetchB ? 4 : 1], an[MTW];
        const bool more = c + 1 < KC;
        if (!kPrefetchB && c > 0)
          for (int j = 0; j < 4; ++j) bv[j] = gld(reinterpret_cast<const T4*>(bptr[j] + 16 * c));
        if (more) {
          if (kPrefetchB)
            for (int j = 0; j < 4; ++j)
              bn[kPrefetchB ? j : 0] = gld(reinterpret_cast<const T4*>(bptr[j] + 16 * (c + 1)));
          for (int i = 0; i < MTW; ++i)
            an[i] = i < nmt ? gld(reinterpret_cast<const T4*>(aptr + (int64_t(i) * KC + c + 1) * 256))
                            : T4{0, 0, 0, 0};
        }
#pragma unroll
        for (int st = 0; st < 4; ++st)
#pragma unroll
          for (int i = 0; i < MTW; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = mfma16x16x4(av[i][st], bv[j][st], acc[i][j]);
        if (more) {
          if (kPrefetchB)
            for (int j = 0; j < 4; ++j) bv[j] = bn[kPrefetchB ? j : 0];
          for (int i = 0; i < MTW; ++i) av[i] = an[i];
        }
      }
      if (FOLD) {
        for (int i = 0; i < MTW; ++i)
          for (int j = 0; j < 4; ++j) {
            for (int r = 0; r < 4; ++r) acc64[FOLD ? i : 0][j][r] += double(acc[i][j][r]);
            acc[i][j] = T4{0, 0, 0, 0};
          }
      }
    }

    // D layout of the 16x16 outputs, column c16 in every lane group g: the
    // FP32 instruction holds rows 4g+r in item r, the FP64 one rows 4r+g
    // (both measured on gfx950).
    const double sc = J.scale[tl.level];
    const bool f64 = sizeof(T) == 8;
    for (int j = 0; j < 4; ++j) {
      const int col = 16 * j + c16;
      if (col >= tl.count) continue;
      double* out = J.Loc + int64_t(gld(J.tgt + tl.first + col)) * ld;
#pragma unroll
      for (int i = 0; i < MTW; ++i) {
        if (i >= nmt) continue;  // constant trip count keeps acc[] in registers
        const int base = 16 * (mt0 + i);
        if (f64) {
          for (int r = 0; r < 4; ++r)
            gst(out + base + 4 * r + g,
                sc * (FOLD ? acc64[FOLD ? i : 0][j][r] : double(acc[i][j][r])));
        } else {
          d4 v;
          for (int r = 0; r < 4; ++r)
            v[r] = sc * (FOLD ? acc64[FOLD ? i : 0][j][r] : double(acc[i][j][r]));
          gst(reinterpret_cast<d4*>(out + base + 4 * g), v);
        }
      }
    }
  }
}

template <typename T, bool FOLD>
static void launch_mtw(int mtw, const JobDev* jobs, const StepTab* tab, int grid, hipStream_t s) {
  switch (mtw) {
    case 1: m2l_kernel<T, 1, FOLD><<<grid, 256, 0, s>>>(jobs, tab); break;
    case 2: m2l_kernel<T, 2, FOLD><<<grid, 256, 0, s>>>(jobs, tab); break;
    case 3: m2l_kernel<T, 3, FOLD><<<grid, 256, 0, s>>>(jobs, tab); break;
    default: m2l_kernel<T, 4, FOLD><<<grid, 256, 0, s>>>(jobs, tab); break;
  }
}

// M-tiles per wavefront: fewest idle M-tile slots, then the largest count
// (fewest M-blocks, so the gathered source columns are read fewest times);
// at most 3, which keeps two wavefronts per SIMD without spills.
int m2l_mtw(int mt) {
  int best = 1, best_waste = 1 << 30;
  for (int w = 1; w <= 3; ++w) {
    const int per_block = 4 * w;
    const int nmb = (mt + per_block - 1) / per_block;
    const int waste = nmb * per_block - mt;
    if (waste < best_waste || (waste == best_waste && w > best)) {
      best = w;
      best_waste = waste;
    }
  }
  return best;
}

int m2l_nmb(int mt) {
  const int w = m2l_mtw(mt);
  return (mt + 4 * w - 1) / (4 * w);
}

// Every job in `tab` must have the same order (same packed operator shape).
void launch_m2l_step(int order, bool fp32, const JobDev* jobs, const StepTab* tab, int grid,
                     hipStream_t s) {
  const int l3 = order * order * order;
  const int mtw = m2l_mtw((l3 + 15) / 16);
  if (fp32)
    launch_mtw<float, true>(mtw, jobs, tab, grid, s);
  else
    launch_mtw<double, false>(mtw, jobs, tab, grid, s);
  FMM_HIP_CHECK(hipGetLastError());
}

// ============================================================ compressed M2L
// Sec. 2.1.2: instead of one large SVD of all 316 operators, each of the 16
// canonical operators Kc gets its own SVD Kc = Uc Sc Vc^T, truncated at
// s_k >= eps s_1.  An offset t = G tc reuses it through the same signed
// permutation g as the dense operators:
//     Kh_t[m][n] ~ sum_k Uc[g(m)][k] s_k Vc[g(n)][k],
// so per far offset the tile computes X = (S Vc^T)_g W (rank x 64) and then
// Loc += (Uc)_g X: 4 l^3 r flops per (target, source) pair instead of 2 l^6.
namespace {

// Factors in MFMA fragment order, per packed operator kid (rank padded to
// rp = 16 ceil(r/16)), both blocks rp * ld elements at off[kid]:
//   p1[((i*kc + c)*64 + lane)*4 + s] = s_k Vc[g(n)][k],  k = 16i + lane%16,
//                                                        n = 16c + 4(lane/16) + s
//   p2[((i*nr + c)*64 + lane)*4 + s] = Uc[g(m)][k],      m = 16i + lane%16,
//                                                        k = 16c + 4(lane/16) + s
// rocSOLVER works column-major: it factorises M = Kc^T (the row-major buffer
// read column-major) as M = U_M S V_M^T and returns U_M and V_M^T, so
// Uc[a][k] = Vt[a*n + k] and Vc[b][k] = U[k*n + b].
// Rank held by position p of the packed factors: inside each block of 16
// the 4 x 4 transpose, so that K-step st of a phase-2 MFMA chunk (positions
// 4g + st over the four lane groups g) takes the four consecutive ranks
// 4 st .. 4 st + 3, and the steps past the kept rank hold only zeros.  The
// order of the ranks in a sum over them is free; both factors use the same.
__host__ __device__ inline int rank_slot(int p) {
  return (p & ~15) | ((p & 3) << 2) | ((p >> 2) & 3);
}

__global__ void svd_pack_kernel(const double* __restrict__ U, const double* __restrict__ Vt,
                                const double* __restrict__ VtM,
                                const double* __restrict__ S, const int* __restrict__ info,
                                const int* __restrict__ rank, const int* __restrict__ rpad,
                                const int64_t* __restrict__ off, int l, int mt, int kc,
                                double* __restrict__ p1_64, float* __restrict__ p1_32,
                                double* __restrict__ p2_64, float* __restrict__ p2_32) {
  const int kid = blockIdx.y;
  const int l3 = l * l * l;
  const int* in = info + 7 * kid;  // canon, pi[3], sg[3]
  const int c = in[0];
  const int r = rank[c], rp = rpad[kid], nr = rp / 16;
  const int64_t nblk = int64_t(rp) * kc * 16;  // elements per factor block
  const double* Uc = U + int64_t(c) * l3 * l3;
  const double* Vc = Vt + int64_t(c) * l3 * l3;
  const double* VcM = VtM + int64_t(c) * l3 * l3;  // the same in coefficient rows
  const double* Sc = S + int64_t(c) * l3;
  auto gmap = [&](int m) {
    int mm[3] = {m / (l * l), (m / l) % l, m % l}, gm[3];
    for (int d = 0; d < 3; ++d) gm[in[1 + d]] = in[4 + d] > 0 ? mm[d] : l - 1 - mm[d];
    return (gm[0] * l + gm[1]) * l + gm[2];
  };
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < nblk;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int s = int(e & 3), lane = int((e >> 2) & 63);
    const int64_t q = e >> 8;
    {  // phase-1 factor: rows k (rp, in rank_slot order), columns n (ld)
      const int cc = int(q % kc), i = int(q / kc);
      const int k = rank_slot(16 * i + (lane & 15)), n = 16 * cc + 4 * (lane >> 4) + s;
      double v = 0.0;
      if (k < r && n < l3) v = Sc[k] * Uc[int64_t(k) * l3 + gmap(n)];
      p1_64[off[kid] + e] = v;
      p1_32[off[kid] + e] = float(v);
    }
    {  // phase-2 factor: rows m (ld), columns k (rp, in rank_slot order); the
       // FP32 factor's rows are Chebyshev coefficients
      const int cc = int(q % nr), i = int(q / nr);
      const int m = 16 * i + (lane & 15), k = rank_slot(16 * cc + 4 * (lane >> 4) + s);
      double v = 0.0, vm = 0.0;
      if (m < l3 && k < r) {
        v = Vc[int64_t(gmap(m)) * l3 + k];
        double sgn;
        const int gu = modal_row(in, l, m, sgn);
        vm = sgn * VcM[int64_t(gu) * l3 + k];
      }
      p2_64[off[kid] + e] = v;
      p2_32[off[kid] + e] = float(vm);
    }
  }
}

std::mutex g_svd_mu;
// (device, order, tolerance, kernel exponent)
std::map<std::tuple<int, int, double, int>, std::unique_ptr<SvdOps>> g_svd;
rocblas_handle g_blas[64] = {nullptr};

}  // namespace

int kid_canon(int kid) { return tables().offs[kid].canon; }

const SvdOps* get_svd_ops(int l, double eps, int kernel, hipStream_t s) {
  int dev = 0;
  FMM_HIP_CHECK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_svd_mu);
  auto key = std::make_tuple(dev, l, eps, kernel);
  auto it = g_svd.find(key);
  if (it != g_svd.end()) return it->second.get();
  const OpSet* op = get_opset(l, kernel, s);
  const StaticTables& T = tables();
  const int l3 = l * l * l;
  auto sv = std::make_unique<SvdOps>();
  sv->order = l;
  sv->eps = eps;

  std::vector<void*> tmp;
  auto talloc = [&](size_t b) {
    void* q = dev_alloc(b);
    tmp.push_back(q);
    return q;
  };
  try {
    // the 16 canonical operators, then their SVDs (batched)
    double xi[kMaxOrder];
    cheb_nodes(l, xi);
    std::vector<int> tc(48), info(7 * kOffsets);
    for (int c = 0; c < 16; ++c)
      for (int d = 0; d < 3; ++d) tc[3 * c + d] = T.canon[c][d];
    for (int k = 0; k < kOffsets; ++k) {
      info[7 * k] = T.offs[k].canon;
      for (int d = 0; d < 3; ++d) {
        info[7 * k + 1 + d] = T.offs[k].pi[d];
        info[7 * k + 4 + d] = T.offs[k].sg[d];
      }
    }
    double* xi_d = static_cast<double*>(talloc(sizeof(double) * l));
    int* tc_d = static_cast<int*>(talloc(sizeof(int) * 48));
    int* info_d = static_cast<int*>(talloc(sizeof(int) * info.size()));
    FMM_HIP_CHECK(hipMemcpyAsync(xi_d, xi, sizeof(double) * l, hipMemcpyHostToDevice, s));
    FMM_HIP_CHECK(hipMemcpyAsync(tc_d, tc.data(), sizeof(int) * 48, hipMemcpyHostToDevice, s));
    FMM_HIP_CHECK(hipMemcpyAsync(info_d, info.data(), sizeof(int) * info.size(),
                                 hipMemcpyHostToDevice, s));
    const size_t nn = size_t(l3) * l3;
    double* A = static_cast<double*>(talloc(sizeof(double) * 16 * nn));
    double* U = static_cast<double*>(talloc(sizeof(double) * 16 * nn));
    double* Vt = static_cast<double*>(talloc(sizeof(double) * 16 * nn));
    double* S = static_cast<double*>(talloc(sizeof(double) * 16 * l3));
    double* E = static_cast<double*>(talloc(sizeof(double) * 16 * l3));
    int* dinfo = static_cast<int*>(talloc(sizeof(int) * 16));
    canon_kernel<<<1024, 256, 0, s>>>(xi_d, tc_d, l, 16, kernel, A);
    FMM_HIP_CHECK(hipGetLastError());
    if (dev < 0 || dev >= 64) throw FmmError{FMM_ERR_HIP, "device index out of range"};
    if (!g_blas[dev] && rocblas_create_handle(&g_blas[dev]) != rocblas_status_success)
      throw FmmError{FMM_ERR_HIP, "rocblas_create_handle failed"};
    if (rocblas_set_stream(g_blas[dev], s) != rocblas_status_success)
      throw FmmError{FMM_ERR_HIP, "rocblas_set_stream failed"};
    const rocblas_status st = rocsolver_dgesvd_strided_batched(
        g_blas[dev], rocblas_svect_all, rocblas_svect_all, l3, l3, A, l3, rocblas_stride(nn), S,
        rocblas_stride(l3), U, l3, rocblas_stride(nn), Vt, l3, rocblas_stride(nn), E,
        rocblas_stride(l3), rocblas_outofplace, dinfo, 16);
    if (st != rocblas_status_success) throw FmmError{FMM_ERR_HIP, "rocsolver gesvd failed"};
    std::vector<double> Sh(16 * size_t(l3));
    int hinfo[16];
    FMM_HIP_CHECK(hipMemcpyAsync(Sh.data(), S, sizeof(double) * Sh.size(), hipMemcpyDeviceToHost, s));
    FMM_HIP_CHECK(hipMemcpyAsync(hinfo, dinfo, sizeof(hinfo), hipMemcpyDeviceToHost, s));
    FMM_HIP_CHECK(hipStreamSynchronize(s));
    for (int c = 0; c < 16; ++c)
      if (hinfo[c] != 0) throw FmmError{FMM_ERR_HIP, "rocsolver gesvd did not converge"};

    // ranks: singular values come sorted, largest first
    int rank_h[16];
    for (int c = 0; c < 16; ++c) {
      const double* sc = &Sh[size_t(c) * l3];
      int r = 0;
      while (r < l3 && sc[r] >= eps * sc[0]) ++r;
      rank_h[c] = std::max(r, 1);
      sv->rank[c] = rank_h[c];
    }
    sv->rpad_h.resize(kOffsets);
    std::vector<int> rk_h(kOffsets);
    std::vector<int64_t> off(kOffsets);
    int64_t tot = 0;
    double wr = 0.0, wf = 0.0;
    for (int k = 0; k < kOffsets; ++k) {
      const int r = rank_h[T.offs[k].canon];
      const int rp = 16 * ((r + 15) / 16);
      sv->rpad_h[k] = rp;
      rk_h[k] = r;
      sv->rmax_pad = std::max(sv->rmax_pad, rp);
      off[k] = tot;
      tot += int64_t(rp) * op->ld;
      wr += r;
      wf += 4.0 * l3 * r;
    }
    sv->weighted_rank = wr / kOffsets;
    sv->flops_per_pair_weighted = int64_t(wf / kOffsets + 0.5);
    int* rank_d = static_cast<int*>(talloc(sizeof(int) * 16));
    FMM_HIP_CHECK(hipMemcpyAsync(rank_d, rank_h, sizeof(rank_h), hipMemcpyHostToDevice, s));
    sv->rpad = static_cast<int*>(dev_alloc(sizeof(int) * kOffsets));
    sv->off = static_cast<int64_t*>(dev_alloc(sizeof(int64_t) * kOffsets));
    FMM_HIP_CHECK(hipMemcpyAsync(sv->rpad, sv->rpad_h.data(), sizeof(int) * kOffsets,
                                 hipMemcpyHostToDevice, s));
    FMM_HIP_CHECK(hipMemcpyAsync(sv->off, off.data(), sizeof(int64_t) * kOffsets,
                                 hipMemcpyHostToDevice, s));
    sv->rk = static_cast<int*>(dev_alloc(sizeof(int) * kOffsets));
    FMM_HIP_CHECK(hipMemcpyAsync(sv->rk, rk_h.data(), sizeof(int) * kOffsets,
                                 hipMemcpyHostToDevice, s));
    sv->p1_64 = static_cast<double*>(dev_alloc(sizeof(double) * tot));
    sv->p2_64 = static_cast<double*>(dev_alloc(sizeof(double) * tot));
    sv->p1_32 = static_cast<float*>(dev_alloc(sizeof(float) * tot));
    sv->p2_32 = static_cast<float*>(dev_alloc(sizeof(float) * tot));
    // Uc[a][k] = Vt[a * l3 + k]: its rows as Chebyshev coefficients, for FP32
    double* VtM = static_cast<double*>(talloc(sizeof(double) * 16 * nn));
    modal_rows_kernel<<<4096, 256, 0, s>>>(Vt, op->cheb, l, l3, 16, VtM);
    FMM_HIP_CHECK(hipGetLastError());
    svd_pack_kernel<<<dim3(64, kOffsets), 256, 0, s>>>(U, Vt, VtM, S, info_d, rank_d, sv->rpad,
                                                        sv->off, l, op->mt, op->kc, sv->p1_64,
                                                        sv->p1_32, sv->p2_64, sv->p2_32);
    FMM_HIP_CHECK(hipGetLastError());
    FMM_HIP_CHECK(hipStreamSynchronize(s));
  } catch (...) {
    (void)hipStreamSynchronize(s);
    for (void* q : tmp) dev_free(q);
    for (void* q : {(void*)sv->rpad, (void*)sv->rk, (void*)sv->off, (void*)sv->p1_64,
                    (void*)sv->p1_32, (void*)sv->p2_64, (void*)sv->p2_32})
      if (q) dev_free(q);
    throw;
  }
  for (void* q : tmp) dev_free(q);
  const SvdOps* r = sv.get();
  g_svd[key] = std::move(sv);
  return r;
}

// Target columns per workgroup of the compressed kernel, 16 * NT, for FP32
// and FP64.  Fewer columns than the tile's 64 cost operator re-reads (from
// L2) but free registers for two wavefronts per SIMD.  Measured on gfx950
// at order 7 with the 4-wavefront kernel: FP32 best at 32 columns in 8
// wavefronts (3 M-tiles each, no spills); FP64 at 16 columns in 4
// wavefronts (within 1% of 32 columns in 8, and half the LDS, so order 9 at
// 1e-9 still fits).  These are the base shapes; the warp-specialised kernel
// takes wider items where they fit (FMM_M2L_SVD_FULL_*).
#ifndef FMM_M2L_SVD_NT_F32
#define FMM_M2L_SVD_NT_F32 2
#endif
#ifndef FMM_M2L_SVD_NT_F64
#define FMM_M2L_SVD_NT_F64 1
#endif
constexpr int svd_nt(bool fp32) { return fp32 ? FMM_M2L_SVD_NT_F32 : FMM_M2L_SVD_NT_F64; }
static_assert(svd_nt(true) == 1 || svd_nt(true) == 2 || svd_nt(true) == 4, "NT");
static_assert(svd_nt(false) == 1 || svd_nt(false) == 2 || svd_nt(false) == 4, "NT");
// Whether phase 2 loads its U fragments one rank chunk ahead (FP32, FP64).
#ifndef FMM_M2L_SVD_P2_PREFETCH_F32
#define FMM_M2L_SVD_P2_PREFETCH_F32 0
#endif
#ifndef FMM_M2L_SVD_P2_PREFETCH_F64
#define FMM_M2L_SVD_P2_PREFETCH_F64 0
#endif
// Rank tiles per pass of phase 1 over the l^3 contraction (each pass reads
// its share of the gathered multipoles once), FP32 and FP64.
#ifndef FMM_M2L_SVD_RPASS_F32
#define FMM_M2L_SVD_RPASS_F32 2
#endif
#ifndef FMM_M2L_SVD_RPASS_F64
#define FMM_M2L_SVD_RPASS_F64 2
#endif
// FP32 mode: where the FP32 accumulators are folded into FP64 sums, every
// J.fold_every far offsets (the plan's fold interval):
//   0  nowhere (FP32 across all far offsets)
//   1  FP64 registers (acc64)
//   2  the item's own FP64 rows of the local expansions in global memory
// Measured at order 7 (fold every 8): mode 2 runs in 5.5 ms where mode 1
// runs in 8.0 ms, because without the FP64 registers two 4-wavefront
// workgroups fit per CU without spills.
#ifndef FMM_M2L_SVD_F32_FOLD_MODE
#define FMM_M2L_SVD_F32_FOLD_MODE 2
#endif
// Wavefronts per SIMD the register allocation must allow, FP32 and FP64.
#ifndef FMM_M2L_SVD_WAVES_F32
#define FMM_M2L_SVD_WAVES_F32 2
#endif
#ifndef FMM_M2L_SVD_WAVES_F64
#define FMM_M2L_SVD_WAVES_F64 2
#endif
// Wavefronts per workgroup (4 or 8), FP32 and FP64.  With 8, two wavefronts
// share each K-group of phase 1 (one per N-tile half) and every wavefront
// owns half as many output rows, which halves its accumulator registers.
#ifndef FMM_M2L_SVD_NWV_F32
#define FMM_M2L_SVD_NWV_F32 4
#endif
#ifndef FMM_M2L_SVD_NWV_F64
#define FMM_M2L_SVD_NWV_F64 4
#endif
constexpr int svd_nwv(bool fp32) { return fp32 ? FMM_M2L_SVD_NWV_F32 : FMM_M2L_SVD_NWV_F64; }
static_assert((svd_nwv(true) == 4 || svd_nwv(true) == 8) &&
                  (svd_nwv(false) == 4 || svd_nwv(false) == 8),
              "4 or 8 wavefronts per workgroup");
static_assert(4 * svd_nt(true) % svd_nwv(true) == 0 && 4 * svd_nt(false) % svd_nwv(false) == 0,
              "8 wavefronts need at least 2 N-tiles");

// One workgroup = NWV wavefronts = one (tile, M-block, N-group) item, the
// N-group being NC = 16 NT of the tile's 64 target columns.  Per far offset:
//   phase 1  X(rp x NC) = (S V^T)_g W.  K-group kg = w % 4 takes the
//            K-chunks kg, kg+4, ... of the l^3 contraction for every rank
//            tile (two per pass); its NWV/4 wavefronts split the N-tiles.
//            Partial sums go to the K-group's LDS slab P[kg];
//   phase 2  Y(l^3 x NC) += U_g X, X read as P[0]+P[1]+P[2]+P[3] (always
//            in that order, so every wavefront sees the same X and the
//            result does not depend on timing).  Wavefront w owns MTW
//            16-row M-tiles of the output.
// The slabs are double-buffered, the buffer alternating with every offset
// the workgroup processes (also across items), so one barrier per offset
// suffices: a wavefront writes buffer b again only after the barrier of the
// next offset, which every wavefront reaches after its reads of buffer b.
template <typename T, int MTW, int NT, int NWV, int FM>
__global__ __launch_bounds__(64 * NWV, sizeof(T) == 4 ? FMM_M2L_SVD_WAVES_F32
                                                      : FMM_M2L_SVD_WAVES_F64) void m2l_svd_kernel(const JobDev* __restrict__ jobs,
                                                         const StepTab* __restrict__ tab) {
  typedef typename Vec4<T>::type T4;
  constexpr bool FOLD = FM == 1;  // FP64 register sums
  constexpr int NC = 16 * NT, NG = 4 / NT;
  constexpr int NTW = NT * 4 / NWV;  // N-tiles per wavefront in phase 1
  constexpr int kRP = sizeof(T) == 4 ? FMM_M2L_SVD_RPASS_F32 : FMM_M2L_SVD_RPASS_F64;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* const lds = reinterpret_cast<T*>(lds_raw);
  int buf = 0;
  const int total = step_total(*tab);
  const int wave = wuni(int(threadIdx.x >> 6)), lane = threadIdx.x & 63;
  const int g = lane >> 4, c16 = lane & 15;
  const bool f64 = sizeof(T) == 8;
  for (int it = blockIdx.x; it < total; it += gridDim.x) {
    int b = it;
    if (int(gridDim.x) == total) {
      const int n8 = (total / 8) * 8;
      if (b < n8) b = (b % 8) * (n8 / 8) + b / 8;
    }
    const int k = step_find(*tab, b);
    const JobDev& J = jobs[tab->job[k]];
    const int local = b - tab->start[k] + tab->first[k];
    const int tile = local / J.nmb, rem = local % J.nmb;
    const int mb = rem / NG, col0 = NC * (rem % NG);
    const M2LTile tl = J.tiles[tile];
    if (col0 >= tl.count) continue;  // the same for the whole workgroup
    const int MT = J.mt, KC = J.kc, ld = J.ld, XS = J.xs;
    const int mt0 = (mb * NWV + wave) * MTW;
    const int nmt = mt0 < MT ? min(MTW, MT - mt0) : 0;
    const int kg = wave & 3, jn0 = (wave >> 2) * NTW;
    constexpr bool F32 = sizeof(T) == 4;
    const T* __restrict__ Wp = F32 ? reinterpret_cast<const T*>(J.W32)
                                   : reinterpret_cast<const T*>(J.W);
    const T* __restrict__ P1 = F32 ? reinterpret_cast<const T*>(J.p1_32)
                                   : reinterpret_cast<const T*>(J.p1_64);
    const T* __restrict__ P2 = F32 ? reinterpret_cast<const T*>(J.p2_32)
                                   : reinterpret_cast<const T*>(J.p2_64);
    T4 acc[MTW][NT];
    d4 acc64[FOLD ? MTW : 1][NT];
#pragma unroll
    for (int i = 0; i < MTW; ++i)
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        acc[i][j] = T4{0, 0, 0, 0};
        if (FOLD) acc64[FOLD ? i : 0][j] = d4{0, 0, 0, 0};
      }
    const int nact = wuni(gld(J.tile_nact + tile));
    bool folded = false;  // FM == 2: Loc rows written once already
    const unsigned char* act = J.tile_act + int64_t(tile) * kSlots;
    const int* srcb = J.tile_src + int64_t(tile) * kSlots * kTileN + col0;
    const int* kidp = J.slot_kid + tl.parity * kSlots;

    for (int ia = 0; ia < nact; ++ia) {
      const int s = wuni(int(gld(act + ia)));
      const int kid = wuni(gld(kidp + s));
      const int rp = wuni(gld(J.svd_rpad + kid)), nr = rp >> 4;
      const int nst = (wuni(gld(J.svd_rank + kid)) - 16 * (nr - 1) + 3) >> 2;  // K-steps, last chunk
      const int64_t off = wuni(gld(J.svd_off + kid));
      T* const P = lds + buf * 4 * NC * XS;
      T* const Pw = P + kg * NC * XS;
      buf ^= 1;
      // ---- phase 1: this wavefront's share of X, into its K-group's slab ----
      const T* bp[NTW];
#pragma unroll
      for (int j = 0; j < NTW; ++j)
        bp[j] = Wp + int64_t(gld(srcb + s * kTileN + 16 * (jn0 + j) + c16)) * ld + 4 * g;
      for (int i0 = 0; i0 < nr; i0 += kRP) {
        const int np = min(kRP, nr - i0);
        const T* a0 = P1 + off + (int64_t(i0) * KC) * 256 + lane * 4;
        T4 x[kRP][NTW];
#pragma unroll
        for (int i = 0; i < kRP; ++i)
#pragma unroll
          for (int j = 0; j < NTW; ++j) x[i][j] = T4{0, 0, 0, 0};
        T4 bv[NTW], av[kRP];
        if (kg < KC) {
#pragma unroll
          for (int j = 0; j < NTW; ++j) bv[j] = gld(reinterpret_cast<const T4*>(bp[j] + 16 * kg));
#pragma unroll
          for (int i = 0; i < kRP; ++i)
            av[i] = i < np ? gld(reinterpret_cast<const T4*>(a0 + (int64_t(i) * KC + kg) * 256))
                           : T4{0, 0, 0, 0};
        }
        for (int c = kg; c < KC; c += 4) {
          T4 bn[NTW], an[kRP];
          const bool more = c + 4 < KC;
          if (more) {
#pragma unroll
            for (int j = 0; j < NTW; ++j)
              bn[j] = gld(reinterpret_cast<const T4*>(bp[j] + 16 * (c + 4)));
#pragma unroll
            for (int i = 0; i < kRP; ++i)
              an[i] = i < np ? gld(reinterpret_cast<const T4*>(a0 + (int64_t(i) * KC + c + 4) * 256))
                             : T4{0, 0, 0, 0};
          }
#pragma unroll
          for (int st = 0; st < 4; ++st)
#pragma unroll
            for (int i = 0; i < kRP; ++i)
#pragma unroll
              for (int j = 0; j < NTW; ++j)
                if (i < np) x[i][j] = mfma16x16x4(av[i][st], bv[j][st], x[i][j]);
          if (more) {
#pragma unroll
            for (int j = 0; j < NTW; ++j) bv[j] = bn[j];
#pragma unroll
            for (int i = 0; i < kRP; ++i) av[i] = an[i];
          }
        }
        // D rows: FP32 item r -> row 4g + r, FP64 item r -> row 4r + g
#pragma unroll
        for (int i = 0; i < kRP; ++i)
#pragma unroll
          for (int j = 0; j < NTW; ++j) {
            if (i >= np) continue;
            T* xrow = Pw + (16 * (jn0 + j) + c16) * XS + 16 * (i0 + i);
            if (f64) {
#pragma unroll
              for (int r = 0; r < 4; ++r) xrow[4 * r + g] = x[i][j][r];
            } else {
              *reinterpret_cast<T4*>(xrow + 4 * g) = x[i][j];
            }
          }
      }
      __syncthreads();
      // ---- phase 2: Loc rows of this wavefront's M-tiles ----
      if (nmt > 0) {
        const T* a2 = P2 + off + int64_t(mt0) * nr * 256 + lane * 4;
        constexpr bool kPre = sizeof(T) == 4 ? FMM_M2L_SVD_P2_PREFETCH_F32
                                             : FMM_M2L_SVD_P2_PREFETCH_F64;
        T4 av[MTW];
        if (kPre) {
#pragma unroll
          for (int i = 0; i < MTW; ++i)
            av[i] = i < nmt ? gld(reinterpret_cast<const T4*>(a2 + int64_t(i) * nr * 256))
                            : T4{0, 0, 0, 0};
        }
        for (int c = 0; c < nr; ++c) {
          T4 bv[NT], an[kPre ? MTW : 1];
          if (!kPre) {
#pragma unroll
            for (int i = 0; i < MTW; ++i)
              av[i] = i < nmt ? gld(reinterpret_cast<const T4*>(a2 + (int64_t(i) * nr + c) * 256))
                              : T4{0, 0, 0, 0};
          } else if (c + 1 < nr) {
#pragma unroll
            for (int i = 0; i < MTW; ++i)
              an[kPre ? i : 0] =
                  i < nmt ? gld(reinterpret_cast<const T4*>(a2 + (int64_t(i) * nr + c + 1) * 256))
                          : T4{0, 0, 0, 0};
          }
#pragma unroll
          for (int j = 0; j < NT; ++j) {
            const int o = (16 * j + c16) * XS + 16 * c + 4 * g;
            T4 v = *reinterpret_cast<const T4*>(P + o);
#pragma unroll
            for (int w = 1; w < 4; ++w) v += *reinterpret_cast<const T4*>(P + w * NC * XS + o);
            bv[j] = v;
          }
          // K-steps past the kept rank hold zeros in both operands
          const int ns = c + 1 < nr ? 4 : nst;
#pragma unroll
          for (int st = 0; st < 4; ++st) {
            if (st >= ns) continue;
#pragma unroll
            for (int i = 0; i < MTW; ++i) {
              if (i >= nmt) continue;
#pragma unroll
              for (int j = 0; j < NT; ++j)
                acc[i][j] = mfma16x16x4(av[i][st], bv[j][st], acc[i][j]);
            }
          }
          if (kPre && c + 1 < nr) {
#pragma unroll
            for (int i = 0; i < MTW; ++i) av[i] = an[kPre ? i : 0];
          }
        }
        const bool fold_now = (ia + 1) % J.fold_every == 0 || ia == nact - 1;
        if (FOLD && fold_now) {
#pragma unroll
          for (int i = 0; i < MTW; ++i)
#pragma unroll
            for (int j = 0; j < NT; ++j) {
#pragma unroll
              for (int r = 0; r < 4; ++r) acc64[FOLD ? i : 0][j][r] += double(acc[i][j][r]);
              acc[i][j] = T4{0, 0, 0, 0};
            }
        }
        if (FM == 2 && fold_now) {
          // fold into this item's rows of Loc (scaled; the first fold
          // stores, later ones add): no other workgroup touches these rows
          const double sc = J.scale[tl.level];
#pragma unroll
          for (int j = 0; j < NT; ++j) {
            const int col = col0 + 16 * j + c16;
            if (col < tl.count) {
              double* out = J.Loc + int64_t(gld(J.tgt + tl.first + col)) * ld;
#pragma unroll
              for (int i = 0; i < MTW; ++i) {
                if (i >= nmt) continue;
                d4* o = reinterpret_cast<d4*>(out + 16 * (mt0 + i) + 4 * g);  // rows 4g..4g+3
                d4 v;
#pragma unroll
                for (int r = 0; r < 4; ++r) v[r] = sc * double(acc[i][j][r]);
                if (folded) v += gld(o);
                gst(o, v);
              }
            }
#pragma unroll
            for (int i = 0; i < MTW; ++i) acc[i][j] = T4{0, 0, 0, 0};
          }
          folded = true;
        }
      }
    }

    if (FM == 2 && folded) continue;  // the folds wrote the rows
    const double sc = J.scale[tl.level];
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      const int col = col0 + 16 * j + c16;
      if (col >= tl.count) continue;
      double* out = J.Loc + int64_t(gld(J.tgt + tl.first + col)) * ld;
#pragma unroll
      for (int i = 0; i < MTW; ++i) {
        if (i >= nmt) continue;
        const int base = 16 * (mt0 + i);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = f64 ? 4 * r + g : 4 * g + r;
          gst(out + base + row, sc * (FOLD ? acc64[FOLD ? i : 0][j][r] : double(acc[i][j][r])));
        }
      }
    }
  }
}

// Warp-specialised form of the same computation, 8 wavefronts: 0-3 are the
// four K-groups of phase 1 (producers), 4-7 own the M-tiles of phase 2
// (consumers, MTW each, as the 4-wavefront kernel).  Iteration ia of an
// item: the producers write X of offset ia into slab buffer ia % 2 while the
// consumers apply X of offset ia - 1 from the other buffer; one barrier ends
// the iteration, so phase 1 of one offset runs beside phase 2 of the
// previous one, and a buffer is written again only after the barrier that
// follows its last read.  Both roles walk the same items and pass nact + 1
// barriers per item; the role is taken on a wavefront-uniform branch, and
// each role keeps only its own registers live.  The arithmetic, including
// its order, is that of m2l_svd_kernel with 4 wavefronts: FP32 folds into
// the item's FP64 Loc rows every J.fold_every offsets; FP64 accumulates in
// registers and writes once.
#ifndef FMM_M2L_SVD_WS_WAVES
#define FMM_M2L_SVD_WS_WAVES 4
#endif
// ...and for workgroups of 8 consumers (12 wavefronts): one of them fills a
// CU at 3 wavefronts per SIMD, and a second would need 6 per SIMD (85
// VGPRs), so they take the 168 VGPRs of 3 per SIMD at no loss of occupancy
// (the 32-column shapes of orders 8 to 10 spilled at 128).
#ifndef FMM_M2L_SVD_WS_WAVES_BIG
#define FMM_M2L_SVD_WS_WAVES_BIG 3
#endif
constexpr int svd_ws_waves(int ncw, int nt) {
  return ncw >= 8 ? FMM_M2L_SVD_WS_WAVES_BIG : FMM_M2L_SVD_WS_WAVES;
}
// Producer stage depth D, FP32 and FP64: where every K-group has at most D
// chunks of the l^3 contraction (ceil(KC / 4) <= D), the kernel built for D
// loads each K-group's chunks all at once; otherwise (or D = 0) they stream
// one chunk ahead.
#ifndef FMM_M2L_SVD_WS_STAGE_F32
#define FMM_M2L_SVD_WS_STAGE_F32 0
#endif
#ifndef FMM_M2L_SVD_WS_STAGE_F64
#define FMM_M2L_SVD_WS_STAGE_F64 0
#endif
// Whether a producer loads the first chunk of its next offset before the
// barrier that ends the current one (streamed path), FP32 and FP64 (the FP64
// registers would spill).
#ifndef FMM_M2L_SVD_WS_XPRE_F32
#define FMM_M2L_SVD_WS_XPRE_F32 1
#endif
#ifndef FMM_M2L_SVD_WS_XPRE_F64
#define FMM_M2L_SVD_WS_XPRE_F64 0
#endif
// Chunks a producer keeps in flight ahead of the one it computes (1 or 2),
// FP32 and FP64.
#ifndef FMM_M2L_SVD_WS_LOOK_F32
#define FMM_M2L_SVD_WS_LOOK_F32 1
#endif
#ifndef FMM_M2L_SVD_WS_LOOK_F64
#define FMM_M2L_SVD_WS_LOOK_F64 1
#endif
// U fragments (M-tiles of rank chunk 0) a consumer loads for its next offset
// before the barrier, FP32 and FP64 (measured at order 7: 0 to 6 within
// noise, so off).
#ifndef FMM_M2L_SVD_WS_CPRE_F32
#define FMM_M2L_SVD_WS_CPRE_F32 0
#endif
#ifndef FMM_M2L_SVD_WS_CPRE_F64
#define FMM_M2L_SVD_WS_CPRE_F64 0
#endif
#ifndef FMM_M2L_SVD_WS_APRE_F32
#define FMM_M2L_SVD_WS_APRE_F32 0
#endif
#ifndef FMM_M2L_SVD_WS_APRE_F64
#define FMM_M2L_SVD_WS_APRE_F64 0
#endif

struct SvdItem {
  const JobDev* J;
  M2LTile tl;
  int tile, mb, col0;
  int part;  // offset range [ia0, ia1) of the tile's active offsets
};

__device__ inline void svd_part_range(const SvdItem& I, int nact, int& ia0, int& ia1) {
  const int K = I.J->m2l_parts;
  ia0 = int(int64_t(I.part) * nact / K);
  ia1 = int(int64_t(I.part + 1) * nact / K);
}

// Per active offset of an item, what both roles look up: the factor offset,
// the slot (for the source columns), the rank chunks and the K-steps of the
// last one.  Filled once per item into LDS, after the slabs, by all threads.
struct SvdMeta {
  int64_t off;
  int s;
  int nr_nst;  // nr | nst << 16 | gmask << 24 (the slot's 16-target groups with a source)
};
constexpr size_t kSvdMetaBytes = sizeof(SvdMeta) * kSlots;

template <bool GS = false>
__device__ inline void svd_meta_fill(const SvdItem& I, int nact, SvdMeta* meta) {
  const JobDev& J = *I.J;
  int ia0, ia1;
  svd_part_range(I, nact, ia0, ia1);
  const unsigned char* act = J.tile_act + int64_t(I.tile) * kSlots;
  const int* kidp = J.slot_kid + I.tl.parity * kSlots;
  for (int t = threadIdx.x; t < ia1 - ia0; t += blockDim.x) {
    const int sl = gld(act + ia0 + t);
    const int kid = gld(kidp + sl);
    const int nr = gld(J.svd_rpad + kid) >> 4;
    const int nst = (gld(J.svd_rank + kid) - 16 * (nr - 1) + 3) >> 2;
    const int gm = GS ? gld(J.tile_gmask + int64_t(I.tile) * kSlots + ia0 + t) : 0xf;
    meta[t] = SvdMeta{gld(J.svd_off + kid), sl, nr | (nst << 16) | (gm << 24)};
  }
  __syncthreads();
}

// The FP64 row that target column col of the item accumulates into: the
// cell's local expansion for part 0, else the part's own row of LocX.
__device__ inline double* svd_out_row(const SvdItem& I, int col) {
  const JobDev& J = *I.J;
  const int64_t t = gld(J.tgt + I.tl.first + col);
  if (I.part == 0) return J.Loc + t * J.ld;
  return J.LocX + (int64_t(I.part - 1) * J.locx_rows + (t - J.locx_first)) * J.ld;
}

// Item `it` of the launch; false when its N-group holds no target column
// (the same for the whole workgroup).
template <int NT>
__device__ inline bool svd_item(const JobDev* __restrict__ jobs, const StepTab* __restrict__ tab,
                                int it, int total, SvdItem& I) {
  constexpr int NC = 16 * NT, NG = 4 / NT;
  int b = it;
  if (int(gridDim.x) == total) {
    const int n8 = (total / 8) * 8;
    if (b < n8) b = (b % 8) * (n8 / 8) + b / 8;
  }
  const int k = step_find(*tab, b);
  const JobDev& J = jobs[tab->job[k]];
  const int local = b - tab->start[k] + tab->first[k];
  I.J = &J;
  const int per_tile = J.nmb * J.m2l_parts;
  I.tile = local / per_tile;
  const int rem0 = local % per_tile;
  I.part = rem0 / J.nmb;
  const int rem = rem0 % J.nmb;
  I.mb = rem / NG;
  I.col0 = NC * (rem % NG);
  I.tl = J.tiles[I.tile];
  return I.col0 < I.tl.count;
}

// The 32-column items of 8 consumers (FP32 at orders 10 to 12, where whole
// tiles would spill) have registers to spare at 3 wavefronts per SIMD: their
// producers take 3 rank tiles per pass, so that the offsets padded to rank
// 48 gather their multipoles once, and keep two chunks in flight (30M-
// particle order-10 cube, M2L 5126 -> 4771 ms; 167 VGPRs, no spills).  The
// other shapes spill with either.
#ifndef FMM_M2L_SVD_RPASS_WIDE_F32
#define FMM_M2L_SVD_RPASS_WIDE_F32 3
#endif
#ifndef FMM_M2L_SVD_WS_LOOK_WIDE_F32
#define FMM_M2L_SVD_WS_LOOK_WIDE_F32 2
#endif

// GS: the N-tiles whose 16 target columns have no source at an offset
// (their multipole columns are the zero row, so their products are zero)
// are skipped, by both roles; a wavefront-uniform test per N-tile, which
// costs the dense cubes 9-11%, so only plans with many empty groups take it
template <typename T, int NT, int D, int NCW, bool GS>
__device__ inline void svd_ws_produce(const JobDev* __restrict__ jobs,
                                      const StepTab* __restrict__ tab, T* const lds,
                                      SvdMeta* const meta, int kg) {
  typedef typename Vec4<T>::type T4;
  constexpr bool F32 = sizeof(T) == 4;
  constexpr int NC = 16 * NT;
  constexpr bool kWide = F32 && NT == 2 && NCW == 8;
  constexpr int kRP = kWide ? FMM_M2L_SVD_RPASS_WIDE_F32
                            : F32 ? FMM_M2L_SVD_RPASS_F32 : FMM_M2L_SVD_RPASS_F64;
  // staged path: the next rank tile's factor fragments load while this one
  // computes (1) or after it (0)
  constexpr bool kAPre = F32 ? FMM_M2L_SVD_WS_APRE_F32 : FMM_M2L_SVD_WS_APRE_F64;
  constexpr bool kXPre = F32 ? FMM_M2L_SVD_WS_XPRE_F32 : FMM_M2L_SVD_WS_XPRE_F64;
  constexpr int kLook = kWide ? FMM_M2L_SVD_WS_LOOK_WIDE_F32
                              : F32 ? FMM_M2L_SVD_WS_LOOK_F32 : FMM_M2L_SVD_WS_LOOK_F64;
  // the chunk pipeline below holds the current chunk and at most two more
  static_assert(kLook == 1 || kLook == 2, "one or two chunks in flight");
  const int lane = threadIdx.x & 63, g = lane >> 4, c16 = lane & 15;
  const int total = step_total(*tab);
  int buf = 0;
  for (int it = blockIdx.x; it < total; it += gridDim.x) {
    SvdItem I;
    if (!svd_item<NT>(jobs, tab, it, total, I)) continue;
    const JobDev& J = *I.J;
    const int KC = J.kc, ld = J.ld, XS = J.xs;
    const int nck = KC > kg ? (KC - kg + 3) / 4 : 0;  // chunks kg, kg + 4, ...
    const T* __restrict__ Wp = F32 ? reinterpret_cast<const T*>(J.W32)
                                   : reinterpret_cast<const T*>(J.W);
    const T* __restrict__ P1 = F32 ? reinterpret_cast<const T*>(J.p1_32)
                                   : reinterpret_cast<const T*>(J.p1_64);
    const int nact = wuni(gld(J.tile_nact + I.tile));
    const unsigned char* act = J.tile_act + int64_t(I.tile) * kSlots;
    const int* srcb = J.tile_src + int64_t(I.tile) * kSlots * kTileN + I.col0;
    const int* kidp = J.slot_kid + I.tl.parity * kSlots;
    int ia0, ia1;
    svd_part_range(I, nact, ia0, ia1);
    svd_meta_fill<GS>(I, nact, meta);
    // each lane's source cells, one offset ahead
    int src_next[NT];
    if (ia0 < ia1) {
      const int s0 = wuni(meta[0].s);
#pragma unroll
      for (int j = 0; j < NT; ++j) src_next[j] = gld(srcb + s0 * kTileN + 16 * j + c16);
    }
    // the first chunk of the next offset, loaded before the barrier
    T4 pre_bv[NT], pre_av[kRP];
    bool have_pre = false;
    for (int ia = ia0; ia <= ia1; ++ia) {
      if (ia < ia1) {
        // phase 1 of offset ia: this K-group's partial X into its slab
        const SvdMeta md = meta[ia - ia0];
        const int nrs = wuni(md.nr_nst);
        const int nr = nrs & 0xffff;
        bool on[NT];
#pragma unroll
        for (int j = 0; j < NT; ++j) on[j] = !GS || ((nrs >> (24 + I.col0 / 16 + j)) & 1);
        const int64_t off = wuni(md.off);
        int src[NT];
#pragma unroll
        for (int j = 0; j < NT; ++j) src[j] = src_next[j];
        if (ia + 1 < ia1) {
          const int sn = wuni(meta[ia + 1 - ia0].s);
#pragma unroll
          for (int j = 0; j < NT; ++j) src_next[j] = gld(srcb + sn * kTileN + 16 * j + c16);
        }
        T* const Pw = lds + buf * 4 * NC * XS + kg * NC * XS;
        const T* bp[NT];
#pragma unroll
        for (int j = 0; j < NT; ++j)
          bp[j] = Wp + int64_t(src[j]) * ld + 4 * g;
        if (D > 0) {  // the host launches D > 0 only where nck <= D
          // the K-group's whole share of the gathered multipoles in
          // registers at once (one memory latency per offset, not per
          // chunk), then one rank tile after the other with the next
          // tile's factor fragments in flight
          T4 wv[D > 0 ? D : 1][NT], an[D > 0 ? D : 1];
          const T* a0 = P1 + off + lane * 4;
#pragma unroll
          for (int u = 0; u < D; ++u) {
#pragma unroll
            for (int j = 0; j < NT; ++j)
              wv[u][j] = u < nck ? gld(reinterpret_cast<const T4*>(bp[j] + 16 * (kg + 4 * u)))
                                 : T4{0, 0, 0, 0};
            an[u] = u < nck ? gld(reinterpret_cast<const T4*>(a0 + int64_t(kg + 4 * u) * 256))
                            : T4{0, 0, 0, 0};
          }
          for (int i = 0; i < nr; ++i) {
            T4 av[D > 0 ? D : 1];
#pragma unroll
            for (int u = 0; u < D; ++u) av[u] = an[u];
            if (kAPre && i + 1 < nr) {
              const T* an0 = a0 + int64_t(i + 1) * KC * 256;
#pragma unroll
              for (int u = 0; u < D; ++u)
                an[u] = u < nck ? gld(reinterpret_cast<const T4*>(an0 + int64_t(kg + 4 * u) * 256))
                                : T4{0, 0, 0, 0};
            }
            T4 x[NT];
#pragma unroll
            for (int j = 0; j < NT; ++j) x[j] = T4{0, 0, 0, 0};
#pragma unroll
            for (int u = 0; u < D; ++u) {
              if (u >= nck) continue;
#pragma unroll
              for (int st = 0; st < 4; ++st)
#pragma unroll
                for (int j = 0; j < NT; ++j)
                  if (on[j]) x[j] = mfma16x16x4(av[u][st], wv[u][j][st], x[j]);
            }
            if (!kAPre && i + 1 < nr) {
              const T* an0 = a0 + int64_t(i + 1) * KC * 256;
#pragma unroll
              for (int u = 0; u < D; ++u)
                an[u] = u < nck ? gld(reinterpret_cast<const T4*>(an0 + int64_t(kg + 4 * u) * 256))
                                : T4{0, 0, 0, 0};
            }
#pragma unroll
            for (int j = 0; j < NT; ++j) {
              T* xrow = Pw + (16 * j + c16) * XS + 16 * i;
              if (!F32) {
#pragma unroll
                for (int r = 0; r < 4; ++r) xrow[4 * r + g] = x[j][r];
              } else {
                *reinterpret_cast<T4*>(xrow + 4 * g) = x[j];
              }
            }
          }
        } else {
        for (int i0 = 0; i0 < nr; i0 += kRP) {
          const int np = min(kRP, nr - i0);
          const T* a0 = P1 + off + (int64_t(i0) * KC) * 256 + lane * 4;
          T4 x[kRP][NT];
#pragma unroll
          for (int i = 0; i < kRP; ++i)
#pragma unroll
            for (int j = 0; j < NT; ++j) x[i][j] = T4{0, 0, 0, 0};
          T4 bv[NT], av[kRP];
          if (kXPre && i0 == 0 && have_pre) {
#pragma unroll
            for (int j = 0; j < NT; ++j) bv[j] = pre_bv[j];
#pragma unroll
            for (int i = 0; i < kRP; ++i) av[i] = pre_av[i];
          } else if (kg < KC) {
#pragma unroll
            for (int j = 0; j < NT; ++j) bv[j] = gld(reinterpret_cast<const T4*>(bp[j] + 16 * kg));
#pragma unroll
            for (int i = 0; i < kRP; ++i)
              av[i] = i < np ? gld(reinterpret_cast<const T4*>(a0 + (int64_t(i) * KC + kg) * 256))
                             : T4{0, 0, 0, 0};
          }
          // chunks in flight: c + 4 (kLook = 1) or also c + 8 (kLook = 2)
          T4 b1[kLook > 1 ? NT : 1], a1[kLook > 1 ? kRP : 1];
          if (kLook > 1 && kg + 4 < KC) {
#pragma unroll
            for (int j = 0; j < NT; ++j)
              b1[kLook > 1 ? j : 0] = gld(reinterpret_cast<const T4*>(bp[j] + 16 * (kg + 4)));
#pragma unroll
            for (int i = 0; i < kRP; ++i)
              a1[kLook > 1 ? i : 0] =
                  i < np ? gld(reinterpret_cast<const T4*>(a0 + (int64_t(i) * KC + kg + 4) * 256))
                         : T4{0, 0, 0, 0};
          }
          for (int c = kg; c < KC; c += 4) {
            T4 bn[NT], an[kRP];
            const int cn = c + 4 * kLook;
            const bool more = cn < KC;
            if (more) {
#pragma unroll
              for (int j = 0; j < NT; ++j)
                bn[j] = gld(reinterpret_cast<const T4*>(bp[j] + 16 * cn));
#pragma unroll
              for (int i = 0; i < kRP; ++i)
                an[i] = i < np
                            ? gld(reinterpret_cast<const T4*>(a0 + (int64_t(i) * KC + cn) * 256))
                            : T4{0, 0, 0, 0};
            }
#pragma unroll
            for (int st = 0; st < 4; ++st)
#pragma unroll
              for (int i = 0; i < kRP; ++i)
#pragma unroll
                for (int j = 0; j < NT; ++j)
                  if (i < np && on[j]) x[i][j] = mfma16x16x4(av[i][st], bv[j][st], x[i][j]);
            if (kLook > 1) {
#pragma unroll
              for (int j = 0; j < NT; ++j) {
                bv[j] = b1[kLook > 1 ? j : 0];
                if (more) b1[kLook > 1 ? j : 0] = bn[j];
              }
#pragma unroll
              for (int i = 0; i < kRP; ++i) {
                av[i] = a1[kLook > 1 ? i : 0];
                if (more) a1[kLook > 1 ? i : 0] = an[i];
              }
            } else if (more) {
#pragma unroll
              for (int j = 0; j < NT; ++j) bv[j] = bn[j];
#pragma unroll
              for (int i = 0; i < kRP; ++i) av[i] = an[i];
            }
          }
          // D rows: FP32 item r -> row 4g + r, FP64 item r -> row 4r + g
#pragma unroll
          for (int i = 0; i < kRP; ++i)
#pragma unroll
            for (int j = 0; j < NT; ++j) {
              if (i >= np) continue;
              T* xrow = Pw + (16 * j + c16) * XS + 16 * (i0 + i);
              if (!F32) {
#pragma unroll
                for (int r = 0; r < 4; ++r) xrow[4 * r + g] = x[i][j][r];
              } else {
                *reinterpret_cast<T4*>(xrow + 4 * g) = x[i][j];
              }
            }
        }
        have_pre = false;
        if (kXPre && ia + 1 < ia1 && kg < KC) {
          const SvdMeta mn = meta[ia + 1 - ia0];
          const int npn = min(kRP, wuni(mn.nr_nst) & 0xffff);
          const T* an0 = P1 + wuni(mn.off) + lane * 4;
#pragma unroll
          for (int j = 0; j < NT; ++j)
            pre_bv[j] = gld(reinterpret_cast<const T4*>(Wp + int64_t(src_next[j]) * ld + 4 * g +
                                                        16 * kg));
#pragma unroll
          for (int i = 0; i < kRP; ++i)
            pre_av[i] = i < npn ? gld(reinterpret_cast<const T4*>(an0 + (int64_t(i) * KC + kg) * 256))
                                : T4{0, 0, 0, 0};
          have_pre = true;
        }
        }
      }
      buf ^= 1;
      __syncthreads();
    }
  }
}

template <typename T, int MTW, int NT, int NCW, bool GS>
__device__ inline void svd_ws_consume(const JobDev* __restrict__ jobs,
                                      const StepTab* __restrict__ tab, const T* const lds,
                                      SvdMeta* const meta, int wg) {
  typedef typename Vec4<T>::type T4;
  constexpr bool F32 = sizeof(T) == 4;
  constexpr int NC = 16 * NT;
  const int lane = threadIdx.x & 63, g = lane >> 4, c16 = lane & 15;
  const int total = step_total(*tab);
  int buf = 0;
  for (int it = blockIdx.x; it < total; it += gridDim.x) {
    SvdItem I;
    if (!svd_item<NT>(jobs, tab, it, total, I)) continue;
    const JobDev& J = *I.J;
    const M2LTile tl = I.tl;
    const int MT = J.mt, ld = J.ld, XS = J.xs;
    const int mt0 = (I.mb * NCW + wg) * MTW;
    const int nmt = mt0 < MT ? min(MTW, MT - mt0) : 0;
    const T* __restrict__ P2 = F32 ? reinterpret_cast<const T*>(J.p2_32)
                                   : reinterpret_cast<const T*>(J.p2_64);
    T4 acc[MTW][NT];
#pragma unroll
    for (int i = 0; i < MTW; ++i)
#pragma unroll
      for (int j = 0; j < NT; ++j) acc[i][j] = T4{0, 0, 0, 0};
    const int nact = wuni(gld(J.tile_nact + I.tile));
    bool folded = false;
    const unsigned char* act = J.tile_act + int64_t(I.tile) * kSlots;
    const int* kidp = J.slot_kid + tl.parity * kSlots;
    int ia0, ia1;
    svd_part_range(I, nact, ia0, ia1);
    svd_meta_fill<GS>(I, nact, meta);
    // the first U fragments (rank chunk 0) of the offset consumed next,
    // loaded before the barrier that precedes it
    constexpr int kCP = F32 ? FMM_M2L_SVD_WS_CPRE_F32 : FMM_M2L_SVD_WS_CPRE_F64;
    T4 cpre[kCP > 0 ? kCP : 1];
    for (int ia = ia0; ia <= ia1; ++ia) {
      if (ia > ia0 && nmt > 0) {
        // phase 2 of offset ia - 1 from the buffer the producers filled
        const int ic = ia - 1;
        const SvdMeta md = meta[ic - ia0];
        const int nrs = wuni(md.nr_nst);
        const int nr = nrs & 0xffff, nst = (nrs >> 16) & 0xff;  // rank chunks; K-steps of the last
        bool on[NT];
#pragma unroll
        for (int j = 0; j < NT; ++j) on[j] = !GS || ((nrs >> (24 + I.col0 / 16 + j)) & 1);
        const int64_t off = wuni(md.off);
        const T* const P = lds + (buf ^ 1) * 4 * NC * XS;
        const T* a2 = P2 + off + int64_t(mt0) * nr * 256 + lane * 4;
        for (int c = 0; c < nr; ++c) {
          T4 bv[NT];
#pragma unroll
          for (int j = 0; j < NT; ++j) {
            bv[j] = T4{0, 0, 0, 0};
            if (!on[j]) continue;
            const int o = (16 * j + c16) * XS + 16 * c + 4 * g;
            T4 v = *reinterpret_cast<const T4*>(P + o);
#pragma unroll
            for (int w = 1; w < 4; ++w) v += *reinterpret_cast<const T4*>(P + w * NC * XS + o);
            bv[j] = v;
          }
          // one U fragment live at a time; each accumulator still takes the
          // K-steps in order, and the steps past the kept rank (zeros in
          // both operands) are skipped
          const int ns = c + 1 < nr ? 4 : nst;
#pragma unroll
          for (int i = 0; i < MTW; ++i) {
            if (i >= nmt) continue;
            const T4 av = i < kCP && c == 0
                              ? cpre[i < kCP ? i : 0]
                              : gld(reinterpret_cast<const T4*>(a2 + (int64_t(i) * nr + c) * 256));
#pragma unroll
            for (int st = 0; st < 4; ++st) {
              if (st >= ns) continue;
#pragma unroll
              for (int j = 0; j < NT; ++j)
                if (on[j]) acc[i][j] = mfma16x16x4(av[st], bv[j][st], acc[i][j]);
            }
          }
        }
        if (F32 && ((ic - ia0 + 1) % J.fold_every == 0 || ic == ia1 - 1)) {
          // fold into this item's rows of Loc (scaled; the first fold
          // stores, later ones add): no other workgroup touches these rows
          const double sc = J.scale[tl.level];
#pragma unroll
          for (int j = 0; j < NT; ++j) {
            const int col = I.col0 + 16 * j + c16;
            if (col < tl.count) {
              double* out = svd_out_row(I, col);
#pragma unroll
              for (int i = 0; i < MTW; ++i) {
                if (i >= nmt) continue;
                d4* o = reinterpret_cast<d4*>(out + 16 * (mt0 + i) + 4 * g);  // rows 4g..4g+3
                d4 v;
#pragma unroll
                for (int r = 0; r < 4; ++r) v[r] = sc * double(acc[i][j][r]);
                if (folded) v += gld(o);
                gst(o, v);
              }
            }
#pragma unroll
            for (int i = 0; i < MTW; ++i) acc[i][j] = T4{0, 0, 0, 0};
          }
          folded = true;
        }
      }
      if (kCP > 0 && ia < ia1 && nmt > 0) {
        const SvdMeta mn = meta[ia - ia0];
        const int nrn = wuni(mn.nr_nst) & 0xffff;
        const T* a2n = P2 + wuni(mn.off) + int64_t(mt0) * nrn * 256 + lane * 4;
#pragma unroll
        for (int i = 0; i < kCP; ++i)
          cpre[i] = i < nmt ? gld(reinterpret_cast<const T4*>(a2n + int64_t(i) * nrn * 256))
                            : T4{0, 0, 0, 0};
      }
      buf ^= 1;
      __syncthreads();
    }
    if (nmt == 0 || (F32 && folded)) continue;
    const double sc = J.scale[tl.level];
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      const int col = I.col0 + 16 * j + c16;
      if (col >= tl.count) continue;
      double* out = svd_out_row(I, col);
#pragma unroll
      for (int i = 0; i < MTW; ++i) {
        if (i >= nmt) continue;
        const int base = 16 * (mt0 + i);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = F32 ? 4 * g + r : 4 * r + g;
          gst(out + base + row, sc * double(acc[i][j][r]));
        }
      }
    }
  }
}

template <typename T, int MTW, int NT, int D, int NCW, bool GS = false>
__global__ __launch_bounds__(64 * (4 + NCW), svd_ws_waves(NCW, NT * int(sizeof(T) / 4))) void m2l_svd_ws_kernel(
    const JobDev* __restrict__ jobs, const StepTab* __restrict__ tab) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  // the per-offset table first (a fixed size, so jobs of different slab
  // widths share one launch), then the two sets of slabs
  static_assert(kSvdMetaBytes % 16 == 0, "slabs stay 16-byte aligned");
  SvdMeta* const meta = reinterpret_cast<SvdMeta*>(lds_raw);
  T* const lds = reinterpret_cast<T*>(lds_raw + kSvdMetaBytes);
  // the role is uniform per wavefront: a scalar branch, no lane masking
  const int wave = wuni(int(threadIdx.x >> 6));
  if (wave < 4) {
    // producers issue ahead of the consumers on their SIMD, so that their
    // gathers are in flight while the consumers' MFMAs run (30M-particle
    // order-10 cube: M2L 4255 -> 4223 ms; the same at levels 1 to 3, while
    // raising the consumers instead costs 1.6%)
    __builtin_amdgcn_s_setprio(1);
    svd_ws_produce<T, NT, D, NCW, GS>(jobs, tab, lds, meta, wave);
  } else {
    svd_ws_consume<T, MTW, NT, NCW, GS>(jobs, tab, lds, meta, wave - 4);
  }
}

// M-tiles per wavefront for the compressed kernel: the whole output in one
// M-block when it fits NWV x 6 tiles (phase 1 then runs once per N-group).
// Whether the warp-specialised kernel runs (FP32, FP64).
#ifndef FMM_M2L_SVD_WS_F32
#define FMM_M2L_SVD_WS_F32 1
#endif
#ifndef FMM_M2L_SVD_WS_F64
#define FMM_M2L_SVD_WS_F64 1
#endif
// Warp-specialised kernel: when NWV consumers of up to 6 M-tiles cannot
// hold all l^3 rows (l >= 8), 8 consumers of up to 8 M-tiles take them in
// one M-block instead of several, each of which would repeat phase 1.
#ifndef FMM_M2L_SVD_WIDE
#define FMM_M2L_SVD_WIDE 1
#endif
constexpr int kSvdWideMtw = 8;
// FP32, warp-specialised: where the slabs of all 64 columns of a tile fit
// the LDS, one item takes the whole tile (NT = 4) with 8 consumers of up to
// 6 M-tiles, so that each operator chunk is read once per tile rather than
// once per 32-column half (M2L time on gfx950: order 7 -2.2%, order 8
// -6.8%).  Beyond 6 M-tiles NT = 4 spills, and the shapes above take over;
// at 16 M-tiles or fewer (l <= 6) the 32-column items are as fast (l = 6)
// or faster (l = 5: by 9%).
#ifndef FMM_M2L_SVD_FULL_F32
#define FMM_M2L_SVD_FULL_F32 1
#endif
// FP64 likewise with 32-column items (NT = 2) where they fit: fp64_svd M2L
// order 7 9.0 -> 8.3 ms, order 8 16.0 -> 13.6 ms (order 9 at 1e-9 needs
// 168 KiB and keeps 16 columns).
#ifndef FMM_M2L_SVD_FULL_F64
#define FMM_M2L_SVD_FULL_F64 1
#endif
constexpr int kSvdFullNt = 4, kSvdFullNt64 = 2, kSvdFullMtw = 6;
constexpr int svd_full_nt(bool fp32) { return fp32 ? kSvdFullNt : kSvdFullNt64; }
constexpr size_t kSvdLdsMax = 160 * 1024;  // LDS per workgroup on gfx950

struct SvdShape {
  int ncw, mtw, nt;  // consumer wavefronts (compressed kernel: wavefronts), M-tiles each,
                     // 16-column N-tiles per item
};

size_t m2l_svd_lds_bytes(int xs, bool fp32, int nt) {
  return size_t(2) * 4 * 16 * nt * xs * (fp32 ? sizeof(float) : sizeof(double)) + kSvdMetaBytes;
}

static SvdShape m2l_svd_shape(int mt, bool fp32, int xs) {
  const int nw = svd_nwv(fp32), nt = svd_nt(fp32);
  const bool ws = fp32 ? FMM_M2L_SVD_WS_F32 : FMM_M2L_SVD_WS_F64;
  const int fnt = svd_full_nt(fp32);
  const bool full = fp32 ? FMM_M2L_SVD_FULL_F32 : FMM_M2L_SVD_FULL_F64;
  if (ws && full && nt < fnt && mt > 16 && 8 * kSvdFullMtw >= mt &&
      m2l_svd_lds_bytes(xs, fp32, fnt) <= kSvdLdsMax)
    for (int w = 1; w <= kSvdFullMtw; ++w)
      if (8 * w >= mt) return {8, w, fnt};
  for (int w = 1; w <= 6; ++w)
    if (nw * w >= mt) return {nw, w, nt};
  if (ws && FMM_M2L_SVD_WIDE && nw < 8)
    for (int w = 4; w <= kSvdWideMtw; ++w)
      if (8 * w >= mt) return {8, w, nt};
  return ws && FMM_M2L_SVD_WIDE && nw < 8 ? SvdShape{8, kSvdWideMtw, nt} : SvdShape{nw, 6, nt};
}

static int svd_kc(int order) { return (order * order * order + 15) / 16; }

int m2l_svd_nt(int order, bool fp32, int xs) { return m2l_svd_shape(svd_kc(order), fp32, xs).nt; }

int m2l_svd_nmb(int mt, bool fp32, int xs) {
  const SvdShape sh = m2l_svd_shape(mt, fp32, xs);
  return (mt + sh.ncw * sh.mtw - 1) / (sh.ncw * sh.mtw) * (4 / sh.nt);
}

// Slab row stride: the padded rank plus 16 bytes, so that consecutive target
// columns start 16 bytes apart modulo the LDS banks.
int m2l_svd_xs(int rmax_pad, bool fp32) { return rmax_pad + (fp32 ? 4 : 2); }

size_t m2l_svd_lds_need(int order, bool fp32, int xs) {
  return m2l_svd_lds_bytes(xs, fp32, m2l_svd_shape(svd_kc(order), fp32, xs).nt);
}

// With the warp-specialised kernel, NWV counts the consumer wavefronts (the
// workgroup has 4 more).

template <typename T, int MTW, int NT, int NCW>
static const void* svd_ws_ptr(bool gs = false) {
  return gs ? reinterpret_cast<const void*>(&m2l_svd_ws_kernel<T, MTW, NT, 0, NCW, true>)
            : reinterpret_cast<const void*>(&m2l_svd_ws_kernel<T, MTW, NT, 0, NCW>);
}

// The warp-specialised kernel of a shape; staged selects the stage depth
// FMM_M2L_SVD_WS_STAGE_* of the NWV-consumer shape, gs the form that skips
// empty 16-target groups (whole-tile and 8-consumer shapes).
template <typename T>
static const void* svd_ws_fn(SvdShape sh, bool staged, bool gs) {
  constexpr int NT = svd_nt(sizeof(T) == 4), NW = svd_nwv(sizeof(T) == 4);
  constexpr int D = sizeof(T) == 4 ? FMM_M2L_SVD_WS_STAGE_F32 : FMM_M2L_SVD_WS_STAGE_F64;
  const int mtw = sh.mtw;
  constexpr int FNT = svd_full_nt(sizeof(T) == 4);
  constexpr bool FULL = sizeof(T) == 4 ? FMM_M2L_SVD_FULL_F32 : FMM_M2L_SVD_FULL_F64;
  if constexpr (FULL && NT < FNT) {
    if (sh.nt == FNT) {
      switch (mtw) {
        case 1: return svd_ws_ptr<T, 1, FNT, 8>(gs);
        case 2: return svd_ws_ptr<T, 2, FNT, 8>(gs);
        case 3: return svd_ws_ptr<T, 3, FNT, 8>(gs);
        case 4: return svd_ws_ptr<T, 4, FNT, 8>(gs);
        case 5: return svd_ws_ptr<T, 5, FNT, 8>(gs);
        default: return svd_ws_ptr<T, kSvdFullMtw, FNT, 8>(gs);
      }
    }
  }
  if (sh.ncw == 8 && NW != 8) {
    switch (mtw) {
      case 4: return svd_ws_ptr<T, 4, NT, 8>(gs);
      case 5: return svd_ws_ptr<T, 5, NT, 8>(gs);
      case 6: return svd_ws_ptr<T, 6, NT, 8>(gs);
      case 7: return svd_ws_ptr<T, 7, NT, 8>(gs);
      default: return svd_ws_ptr<T, kSvdWideMtw, NT, 8>(gs);
    }
  }
#define FMM_WS_FN(M)                                                                     \
  return staged ? reinterpret_cast<const void*>(&m2l_svd_ws_kernel<T, M, NT, D, NW>)    \
                : svd_ws_ptr<T, M, NT, NW>()
  switch (mtw) {
    case 1: FMM_WS_FN(1);
    case 2: FMM_WS_FN(2);
    case 3: FMM_WS_FN(3);
    case 4: FMM_WS_FN(4);
    case 5: FMM_WS_FN(5);
    default: FMM_WS_FN(6);
  }
#undef FMM_WS_FN
}

template <typename T, int FOLD>
static void launch_svd_mtw(SvdShape sh, int kc, const JobDev* jobs, const StepTab* tab, int grid,
                           size_t lds, hipStream_t s, bool gs) {
  constexpr int NT = svd_nt(sizeof(T) == 4), NW = svd_nwv(sizeof(T) == 4), B = 64 * NW;
  constexpr bool WS = sizeof(T) == 4 ? FMM_M2L_SVD_WS_F32 : FMM_M2L_SVD_WS_F64;
  if (WS) {
    constexpr int D = sizeof(T) == 4 ? FMM_M2L_SVD_WS_STAGE_F32 : FMM_M2L_SVD_WS_STAGE_F64;
    const bool staged = D > 0 && (kc + 3) / 4 <= D && sh.ncw == NW && sh.nt == NT;
    const void* f = svd_ws_fn<T>(sh, staged, gs);
    void* args[] = {&jobs, &tab};
    FMM_HIP_CHECK(hipLaunchKernel(f, dim3(grid), dim3(64 * (4 + sh.ncw)), args, lds, s));
    return;
  }
  switch (sh.mtw) {
    case 1: m2l_svd_kernel<T, 1, NT, NW, FOLD><<<grid, B, lds, s>>>(jobs, tab); break;
    case 2: m2l_svd_kernel<T, 2, NT, NW, FOLD><<<grid, B, lds, s>>>(jobs, tab); break;
    case 3: m2l_svd_kernel<T, 3, NT, NW, FOLD><<<grid, B, lds, s>>>(jobs, tab); break;
    case 4: m2l_svd_kernel<T, 4, NT, NW, FOLD><<<grid, B, lds, s>>>(jobs, tab); break;
    case 5: m2l_svd_kernel<T, 5, NT, NW, FOLD><<<grid, B, lds, s>>>(jobs, tab); break;
    default: m2l_svd_kernel<T, 6, NT, NW, FOLD><<<grid, B, lds, s>>>(jobs, tab); break;
  }
}

bool m2l_svd_splits(bool fp32) { return fp32 ? FMM_M2L_SVD_WS_F32 : FMM_M2L_SVD_WS_F64; }

int m2l_svd_slots(int order, bool fp32, int xs) {
  const int kc = svd_kc(order);
  const SvdShape sh = m2l_svd_shape(kc, fp32, xs);
  const int D = fp32 ? FMM_M2L_SVD_WS_STAGE_F32 : FMM_M2L_SVD_WS_STAGE_F64;
  const bool staged =
      D > 0 && (kc + 3) / 4 <= D && sh.ncw == svd_nwv(fp32) && sh.nt == svd_nt(fp32);
  const void* f = fp32 ? svd_ws_fn<float>(sh, staged, false) : svd_ws_fn<double>(sh, staged, false);
  int per_cu = 0, dev = 0, cus = 0;
  FMM_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per_cu, f, 64 * (4 + sh.ncw), m2l_svd_lds_bytes(xs, fp32, sh.nt)));
  FMM_HIP_CHECK(hipGetDevice(&dev));
  FMM_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  return std::max(1, per_cu) * std::max(1, cus);
}

void launch_m2l_svd_step(int order, bool fp32, const JobDev* jobs, const StepTab* tab, int grid,
                         int xs, hipStream_t s, bool gskip) {
  const int kc = svd_kc(order);
  const SvdShape sh = m2l_svd_shape(kc, fp32, xs);
  const size_t lds = m2l_svd_lds_bytes(xs, fp32, sh.nt);
  if (fp32)
    launch_svd_mtw<float, FMM_M2L_SVD_F32_FOLD_MODE>(sh, kc, jobs, tab, grid, lds, s, gskip);
  else
    launch_svd_mtw<double, 0>(sh, kc, jobs, tab, grid, lds, s, gskip);
  FMM_HIP_CHECK(hipGetLastError());
}

}  // namespace fmm
