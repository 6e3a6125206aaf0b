// Mutual near field (the reduction form of the P2P kernel, Sec. 5: each pair
// of neighbour leaves is computed once and feeds both).
//
// A work item is a pair of distinct neighbour leaves (A, B), with B at a
// forward offset of A (plan.hip builds the 26 pair lists; within one list no
// two pairs share a leaf, so an item owns the outputs of both leaves).  The
// leaves' own pairs are taken beforehand by the one-sided kernel restricted
// to the leaf itself, which writes the outputs; every item adds to them.
//
// One wavefront per item.  A's particles (up to 64 at a time) sit in the
// lanes; a chunk of up to 64 of B's is staged in LDS twice over, slots j and
// 64 + j, so that lane l reads B's particle (l + s) mod 64 at step s without
// a wrap.  Step s computes the pair (A_l, B_{(l+s) mod 64}) once: A's terms
// go to lane l's sums, and B's terms to B's sums, which travel with B's
// particle: before every step each lane takes the B sums of the lane above
// (a DPP rotation of the wavefront, folded into the add), so that at step s
// lane l holds the sums of the particle it reads.  A pair (a, b) of the
// chunks comes up at the step s = b - a mod 64; with ca and cb particles the
// differences run from 1 - ca to cb - 1, so min(64, ca + cb - 1) steps from
// s = 1 - ca cover every pair once.  The steps go eight at a time: the extra
// ones pair a padding slot (no charge, far away) with every lane and add
// zeros.
//
// Arithmetic as in the one-sided kernel: FP64 differences, then FP32 (mixed
// modes) or FP64 for r^2, the reciprocal (square) root and the products; the
// FP32 sums over one chunk are folded into FP64 once per chunk pair.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_util.h"
#include "fmm_internal.h"
#include "jobs.h"

namespace fmm {
namespace {

typedef double src4 __attribute__((ext_vector_type(4)));  // x, y, z, q of one B particle

constexpr int kUnroll = 8;
// padding particles: A's at +kPad, B's at -kPad, so that no two coincide and
// every pair with a padding particle has an infinite (FP32) or huge (FP64)
// distance and a zero charge on the padding side
constexpr double kPad = 1e30;
constexpr int kRol1 = 0x134;  // DPP wavefront rotation: lane i reads lane i + 1 (mod 64)

__device__ __forceinline__ double q_slot(float q) {
  return __longlong_as_double(static_cast<long long>(__float_as_uint(q)));
}
__device__ __forceinline__ float q_of_slot(double d) {
  return __uint_as_float(static_cast<unsigned>(__double_as_longlong(d)));
}

// the value of lane (i + 1) mod 64; zero-filled form so that the compiler
// folds it into the add that follows
__device__ __forceinline__ float rot(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), kRol1, 0xf, 0xf, true));
}
__device__ __forceinline__ double rot(double v) {
  const long long u = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, int(u), kRol1, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, int(u >> 32), kRol1, 0xf, 0xf, true);
  return __builtin_bit_cast(double, (static_cast<long long>(hi) << 32) |
                                        static_cast<long long>(static_cast<unsigned>(lo)));
}

// acc from the lane above, plus (minus) t: one DPP add (no contraction with the
// product that forms t, which would keep the rotation a separate move)
__device__ __forceinline__ float rot_add(float acc, float t) {
#pragma clang fp contract(off)
  return rot(acc) + t;
}
__device__ __forceinline__ double rot_add(double acc, double t) { return rot(acc) + t; }
__device__ __forceinline__ float rot_sub(float acc, float t) {
#pragma clang fp contract(off)
  return rot(acc) - t;
}
__device__ __forceinline__ double rot_sub(double acc, double t) { return rot(acc) - t; }

// Sums of one side: potential and field (the force without the particle's
// own charge).
template <typename T>
struct Acc {
  T p, x, y, z;
};

// One pair for the kernel |x - y|^-KP: d = x_a - x_b; A gains q_b r^-KP and
// KP q_b r^-(KP+2) d, B gains q_a r^-KP and -KP q_a r^-(KP+2) d, B's sums
// arriving from the lane above first.
template <int KP, typename T>
__device__ __forceinline__ void mutual_pair(T dx, T dy, T dz, T qa, T qb, Acc<T>& A, Acc<T>& B) {
  const T r2 = dx * dx + dy * dy + dz * dz;
  T ir2, ira, irb;
  if constexpr (sizeof(T) == 4) {
    if (KP == 2) {
      ir2 = __builtin_amdgcn_rcpf(r2);
      ira = irb = ir2;
    } else {
      const T ir = __builtin_amdgcn_rsqf(r2);
      ir2 = ir * ir;
      ira = irb = ir;
    }
  } else {
    if (KP == 2) {
      ir2 = 1.0 / r2;
      ira = irb = ir2;
    } else {
      const T ir = rsqrt(r2);
      ir2 = ir * ir;
      ira = irb = ir;
    }
  }
  const T ta = qb * ira, tb = qa * irb;
  const T sa = (KP == 2 ? T(2) * ta : ta) * ir2;
  const T sb = (KP == 2 ? T(2) * tb : tb) * ir2;
  A.p += ta;
  A.x += sa * dx;
  A.y += sa * dy;
  A.z += sa * dz;
  B.p = rot_add(B.p, tb);
  B.x = rot_sub(B.x, sb * dx);
  B.y = rot_sub(B.y, sb * dy);
  B.z = rot_sub(B.z, sb * dz);
}

template <int KP, bool F32>
__device__ __forceinline__ void mutual_item(const JobDev& J, int a, int b, src4* src) {
  typedef typename std::conditional<F32, float, double>::type T;
  const int lane = threadIdx.x;
  const double *px = J.px, *py = J.py, *pz = J.pz;
  const int a0 = wuni(gld(J.leaf_start + a)), na = wuni(gld(J.leaf_start + a + 1)) - a0;
  const int b0 = wuni(gld(J.leaf_start + b)), nb = wuni(gld(J.leaf_start + b + 1)) - b0;
  for (int ia = 0; ia < na; ia += 64) {
    const int ca = min(64, na - ia);
    const bool va = lane < ca;
    const int i = a0 + ia + lane;
    double xa = kPad, ya = kPad, za = kPad;
    T qa = 0;
    if (va) {
      xa = gld(px + i);
      ya = gld(py + i);
      za = gld(pz + i);
      qa = F32 ? T(gld(&J.prel[i].w)) : T(gld(J.qs + i));
    }
    Acc<double> A64{0.0, 0.0, 0.0, 0.0};
    for (int jb = 0; jb < nb; jb += 64) {
      const int cb = min(64, nb - jb);
      const int j = b0 + jb + lane;
      src4 u{-kPad, -kPad, -kPad, F32 ? q_slot(0.f) : 0.0};
      if (lane < cb) {
        u.x = gld(px + j);
        u.y = gld(py + j);
        u.z = gld(pz + j);
        u.w = F32 ? q_slot(gld(&J.prel[j].w)) : gld(J.qs + j);
      }
      __syncthreads();  // the previous chunk's reads (and output updates) are done
      src[lane] = u;
      src[64 + lane] = u;
      __syncthreads();
      const int steps = min(64, (ca + cb - 1 + kUnroll - 1) / kUnroll * kUnroll);
      const int s0 = (65 - ca) & 63;
      const src4* row = src + ((lane + s0) & 63);
      Acc<T> As{0, 0, 0, 0}, Bs{0, 0, 0, 0};
      for (int st = 0; st < steps; st += kUnroll) {
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) {
          const src4 v = row[st + k];
          const T qb = F32 ? T(q_of_slot(v.w)) : T(v.w);
          mutual_pair<KP, T>(T(xa - v.x), T(ya - v.y), T(za - v.z), qa, qb, As, Bs);
        }
      }
      A64.p += double(As.p);
      A64.x += double(As.x);
      A64.y += double(As.y);
      A64.z += double(As.z);
      // lane l now holds the sums of B's slot (l + s0 + steps - 1) mod 64
      const int sb = (lane + s0 + steps - 1) & 63;
      if (sb < cb) {
        const int jj = b0 + jb + sb;
        const double qj = gld(J.qs + jj);
        const int64_t j3 = 3 * int64_t(jj);
        gst(J.phi_n + jj, gld(J.phi_n + jj) + double(Bs.p));
        gst(J.f_n + j3, gld(J.f_n + j3) + qj * double(Bs.x));
        gst(J.f_n + j3 + 1, gld(J.f_n + j3 + 1) + qj * double(Bs.y));
        gst(J.f_n + j3 + 2, gld(J.f_n + j3 + 2) + qj * double(Bs.z));
      }
    }
    if (va) {
      const double qi = gld(J.qs + i);
      const int64_t i3 = 3 * int64_t(i);
      gst(J.phi_n + i, gld(J.phi_n + i) + A64.p);
      gst(J.f_n + i3, gld(J.f_n + i3) + qi * A64.x);
      gst(J.f_n + i3 + 1, gld(J.f_n + i3 + 1) + qi * A64.y);
      gst(J.f_n + i3 + 2, gld(J.f_n + i3 + 2) + qi * A64.z);
    }
  }
}

// Block = one wavefront = one pair (list[blockIdx.x], its neighbour in the
// forward slot `slot`).
template <bool F32>
__global__ __launch_bounds__(64) void p2p_mutual_kernel(const JobDev* __restrict__ job,
                                                        const int* __restrict__ list, int slot) {
  __shared__ src4 src[128];
  const JobDev& J = *job;
  const int a = wuni(gld(list + blockIdx.x));
  const int b = wuni(gld(J.near + 27 * a + slot));
  if (J.kernel == 2)
    mutual_item<2, F32>(J, a, b, src);
  else
    mutual_item<1, F32>(J, a, b, src);
}

}  // namespace

void launch_p2p_mutual(const fmm_plan_s* p, bool fp32, hipStream_t s) {
  for (int k = 0; k < 2 * kMutualSlots; ++k) {
    const int64_t lo = p->mutual_off[k], cnt = p->mutual_off[k + 1] - lo;
    if (cnt <= 0) continue;
    const int slot = kMutualFirstSlot + k / 2;
    if (fp32)
      p2p_mutual_kernel<true><<<unsigned(cnt), 64, 0, s>>>(p->job_d, p->mutual_list + lo, slot);
    else
      p2p_mutual_kernel<false><<<unsigned(cnt), 64, 0, s>>>(p->job_d, p->mutual_list + lo, slot);
    FMM_HIP_CHECK(hipGetLastError());
  }
}

}  // namespace fmm
