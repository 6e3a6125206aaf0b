// Evaluation kernels: P2M, M2M, L2L, L2P, P2P, gather and combine.
//
// Interpolation (Sec. 2.1, Eq. 3-5): S(xb_m; u) = 1/l + 2/l sum_{n=1}^{l-1}
// T_n(xb_m) T_n(u), tensorised over x, y, z (Eq. 4).  With the table
// C[m][n] = (n == 0 ? 1 : 2 T_n(xb_m)) / l this is S_m(u) = sum_n C[m][n] T_n(u)
// (the outer-product form of Sec. 2.1.1: O(l^3) per particle).  M2M and L2L
// apply the child-to-parent interpolation as three 1-D l x l contractions
// (Sec. 2.1.1, O(l^4) per cell).
//
// Every kernel walks the items of a StepTab (one or many plans, see jobs.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <vector>

#include "device_util.h"
#include "fmm_internal.h"
#include "jobs.h"

namespace fmm {

#define FOR_ITEMS(tab)                                                   \
  for (int it_ = blockIdx.x, tot_ = step_total(*(tab)); it_ < tot_;      \
       it_ += gridDim.x)

__device__ inline void leaf_centre(const LeafGeom& g, uint64_t key, double* c) {
  int k[3];
  demorton3(key, g.bits, k);
  c[0] = g.lo0 + (k[0] + 0.5) * g.w;
  c[1] = g.lo1 + (k[1] + 0.5) * g.w;
  c[2] = g.lo2 + (k[2] + 0.5) * g.w;
}

// ------------------------------------------------------------------- P2M
// Item = leaf.  Thread (m1, m2) accumulates the l coefficients W[m1][m2][*]
// over the leaf's particles: W += q Sx[m1] Sy[m2] Sz[*].
constexpr int kP2MChunk = 64;

// Minimum wavefronts per SIMD the register allocation of P2M and L2P must
// allow (0: the compiler's choice).
#ifndef FMM_P2M_WAVES
#define FMM_P2M_WAVES 0
#endif
#ifndef FMM_L2P_WAVES
#define FMM_L2P_WAVES 0
#endif
#if FMM_P2M_WAVES > 0
#define FMM_P2M_BOUNDS __launch_bounds__(256, FMM_P2M_WAVES)
#else
#define FMM_P2M_BOUNDS __launch_bounds__(256)
#endif
#if FMM_L2P_WAVES > 0
#define FMM_L2P_BOUNDS __launch_bounds__(64, FMM_L2P_WAVES)
#else
#define FMM_L2P_BOUNDS __launch_bounds__(64)
#endif

template <int L>
__global__ FMM_P2M_BOUNDS void p2m_kernel(const JobDev* __restrict__ jobs,
                                                  const StepTab* __restrict__ tab) {
  __shared__ double C[L * L];
  __shared__ double S[kP2MChunk][3][L];
  const int t = threadIdx.x, nt = blockDim.x;
  const int m1 = t / L, m2 = t % L;
  const bool owner = t < L * L;
  FOR_ITEMS(tab) {
    const int k = step_find(*tab, it_);
    const JobDev& J = jobs[tab->job[k]];
    const int a = it_ - tab->start[k];
    for (int e = t; e < L * L; e += nt) C[e] = J.cheb[e];
    double c[3];
    leaf_centre(J.geo, J.leaf_keys[a], c);
    const double ia = 2.0 / J.geo.w;
    double acc[L];
    for (int e = 0; e < L; ++e) acc[e] = 0.0;
    const int s0 = wuni(gld(J.leaf_start + a)), s1 = wuni(gld(J.leaf_start + a + 1));
    __syncthreads();
    for (int base = s0; base < s1; base += kP2MChunk) {
      const int cnt = min(kP2MChunk, s1 - base);
      for (int e = t; e < 3 * cnt; e += nt) {
        const int j = e / 3, d = e % 3;
        const int i = base + j;
        const double x = gld(d == 0 ? J.px + i : (d == 1 ? J.py + i : J.pz + i));
        const double u = (x - c[d]) * ia;
        double T[L];
        T[0] = 1.0;
        if (L > 1) T[1] = u;
        for (int n = 2; n < L; ++n) T[n] = 2.0 * u * T[n - 1] - T[n - 2];
        const double f = d == 0 ? gld(J.qs + i) : 1.0;
        // one row of C at a time (unrolled, the compiler holds all l^2 of
        // them: 256 VGPRs at order 10, one wavefront per SIMD)
#pragma unroll 1
        for (int m = 0; m < L; ++m) {
          double v = 0.0;
          for (int n = 0; n < L; ++n) v += C[m * L + n] * T[n];
          S[j][d][m] = f * v;
        }
      }
      __syncthreads();
      if (owner)
        for (int j = 0; j < cnt; ++j) {
          const double f = S[j][0][m1] * S[j][1][m2];
          for (int m3 = 0; m3 < L; ++m3) acc[m3] += f * S[j][2][m3];
        }
      __syncthreads();
    }
    const int64_t row = (J.lev_off[J.height - 1] + a) * int64_t(J.ld);
    if (J.w32_leaf) {
      // mixed modes keep the leaf multipoles in FP32 only
      float* out = J.W32 + row;
      if (owner)
        for (int m3 = 0; m3 < L; ++m3) gst(out + (m1 * L + m2) * L + m3, float(acc[m3]));
      for (int e = L * L * L + t; e < J.ld; e += nt) gst(out + e, 0.f);
    } else {
      double* out = J.W + row;
      if (owner)
        for (int m3 = 0; m3 < L; ++m3) gst(out + (m1 * L + m2) * L + m3, acc[m3]);
      for (int e = L * L * L + t; e < J.ld; e += nt) gst(out + e, 0.0);
    }
  }
}

// ------------------------------------------------------------- M2M / L2L
// Three 1-D contractions with the child-to-parent matrices
// Sc[s][m][m'] = S(xb_m; (s + xb_m')/2), s in {-1,+1} by the child octant bit
// (Eq. 5 applied per dimension).  One wavefront per child: the child's l^3
// values sit in LDS, each lane keeps whole lines of l values in registers,
// and the matrix rows are read as wavefront-wide broadcasts, so that a
// contraction reads every value once rather than once per output (the form
// with one LDS operand per FMA was bound by LDS bandwidth at orders 7 to 10).
// Every output is summed over q in increasing order from zero, and the
// children of a cell in key order, as in the paper's one-child-at-a-time
// form.
constexpr int kTransThreads = 512;  // one wavefront per child of a cell

// Orders the LDS accesses of every lane of this wavefront before the call
// ahead of those after it.  The hardware performs a wavefront's LDS accesses
// in order; the fences keep the compiler from reusing a value loaded before
// them or moving an access across them, which it may otherwise do whenever
// it can show that no access of the lane itself conflicts (the rotated
// contraction below reads what other lanes wrote).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// out[m][a][b] = sum_q M[m][q] in[a][b][q] for one L^3 cube: a contraction
// along the last index whose result has its indices rotated, so that the
// next one again runs along the last index (three restore the order).  M is
// row-major in LDS.  One wavefront: lane takes lines a L + b = lane + 64 r;
// every lane reads all its lines before any lane writes (so `out` may be
// `in`), and each output goes to `emit` with its index m L^2 + a L + b and
// its (m, round).
template <int L, typename Emit>
__device__ __forceinline__ void rot_contract(const double* in, const double* M, int lane,
                                             Emit emit) {
  constexpr int L2 = L * L, R = (L2 + 63) / 64;
  double v[R][L];
  wave_lds_sync();  // the previous contraction's writes, from every lane
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int line = lane + 64 * r;
#pragma unroll
    for (int q = 0; q < L; ++q) v[r][q] = line < L2 ? in[line * L + q] : 0.0;
  }
  wave_lds_sync();  // every line read before the first write
#pragma unroll
  for (int m = 0; m < L; ++m) {
    double row[L];
#pragma unroll
    for (int q = 0; q < L; ++q) row[q] = M[m * L + q];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int line = lane + 64 * r;
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < L; ++q) acc += row[q] * v[r][q];
      if (line < L2) emit(m * L2 + line, acc, m, r);
    }
  }
}

// Dynamic LDS (doubles): M2M one cube per child; L2L the parent's cube and
// one per child.  The matrices (both octant signs, and for L2L transposed)
// take 2 l^2 more.
size_t m2m_lds_bytes(int L) { return sizeof(double) * size_t(8 * L * L * L + 2 * L * L); }
size_t l2l_lds_bytes(int L) { return sizeof(double) * size_t(9 * L * L * L + 2 * L * L); }

// Parent cell p at level lv: W_p = sum over children c (key order) of
// (Sx (x) Sy (x) Sz)_c W_c.
template <int L>
__device__ void m2m_item(const JobDev& J, int lv, int p, double* lds) {
  constexpr int L2 = L * L, L3 = L2 * L;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  double* const Sc = lds;  // Sc[s][m][q]
  double* const X = lds + 2 * L2;
  const int ld = J.ld;
  const int c0 = J.child_start[lv][p], nc = J.child_start[lv][p + 1] - c0;
  for (int e = t; e < 2 * L2; e += kTransThreads) Sc[e] = J.child[e];
  double* const Xw = X + w * L3;
  int oct = 0;
  if (w < nc) {
    oct = wuni(int(gld(J.keys[lv + 1] + c0 + w) & 7u));
    const int64_t crow = (J.lev_off[lv + 1] + c0 + w) * int64_t(ld);
    // all of the child's loads in flight at once (a loop bounded at run time
    // waits for each before issuing the next); leaf children of the mixed
    // modes are stored in FP32, the contraction is FP64
    constexpr int NE = (L3 + 63) / 64;
    double v[NE];
    if (J.w32_leaf && lv + 1 == J.height - 1) {
#pragma unroll
      for (int k = 0; k < NE; ++k)
        v[k] = lane + 64 * k < L3 ? double(gld(J.W32 + crow + lane + 64 * k)) : 0.0;
    } else {
#pragma unroll
      for (int k = 0; k < NE; ++k) v[k] = lane + 64 * k < L3 ? gld(J.W + crow + lane + 64 * k) : 0.0;
    }
#pragma unroll
    for (int k = 0; k < NE; ++k)
      if (lane + 64 * k < L3) Xw[lane + 64 * k] = v[k];
  }
  __syncthreads();
  if (w < nc) {
    auto to_x = [&](int i, double v, int, int) { Xw[i] = v; };
    rot_contract<L>(Xw, Sc + ((oct >> 2) & 1) * L2, lane, to_x);  // along z
    rot_contract<L>(Xw, Sc + ((oct >> 1) & 1) * L2, lane, to_x);  // along y
    rot_contract<L>(Xw, Sc + (oct & 1) * L2, lane, to_x);         // along x
  }
  __syncthreads();
  double* out = J.W + (J.lev_off[lv] + p) * int64_t(ld);
  for (int e = t; e < L3; e += kTransThreads) {
    double acc = 0.0;
    for (int cc = 0; cc < nc; ++cc) acc += X[cc * L3 + e];
    out[e] = acc;
  }
  for (int e = L3 + t; e < ld; e += kTransThreads) out[e] = 0.0;
  __syncthreads();
}

// Item = parent cell at level tab->level[k]; every plan of the launch has
// order L.
template <int L>
__global__ __launch_bounds__(kTransThreads) void m2m_kernel(const JobDev* __restrict__ jobs,
                                                            const StepTab* __restrict__ tab) {
  extern __shared__ double dyn_lds[];
  FOR_ITEMS(tab) {
    const int k = step_find(*tab, it_);
    m2m_item<L>(jobs[tab->job[k]], tab->level[k], it_ - tab->start[k], dyn_lds);
  }
}

// Parent cell p at level lv - 1: every child c (level lv) gets
// Loc_c += (Sx (x) Sy (x) Sz)_c^T Loc_p on node values, or the exact
// re-expansion (Rx (x) Ry (x) Rz)_c Loc_p on Chebyshev coefficients.
template <int L>
__device__ void l2l_item(const JobDev& J, int lv, int p, double* lds) {
  constexpr int L2 = L * L, L3 = L2 * L;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  // node values: St[s][m][q] = Sc[s][q][m]; Chebyshev coefficients (the
  // mixed modes): the re-expansion R_s[m][q] on the child's interval
  double* const St = lds;
  double* const P = lds + 2 * L2;
  double* const X = P + L3;
  const int ld = J.ld;
  const bool modal = wuni(J.modal);
  for (int e = t; e < 2 * L2; e += kTransThreads) {
    const int s = e / L2, m = (e / L) % L, q = e % L;
    St[e] = modal ? J.child_modal[e] : J.child[s * L2 + q * L + m];
  }
  const double* lp = J.Loc + (J.lev_off[lv - 1] + p) * int64_t(ld);
  {
    constexpr int NE = (L3 + kTransThreads - 1) / kTransThreads;
    double v[NE];
#pragma unroll
    for (int k = 0; k < NE; ++k) v[k] = t + kTransThreads * k < L3 ? gld(lp + t + kTransThreads * k) : 0.0;
#pragma unroll
    for (int k = 0; k < NE; ++k)
      if (t + kTransThreads * k < L3) P[t + kTransThreads * k] = v[k];
  }
  const int c0 = J.child_start[lv - 1][p], nc = J.child_start[lv - 1][p + 1] - c0;
  __syncthreads();
  if (w < nc) {
    const int oct = wuni(int(gld(J.keys[lv] + c0 + w) & 7u));
    double* const Xw = X + w * L3;
    double* const out = J.Loc + (J.lev_off[lv] + c0 + w) * int64_t(ld);
    // the child's expansion where this lane adds to it in the last pass,
    // loaded before the passes so that the adds do not wait on memory
    constexpr int R = (L2 + 63) / 64;
    double cur[R][L];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int m = 0; m < L; ++m)
        cur[r][m] = lane + 64 * r < L2 ? gld(out + m * L2 + lane + 64 * r) : 0.0;
    auto to_x = [&](int i, double v, int, int) { Xw[i] = v; };
    rot_contract<L>(P, St + ((oct >> 2) & 1) * L2, lane, to_x);  // along z, transposed
    rot_contract<L>(Xw, St + ((oct >> 1) & 1) * L2, lane, to_x);  // along y
    rot_contract<L>(Xw, St + (oct & 1) * L2, lane, [&](int i, double v, int m, int r) {
      gst(out + i, cur[r][m] + v);  // along x, accumulated
    });
  }
  __syncthreads();
}

// Item = parent cell at level tab->level[k] - 1 (tab->level[k] is the
// children's level); every plan of the launch has order L.
template <int L>
__global__ __launch_bounds__(kTransThreads) void l2l_kernel(const JobDev* __restrict__ jobs,
                                                            const StepTab* __restrict__ tab) {
  extern __shared__ double dyn_lds[];
  FOR_ITEMS(tab) {
    const int k = step_find(*tab, it_);
    l2l_item<L>(jobs[tab->job[k]], tab->level[k], it_ - tab->start[k], dyn_lds);
  }
}

// ------------------------------------------------------------------- L2P
// Item = leaf; two lanes per particle (a leaf holds about 30 at the usual
// occupancy, so a wavefront's second half would idle otherwise); the leaf's
// local expansion sits in LDS and each half-wavefront reads one coefficient
// (broadcast).
// phi = sum_m S_m(u) Loc[m];  F = -q (1/a) grad_u sum_m S_m(u) Loc[m], with
// S_m(u) = sum_n C[m][n] T_n(u) for node values and S_m = T_m for Chebyshev
// coefficients (C the identity).
template <int L>
__global__ FMM_L2P_BOUNDS void l2p_kernel(const JobDev* __restrict__ jobs,
                                                 const StepTab* __restrict__ tab) {
  __shared__ double C[L * L];
  __shared__ double Lc[L * L * L];
  const int t = threadIdx.x;
  FOR_ITEMS(tab) {
    const int k = step_find(*tab, it_);
    const JobDev& J = jobs[tab->job[k]];
    const int a = it_ - tab->start[k];
    const bool modal = wuni(J.modal);
    for (int e = t; e < L * L; e += 64) C[e] = modal ? (e / L == e % L ? 1.0 : 0.0) : J.cheb[e];
    const double* lsrc = J.Loc + (J.lev_off[J.height - 1] + a) * J.ld;
    {  // all loads in flight at once
      constexpr int NE = (L * L * L + 63) / 64;
      double v[NE];
#pragma unroll
      for (int k = 0; k < NE; ++k) v[k] = t + 64 * k < L * L * L ? gld(lsrc + t + 64 * k) : 0.0;
#pragma unroll
      for (int k = 0; k < NE; ++k)
        if (t + 64 * k < L * L * L) Lc[t + 64 * k] = v[k];
    }
    double c[3];
    leaf_centre(J.geo, J.leaf_keys[a], c);
    const double ia = 2.0 / J.geo.w;
    __syncthreads();
    const int s0 = J.leaf_start[a], s1 = J.leaf_start[a + 1];
    // Two lanes per particle, t and t + 32, each take half of the m1 sum
    // (m1 < H and m1 >= H); the halves are added once, to the same value in
    // both lanes, and the first lane writes.
    constexpr int H = (L + 1) / 2;
    const int half = t >> 5;
    for (int i0 = s0; i0 < s1; i0 += 32) {
      const int i = i0 + (t & 31);
      const bool valid = i < s1;
      const int ip = valid ? i : s0;
      double S[3][L], dS[3][L];
      const double xyz[3] = {J.px[ip], J.py[ip], J.pz[ip]};
      for (int d = 0; d < 3; ++d) {
        const double u = (xyz[d] - c[d]) * ia;
        double T[L], dT[L];
        T[0] = 1.0;
        dT[0] = 0.0;
        if (L > 1) {
          T[1] = u;
          dT[1] = 1.0;
        }
        for (int n = 2; n < L; ++n) {
          T[n] = 2.0 * u * T[n - 1] - T[n - 2];
          dT[n] = 2.0 * T[n - 1] + 2.0 * u * dT[n - 1] - dT[n - 2];
        }
        for (int m = 0; m < L; ++m) {
          double v = 0.0, dv = 0.0;
          for (int n = 0; n < L; ++n) {
            v += C[m * L + n] * T[n];
            dv += C[m * L + n] * dT[n];
          }
          S[d][m] = v;
          dS[d][m] = dv;
        }
      }
      // this lane's dimension-0 factors; past m1 = L - 1 they are zero
      double s0h[H], d0h[H];
      for (int j = 0; j < H; ++j) {
        const int hi = H + j < L ? H + j : L - 1;
        s0h[j] = half ? (H + j < L ? S[0][hi] : 0.0) : S[0][j];
        d0h[j] = half ? (H + j < L ? dS[0][hi] : 0.0) : dS[0][j];
      }
      double ph = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
      for (int j = 0; j < H; ++j) {
        const int m1 = min(half * H + j, L - 1);
        double b0 = 0.0, by = 0.0, bz = 0.0;
        for (int m2 = 0; m2 < L; ++m2) {
          double a0 = 0.0, a1 = 0.0;
          const double* row = Lc + (m1 * L + m2) * L;
          for (int m3 = 0; m3 < L; ++m3) {
            a0 += row[m3] * S[2][m3];
            a1 += row[m3] * dS[2][m3];
          }
          b0 += S[1][m2] * a0;
          by += dS[1][m2] * a0;
          bz += S[1][m2] * a1;
        }
        ph += s0h[j] * b0;
        gx += d0h[j] * b0;
        gy += s0h[j] * by;
        gz += s0h[j] * bz;
      }
      ph += __shfl_xor(ph, 32, 64);
      gx += __shfl_xor(gx, 32, 64);
      gy += __shfl_xor(gy, 32, 64);
      gz += __shfl_xor(gz, 32, 64);
      if (!valid || half) continue;
      const double fq = -J.qs[i] * ia;
      J.phi_f[i] = ph;
      const int64_t i3 = 3 * int64_t(i);  // forces of n > 2^31/3 particles
      J.f_f[i3] = fq * gx;
      J.f_f[i3 + 1] = fq * gy;
      J.f_f[i3 + 2] = fq * gz;
    }
    __syncthreads();
  }
}

// Item = leaf, one wavefront, for plans whose leaves hold few particles
// (kL2PSparseMax): lanes over the l^3 terms of each particle's sums.  The
// leaf's l^3 coefficients are loaded at once into registers (one memory
// latency per leaf); the 1-D factors S_d(m) and their derivatives of up to
// kL2PSparseNP particles (computed as in l2p_kernel) go to LDS; then, one
// particle at a time, lane k sums the terms e = k, k + 64, ... of phi and the
// three gradient components, and the 64 partial sums of each are added in a
// fixed two-level order (eight runs of eight lanes, then the eight run sums).
constexpr int kL2PSparseNP = 8;

template <int L>
__global__ __launch_bounds__(64) void l2p_sparse_kernel(const JobDev* __restrict__ jobs,
                                                        const StepTab* __restrict__ tab) {
  constexpr int L2 = L * L, L3 = L2 * L, NP = kL2PSparseNP, NE = (L3 + 63) / 64;
  __shared__ double C[L2];
  __shared__ double Sd[NP][6][L];  // S_0, S_1, S_2, dS_0, dS_1, dS_2
  __shared__ double red[4][64];
  __shared__ double red2[4][8];
  const int lane = threadIdx.x;
  FOR_ITEMS(tab) {
    const int k = step_find(*tab, it_);
    const JobDev& J = jobs[tab->job[k]];
    const int a = it_ - tab->start[k];
    const double* lsrc = J.Loc + (J.lev_off[J.height - 1] + a) * J.ld;
    double lcv[NE];
#pragma unroll
    for (int t = 0; t < NE; ++t) {
      const int e = lane + 64 * t;
      lcv[t] = e < L3 ? gld(lsrc + e) : 0.0;
    }
    const bool modal = wuni(J.modal);
    for (int e = lane; e < L2; e += 64) C[e] = modal ? (e / L == e % L ? 1.0 : 0.0) : J.cheb[e];
    double c[3];
    leaf_centre(J.geo, J.leaf_keys[a], c);
    const double ia = 2.0 / J.geo.w;
    const int s0 = wuni(gld(J.leaf_start + a)), s1 = wuni(gld(J.leaf_start + a + 1));
    __syncthreads();
    for (int i0 = s0; i0 < s1; i0 += NP) {
      const int np = min(NP, s1 - i0);
      for (int v = lane; v < np * 3 * L; v += 64) {
        const int j = v / (3 * L), d = (v / L) % 3, m = v % L;
        const int i = i0 + j;
        const double x = gld(d == 0 ? J.px + i : (d == 1 ? J.py + i : J.pz + i));
        const double u = (x - c[d]) * ia;
        double T[L], dT[L];
        T[0] = 1.0;
        dT[0] = 0.0;
        if (L > 1) {
          T[1] = u;
          dT[1] = 1.0;
        }
        for (int n = 2; n < L; ++n) {
          T[n] = 2.0 * u * T[n - 1] - T[n - 2];
          dT[n] = 2.0 * T[n - 1] + 2.0 * u * dT[n - 1] - dT[n - 2];
        }
        double sv = 0.0, dv = 0.0;
        for (int n = 0; n < L; ++n) {
          sv += C[m * L + n] * T[n];
          dv += C[m * L + n] * dT[n];
        }
        Sd[j][d][m] = sv;
        Sd[j][3 + d][m] = dv;
      }
      __syncthreads();
      for (int j = 0; j < np; ++j) {
        double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
#pragma unroll
        for (int t = 0; t < NE; ++t) {
          const int e = lane + 64 * t;
          if (e < L3) {
            const int m1 = e / L2, m2 = (e / L) % L, m3 = e % L;
            const double s1 = Sd[j][0][m1], s2 = Sd[j][1][m2], s3 = Sd[j][2][m3];
            const double t23 = lcv[t] * s2 * s3;
            const double t1 = lcv[t] * s1;
            p0 += s1 * t23;
            p1 += Sd[j][3][m1] * t23;
            p2 += t1 * Sd[j][4][m2] * s3;
            p3 += t1 * s2 * Sd[j][5][m3];
          }
        }
        red[0][lane] = p0;
        red[1][lane] = p1;
        red[2][lane] = p2;
        red[3][lane] = p3;
        __syncthreads();
        if (lane < 32) {  // (value, run of eight)
          const int q = lane >> 3, r = lane & 7;
          double v = 0.0;
#pragma unroll
          for (int l = 0; l < 8; ++l) v += red[q][8 * r + l];
          red2[q][r] = v;
        }
        __syncthreads();
        if (lane < 4) {
          double v = 0.0;
#pragma unroll
          for (int r = 0; r < 8; ++r) v += red2[lane][r];
          red[lane][0] = v;
        }
        __syncthreads();
        if (lane == 0) {
          const int i = i0 + j;
          const double fq = -J.qs[i] * ia;
          J.phi_f[i] = red[0][0];
          const int64_t i3 = 3 * int64_t(i);
          J.f_f[i3] = fq * red[1][0];
          J.f_f[i3 + 1] = fq * red[2][0];
          J.f_f[i3 + 2] = fq * red[3][0];
        }
        __syncthreads();
      }
    }
  }
}

// ------------------------------------------------------------------- P2P
// Item = target leaf, one wavefront.  Source leaves of the near list are
// staged through LDS in tiles of 64 particles.  When the leaf holds P <= 32
// targets, the 64 lanes split into 64/P groups that take interleaved
// sources, and the partial sums are combined with wavefront butterflies.
__device__ inline int p2p_groups(int nt) {
  int P = 1;
  while (P < nt && P < 64) P <<= 1;
  return P;
}

// One near-field pair for the kernel |x - y|^-KP: adds the potential term
// q r^-KP to ph and the force factor KP q r^-(KP+2) times d to (fx, fy, fz);
// the target charge multiplies the force at the end.  Zero distance adds 0.
// CHECK: whether the pair may be at zero distance.  Particles at one position
// share a leaf, so only the target leaf's own particles need the test; the
// padding of a source tile (q = 0, 1e30 away) contributes exact zeros.
template <int KP, bool CHECK = true>
__device__ __forceinline__ void pair_f64(double dx, double dy, double dz, double q, double& ph,
                                         double& fx, double& fy, double& fz) {
  const double r2 = dx * dx + dy * dy + dz * dz;
  double t, s;
  if (KP == 2) {
    const double ir2 = !CHECK || r2 > 0.0 ? 1.0 / r2 : 0.0;
    t = q * ir2;
    s = 2.0 * t * ir2;
  } else {
    const double ir = !CHECK || r2 > 0.0 ? rsqrt(r2) : 0.0;
    t = q * ir;
    s = t * ir * ir;
  }
  ph += t;
  fx += s * dx;
  fy += s * dy;
  fz += s * dz;
}

// The same in FP32 (v_rsq_f32 for 1/r, v_rcp_f32 for 1/r^2).
template <int KP, bool CHECK = true>
__device__ __forceinline__ void pair_f32(float dx, float dy, float dz, float q, float& ph,
                                         float& fx, float& fy, float& fz) {
  const float r2 = dx * dx + dy * dy + dz * dz;
  float t, s;
  if (KP == 2) {
    const float ir2 = !CHECK || r2 > 0.f ? __builtin_amdgcn_rcpf(r2) : 0.f;
    t = q * ir2;
    s = 2.f * t * ir2;
  } else {
    const float ir = !CHECK || r2 > 0.f ? __builtin_amdgcn_rsqf(r2) : 0.f;
    t = q * ir;
    s = t * ir * ir;
  }
  ph += t;
  fx += s * dx;
  fy += s * dy;
  fz += s * dz;
}

// Next chunk (up to 64 consecutive particles of one source leaf) of the near
// list, in slot order: advances (sl, jb, j1) and returns false past the last
// one.  Lane s < 27 holds the particle range [nj0, nj1) of near slot s (empty
// for an absent neighbour).  Start from sl = -1, jb = j1 = 0.  No memory
// access: the loads of the chunk in flight are not waited for.
__device__ __forceinline__ bool near_next(int nj0, int nj1, int& sl, int& jb, int& j1) {
  jb += 64;
  while (jb >= j1) {
    if (++sl >= 27) return false;
    jb = __builtin_amdgcn_readlane(nj0, sl);
    j1 = __builtin_amdgcn_readlane(nj1, sl);
  }
  return true;
}

// One target leaf.  The source chunks pass through LDS one at a time; the
// next chunk's loads are in flight while the current one is computed.  FP32:
// the pair difference is taken in FP64 and rounded once (a relative error of
// 2^-24 of the distance itself, however close the pair), r^2, the reciprocal
// (square) root and the products are FP32, and the partial sums over one
// source chunk (at most 64 particles, so their rounding does not grow with
// the leaves' occupancy) are kept in FP32 and folded into FP64 accumulators.
// Pairs are taken in the same order as one leaf, one chunk at a time.
typedef double src4 __attribute__((ext_vector_type(4)));  // x, y, z, q of one source

// FP32 charges travel in the q slot as their own bits (low word), so the
// pair loop reads them without a conversion.
__device__ __forceinline__ double q_slot(float q) {
  return __longlong_as_double(static_cast<long long>(__float_as_uint(q)));
}
__device__ __forceinline__ float q_of_slot(double d) {
  return __uint_as_float(static_cast<unsigned>(__double_as_longlong(d)));
}

// A source tile's passes for one lane group: sources k = split + S i,
// i < npass (a wavefront-uniform count, so the loop needs no lane masks),
// two per iteration, in increasing i.  Slots past the tile's sources hold
// the padding source, which adds zeros.
constexpr int kSelfSlot = 13;   // the near-list slot of the target leaf itself
constexpr int kSrcSlots = 128;  // 64 staged sources, then padding for the last passes
constexpr double kFarAway = 1e30;

template <int KP, bool CHECK>
__device__ __forceinline__ void p2p_passes_f32(const src4* src, int split, int S, int npass,
                                               double xi, double yi, double zi, float& p32,
                                               float& x32, float& y32, float& z32) {
  int i = 0;
  for (; i + 1 < npass; i += 2) {
    const src4 u = src[split + S * i], v = src[split + S * (i + 1)];
    pair_f32<KP, CHECK>(float(xi - u.x), float(yi - u.y), float(zi - u.z), q_of_slot(u.w), p32,
                        x32, y32, z32);
    pair_f32<KP, CHECK>(float(xi - v.x), float(yi - v.y), float(zi - v.z), q_of_slot(v.w), p32,
                        x32, y32, z32);
  }
  if (i < npass) {
    const src4 u = src[split + S * i];
    pair_f32<KP, CHECK>(float(xi - u.x), float(yi - u.y), float(zi - u.z), q_of_slot(u.w), p32,
                        x32, y32, z32);
  }
}

template <int KP, bool CHECK>
__device__ __forceinline__ void p2p_passes_f64(const src4* src, int split, int S, int npass,
                                               double xi, double yi, double zi, double& ph,
                                               double& fx, double& fy, double& fz) {
  for (int i = 0; i < npass; ++i) {
    const src4 u = src[split + S * i];
    pair_f64<KP, CHECK>(xi - u.x, yi - u.y, zi - u.z, u.w, ph, fx, fy, fz);
  }
}

// SELF: only the leaf's own particles (the within-leaf part of the mutual
// near field, whose pairs of distinct leaves go through p2p_mutual.hip).
template <int KP, bool F32, bool SELF>
__device__ __forceinline__ void p2p_leaf(const JobDev& J, int a, src4* src) {
  const int lane = threadIdx.x;
  const double *px = J.px, *py = J.py, *pz = J.pz;
  const int t0 = wuni(gld(J.leaf_start + a)), nt = wuni(gld(J.leaf_start + a + 1)) - t0;
  const int P = p2p_groups(nt);
  const int S = 64 / P;
  const int split = lane / P;
  int nj0 = 0, nj1 = 0;
  if (SELF ? lane == kSelfSlot : lane < 27) {
    const int b = gld(J.near + 27 * a + lane);
    if (b >= 0) {
      nj0 = gld(J.leaf_start + b);
      nj1 = gld(J.leaf_start + b + 1);
    }
  }
  // the source charge as stored (FP32 or FP64), widened when staged
  typedef typename std::conditional<F32, float, double>::type QT;
  const QT* qsrc = F32 ? reinterpret_cast<const QT*>(J.prel) : reinterpret_cast<const QT*>(J.qs);
  const int qstride = F32 ? 4 : 1, qoff = F32 ? 3 : 0;
  for (int tb = 0; tb < nt; tb += 64) {
    const int ti = tb + (lane % P);
    const bool valid = ti < nt;
    const int it = t0 + (valid ? ti : 0);
    const double xi = gld(px + it), yi = gld(py + it), zi = gld(pz + it);
    double ph = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
    float p32 = 0.f, x32 = 0.f, y32 = 0.f, z32 = 0.f;
    int sl = -1, jb = 0, j1 = 0;
    bool have = near_next(nj0, nj1, sl, jb, j1);
    int cnt = have ? min(64, j1 - jb) : 0;
    double rx = kFarAway, ry = kFarAway, rz = kFarAway;
    QT rq = 0;
    if (lane < cnt) {
      rx = gld(px + jb + lane);
      ry = gld(py + jb + lane);
      rz = gld(pz + jb + lane);
      rq = gld(qsrc + int64_t(jb + lane) * qstride + qoff);
    }
    while (have) {
      const int ccnt = cnt, csl = sl;
      __syncthreads();  // the previous chunk's reads are done
      src[lane] = src4{rx, ry, rz, F32 ? q_slot(float(rq)) : double(rq)};
      __syncthreads();
      have = near_next(nj0, nj1, sl, jb, j1);
      cnt = have ? min(64, j1 - jb) : 0;
      rx = ry = rz = kFarAway;
      rq = 0;
      if (lane < cnt) {
        rx = gld(px + jb + lane);
        ry = gld(py + jb + lane);
        rz = gld(pz + jb + lane);
        rq = gld(qsrc + int64_t(jb + lane) * qstride + qoff);
      }
      const int npass = (ccnt + S - 1) / S;
      if (F32) {
        if (csl == kSelfSlot)
          p2p_passes_f32<KP, true>(src, split, S, npass, xi, yi, zi, p32, x32, y32, z32);
        else
          p2p_passes_f32<KP, false>(src, split, S, npass, xi, yi, zi, p32, x32, y32, z32);
        ph += double(p32);
        fx += double(x32);
        fy += double(y32);
        fz += double(z32);
        p32 = x32 = y32 = z32 = 0.f;
      } else if (csl == kSelfSlot) {
        p2p_passes_f64<KP, true>(src, split, S, npass, xi, yi, zi, ph, fx, fy, fz);
      } else {
        p2p_passes_f64<KP, false>(src, split, S, npass, xi, yi, zi, ph, fx, fy, fz);
      }
    }
    for (int o = P; o < 64; o <<= 1) {
      ph += __shfl_xor(ph, o, 64);
      fx += __shfl_xor(fx, o, 64);
      fy += __shfl_xor(fy, o, 64);
      fz += __shfl_xor(fz, o, 64);
    }
    if (valid && split == 0) {
      const int i = t0 + ti;
      const double qi = gld(J.qs + i);
      gst(J.phi_n + i, ph);
      const int64_t i3 = 3 * int64_t(i);
      gst(J.f_n + i3, qi * fx);
      gst(J.f_n + i3 + 1, qi * fy);
      gst(J.f_n + i3 + 2, qi * fz);
    }
  }
}

template <bool SELF>
__global__ __launch_bounds__(64) void p2p_f64_kernel(const JobDev* __restrict__ jobs,
                                                     const StepTab* __restrict__ tab) {
  __shared__ src4 src[kSrcSlots];
  // slots past the 64 staged sources: the padding source, set once (the
  // first staging's barrier orders it before any read)
  src[64 + threadIdx.x] = src4{kFarAway, kFarAway, kFarAway, 0.0};
  FOR_ITEMS(tab) {
    const int k = step_find(*tab, it_);
    const JobDev& J = jobs[tab->job[k]];
    const int a = it_ - tab->start[k];
    if (J.kernel == 2)
      p2p_leaf<2, false, SELF>(J, a, src);
    else
      p2p_leaf<1, false, SELF>(J, a, src);
    __syncthreads();
  }
}

template <bool SELF>
__global__ __launch_bounds__(64) void p2p_f32_kernel(const JobDev* __restrict__ jobs,
                                                     const StepTab* __restrict__ tab) {
  __shared__ src4 src[kSrcSlots];
  // slots past the 64 staged sources: the padding source, set once (the
  // first staging's barrier orders it before any read)
  src[64 + threadIdx.x] = src4{kFarAway, kFarAway, kFarAway, 0.0};
  FOR_ITEMS(tab) {
    const int k = step_find(*tab, it_);
    const JobDev& J = jobs[tab->job[k]];
    const int a = it_ - tab->start[k];
    if (J.kernel == 2)
      p2p_leaf<2, true, SELF>(J, a, src);
    else
      p2p_leaf<1, true, SELF>(J, a, src);
    __syncthreads();
  }
}

// ------------------------------------------ M2L parts and coefficient rows
// Item = row of levels >= 2 of a job whose M2L ran in parts or in FP32:
// Loc += the partial local expansions of parts 1 .. K-1, added in part order
// (one FP64 sum per element, the same order every run).  Item = row.
__global__ __launch_bounds__(256) void loc_sum_kernel(const JobDev* __restrict__ jobs,
                                                      const StepTab* __restrict__ tab) {
  const int t = threadIdx.x;
  FOR_ITEMS(tab) {
    const int k = step_find(*tab, it_);
    const JobDev& J = jobs[tab->job[k]];
    const int64_t r = it_ - tab->start[k];
    const int64_t n = J.locx_rows * J.ld;
    double* loc = J.Loc + (J.locx_first + r) * J.ld;
    const double* x = J.LocX + r * J.ld;
    const int parts = wuni(J.m2l_parts);
    for (int e = t; e < J.ld; e += 256) {
      double v = gld(loc + e);
      for (int p = 1; p < parts; ++p) v += gld(x + (p - 1) * n + e);
      gst(loc + e, v);
    }
  }
}

// ------------------------------------------------------- gather / combine
// Items are chunks of 256 particles.
constexpr int kChunk = 256;

__device__ inline void gather_chunk(const JobDev& J, const double* q, int chunk) {
  const int i = chunk * kChunk + threadIdx.x;
  if (i >= J.n) return;
  const double v = q[J.perm[i]];
  J.qs[i] = v;
  J.prel[i].w = float(v);
}

// out[perm[i]] = near[i] + far[i] in FP64; far is absent below height 3.
// With part outputs the near and far results are un-permuted as they are.
__device__ inline void combine_chunk(const JobDev& J, const CallDev& C, int chunk) {
  const int i = chunk * kChunk + threadIdx.x;
  if (i >= J.n) return;
  const int64_t o = J.perm[i];
  const bool far = J.has_far;
  const double a = J.phi_n[i], b = far ? J.phi_f[i] : 0.0;
  const int64_t i3 = 3 * int64_t(i), o3 = 3 * o;
  const double ax = J.f_n[i3], ay = J.f_n[i3 + 1], az = J.f_n[i3 + 2];
  const double bx = far ? J.f_f[i3] : 0.0, by = far ? J.f_f[i3 + 1] : 0.0,
               bz = far ? J.f_f[i3 + 2] : 0.0;
  if (C.phi) {
    C.phi[o] = a + b;
    C.f[o3] = ax + bx;
    C.f[o3 + 1] = ay + by;
    C.f[o3 + 2] = az + bz;
  }
  if (C.pn) {
    C.pn[o] = a;
    C.fn[o3] = ax;
    C.fn[o3 + 1] = ay;
    C.fn[o3 + 2] = az;
    C.pf[o] = b;
    C.ff[o3] = bx;
    C.ff[o3 + 1] = by;
    C.ff[o3 + 2] = bz;
  }
}

__global__ __launch_bounds__(kChunk) void gather_kernel(const JobDev* __restrict__ jobs,
                                                        const StepTab* __restrict__ tab,
                                                        const CallDev* __restrict__ calls) {
  FOR_ITEMS(tab) {
    const int k = step_find(*tab, it_);
    const int j = tab->job[k];
    gather_chunk(jobs[j], calls[j].q, it_ - tab->start[k]);
  }
}

__global__ __launch_bounds__(kChunk) void combine_kernel(const JobDev* __restrict__ jobs,
                                                         const StepTab* __restrict__ tab,
                                                         const CallDev* __restrict__ calls) {
  FOR_ITEMS(tab) {
    const int k = step_find(*tab, it_);
    const int j = tab->job[k];
    combine_chunk(jobs[j], calls[j], it_ - tab->start[k]);
  }
}

// single-plan forms: the call's pointers travel as kernel arguments
__global__ __launch_bounds__(kChunk) void gather1_kernel(const JobDev* __restrict__ job,
                                                         const double* __restrict__ q) {
  gather_chunk(*job, q, blockIdx.x);
}

__global__ __launch_bounds__(kChunk) void combine1_kernel(const JobDev* __restrict__ job,
                                                          CallDev call) {
  combine_chunk(*job, call, blockIdx.x);
}

// FP32 copy of the multipoles of levels 2 .. h-2 (the leaf level is written
// in FP32 by P2M in the mixed modes); item = one row.
__global__ __launch_bounds__(256) void cast_kernel(const JobDev* __restrict__ jobs,
                                                   const StepTab* __restrict__ tab) {
  FOR_ITEMS(tab) {
    const int k = step_find(*tab, it_);
    const JobDev& J = jobs[tab->job[k]];
    const int64_t row = J.lev_off[2] + (it_ - tab->start[k]);
    for (int e = threadIdx.x; e < J.ld; e += 256) J.W32[row * J.ld + e] = float(J.W[row * J.ld + e]);
  }
}

// ---------------------------------------------------------------- driver
#define FMM_ORDER_SWITCH(L, CALL) \
  switch (L) {                    \
    case 1: CALL(1); break;       \
    case 2: CALL(2); break;       \
    case 3: CALL(3); break;       \
    case 4: CALL(4); break;       \
    case 5: CALL(5); break;       \
    case 6: CALL(6); break;       \
    case 7: CALL(7); break;       \
    case 8: CALL(8); break;       \
    case 9: CALL(9); break;       \
    case 10: CALL(10); break;     \
    case 11: CALL(11); break;     \
    default: CALL(12); break;     \
  }

void launch_m2l_step(int order, bool fp32, const JobDev* jobs, const StepTab* tab, int grid,
                     hipStream_t s);
void launch_m2l_svd_step(int order, bool fp32, const JobDev* jobs, const StepTab* tab, int grid,
                         int xs, hipStream_t s, bool gskip);

void launch_step(StepKind kind, int L, bool fp32, const JobDev* jobs, const StepTab* tab,
                 const CallDev* calls, int grid, hipStream_t s, int xs, bool gskip) {
  const unsigned g = unsigned(grid);
  switch (kind) {
    case kStepGather:
      gather_kernel<<<g, kChunk, 0, s>>>(jobs, tab, calls);
      break;
    case kStepP2M: {
      const int thr = L * L <= 64 ? 64 : (L * L <= 128 ? 128 : 256);
#define P2M_CALL(LL) p2m_kernel<LL><<<g, thr, 0, s>>>(jobs, tab)
      FMM_ORDER_SWITCH(L, P2M_CALL)
#undef P2M_CALL
      break;
    }
    case kStepM2M:
#define M2M_CALL(LL) m2m_kernel<LL><<<g, kTransThreads, m2m_lds_bytes(LL), s>>>(jobs, tab)
      FMM_ORDER_SWITCH(L, M2M_CALL)
#undef M2M_CALL
      break;
    case kStepCast:
      cast_kernel<<<g, 256, 0, s>>>(jobs, tab);
      break;
    case kStepLocSum:
      loc_sum_kernel<<<g, 256, 0, s>>>(jobs, tab);
      break;
    case kStepM2L:
      launch_m2l_step(L, fp32, jobs, tab, grid, s);
      break;
    case kStepM2LSvd:
      launch_m2l_svd_step(L, fp32, jobs, tab, grid, xs, s, gskip);
      break;
    case kStepL2L:
#define L2L_CALL(LL) l2l_kernel<LL><<<g, kTransThreads, l2l_lds_bytes(LL), s>>>(jobs, tab)
      FMM_ORDER_SWITCH(L, L2L_CALL)
#undef L2L_CALL
      break;
    case kStepL2P:
#define L2P_CALL(LL) l2p_kernel<LL><<<g, 64, 0, s>>>(jobs, tab)
      FMM_ORDER_SWITCH(L, L2P_CALL)
#undef L2P_CALL
      break;
    case kStepL2PSparse:
#define L2P_CALL(LL) l2p_sparse_kernel<LL><<<g, 64, 0, s>>>(jobs, tab)
      FMM_ORDER_SWITCH(L, L2P_CALL)
#undef L2P_CALL
      break;
    case kStepP2P:
      if (fp32) p2p_f32_kernel<false><<<g, 64, 0, s>>>(jobs, tab);
      else p2p_f64_kernel<false><<<g, 64, 0, s>>>(jobs, tab);
      break;
    case kStepP2PSelf:
      if (fp32) p2p_f32_kernel<true><<<g, 64, 0, s>>>(jobs, tab);
      else p2p_f64_kernel<true><<<g, 64, 0, s>>>(jobs, tab);
      break;
    case kStepCombine:
      combine_kernel<<<g, kChunk, 0, s>>>(jobs, tab, calls);
      break;
  }
  FMM_HIP_CHECK(hipGetLastError());
}

// Where the forked schedule starts the near field: 0 = just before the M2L
// launch, 1 = just after it, 2 = after the L2L levels, 3 = before the last
// L2L level.  Measured (1M cube, order 7, compressed mixed mode, evaluate
// only): after 6.84 ms, serial 6.90 ms, before 6.98 ms; later, with the
// faster M2L: 1 5.24 ms, 2 5.23 ms, 3 5.21 ms (within the spread).
#ifndef FMM_FORK_AFTER_M2L
#define FMM_FORK_AFTER_M2L 1
#endif

namespace {
// the step's timing events, if set, around a launch on stream s
struct Timed {
  int step;
  hipStream_t s;
  Timed(int st, hipStream_t str) : step(st), s(str) {
    if (g_time_ev[step][0]) FMM_HIP_CHECK(hipEventRecord(g_time_ev[step][0], s));
  }
  // a failed record here only loses a timing; launch errors are reported by
  // the launch itself
  ~Timed() {
    if (g_time_ev[step][1]) (void)hipEventRecord(g_time_ev[step][1], s);
  }
};
}  // namespace

// One plan: the step tables were built at plan time; every launch has one
// block per item.  In the forked schedule the near field runs on the plan's
// side stream, forked after the M2L launch and joined before the combine, so
// it fills the GPU beside the L2L levels and L2P, which do not.  (Forked
// earlier, its 64-thread blocks flood the GPU and delay P2M and M2M, and it
// cannot share CUs with M2L, whose wavefronts hold the register files.)
void evaluate(fmm_plan_s* p, const double* q, double* phi, double* f, double* phi_n,
              double* f_n, double* phi_f, double* f_f, hipStream_t s) {
  const int L = p->order, h = p->height;
  const bool mixed = p->precision == FMM_MIXED_FP32 || p->precision == FMM_MIXED_SVD;
  const JobDev* J = p->job_d;
  const unsigned chunks = unsigned((p->n + kChunk - 1) / kChunk);
  gather1_kernel<<<chunks, kChunk, 0, s>>>(J, q);
  FMM_HIP_CHECK(hipGetLastError());
  // the pipelined schedule forks the near field like the forked one
  const bool pipelined = p->schedule == FMM_SCHEDULE_PIPELINED;
  const bool forked = p->schedule == FMM_SCHEDULE_FORKED || pipelined;
  // the near field: one-sided, or the leaves' own pairs and then the mutual
  // pair lists of distinct neighbour leaves (Sec. 5)
  auto near_field = [&](hipStream_t st) {
    Timed t(FMM_TIME_P2P, st);
    if (p->near_mode == FMM_NEAR_MUTUAL) {
      launch_step(kStepP2PSelf, L, mixed, J, p->tab_d + kTabLeaf, nullptr, int(p->nleaf), st);
      launch_p2p_mutual(p, mixed, st);
    } else {
      launch_step(kStepP2P, L, mixed, J, p->tab_d + kTabLeaf, nullptr, int(p->nleaf), st);
    }
  };
  auto fork_near = [&]() {
    FMM_HIP_CHECK(hipEventRecord(p->ev_fork, s));
    FMM_HIP_CHECK(hipStreamWaitEvent(p->side, p->ev_fork, 0));
    near_field(p->side);
    FMM_HIP_CHECK(hipEventRecord(p->ev_join, p->side));
  };
  if (forked && h < 3) fork_near();
  const StepKind m2l_kind = p->svd ? kStepM2LSvd : kStepM2L;
  auto m2l_launch = [&](int tab, hipStream_t st) {
    if (p->tab_h[tab].start[1] > 0)
      launch_step(m2l_kind, L, mixed, J, p->tab_d + tab, nullptr, p->tab_h[tab].start[1], st,
                  p->job_h.xs, p->m2l_gskip);
  };
  auto loc_sum = [&]() {
    if (p->tab_h[kTabLocSum].start[1] > 0) {
      Timed t(FMM_TIME_LOC_SUM, s);
      launch_step(kStepLocSum, L, false, J, p->tab_d + kTabLocSum, nullptr,
                  p->tab_h[kTabLocSum].start[1], s);
    }
  };
  if (h >= 3) {
    {
      Timed t(FMM_TIME_P2M, s);
      launch_step(kStepP2M, L, false, J, p->tab_d + kTabLeaf, nullptr, int(p->nleaf), s);
    }
    // pipelined: the leaf level's M2L needs only the leaf multipoles, so it
    // starts on the side stream beside the M2M chain (Sec. 3.3: M2L of one
    // level overlaps M2M of the next coarser one)
    if (pipelined && p->ntiles > 0) {
      FMM_HIP_CHECK(hipEventRecord(p->ev_fork, s));
      FMM_HIP_CHECK(hipStreamWaitEvent(p->side, p->ev_fork, 0));
      {
        Timed t(FMM_TIME_M2L, p->side);
        m2l_launch(kTabM2LLeaf, p->side);
      }
      FMM_HIP_CHECK(hipEventRecord(p->ev_join, p->side));
    }
    {
      Timed t(FMM_TIME_M2M, s);
      for (int st = 0; st + 4 <= h; ++st)
        launch_step(kStepM2M, L, false, J, p->tab_d + kTabM2M + st, nullptr,
                    p->tab_h[kTabM2M + st].start[1], s);
    }
    if (mixed && p->tab_h[kTabCast].start[1] > 0)
      launch_step(kStepCast, L, true, J, p->tab_d + kTabCast, nullptr,
                  p->tab_h[kTabCast].start[1], s);
    if (forked && !FMM_FORK_AFTER_M2L) fork_near();
    if (pipelined) {
      if (p->ntiles > 0) {
        m2l_launch(kTabM2LCoarse, s);
        FMM_HIP_CHECK(hipStreamWaitEvent(s, p->ev_join, 0));
        loc_sum();
      }
    } else if (p->ntiles > 0) {
      {
        Timed t(FMM_TIME_M2L, s);
        m2l_launch(kTabM2L, s);
      }
      loc_sum();
    }
    if (forked && FMM_FORK_AFTER_M2L == 1) fork_near();
    {
      Timed t(FMM_TIME_L2L, s);
      for (int st = 0; st + 4 <= h; ++st) {
        if (forked && FMM_FORK_AFTER_M2L == 3 && st + 4 == h) fork_near();
        launch_step(kStepL2L, L, false, J, p->tab_d + kTabL2L + st, nullptr,
                    p->tab_h[kTabL2L + st].start[1], s);
      }
    }
    if (forked && (FMM_FORK_AFTER_M2L == 2 || (FMM_FORK_AFTER_M2L == 3 && h < 4))) fork_near();
    {
      Timed t(FMM_TIME_L2P, s);
      launch_step(p->job_h.l2p_sparse ? kStepL2PSparse : kStepL2P, L, false, J,
                  p->tab_d + kTabLeaf, nullptr, int(p->nleaf), s);
    }
  }
  if (forked) {
    FMM_HIP_CHECK(hipStreamWaitEvent(s, p->ev_join, 0));
  } else {
    near_field(s);
  }
  CallDev c{q, phi, f, phi_n, f_n, phi_f, f_f};
  combine1_kernel<<<chunks, kChunk, 0, s>>>(J, c);
  FMM_HIP_CHECK(hipGetLastError());
}


bool timing_hooks_set() {
  for (int i = 0; i < kTimedSteps; ++i)
    if (g_time_ev[i][0] || g_time_ev[i][1]) return true;
  return false;
}

void release_graph(fmm_plan_s* p) {
  if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->graph_exec = nullptr;
  p->graph = nullptr;
  p->graph_gather = p->graph_combine = nullptr;
  p->graph_version = -1;
  p->graph_schedule = -1;
}

// Capture: evaluate() on the plan's private stream (the near-field fork and
// join become branches of the graph), then find the two kernel nodes that
// take the call's pointers.  No memset or allocation happens in evaluate().
static void capture_graph(fmm_plan_s* p, const double* q, double* phi, double* f) {
  release_graph(p);
  if (!p->capture) p->capture = side_stream_get(p->device);
  // the side stream joins the capture: nothing of an eager evaluation may be
  // pending on it
  FMM_HIP_CHECK(hipStreamSynchronize(p->side));
  FMM_HIP_CHECK(hipStreamBeginCapture(p->capture, hipStreamCaptureModeThreadLocal));
  try {
    evaluate(p, q, phi, f, nullptr, nullptr, nullptr, nullptr, p->capture);
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(p->capture, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  FMM_HIP_CHECK(hipStreamEndCapture(p->capture, &p->graph));
  size_t nn = 0;
  FMM_HIP_CHECK(hipGraphGetNodes(p->graph, nullptr, &nn));
  std::vector<hipGraphNode_t> nodes(nn);
  FMM_HIP_CHECK(hipGraphGetNodes(p->graph, nodes.data(), &nn));
  for (hipGraphNode_t nd : nodes) {
    hipGraphNodeType t;
    FMM_HIP_CHECK(hipGraphNodeGetType(nd, &t));
    if (t != hipGraphNodeTypeKernel) continue;
    hipKernelNodeParams kp;
    FMM_HIP_CHECK(hipGraphKernelNodeGetParams(nd, &kp));
    if (kp.func == reinterpret_cast<void*>(&gather1_kernel)) p->graph_gather = nd;
    if (kp.func == reinterpret_cast<void*>(&combine1_kernel)) p->graph_combine = nd;
  }
  if (!p->graph_gather || !p->graph_combine) {
    release_graph(p);
    throw FmmError{FMM_ERR_HIP, "internal: captured evaluation lacks its gather or combine"};
  }
  FMM_HIP_CHECK(hipGraphInstantiate(&p->graph_exec, p->graph, nullptr, nullptr, 0));
  p->graph_version = p->job_version;
  p->graph_schedule = p->schedule;
}

void evaluate_graph(fmm_plan_s* p, const double* q, double* phi, double* f, hipStream_t s) {
  if (!p->graph_exec || p->graph_version != p->job_version || p->graph_schedule != p->schedule)
    capture_graph(p, q, phi, f);
  // the call's pointers into the two nodes that take them
  const JobDev* J = p->job_d;
  hipKernelNodeParams kp;
  FMM_HIP_CHECK(hipGraphKernelNodeGetParams(p->graph_gather, &kp));
  void* ga[] = {&J, &q};
  kp.kernelParams = ga;
  kp.extra = nullptr;
  FMM_HIP_CHECK(hipGraphExecKernelNodeSetParams(p->graph_exec, p->graph_gather, &kp));
  CallDev c{q, phi, f, nullptr, nullptr, nullptr, nullptr};
  FMM_HIP_CHECK(hipGraphKernelNodeGetParams(p->graph_combine, &kp));
  void* ca[] = {&J, &c};
  kp.kernelParams = ca;
  kp.extra = nullptr;
  FMM_HIP_CHECK(hipGraphExecKernelNodeSetParams(p->graph_exec, p->graph_combine, &kp));
  FMM_HIP_CHECK(hipGraphLaunch(p->graph_exec, s));
}

}  // namespace fmm
