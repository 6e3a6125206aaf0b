// Evaluation kernels: P2M, M2M, L2L, L2P, P2P and the final combine.
//
// Interpolation (Sec. 2.1, Eq. 3-5): S(xb_m; u) = 1/l + 2/l sum_{n=1}^{l-1}
// T_n(xb_m) T_n(u), tensorised over x, y, z (Eq. 4).  With the table
// C[m][n] = (n == 0 ? 1 : 2 T_n(xb_m)) / l this is S_m(u) = sum_n C[m][n] T_n(u)
// (the outer-product form of Sec. 2.1.1: O(l^3) per particle).  M2M and L2L
// apply the child-to-parent interpolation as three 1-D l x l contractions
// (Sec. 2.1.1, O(l^4) per cell).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_util.h"
#include "fmm_internal.h"

namespace fmm {

struct LeafGeom {
  double lo0, lo1, lo2, w;  // leaf width w, centre lo + (k + 1/2) w
  int bits;
};

__device__ inline void leaf_centre(const LeafGeom& g, uint64_t key, double* c) {
  int k[3];
  demorton3(key, g.bits, k);
  c[0] = g.lo0 + (k[0] + 0.5) * g.w;
  c[1] = g.lo1 + (k[1] + 0.5) * g.w;
  c[2] = g.lo2 + (k[2] + 0.5) * g.w;
}

// ------------------------------------------------------------------- P2M
// One workgroup per leaf; thread (m1, m2) accumulates the l coefficients
// W[m1][m2][*] over the leaf's particles: W += q Sx[m1] Sy[m2] Sz[*].
constexpr int kP2MChunk = 64;

template <int L>
__global__ __launch_bounds__(256) void p2m_kernel(
    const double* __restrict__ px, const double* __restrict__ py,
    const double* __restrict__ pz, const double* __restrict__ qs,
    const int* __restrict__ leaf_start, const uint64_t* __restrict__ leaf_keys,
    LeafGeom geo, const double* __restrict__ cheb, double* __restrict__ W,
    int64_t gid0, int ld) {
  __shared__ double C[L * L];
  __shared__ double S[kP2MChunk][3][L];
  const int a = blockIdx.x, t = threadIdx.x, nt = blockDim.x;
  for (int k = t; k < L * L; k += nt) C[k] = cheb[k];
  double c[3];
  leaf_centre(geo, leaf_keys[a], c);
  const double ia = 2.0 / geo.w;
  const int m1 = t / L, m2 = t % L;
  const bool owner = t < L * L;
  double acc[L];
  for (int k = 0; k < L; ++k) acc[k] = 0.0;
  const int s0 = leaf_start[a], s1 = leaf_start[a + 1];
  __syncthreads();
  for (int base = s0; base < s1; base += kP2MChunk) {
    const int cnt = min(kP2MChunk, s1 - base);
    for (int e = t; e < 3 * cnt; e += nt) {
      const int j = e / 3, d = e % 3;
      const int i = base + j;
      const double x = d == 0 ? px[i] : (d == 1 ? py[i] : pz[i]);
      const double u = (x - c[d]) * ia;
      double T[L];
      T[0] = 1.0;
      if (L > 1) T[1] = u;
      for (int n = 2; n < L; ++n) T[n] = 2.0 * u * T[n - 1] - T[n - 2];
      const double f = d == 0 ? qs[i] : 1.0;
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
  double* out = W + (gid0 + a) * ld;
  if (owner)
    for (int m3 = 0; m3 < L; ++m3) out[(m1 * L + m2) * L + m3] = acc[m3];
  for (int k = L * L * L + t; k < ld; k += nt) out[k] = 0.0;
}

// ------------------------------------------------------------- M2M / L2L
// Three 1-D contractions with the child-to-parent matrices
// Sc[s][m][m'] = S(xb_m; (s + xb_m')/2), s in {-1,+1} by the child octant bit.
constexpr int kTransThreads = 256;
constexpr int kTransMaxR = (kMaxOrder * kMaxOrder * kMaxOrder + kTransThreads - 1) / kTransThreads;

__global__ __launch_bounds__(kTransThreads) void m2m_kernel(
    const int* __restrict__ child_start, const uint64_t* __restrict__ child_keys,
    int64_t gid_p0, int64_t gid_c0, const double* __restrict__ child_mat, int L,
    int ld, double* __restrict__ W) {
  __shared__ double Sc[2 * kMaxOrder * kMaxOrder];
  __shared__ double b0[kMaxOrder * kMaxOrder * kMaxOrder];
  __shared__ double b1[kMaxOrder * kMaxOrder * kMaxOrder];
  const int p = blockIdx.x, t = threadIdx.x;
  const int L2 = L * L, L3 = L2 * L;
  for (int k = t; k < 2 * L2; k += kTransThreads) Sc[k] = child_mat[k];
  double acc[kTransMaxR];
  for (int r = 0; r < kTransMaxR; ++r) acc[r] = 0.0;
  const int c0 = child_start[p], c1 = child_start[p + 1];
  for (int c = c0; c < c1; ++c) {
    const int o = int(child_keys[c] & 7u);
    const double* Sx = Sc + ((o & 1) ? L2 : 0);
    const double* Sy = Sc + (((o >> 1) & 1) ? L2 : 0);
    const double* Sz = Sc + (((o >> 2) & 1) ? L2 : 0);
    const double* wc = W + (gid_c0 + c) * ld;
    __syncthreads();
    for (int k = t; k < L3; k += kTransThreads) b0[k] = wc[k];
    __syncthreads();
    for (int k = t; k < L3; k += kTransThreads) {  // along z
      const int ab = k / L, m3 = k % L;
      double v = 0.0;
      for (int q = 0; q < L; ++q) v += Sz[m3 * L + q] * b0[ab * L + q];
      b1[k] = v;
    }
    __syncthreads();
    for (int k = t; k < L3; k += kTransThreads) {  // along y
      const int a1 = k / L2, m2 = (k / L) % L, m3 = k % L;
      double v = 0.0;
      for (int q = 0; q < L; ++q) v += Sy[m2 * L + q] * b1[(a1 * L + q) * L + m3];
      b0[k] = v;
    }
    __syncthreads();
    for (int r = 0, k = t; k < L3; ++r, k += kTransThreads) {  // along x
      const int m1 = k / L2, rest = k % L2;
      double v = 0.0;
      for (int q = 0; q < L; ++q) v += Sx[m1 * L + q] * b0[q * L2 + rest];
      acc[r] += v;
    }
  }
  double* out = W + (gid_p0 + p) * ld;
  for (int r = 0, k = t; k < L3; ++r, k += kTransThreads) out[k] = acc[r];
  for (int k = L3 + t; k < ld; k += kTransThreads) out[k] = 0.0;
}

__global__ __launch_bounds__(kTransThreads) void l2l_kernel(
    const int* __restrict__ parent, const uint64_t* __restrict__ child_keys,
    int64_t gid_p0, int64_t gid_c0, const double* __restrict__ child_mat, int L,
    int ld, double* __restrict__ Loc) {
  __shared__ double Sc[2 * kMaxOrder * kMaxOrder];
  __shared__ double b0[kMaxOrder * kMaxOrder * kMaxOrder];
  __shared__ double b1[kMaxOrder * kMaxOrder * kMaxOrder];
  const int c = blockIdx.x, t = threadIdx.x;
  const int L2 = L * L, L3 = L2 * L;
  for (int k = t; k < 2 * L2; k += kTransThreads) Sc[k] = child_mat[k];
  const int o = int(child_keys[c] & 7u);
  const double* lp = Loc + (gid_p0 + parent[c]) * ld;
  for (int k = t; k < L3; k += kTransThreads) b0[k] = lp[k];
  __syncthreads();
  const double* Sx = Sc + ((o & 1) ? L2 : 0);
  const double* Sy = Sc + (((o >> 1) & 1) ? L2 : 0);
  const double* Sz = Sc + (((o >> 2) & 1) ? L2 : 0);
  for (int k = t; k < L3; k += kTransThreads) {  // along z, transposed
    const int ab = k / L, m3 = k % L;
    double v = 0.0;
    for (int q = 0; q < L; ++q) v += Sz[q * L + m3] * b0[ab * L + q];
    b1[k] = v;
  }
  __syncthreads();
  for (int k = t; k < L3; k += kTransThreads) {  // along y
    const int a1 = k / L2, m2 = (k / L) % L, m3 = k % L;
    double v = 0.0;
    for (int q = 0; q < L; ++q) v += Sy[q * L + m2] * b1[(a1 * L + q) * L + m3];
    b0[k] = v;
  }
  __syncthreads();
  double* lc = Loc + (gid_c0 + c) * ld;
  for (int k = t; k < L3; k += kTransThreads) {  // along x, accumulate
    const int m1 = k / L2, rest = k % L2;
    double v = 0.0;
    for (int q = 0; q < L; ++q) v += Sx[q * L + m1] * b0[q * L2 + rest];
    lc[k] += v;
  }
}

// ------------------------------------------------------------------- L2P
// One thread per particle; the leaf's local expansion sits in LDS and every
// lane reads the same coefficient (broadcast).  phi = sum_m S_m(u) Loc[m];
// F = -q (1/a) grad_u sum_m S_m(u) Loc[m].
template <int L>
__global__ __launch_bounds__(64) void l2p_kernel(
    const double* __restrict__ px, const double* __restrict__ py,
    const double* __restrict__ pz, const double* __restrict__ qs,
    const int* __restrict__ leaf_start, const uint64_t* __restrict__ leaf_keys,
    LeafGeom geo, const double* __restrict__ cheb, const double* __restrict__ Loc,
    int64_t gid0, int ld, double* __restrict__ phi, double* __restrict__ f) {
  __shared__ double C[L * L];
  __shared__ double Lc[L * L * L];
  const int a = blockIdx.x, t = threadIdx.x;
  for (int k = t; k < L * L; k += 64) C[k] = cheb[k];
  const double* lsrc = Loc + (gid0 + a) * ld;
  for (int k = t; k < L * L * L; k += 64) Lc[k] = lsrc[k];
  double c[3];
  leaf_centre(geo, leaf_keys[a], c);
  const double ia = 2.0 / geo.w;
  __syncthreads();
  const int s0 = leaf_start[a], s1 = leaf_start[a + 1];
  for (int i = s0 + t; i < s1; i += 64) {
    double S[3][L], dS[3][L];
    const double xyz[3] = {px[i], py[i], pz[i]};
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
    double ph = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    for (int m1 = 0; m1 < L; ++m1) {
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
      ph += S[0][m1] * b0;
      gx += dS[0][m1] * b0;
      gy += S[0][m1] * by;
      gz += S[0][m1] * bz;
    }
    const double fq = -qs[i] * ia;
    phi[i] = ph;
    f[3 * i] = fq * gx;
    f[3 * i + 1] = fq * gy;
    f[3 * i + 2] = fq * gz;
  }
}

// ------------------------------------------------------------------- P2P
// One wavefront per target leaf.  Source leaves of the near list are staged
// through LDS in tiles of 64 particles.  When the leaf holds P <= 32 targets,
// the 64 lanes split into 64/P groups that take interleaved sources, and the
// partial sums are combined with wavefront butterfly shuffles.
__device__ inline int p2p_groups(int nt) {
  int P = 1;
  while (P < nt && P < 64) P <<= 1;
  return P;
}

__global__ __launch_bounds__(64) void p2p_f64_kernel(
    const double* __restrict__ px, const double* __restrict__ py,
    const double* __restrict__ pz, const double* __restrict__ qs,
    const int* __restrict__ leaf_start, const int* __restrict__ near,
    double* __restrict__ phi, double* __restrict__ f) {
  __shared__ double sx[64], sy[64], sz[64], sq[64];
  const int a = blockIdx.x, lane = threadIdx.x;
  const int t0 = leaf_start[a], nt = leaf_start[a + 1] - t0;
  const int P = p2p_groups(nt);
  const int S = 64 / P;
  const int split = lane / P;
  for (int tb = 0; tb < nt; tb += 64) {
    const int ti = tb + (lane % P);
    const bool valid = ti < nt;
    const int it = t0 + (valid ? ti : 0);
    const double xi = px[it], yi = py[it], zi = pz[it];
    double ph = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
    for (int sl = 0; sl < 27; ++sl) {
      const int b = near[27 * a + sl];
      if (b < 0) continue;
      const int j0 = leaf_start[b], j1 = leaf_start[b + 1];
      for (int jb = j0; jb < j1; jb += 64) {
        const int cnt = min(64, j1 - jb);
        __syncthreads();
        if (lane < cnt) {
          sx[lane] = px[jb + lane];
          sy[lane] = py[jb + lane];
          sz[lane] = pz[jb + lane];
          sq[lane] = qs[jb + lane];
        }
        __syncthreads();
        for (int k = split; k < cnt; k += S) {
          const double dx = xi - sx[k], dy = yi - sy[k], dz = zi - sz[k];
          const double r2 = dx * dx + dy * dy + dz * dz;
          const double ir = r2 > 0.0 ? rsqrt(r2) : 0.0;
          const double qir = sq[k] * ir;
          ph += qir;
          const double s3 = qir * ir * ir;
          fx += s3 * dx;
          fy += s3 * dy;
          fz += s3 * dz;
        }
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
      const double qi = qs[i];
      phi[i] = ph;
      f[3 * i] = qi * fx;
      f[3 * i + 1] = qi * fy;
      f[3 * i + 2] = qi * fz;
    }
  }
}

// FP32 near field.  The pair difference is taken in FP64 (full rate on this
// chip) and rounded once, so it carries a relative error of 2^-24 of the
// distance itself however close the pair is; r^2, rsqrt (v_rsq_f32) and the
// products are FP32; partial sums over one source leaf are kept in FP32 and
// folded into FP64 accumulators.
__global__ __launch_bounds__(64) void p2p_f32_kernel(
    const double* __restrict__ px, const double* __restrict__ py,
    const double* __restrict__ pz, const float4* __restrict__ prel,
    const int* __restrict__ leaf_start, const int* __restrict__ near,
    const double* __restrict__ qs, double* __restrict__ phi, double* __restrict__ f) {
  __shared__ double sx[64], sy[64], sz[64];
  __shared__ float sq[64];
  const int a = blockIdx.x, lane = threadIdx.x;
  const int t0 = leaf_start[a], nt = leaf_start[a + 1] - t0;
  const int P = p2p_groups(nt);
  const int S = 64 / P;
  const int split = lane / P;
  for (int tb = 0; tb < nt; tb += 64) {
    const int ti = tb + (lane % P);
    const bool valid = ti < nt;
    const int it = t0 + (valid ? ti : 0);
    const double xi = px[it], yi = py[it], zi = pz[it];
    double ph = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
    for (int sl = 0; sl < 27; ++sl) {
      const int b = near[27 * a + sl];
      if (b < 0) continue;
      const int j0 = leaf_start[b], j1 = leaf_start[b + 1];
      float p32 = 0.f, x32 = 0.f, y32 = 0.f, z32 = 0.f;
      for (int jb = j0; jb < j1; jb += 64) {
        const int cnt = min(64, j1 - jb);
        __syncthreads();
        if (lane < cnt) {
          sx[lane] = px[jb + lane];
          sy[lane] = py[jb + lane];
          sz[lane] = pz[jb + lane];
          sq[lane] = prel[jb + lane].w;
        }
        __syncthreads();
        for (int k = split; k < cnt; k += S) {
          const float dx = float(xi - sx[k]), dy = float(yi - sy[k]), dz = float(zi - sz[k]);
          const float r2 = dx * dx + dy * dy + dz * dz;
          const float ir = r2 > 0.f ? __builtin_amdgcn_rsqf(r2) : 0.f;
          const float qir = sq[k] * ir;
          p32 += qir;
          const float s3 = qir * ir * ir;
          x32 += s3 * dx;
          y32 += s3 * dy;
          z32 += s3 * dz;
        }
      }
      ph += double(p32);
      fx += double(x32);
      fy += double(y32);
      fz += double(z32);
    }
    for (int o = P; o < 64; o <<= 1) {
      ph += __shfl_xor(ph, o, 64);
      fx += __shfl_xor(fx, o, 64);
      fy += __shfl_xor(fy, o, 64);
      fz += __shfl_xor(fz, o, 64);
    }
    if (valid && split == 0) {
      const int i = t0 + ti;
      const double qi = qs[i];
      phi[i] = ph;
      f[3 * i] = qi * fx;
      f[3 * i + 1] = qi * fy;
      f[3 * i + 2] = qi * fz;
    }
  }
}

// ------------------------------------------------------- gather / combine
__global__ void gather_q_kernel(const double* __restrict__ q, const int* __restrict__ perm,
                                int64_t n, double* __restrict__ qs, float4* __restrict__ prel) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = q[perm[i]];
  qs[i] = v;
  prel[i].w = float(v);
}

__global__ void cast_kernel(const double* __restrict__ in, float* __restrict__ out, int64_t n) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = float(in[i]);
}

// out[perm[i]] = near[i] + far[i] (FP64); far absent when the tree has no
// level >= 2.  With separate outputs the parts are un-permuted as they are.
__global__ void combine_kernel(const int* __restrict__ perm, int64_t n,
                               const double* __restrict__ pn, const double* __restrict__ fn,
                               const double* __restrict__ pf, const double* __restrict__ ff,
                               double* __restrict__ phi, double* __restrict__ f,
                               double* __restrict__ phi_n, double* __restrict__ f_n,
                               double* __restrict__ phi_f, double* __restrict__ f_f) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t o = perm[i];
  const double a = pn[i], b = pf ? pf[i] : 0.0;
  const double ax = fn[3 * i], ay = fn[3 * i + 1], az = fn[3 * i + 2];
  const double bx = ff ? ff[3 * i] : 0.0, by = ff ? ff[3 * i + 1] : 0.0,
               bz = ff ? ff[3 * i + 2] : 0.0;
  if (phi) {
    phi[o] = a + b;
    f[3 * o] = ax + bx;
    f[3 * o + 1] = ay + by;
    f[3 * o + 2] = az + bz;
  }
  if (phi_n) {
    phi_n[o] = a;
    f_n[3 * o] = ax;
    f_n[3 * o + 1] = ay;
    f_n[3 * o + 2] = az;
    phi_f[o] = b;
    f_f[3 * o] = bx;
    f_f[3 * o + 1] = by;
    f_f[3 * o + 2] = bz;
  }
}

// ---------------------------------------------------------------- driver
template <template <int> class K>
struct ByOrder;

#define FMM_ORDER_SWITCH(L, CALL)                 \
  switch (L) {                                    \
    case 1: CALL(1); break;                       \
    case 2: CALL(2); break;                       \
    case 3: CALL(3); break;                       \
    case 4: CALL(4); break;                       \
    case 5: CALL(5); break;                       \
    case 6: CALL(6); break;                       \
    case 7: CALL(7); break;                       \
    case 8: CALL(8); break;                       \
    case 9: CALL(9); break;                       \
    case 10: CALL(10); break;                     \
    case 11: CALL(11); break;                     \
    default: CALL(12); break;                     \
  }

static inline unsigned grid_for(int64_t n, int b) { return unsigned((n + b - 1) / b); }

void evaluate(fmm_plan_s* p, const double* q, double* phi, double* f, double* phi_n,
              double* f_n, double* phi_f, double* f_f, hipStream_t s) {
  const int64_t n = p->n;
  const int h = p->height, L = p->order;
  const OpSet* op = p->ops;
  const bool mixed = p->precision == FMM_MIXED_FP32;
  const int64_t nl = p->nleaf;
  const LevelView& leaf = p->lev[h - 1];
  LeafGeom geo{p->lo[0], p->lo[1], p->lo[2], p->L / double(int64_t(1) << (h - 1)), h - 1};

  gather_q_kernel<<<grid_for(n, 256), 256, 0, s>>>(q, p->perm, n, p->qs, p->prel);
  FMM_HIP_CHECK(hipGetLastError());

  const bool far = h >= 3;
  if (far) {
    const int p2m_threads = L * L <= 64 ? 64 : (L * L <= 128 ? 128 : 256);
#define P2M_CALL(LL)                                                                     \
  p2m_kernel<LL><<<unsigned(nl), p2m_threads, 0, s>>>(p->px, p->py, p->pz, p->qs,       \
                                                      p->leaf_start, leaf.keys, geo,     \
                                                      op->cheb, p->W, leaf.off, op->ld)
    FMM_ORDER_SWITCH(L, P2M_CALL)
#undef P2M_CALL
    FMM_HIP_CHECK(hipGetLastError());
    for (int l = h - 2; l >= 2; --l) {
      m2m_kernel<<<unsigned(p->lev[l].ncell), kTransThreads, 0, s>>>(
          p->lev[l].child_start, p->lev[l + 1].keys, p->lev[l].off, p->lev[l + 1].off,
          op->child, L, op->ld, p->W);
      FMM_HIP_CHECK(hipGetLastError());
    }
    if (mixed) {
      const int64_t first = p->lev[2].off * op->ld;
      const int64_t cnt = (p->ncell_total + 1) * op->ld - first;
      cast_kernel<<<grid_for(cnt, 256), 256, 0, s>>>(p->W + first, p->W32 + first, cnt);
      FMM_HIP_CHECK(hipGetLastError());
    }
    launch_m2l(p, mixed, s);
    for (int l = 2; l <= h - 2; ++l) {
      l2l_kernel<<<unsigned(p->lev[l + 1].ncell), kTransThreads, 0, s>>>(
          p->lev[l + 1].parent, p->lev[l + 1].keys, p->lev[l].off, p->lev[l + 1].off,
          op->child, L, op->ld, p->Loc);
      FMM_HIP_CHECK(hipGetLastError());
    }
#define L2P_CALL(LL)                                                                     \
  l2p_kernel<LL><<<unsigned(nl), 64, 0, s>>>(p->px, p->py, p->pz, p->qs, p->leaf_start,  \
                                             leaf.keys, geo, op->cheb, p->Loc, leaf.off, \
                                             op->ld, p->phi_f, p->f_f)
    FMM_ORDER_SWITCH(L, L2P_CALL)
#undef L2P_CALL
    FMM_HIP_CHECK(hipGetLastError());
  }

  if (mixed)
    p2p_f32_kernel<<<unsigned(nl), 64, 0, s>>>(p->px, p->py, p->pz, p->prel, p->leaf_start,
                                               p->near, p->qs, p->phi_n, p->f_n);
  else
    p2p_f64_kernel<<<unsigned(nl), 64, 0, s>>>(p->px, p->py, p->pz, p->qs, p->leaf_start,
                                               p->near, p->phi_n, p->f_n);
  FMM_HIP_CHECK(hipGetLastError());

  combine_kernel<<<grid_for(n, 256), 256, 0, s>>>(
      p->perm, n, p->phi_n, p->f_n, far ? p->phi_f : nullptr, far ? p->f_f : nullptr, phi, f,
      phi_n, f_n, phi_f, f_f);
  FMM_HIP_CHECK(hipGetLastError());
}

}  // namespace fmm
