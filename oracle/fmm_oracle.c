/*
 * Oracle for the FMM evaluation pass: plain FP64, CPU only.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  It shares no code
 * with the HIP implementation.
 *
 * Every step is written the plain way, in the order the method defines it,
 * with no blocking, fusion or reordering:
 *   direct sum         Eq. (1) with P and F of Eq. (2)
 *   Chebyshev basis    Eq. (5): S(xb_m; u) = 1/l + 2/l sum_{n=1}^{l-1} T_n(xb_m) T_n(u)
 *   tensor basis       Eq. (4): S_m(x) = S_{m1}(x1) S_{m2}(x2) S_{m3}(x3)
 *   P2M, M2M, L2L, L2P interpolation operators of Eq. (3) (Sec. 2.1)
 *   M2L                point-wise kernel between Chebyshev nodes, Eq. (3);
 *                      dense matrices, evaluated per (level, offset)
 *   P2P                Eq. (1) restricted to the near field (Sec. 2)
 *   octree / Morton    Sec. 3.2 (tree of height h) and Sec. 4.2 (Morton order)
 *   lists              Sec. 2.1.2: near field = the 27 cells around a cell,
 *                      far field = children of the parent's near cells that
 *                      are not near the cell (at most 189)
 *
 * Readings where the paper is silent (kept identical in the HIP path only by
 * agreement on the definition, never by shared code):
 *   - root box: per-axis minimum lo, side L = max extent (L = 1 if zero);
 *   - leaf coordinate k = min(floor((x - lo) / L * 2^(h-1)), 2^(h-1) - 1);
 *   - Morton key: bit b of kx, ky, kz at key bits 3b, 3b+1, 3b+2;
 *   - particles sorted by (key, original index);
 *   - F_i carries the target charge: F_i = q_i sum_j q_j (x_i-x_j)/r^3;
 *   - zero-distance pairs (and j = i) are skipped;
 *   - order l = number of Chebyshev nodes per dimension.
 *
 * Compiled with -ffp-contract=off so every expression rounds as written.
 */
#include "fmm_oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define MAXO ORACLE_MAX_ORDER
#define MAXH ORACLE_MAX_HEIGHT

static const double kPi = 3.14159265358979323846;

static int g_threads = 0;
void oracle_set_threads(int nthreads) { g_threads = nthreads > 0 ? nthreads : 0; }
int oracle_get_threads(void) {
  return g_threads > 0 ? g_threads : omp_get_max_threads();
}

/* ------------------------------------------------------------------------ */
/* Eq. (1)-(2) for the kernel family P(x, y) = |x - y|^-p, p = 1 (the paper's
 * Laplace kernel) or p = 2 (a second homogeneous kernel, Sec. 2.1: the
 * black-box scheme needs only point evaluations of P).  One source j acting
 * on target i: phi += q_j r^-p, and the force factor -grad_x P = p r^-(p+2) d
 * with d = x_i - x_j.  Zero-distance pairs are skipped.                      */
static inline void pair_accumulate(int p, const double* xi, const double* xj,
                                   double qj, double* phi, double* fx,
                                   double* fy, double* fz) {
  double dx = xi[0] - xj[0];
  double dy = xi[1] - xj[1];
  double dz = xi[2] - xj[2];
  double r2 = (dx * dx + dy * dy) + dz * dz;
  if (r2 == 0.0) return;
  double s;
  if (p == 2) {
    double ir2 = 1.0 / r2;
    *phi += qj * ir2;
    s = 2.0 * qj * ir2 * ir2;
  } else {
    double ir = 1.0 / sqrt(r2);
    *phi += qj * ir;
    s = qj * ir * ir * ir;
  }
  *fx += s * dx;
  *fy += s * dy;
  *fz += s * dz;
}

/* the kernel at distance^2 r2 (r2 > 0) */
static inline double kernel_value(int p, double r2) {
  return p == 2 ? 1.0 / r2 : 1.0 / sqrt(r2);
}

static int valid_kernel(int p) { return p == 1 || p == 2; }

int oracle_direct(const double* pos, int64_t n, const double* q, double* phi,
                  double* f) {
  return oracle_direct_k(pos, n, q, phi, f, 1);
}

int oracle_direct_k(const double* pos, int64_t n, const double* q, double* phi,
                    double* f, int p) {
  if (n < 0 || (n > 0 && (!pos || !q || !phi || !f)) || !valid_kernel(p)) return -1;
#pragma omp parallel for schedule(static) num_threads(oracle_get_threads())
  for (int64_t i = 0; i < n; ++i) {
    double ph = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
    for (int64_t j = 0; j < n; ++j)
      pair_accumulate(p, &pos[3 * i], &pos[3 * j], q[j], &ph, &fx, &fy, &fz);
    phi[i] = ph;
    f[3 * i + 0] = q[i] * fx;
    f[3 * i + 1] = q[i] * fy;
    f[3 * i + 2] = q[i] * fz;
  }
  return 0;
}

int oracle_direct_sampled(const double* pos, int64_t n, const double* q,
                          const int64_t* idx, int64_t s, double* phi,
                          double* f) {
  return oracle_direct_sampled_k(pos, n, q, idx, s, phi, f, 1);
}

int oracle_direct_sampled_k(const double* pos, int64_t n, const double* q,
                            const int64_t* idx, int64_t s, double* phi,
                            double* f, int p) {
  if (n < 0 || s < 0 || (s > 0 && (!pos || !q || !idx || !phi || !f)) ||
      !valid_kernel(p))
    return -1;
  for (int64_t k = 0; k < s; ++k)
    if (idx[k] < 0 || idx[k] >= n) return -1;
#pragma omp parallel for schedule(static) num_threads(oracle_get_threads())
  for (int64_t k = 0; k < s; ++k) {
    int64_t i = idx[k];
    double ph = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
    for (int64_t j = 0; j < n; ++j)
      pair_accumulate(p, &pos[3 * i], &pos[3 * j], q[j], &ph, &fx, &fy, &fz);
    phi[k] = ph;
    f[3 * k + 0] = q[i] * fx;
    f[3 * k + 1] = q[i] * fy;
    f[3 * k + 2] = q[i] * fz;
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Eq. (5): Chebyshev roots and the 1-D interpolation polynomial.            */
typedef struct {
  int l;
  double xi[MAXO];       /* nodes xb_m, m = 0..l-1 */
  double Txi[MAXO][MAXO]; /* T_n(xb_m) */
} basis_t;

/* T_0..T_{l-1} at x by the three-term recurrence */
static void cheb_T(int l, double x, double* T) {
  T[0] = 1.0;
  if (l > 1) T[1] = x;
  for (int n = 2; n < l; ++n) T[n] = 2.0 * x * T[n - 1] - T[n - 2];
}

/* derivatives T'_0..T'_{l-1} at x, given T: T'_n = 2T_{n-1} + 2x T'_{n-1} - T'_{n-2} */
static void cheb_dT(int l, double x, const double* T, double* dT) {
  dT[0] = 0.0;
  if (l > 1) dT[1] = 1.0;
  for (int n = 2; n < l; ++n)
    dT[n] = 2.0 * T[n - 1] + 2.0 * x * dT[n - 1] - dT[n - 2];
}

static void basis_init(basis_t* b, int l) {
  b->l = l;
  /* roots of T_l: cos((2m+1) pi / (2l)), m = 0..l-1 (the paper's m = 1..l) */
  for (int m = 0; m < l; ++m) b->xi[m] = cos((2.0 * m + 1.0) * kPi / (2.0 * l));
  /* exact mirror symmetry and an exact zero node for odd l */
  for (int m = 0; m < l / 2; ++m) b->xi[l - 1 - m] = -b->xi[m];
  if (l % 2) b->xi[l / 2] = 0.0;
  for (int m = 0; m < l; ++m) cheb_T(l, b->xi[m], b->Txi[m]);
}

/* S(xb_m; u) for m = 0..l-1 */
static void basis_S(const basis_t* b, double u, double* S) {
  const int l = b->l;
  double Tu[MAXO];
  cheb_T(l, u, Tu);
  for (int m = 0; m < l; ++m) {
    double s = 0.0;
    for (int n = 1; n < l; ++n) s += b->Txi[m][n] * Tu[n];
    S[m] = 1.0 / l + 2.0 / l * s;
  }
}

/* S and dS/du for m = 0..l-1 */
static void basis_S_dS(const basis_t* b, double u, double* S, double* dS) {
  const int l = b->l;
  double Tu[MAXO], dTu[MAXO];
  cheb_T(l, u, Tu);
  cheb_dT(l, u, Tu, dTu);
  for (int m = 0; m < l; ++m) {
    double s = 0.0, ds = 0.0;
    for (int n = 1; n < l; ++n) {
      s += b->Txi[m][n] * Tu[n];
      ds += b->Txi[m][n] * dTu[n];
    }
    S[m] = 1.0 / l + 2.0 / l * s;
    dS[m] = 2.0 / l * ds;
  }
}

int oracle_cheb_nodes(int l, double* xi) {
  if (l < 1 || l > MAXO || !xi) return -1;
  basis_t b;
  basis_init(&b, l);
  for (int m = 0; m < l; ++m) xi[m] = b.xi[m];
  return 0;
}

double oracle_cheb_S(int l, int m, double u) {
  if (l < 1 || l > MAXO || m < 0 || m >= l) return NAN;
  basis_t b;
  basis_init(&b, l);
  double S[MAXO];
  basis_S(&b, u, S);
  return S[m];
}

double oracle_cheb_dS(int l, int m, double u) {
  if (l < 1 || l > MAXO || m < 0 || m >= l) return NAN;
  basis_t b;
  basis_init(&b, l);
  double S[MAXO], dS[MAXO];
  basis_S_dS(&b, u, S, dS);
  return dS[m];
}

/* ------------------------------------------------------------------------ */
/* Interpolation operators (Eq. 3-4).  Coefficient index m = (m1*l+m2)*l+m3 */
/* with m1 along x, m2 along y, m3 along z.                                 */

/* P2M: W[m] += sum_j q_j S_m((y_j - c) / a) */
static void p2m_points(const basis_t* b, int64_t n, const double* pos,
                       const double* q, const double* c, double a,
                       double* W) {
  const int l = b->l;
  double Sx[MAXO], Sy[MAXO], Sz[MAXO];
  for (int64_t j = 0; j < n; ++j) {
    basis_S(b, (pos[3 * j + 0] - c[0]) / a, Sx);
    basis_S(b, (pos[3 * j + 1] - c[1]) / a, Sy);
    basis_S(b, (pos[3 * j + 2] - c[2]) / a, Sz);
    for (int m1 = 0; m1 < l; ++m1)
      for (int m2 = 0; m2 < l; ++m2)
        for (int m3 = 0; m3 < l; ++m3)
          W[(m1 * l + m2) * l + m3] += q[j] * Sx[m1] * Sy[m2] * Sz[m3];
  }
}

/* Child-to-parent interpolation matrix for child octant o:
 * M[m][m'] = prod_d S(xb_{m_d}; (sigma_d + xb_{m'_d}) / 2),
 * sigma_d = +1 if bit d of o is set, else -1.  The child's node m' sits at
 * (sigma + xb_{m'}) / 2 in the parent's normalised coordinates. */
static double* child_matrix(const basis_t* b, int o) {
  const int l = b->l, l3 = l * l * l;
  double S1[3][MAXO][MAXO]; /* S1[d][m][m'] */
  for (int d = 0; d < 3; ++d) {
    double sigma = ((o >> d) & 1) ? 1.0 : -1.0;
    for (int mp = 0; mp < l; ++mp) {
      double S[MAXO];
      basis_S(b, (sigma + b->xi[mp]) / 2.0, S);
      for (int m = 0; m < l; ++m) S1[d][m][mp] = S[m];
    }
  }
  double* M = (double*)malloc(sizeof(double) * (size_t)l3 * l3);
  if (!M) return NULL;
  for (int m1 = 0; m1 < l; ++m1)
    for (int m2 = 0; m2 < l; ++m2)
      for (int m3 = 0; m3 < l; ++m3)
        for (int p1 = 0; p1 < l; ++p1)
          for (int p2 = 0; p2 < l; ++p2)
            for (int p3 = 0; p3 < l; ++p3)
              M[(size_t)((m1 * l + m2) * l + m3) * l3 + (p1 * l + p2) * l + p3] =
                  S1[0][m1][p1] * S1[1][m2][p2] * S1[2][m3][p3];
  return M;
}

/* M2M: Wp[m] += sum_{m'} M[m][m'] Wc[m'] */
static void m2m_apply(int l3, const double* M, const double* Wc, double* Wp) {
  for (int m = 0; m < l3; ++m) {
    double s = 0.0;
    for (int mp = 0; mp < l3; ++mp) s += M[(size_t)m * l3 + mp] * Wc[mp];
    Wp[m] += s;
  }
}

/* L2L: Lc[m'] += sum_m M[m][m'] Lp[m] */
static void l2l_apply(int l3, const double* M, const double* Lp, double* Lc) {
  for (int mp = 0; mp < l3; ++mp) {
    double s = 0.0;
    for (int m = 0; m < l3; ++m) s += M[(size_t)m * l3 + mp] * Lp[m];
    Lc[mp] += s;
  }
}

/* L2P: phi = sum_m S_m(u) Loc[m]; F = -q (1/a) sum_m grad_u S_m(u) Loc[m] */
static void l2p_point(const basis_t* b, const double* x, double qi,
                      const double* c, double a, const double* Loc,
                      double* phi, double* f) {
  const int l = b->l;
  double Sx[MAXO], Sy[MAXO], Sz[MAXO], dSx[MAXO], dSy[MAXO], dSz[MAXO];
  basis_S_dS(b, (x[0] - c[0]) / a, Sx, dSx);
  basis_S_dS(b, (x[1] - c[1]) / a, Sy, dSy);
  basis_S_dS(b, (x[2] - c[2]) / a, Sz, dSz);
  double p = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
  for (int m1 = 0; m1 < l; ++m1)
    for (int m2 = 0; m2 < l; ++m2)
      for (int m3 = 0; m3 < l; ++m3) {
        double v = Loc[(m1 * l + m2) * l + m3];
        p += Sx[m1] * Sy[m2] * Sz[m3] * v;
        gx += dSx[m1] * Sy[m2] * Sz[m3] * v;
        gy += Sx[m1] * dSy[m2] * Sz[m3] * v;
        gz += Sx[m1] * Sy[m2] * dSz[m3] * v;
      }
  *phi = p;
  f[0] = -qi * (gx / a);
  f[1] = -qi * (gy / a);
  f[2] = -qi * (gz / a);
}

/* M2L: K[m][n] = P(x_m, y_n) with x_m = c + a xb_m (target cell) and
 * y_n = c + w t + a xb_n (source cell), i.e. |a (xb_m - xb_n) - w t|^-p. */
static void m2l_matrix(int p, const basis_t* b, double a, double w, const int* t,
                       double* K) {
  const int l = b->l, l3 = l * l * l;
  for (int m1 = 0; m1 < l; ++m1)
    for (int m2 = 0; m2 < l; ++m2)
      for (int m3 = 0; m3 < l; ++m3)
        for (int n1 = 0; n1 < l; ++n1)
          for (int n2 = 0; n2 < l; ++n2)
            for (int n3 = 0; n3 < l; ++n3) {
              double dx = a * (b->xi[m1] - b->xi[n1]) - w * t[0];
              double dy = a * (b->xi[m2] - b->xi[n2]) - w * t[1];
              double dz = a * (b->xi[m3] - b->xi[n3]) - w * t[2];
              double r2 = (dx * dx + dy * dy) + dz * dz;
              K[(size_t)((m1 * l + m2) * l + m3) * l3 + (n1 * l + n2) * l + n3] =
                  kernel_value(p, r2);
            }
}

int oracle_p2m(int l, int64_t n, const double* pos, const double* q,
               const double* c, double a, double* W) {
  if (l < 1 || l > MAXO || n < 0 || !c || !W || (n > 0 && (!pos || !q)) ||
      !(a > 0.0))
    return -1;
  basis_t b;
  basis_init(&b, l);
  p2m_points(&b, n, pos, q, c, a, W);
  return 0;
}

int oracle_m2m(int l, int octant, const double* Wc, double* Wp) {
  if (l < 1 || l > MAXO || octant < 0 || octant > 7 || !Wc || !Wp) return -1;
  basis_t b;
  basis_init(&b, l);
  double* M = child_matrix(&b, octant);
  if (!M) return -2;
  m2m_apply(l * l * l, M, Wc, Wp);
  free(M);
  return 0;
}

int oracle_l2l(int l, int octant, const double* Lp, double* Lc) {
  if (l < 1 || l > MAXO || octant < 0 || octant > 7 || !Lp || !Lc) return -1;
  basis_t b;
  basis_init(&b, l);
  double* M = child_matrix(&b, octant);
  if (!M) return -2;
  l2l_apply(l * l * l, M, Lp, Lc);
  free(M);
  return 0;
}

int oracle_l2p(int l, int64_t n, const double* pos, const double* q,
               const double* c, double a, const double* Loc, double* phi,
               double* f) {
  if (l < 1 || l > MAXO || n < 0 || !c || !Loc || !(a > 0.0) ||
      (n > 0 && (!pos || !q || !phi || !f)))
    return -1;
  basis_t b;
  basis_init(&b, l);
  for (int64_t i = 0; i < n; ++i)
    l2p_point(&b, &pos[3 * i], q[i], c, a, Loc, &phi[i], &f[3 * i]);
  return 0;
}

int oracle_m2l_matrix(int l, double a, double w, const int* t, double* K) {
  return oracle_m2l_matrix_k(l, a, w, t, K, 1);
}

int oracle_m2l_matrix_k(int l, double a, double w, const int* t, double* K,
                        int p) {
  if (l < 1 || l > MAXO || !t || !K || !(a > 0.0) || !(w > 0.0) ||
      !valid_kernel(p))
    return -1;
  basis_t b;
  basis_init(&b, l);
  m2l_matrix(p, &b, a, w, t, K);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Octree in Morton order.                                                  */
struct oracle_tree {
  int64_t n;
  int h;
  double lo[3], L;
  double* pos_s;     /* [n][3] positions in sorted order */
  uint64_t* key;     /* [n] sorted keys */
  int64_t* perm;     /* sorted position -> original index */
  int64_t* inv;      /* original index -> sorted position */
  int64_t* leaf_of;  /* sorted position -> leaf */
  int64_t nleaf;
  int64_t* leaf_start; /* [nleaf+1] */
  int64_t ncell[MAXH];
  uint64_t* ckey[MAXH];     /* sorted unique cell keys per level */
  int64_t* parent[MAXH];    /* parent index (level l-1), l >= 1 */
  int64_t* child_start[MAXH]; /* children of level-l cells in level l+1: [ncell+1] */
  int64_t* near_off;
  int64_t* near_idx;
  int64_t* far_off[MAXH];
  int64_t* far_idx[MAXH];
};

static uint64_t morton_encode(uint64_t x, uint64_t y, uint64_t z, int bits) {
  uint64_t k = 0;
  for (int b = 0; b < bits; ++b) {
    k |= ((x >> b) & 1ull) << (3 * b);
    k |= ((y >> b) & 1ull) << (3 * b + 1);
    k |= ((z >> b) & 1ull) << (3 * b + 2);
  }
  return k;
}

static void morton_decode(uint64_t k, int bits, int64_t* c) {
  c[0] = c[1] = c[2] = 0;
  for (int b = 0; b < bits; ++b) {
    c[0] |= (int64_t)((k >> (3 * b)) & 1ull) << b;
    c[1] |= (int64_t)((k >> (3 * b + 1)) & 1ull) << b;
    c[2] |= (int64_t)((k >> (3 * b + 2)) & 1ull) << b;
  }
}

/* index of key in sorted unique array, or -1 */
static int64_t find_key(const uint64_t* keys, int64_t n, uint64_t k) {
  int64_t lo = 0, hi = n - 1;
  while (lo <= hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (keys[mid] == k) return mid;
    if (keys[mid] < k) lo = mid + 1;
    else hi = mid - 1;
  }
  return -1;
}

typedef struct {
  uint64_t key;
  int64_t idx;
} keyidx_t;

static int cmp_keyidx(const void* a, const void* b) {
  const keyidx_t* x = (const keyidx_t*)a;
  const keyidx_t* y = (const keyidx_t*)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  if (x->idx != y->idx) return x->idx < y->idx ? -1 : 1;
  return 0;
}

static int cmp_i64(const void* a, const void* b) {
  int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
  return (x > y) - (x < y);
}

void oracle_tree_free(oracle_tree* t) {
  if (!t) return;
  free(t->pos_s);
  free(t->key);
  free(t->perm);
  free(t->inv);
  free(t->leaf_of);
  free(t->leaf_start);
  for (int l = 0; l < MAXH; ++l) {
    free(t->ckey[l]);
    free(t->parent[l]);
    free(t->child_start[l]);
    free(t->far_off[l]);
    free(t->far_idx[l]);
  }
  free(t->near_off);
  free(t->near_idx);
  free(t);
}

oracle_tree* oracle_tree_build(const double* pos, int64_t n, int h) {
  if (!pos || n < 1 || h < 1 || h > MAXH) return NULL;
  for (int64_t i = 0; i < 3 * n; ++i)
    if (!isfinite(pos[i])) return NULL;
  oracle_tree* t = (oracle_tree*)calloc(1, sizeof(oracle_tree));
  if (!t) return NULL;
  t->n = n;
  t->h = h;
  const int bits = h - 1;
  const int64_t side = (int64_t)1 << bits; /* leaves per dimension */

  /* root cube */
  double hi[3];
  for (int d = 0; d < 3; ++d) t->lo[d] = hi[d] = pos[d];
  for (int64_t i = 1; i < n; ++i)
    for (int d = 0; d < 3; ++d) {
      if (pos[3 * i + d] < t->lo[d]) t->lo[d] = pos[3 * i + d];
      if (pos[3 * i + d] > hi[d]) hi[d] = pos[3 * i + d];
    }
  t->L = 0.0;
  for (int d = 0; d < 3; ++d)
    if (hi[d] - t->lo[d] > t->L) t->L = hi[d] - t->lo[d];
  if (t->L == 0.0) t->L = 1.0;

  /* keys and the stable sort by (key, original index) */
  keyidx_t* ki = (keyidx_t*)malloc(sizeof(keyidx_t) * (size_t)n);
  if (!ki) { oracle_tree_free(t); return NULL; }
  for (int64_t i = 0; i < n; ++i) {
    uint64_t k3[3];
    for (int d = 0; d < 3; ++d) {
      double u = (pos[3 * i + d] - t->lo[d]) / t->L;
      double s = floor(u * (double)side);
      int64_t k = (int64_t)s;
      if (k > side - 1) k = side - 1;
      if (k < 0) k = 0;
      k3[d] = (uint64_t)k;
    }
    ki[i].key = morton_encode(k3[0], k3[1], k3[2], bits);
    ki[i].idx = i;
  }
  qsort(ki, (size_t)n, sizeof(keyidx_t), cmp_keyidx);

  t->pos_s = (double*)malloc(sizeof(double) * 3 * (size_t)n);
  t->key = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
  t->perm = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  t->inv = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  t->leaf_of = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  t->leaf_start = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n + 1));
  if (!t->pos_s || !t->key || !t->perm || !t->inv || !t->leaf_of ||
      !t->leaf_start) {
    free(ki);
    oracle_tree_free(t);
    return NULL;
  }
  for (int64_t i = 0; i < n; ++i) {
    t->key[i] = ki[i].key;
    t->perm[i] = ki[i].idx;
    t->inv[ki[i].idx] = i;
    for (int d = 0; d < 3; ++d) t->pos_s[3 * i + d] = pos[3 * ki[i].idx + d];
  }
  free(ki);

  /* leaves: runs of equal keys */
  int64_t nl = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (i == 0 || t->key[i] != t->key[i - 1]) t->leaf_start[nl++] = i;
    t->leaf_of[i] = nl - 1;
  }
  t->leaf_start[nl] = n;
  t->nleaf = nl;

  /* cells per level; leaf level = h-1 */
  t->ncell[h - 1] = nl;
  t->ckey[h - 1] = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)nl);
  for (int64_t c = 0; c < nl; ++c) t->ckey[h - 1][c] = t->key[t->leaf_start[c]];
  for (int l = h - 2; l >= 0; --l) {
    int64_t nc = t->ncell[l + 1];
    const uint64_t* ck = t->ckey[l + 1];
    t->ckey[l] = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)nc);
    t->parent[l + 1] = (int64_t*)malloc(sizeof(int64_t) * (size_t)nc);
    t->child_start[l] = (int64_t*)malloc(sizeof(int64_t) * ((size_t)nc + 1));
    int64_t np = 0;
    for (int64_t c = 0; c < nc; ++c) {
      uint64_t pk = ck[c] >> 3;
      if (c == 0 || pk != (ck[c - 1] >> 3)) {
        t->child_start[l][np] = c;
        t->ckey[l][np++] = pk;
      }
      t->parent[l + 1][c] = np - 1;
    }
    t->child_start[l][np] = nc;
    t->ncell[l] = np;
  }

  /* near lists over leaves: all non-empty leaves within one cell in every
   * dimension (the leaf itself included), ascending key. */
  t->near_off = (int64_t*)malloc(sizeof(int64_t) * ((size_t)nl + 1));
  t->near_idx = (int64_t*)malloc(sizeof(int64_t) * 27 * (size_t)nl);
  int64_t cnt = 0;
  for (int64_t a = 0; a < nl; ++a) {
    int64_t ca[3], buf[27];
    int nb = 0;
    morton_decode(t->ckey[h - 1][a], bits, ca);
    for (int dx = -1; dx <= 1; ++dx)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dz = -1; dz <= 1; ++dz) {
          int64_t b0 = ca[0] + dx, b1 = ca[1] + dy, b2 = ca[2] + dz;
          if (b0 < 0 || b1 < 0 || b2 < 0 || b0 >= side || b1 >= side ||
              b2 >= side)
            continue;
          int64_t j = find_key(t->ckey[h - 1], nl,
                               morton_encode(b0, b1, b2, bits));
          if (j >= 0) buf[nb++] = j;
        }
    qsort(buf, (size_t)nb, sizeof(int64_t), cmp_i64);
    t->near_off[a] = cnt;
    for (int k = 0; k < nb; ++k) t->near_idx[cnt++] = buf[k];
  }
  t->near_off[nl] = cnt;

  /* far lists per level >= 2: children of the parent's near cells that are
   * not adjacent to the cell, ascending key. */
  for (int l = 2; l < h; ++l) {
    const int64_t nc = t->ncell[l];
    const int64_t sd = (int64_t)1 << l;
    t->far_off[l] = (int64_t*)malloc(sizeof(int64_t) * ((size_t)nc + 1));
    t->far_idx[l] = (int64_t*)malloc(sizeof(int64_t) * 189 * ((size_t)nc + 1));
    int64_t fc = 0;
    for (int64_t c = 0; c < nc; ++c) {
      int64_t cc[3], buf[216];
      int nb = 0;
      morton_decode(t->ckey[l][c], l, cc);
      for (int ex = -1; ex <= 1; ++ex)
        for (int ey = -1; ey <= 1; ++ey)
          for (int ez = -1; ez <= 1; ++ez) {
            int64_t p0 = (cc[0] >> 1) + ex, p1 = (cc[1] >> 1) + ey,
                    p2 = (cc[2] >> 1) + ez;
            if (p0 < 0 || p1 < 0 || p2 < 0 || p0 >= sd / 2 || p1 >= sd / 2 ||
                p2 >= sd / 2)
              continue;
            for (int o = 0; o < 8; ++o) {
              int64_t b0 = 2 * p0 + (o & 1), b1 = 2 * p1 + ((o >> 1) & 1),
                      b2 = 2 * p2 + ((o >> 2) & 1);
              int64_t d0 = llabs(b0 - cc[0]), d1 = llabs(b1 - cc[1]),
                      d2 = llabs(b2 - cc[2]);
              int64_t dm = d0 > d1 ? d0 : d1;
              dm = dm > d2 ? dm : d2;
              if (dm <= 1) continue;
              int64_t j = find_key(t->ckey[l], nc, morton_encode(b0, b1, b2, l));
              if (j >= 0) buf[nb++] = j;
            }
          }
      qsort(buf, (size_t)nb, sizeof(int64_t), cmp_i64);
      t->far_off[l][c] = fc;
      for (int k = 0; k < nb; ++k) t->far_idx[l][fc++] = buf[k];
    }
    t->far_off[l][nc] = fc;
  }
  return t;
}

int oracle_tree_info(const oracle_tree* t, int64_t* info) {
  if (!t || !info) return -1;
  info[0] = t->n;
  info[1] = t->h;
  info[2] = t->nleaf;
  for (int l = 0; l < t->h; ++l) info[3 + l] = t->ncell[l];
  return 0;
}

int oracle_tree_box(const oracle_tree* t, double* box) {
  if (!t || !box) return -1;
  for (int d = 0; d < 3; ++d) box[d] = t->lo[d];
  box[3] = t->L;
  return 0;
}

int oracle_tree_keys(const oracle_tree* t, uint64_t* keys) {
  if (!t || !keys) return -1;
  memcpy(keys, t->key, sizeof(uint64_t) * (size_t)t->n);
  return 0;
}

int oracle_tree_perm(const oracle_tree* t, int64_t* perm) {
  if (!t || !perm) return -1;
  memcpy(perm, t->perm, sizeof(int64_t) * (size_t)t->n);
  return 0;
}

int oracle_tree_leaf_start(const oracle_tree* t, int64_t* start) {
  if (!t || !start) return -1;
  memcpy(start, t->leaf_start, sizeof(int64_t) * ((size_t)t->nleaf + 1));
  return 0;
}

int oracle_tree_cell_keys(const oracle_tree* t, int level, uint64_t* keys) {
  if (!t || !keys || level < 0 || level >= t->h) return -1;
  memcpy(keys, t->ckey[level], sizeof(uint64_t) * (size_t)t->ncell[level]);
  return 0;
}

int oracle_tree_near(const oracle_tree* t, int64_t* off, int64_t* idx) {
  if (!t || !off) return -1;
  memcpy(off, t->near_off, sizeof(int64_t) * ((size_t)t->nleaf + 1));
  if (idx)
    memcpy(idx, t->near_idx, sizeof(int64_t) * (size_t)t->near_off[t->nleaf]);
  return 0;
}

int oracle_tree_far(const oracle_tree* t, int level, int64_t* off,
                    int64_t* idx) {
  if (!t || !off || level < 2 || level >= t->h) return -1;
  const int64_t nc = t->ncell[level];
  memcpy(off, t->far_off[level], sizeof(int64_t) * ((size_t)nc + 1));
  if (idx)
    memcpy(idx, t->far_idx[level],
           sizeof(int64_t) * (size_t)t->far_off[level][nc]);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* FMM evaluation.                                                          */

/* geometry of a cell at a level: centre c and half-width a */
static void cell_geometry(const oracle_tree* t, int level, uint64_t key,
                          double* c, double* a) {
  int64_t k[3];
  morton_decode(key, level, k);
  double w = t->L / (double)((int64_t)1 << level);
  for (int d = 0; d < 3; ++d) c[d] = t->lo[d] + ((double)k[d] + 0.5) * w;
  *a = w / 2.0;
}

int oracle_fmm(const oracle_tree* t, int l, const double* q,
               const int64_t* targets, int64_t nt, double* phi, double* f,
               double* phi_near, double* f_near, double* phi_far,
               double* f_far) {
  return oracle_fmm_ops(t, l, q, targets, nt, NULL, phi, f, phi_near, f_near,
                        phi_far, f_far, 1);
}

int oracle_fmm_ops(const oracle_tree* t, int l, const double* q,
                   const int64_t* targets, int64_t nt, const double* unit_ops,
                   double* phi, double* f, double* phi_near, double* f_near,
                   double* phi_far, double* f_far, int p) {
  if (!t || !q || l < 1 || l > MAXO || !valid_kernel(p)) return -1;
  const int64_t n = t->n;
  const int h = t->h;
  if (!targets) nt = n;
  if (nt < 0) return -1;
  for (int64_t k = 0; targets && k < nt; ++k)
    if (targets[k] < 0 || targets[k] >= n) return -1;
  const int nth = oracle_get_threads();
  const int l3 = l * l * l;
  basis_t B;
  basis_init(&B, l);

  /* charges in sorted order */
  double* qs = (double*)malloc(sizeof(double) * (size_t)n);
  int64_t* tsorted = (int64_t*)malloc(sizeof(int64_t) * ((size_t)nt + 1));
  double* pn = (double*)calloc((size_t)nt + 1, sizeof(double));
  double* fn = (double*)calloc(3 * (size_t)nt + 1, sizeof(double));
  double* pf = (double*)calloc((size_t)nt + 1, sizeof(double));
  double* ff = (double*)calloc(3 * (size_t)nt + 1, sizeof(double));
  if (!qs || !tsorted || !pn || !fn || !pf || !ff) return -2;
  for (int64_t i = 0; i < n; ++i) qs[i] = q[t->perm[i]];
  for (int64_t k = 0; k < nt; ++k)
    tsorted[k] = targets ? t->inv[targets[k]] : t->inv[k];

  /* ---- far field: exists only when levels >= 2 have cells below the
   * leaf level or at it, i.e. h >= 3 ---- */
  if (h >= 3) {
    double* W[MAXH] = {0};
    double* Loc[MAXH] = {0};
    char* need[MAXH] = {0};
    for (int lv = 2; lv < h; ++lv) {
      W[lv] = (double*)calloc((size_t)t->ncell[lv] * l3, sizeof(double));
      Loc[lv] = (double*)calloc((size_t)t->ncell[lv] * l3, sizeof(double));
      need[lv] = (char*)calloc((size_t)t->ncell[lv] + 1, 1);
      if (!W[lv] || !Loc[lv] || !need[lv]) return -2;
    }
    const int lf = h - 1;

    /* P2M at every leaf */
#pragma omp parallel for schedule(dynamic, 16) num_threads(nth)
    for (int64_t c = 0; c < t->nleaf; ++c) {
      double cc[3], a;
      cell_geometry(t, lf, t->ckey[lf][c], cc, &a);
      int64_t s0 = t->leaf_start[c], s1 = t->leaf_start[c + 1];
      p2m_points(&B, s1 - s0, &t->pos_s[3 * s0], &qs[s0], cc, a,
                 &W[lf][(size_t)c * l3]);
    }

    /* child interpolation matrices for the 8 octants */
    double* M[8];
    for (int o = 0; o < 8; ++o) {
      M[o] = child_matrix(&B, o);
      if (!M[o]) return -2;
    }

    /* M2M upward, levels h-2 .. 2 */
    for (int lv = h - 2; lv >= 2; --lv) {
#pragma omp parallel for schedule(dynamic, 4) num_threads(nth)
      for (int64_t p = 0; p < t->ncell[lv]; ++p)
        for (int64_t c = t->child_start[lv][p]; c < t->child_start[lv][p + 1];
             ++c) {
          int o = (int)(t->ckey[lv + 1][c] & 7ull);
          m2m_apply(l3, M[o], &W[lv + 1][(size_t)c * l3],
                    &W[lv][(size_t)p * l3]);
        }
    }

    /* cells whose local expansion is needed: the targets' leaves and all
     * their ancestors down to level 2 */
    for (int64_t k = 0; k < nt; ++k) {
      int64_t c = t->leaf_of[tsorted[k]];
      for (int lv = lf; lv >= 2; --lv) {
        need[lv][c] = 1;
        if (lv > 0) c = t->parent[lv][c];
      }
    }

    /* downward pass: M2L at level lv, then L2L from level lv-1 */
    for (int lv = 2; lv < h; ++lv) {
      const int64_t nc = t->ncell[lv];
      const double w = t->L / (double)((int64_t)1 << lv);
      const double a = w / 2.0;
      /* M2L matrices for the offsets this level uses */
      double* K[343] = {0};
      char used[343] = {0};
      for (int64_t c = 0; c < nc; ++c) {
        if (!need[lv][c]) continue;
        int64_t cc[3];
        morton_decode(t->ckey[lv][c], lv, cc);
        for (int64_t e = t->far_off[lv][c]; e < t->far_off[lv][c + 1]; ++e) {
          int64_t bb[3];
          morton_decode(t->ckey[lv][t->far_idx[lv][e]], lv, bb);
          int id = (int)((bb[0] - cc[0] + 3) * 49 + (bb[1] - cc[1] + 3) * 7 +
                         (bb[2] - cc[2] + 3));
          used[id] = 1;
        }
      }
      int ids[343], nid = 0;
      for (int id = 0; id < 343; ++id)
        if (used[id]) ids[nid++] = id;
      for (int k = 0; k < nid; ++k) {
        K[ids[k]] = (double*)malloc(sizeof(double) * (size_t)l3 * l3);
        if (!K[ids[k]]) return -2;
      }
#pragma omp parallel for schedule(dynamic, 1) num_threads(nth)
      for (int k = 0; k < nid; ++k) {
        int id = ids[k];
        int tt[3] = {id / 49 - 3, (id / 7) % 7 - 3, id % 7 - 3};
        if (unit_ops) {
          /* given operator between half-width-1 cells, scaled to this level
           * by the kernel's homogeneity: P(a x, a y) = a^-p P(x, y) */
          const double* src = unit_ops + (size_t)id * l3 * l3;
          const double sc = p == 2 ? 1.0 / (a * a) : 1.0 / a;
          for (size_t e = 0; e < (size_t)l3 * l3; ++e) K[id][e] = src[e] * sc;
        } else {
          m2l_matrix(p, &B, a, w, tt, K[id]);
        }
      }

#pragma omp parallel for schedule(dynamic, 4) num_threads(nth)
      for (int64_t c = 0; c < nc; ++c) {
        if (!need[lv][c]) continue;
        double* Lc = &Loc[lv][(size_t)c * l3];
        int64_t cc[3];
        morton_decode(t->ckey[lv][c], lv, cc);
        for (int64_t e = t->far_off[lv][c]; e < t->far_off[lv][c + 1]; ++e) {
          int64_t b = t->far_idx[lv][e];
          int64_t bb[3];
          morton_decode(t->ckey[lv][b], lv, bb);
          int id = (int)((bb[0] - cc[0] + 3) * 49 + (bb[1] - cc[1] + 3) * 7 +
                         (bb[2] - cc[2] + 3));
          const double* Km = K[id];
          const double* Wb = &W[lv][(size_t)b * l3];
          for (int m = 0; m < l3; ++m) {
            double s = 0.0;
            for (int nn = 0; nn < l3; ++nn) s += Km[(size_t)m * l3 + nn] * Wb[nn];
            Lc[m] += s;
          }
        }
        if (lv >= 3) {
          int64_t p = t->parent[lv][c];
          int o = (int)(t->ckey[lv][c] & 7ull);
          l2l_apply(l3, M[o], &Loc[lv - 1][(size_t)p * l3], Lc);
        }
      }
      for (int k = 0; k < nid; ++k) free(K[ids[k]]);
    }

    /* L2P at the targets */
#pragma omp parallel for schedule(dynamic, 64) num_threads(nth)
    for (int64_t k = 0; k < nt; ++k) {
      int64_t i = tsorted[k];
      int64_t c = t->leaf_of[i];
      double cc[3], a;
      cell_geometry(t, lf, t->ckey[lf][c], cc, &a);
      l2p_point(&B, &t->pos_s[3 * i], qs[i], cc, a, &Loc[lf][(size_t)c * l3],
                &pf[k], &ff[3 * k]);
    }

    for (int o = 0; o < 8; ++o) free(M[o]);
    for (int lv = 2; lv < h; ++lv) {
      free(W[lv]);
      free(Loc[lv]);
      free(need[lv]);
    }
  }

  /* ---- near field: P2P over the near list, sources in list order ---- */
#pragma omp parallel for schedule(dynamic, 64) num_threads(nth)
  for (int64_t k = 0; k < nt; ++k) {
    int64_t i = tsorted[k];
    int64_t a = t->leaf_of[i];
    double ph = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
    for (int64_t e = t->near_off[a]; e < t->near_off[a + 1]; ++e) {
      int64_t b = t->near_idx[e];
      for (int64_t j = t->leaf_start[b]; j < t->leaf_start[b + 1]; ++j)
        pair_accumulate(p, &t->pos_s[3 * i], &t->pos_s[3 * j], qs[j], &ph, &fx,
                        &fy, &fz);
    }
    pn[k] = ph;
    fn[3 * k + 0] = qs[i] * fx;
    fn[3 * k + 1] = qs[i] * fy;
    fn[3 * k + 2] = qs[i] * fz;
  }

  /* ---- outputs: near + far ---- */
  for (int64_t k = 0; k < nt; ++k) {
    if (phi) phi[k] = pn[k] + pf[k];
    if (phi_near) phi_near[k] = pn[k];
    if (phi_far) phi_far[k] = pf[k];
    for (int d = 0; d < 3; ++d) {
      if (f) f[3 * k + d] = fn[3 * k + d] + ff[3 * k + d];
      if (f_near) f_near[3 * k + d] = fn[3 * k + d];
      if (f_far) f_far[3 * k + d] = ff[3 * k + d];
    }
  }
  free(qs);
  free(tsorted);
  free(pn);
  free(fn);
  free(pf);
  free(ff);
  return 0;
}
