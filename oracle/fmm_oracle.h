/*
 * Oracle for the FMM evaluation pass: a plain, slow FP64 CPU implementation.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  It shares no code with the HIP
 * path (no headers, tables or helpers in common) and never calls it.
 *
 * What it computes (paper "Pipelining the Fast Multipole Method over a Runtime
 * System", Sec. 2 and 2.1):
 *   - the pairwise summation of Eq. (1) with the Laplace kernel of Eq. (2),
 *     as a direct O(N^2) sum;
 *   - the black-box Chebyshev FMM of Eq. (3)-(5): octree of height h (levels
 *     0..h-1, leaf level h-1), Morton-ordered cells (Sec. 4.2), P2M, M2M, M2L,
 *     L2L, L2P and the near-field P2P, with dense M2L matrices evaluated
 *     point-wise per level and offset (Sec. 2.1.2 without compression).
 *
 * Conventions:
 *   positions  [n][3] row-major float64; charges [n]; potential [n];
 *   forces [n][3].  Potential phi_i = sum_{j, r_ij>0} q_j / r_ij and force
 *   F_i = q_i sum_{j, r_ij>0} q_j (x_i - x_j) / r_ij^3 (= -q_i grad phi).
 *   Pairs at distance zero (including j = i) contribute nothing.
 *   order l = Chebyshev nodes per dimension (l^3 coefficients per cell).
 *
 * All entry points return 0 on success and a negative value on bad
 * arguments; none of them touches a GPU.
 */
#ifndef FMM_ORACLE_H
#define FMM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORACLE_MAX_HEIGHT 21
#define ORACLE_MAX_ORDER 16

/* ---- direct summation (Eq. 1 with the kernels of Eq. 2) ---- */
int oracle_direct(const double* pos, int64_t n, const double* q, double* phi,
                  double* f);
/* exact sums at s chosen targets idx[0..s) over all n sources */
int oracle_direct_sampled(const double* pos, int64_t n, const double* q,
                          const int64_t* idx, int64_t s, double* phi,
                          double* f);
/* The same two for the kernel P = |x - y|^-p, p = 1 (1/r, the calls above)
 * or p = 2 (1/r^2; force q_i sum_j q_j 2 (x_i - x_j) / r^4).  Other p: -1. */
int oracle_direct_k(const double* pos, int64_t n, const double* q, double* phi,
                    double* f, int p);
int oracle_direct_sampled_k(const double* pos, int64_t n, const double* q,
                            const int64_t* idx, int64_t s, double* phi,
                            double* f, int p);

/* ---- Chebyshev interpolation (Eq. 5) ---- */
int oracle_cheb_nodes(int l, double* xi);                  /* xi[l] */
double oracle_cheb_S(int l, int m, double u);              /* S(xi_m; u) */
double oracle_cheb_dS(int l, int m, double u);             /* d/du S(xi_m; u) */

/* ---- single operators (for pinning against closed forms) ---- */
/* W[l^3] += P2M of n particles into the cell (center c, half-width a) */
int oracle_p2m(int l, int64_t n, const double* pos, const double* q,
               const double* c, double a, double* W);
/* Wp[l^3] += M2M of a child multipole at child octant o (bit0=x,1=y,2=z) */
int oracle_m2m(int l, int octant, const double* Wc, double* Wp);
/* Lc[l^3] += L2L of a parent local expansion to its child at octant o */
int oracle_l2l(int l, int octant, const double* Lp, double* Lc);
/* phi[i], f[i][3] = far-field L2P of Loc at n targets (overwrite) */
int oracle_l2p(int l, int64_t n, const double* pos, const double* q,
               const double* c, double a, const double* Loc, double* phi,
               double* f);
/* K[l^3][l^3]: M2L matrix between cells of half-width a, width w, whose
 * centres differ by w*t (source minus target). */
int oracle_m2l_matrix(int l, double a, double w, const int* t, double* K);
/* the same for the kernel |x - y|^-p (p = 1 or 2) */
int oracle_m2l_matrix_k(int l, double a, double w, const int* t, double* K,
                        int p);

/* ---- octree (plan) ---- */
typedef struct oracle_tree oracle_tree;
oracle_tree* oracle_tree_build(const double* pos, int64_t n, int h);
void oracle_tree_free(oracle_tree* t);
/* info[0]=n, [1]=h, [2]=n_leaf, [3+l]=cells at level l (l<h) */
int oracle_tree_info(const oracle_tree* t, int64_t* info);
/* box[0..2]=lo, box[3]=L */
int oracle_tree_box(const oracle_tree* t, double* box);
int oracle_tree_keys(const oracle_tree* t, uint64_t* keys_sorted); /* [n] */
int oracle_tree_perm(const oracle_tree* t, int64_t* perm);          /* [n] */
int oracle_tree_leaf_start(const oracle_tree* t, int64_t* start);   /* [n_leaf+1] */
int oracle_tree_cell_keys(const oracle_tree* t, int level, uint64_t* keys);
/* near CSR over leaves: off[n_leaf+1]; idx may be NULL to query off only */
int oracle_tree_near(const oracle_tree* t, int64_t* off, int64_t* idx);
/* far CSR over cells of a level (>=2): indices into the level's cells */
int oracle_tree_far(const oracle_tree* t, int level, int64_t* off,
                    int64_t* idx);

/* ---- FMM evaluation ----
 * targets == NULL: all n particles, outputs in input order.
 * targets != NULL: only particles targets[0..nt), outputs in that order.
 * Any of the output pointers may be NULL.  phi/f are near + far. */
int oracle_fmm(const oracle_tree* t, int l, const double* q,
               const int64_t* targets, int64_t nt, double* phi, double* f,
               double* phi_near, double* f_near, double* phi_far,
               double* f_far);

/* As oracle_fmm, for the kernel |x - y|^-p (p = 1 or 2), and, when
 * unit_ops is not NULL, with M2L through given unit operators instead of
 * kernel evaluations: unit_ops[id][l^3][l^3] for the offset t with
 * id = (tx+3)*49 + (ty+3)*7 + (tz+3) is the operator between cells of width
 * 2 (half-width 1); level lv uses it scaled by a_lv^-p (the kernel is
 * homogeneous of degree -p).  Used for the compressed M2L of Sec. 2.1.2,
 * whose truncated operators the caller computes. */
int oracle_fmm_ops(const oracle_tree* t, int l, const double* q,
                   const int64_t* targets, int64_t nt, const double* unit_ops,
                   double* phi, double* f, double* phi_near, double* f_near,
                   double* phi_far, double* f_far, int p);

/* number of OpenMP threads the oracle uses (0 = library default) */
void oracle_set_threads(int nthreads);
int oracle_get_threads(void);

#ifdef __cplusplus
}
#endif
#endif
