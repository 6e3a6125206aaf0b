/*
 * Memory-safety driver for the oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Built together with fmm_oracle.c under AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_oracle_sanitizers.py, it calls
 * every entry point of fmm_oracle.h on small seeded inputs (a uniform cube,
 * a degenerate set of coincident points, and a height-1 tree) so that any
 * out-of-bounds access, use after free, leak or undefined operation in the
 * oracle is reported.  It also checks two facts that hold exactly: the
 * one-level FMM is the direct sum bit for bit (no far field), and the
 * sampled direct sum equals the full one at the sampled targets.
 * Exit status 0 when every call succeeded and both facts hold.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "fmm_oracle.h"

static uint64_t lcg_state = 88172645463325252ull;
static double uniform01(void) {
  /* xorshift64: enough for inputs, nothing of the method depends on it */
  lcg_state ^= lcg_state << 13;
  lcg_state ^= lcg_state >> 7;
  lcg_state ^= lcg_state << 17;
  return (double)(lcg_state >> 11) * (1.0 / 9007199254740992.0);
}

static int fail(const char* what) {
  fprintf(stderr, "asan_check: %s\n", what);
  return 1;
}

static int run_tree(const double* pos, int64_t n, const double* q, int h, int l) {
  oracle_tree* t = oracle_tree_build(pos, n, h);
  if (!t) return fail("tree build");
  int64_t info[3 + ORACLE_MAX_HEIGHT];
  double box[4];
  if (oracle_tree_info(t, info) || oracle_tree_box(t, box)) return fail("tree info");
  const int64_t n_leaf = info[2];
  uint64_t* keys = malloc(sizeof(uint64_t) * n);
  int64_t* perm = malloc(sizeof(int64_t) * n);
  int64_t* start = malloc(sizeof(int64_t) * (n_leaf + 1));
  int64_t* noff = malloc(sizeof(int64_t) * (n_leaf + 1));
  if (oracle_tree_keys(t, keys) || oracle_tree_perm(t, perm) ||
      oracle_tree_leaf_start(t, start) || oracle_tree_near(t, noff, NULL))
    return fail("tree export");
  int64_t* nidx = malloc(sizeof(int64_t) * (noff[n_leaf] + 1));
  if (oracle_tree_near(t, noff, nidx)) return fail("near lists");
  for (int lv = 0; lv < h; ++lv) {
    uint64_t* ck = malloc(sizeof(uint64_t) * info[3 + lv]);
    if (oracle_tree_cell_keys(t, lv, ck)) return fail("cell keys");
    if (lv >= 2) {
      int64_t* foff = malloc(sizeof(int64_t) * (info[3 + lv] + 1));
      if (oracle_tree_far(t, lv, foff, NULL)) return fail("far offsets");
      int64_t* fidx = malloc(sizeof(int64_t) * (foff[info[3 + lv]] + 1));
      if (oracle_tree_far(t, lv, foff, fidx)) return fail("far lists");
      free(fidx);
      free(foff);
    }
    free(ck);
  }
  double* phi = malloc(sizeof(double) * n);
  double* f = malloc(sizeof(double) * 3 * n);
  double* pn = malloc(sizeof(double) * n);
  double* fn = malloc(sizeof(double) * 3 * n);
  double* pf = malloc(sizeof(double) * n);
  double* ff = malloc(sizeof(double) * 3 * n);
  if (oracle_fmm(t, l, q, NULL, n, phi, f, pn, fn, pf, ff)) return fail("fmm");
  int64_t tg[3] = {0, n / 2, n - 1};
  if (oracle_fmm(t, l, q, tg, 3, phi, f, NULL, NULL, NULL, NULL)) return fail("fmm targets");
  if (oracle_fmm_ops(t, l, q, tg, 3, NULL, phi, f, NULL, NULL, NULL, NULL, 2))
    return fail("fmm 1/r^2");
  free(phi), free(f), free(pn), free(fn), free(pf), free(ff);
  free(keys), free(perm), free(start), free(noff), free(nidx);
  oracle_tree_free(t);
  return 0;
}

int main(void) {
  oracle_set_threads(2);
  const int64_t n = 900;
  double* pos = malloc(sizeof(double) * 3 * n);
  double* q = malloc(sizeof(double) * n);
  for (int64_t i = 0; i < 3 * n; ++i) pos[i] = uniform01();
  for (int64_t i = 0; i < n; ++i) q[i] = 2.0 * uniform01() - 1.0;

  /* single operators */
  const int l = 4, l3 = l * l * l;
  double xi[ORACLE_MAX_ORDER], c[3] = {0.5, 0.5, 0.5};
  double* W = calloc(l3, sizeof(double));
  double* Wp = calloc(l3, sizeof(double));
  double* K = malloc(sizeof(double) * l3 * l3);
  double ph1[4], f1[12];
  const int t[3] = {2, -3, 0};
  if (oracle_cheb_nodes(l, xi)) return fail("nodes");
  (void)oracle_cheb_S(l, 1, 0.3);
  (void)oracle_cheb_dS(l, 2, -0.7);
  if (oracle_p2m(l, 4, pos, q, c, 0.5, W) || oracle_m2m(l, 5, W, Wp) ||
      oracle_l2l(l, 3, Wp, W) || oracle_l2p(l, 4, pos, q, c, 0.5, W, ph1, f1) ||
      oracle_m2l_matrix(l, 0.5, 1.0, t, K) || oracle_m2l_matrix_k(l, 0.5, 1.0, t, K, 2))
    return fail("single operators");

  /* direct sums: the sampled sum equals the full one */
  double* phi = malloc(sizeof(double) * n);
  double* f = malloc(sizeof(double) * 3 * n);
  double sp[3], sf[9];
  int64_t idx[3] = {7, 450, 899};
  if (oracle_direct(pos, n, q, phi, f) || oracle_direct_sampled(pos, n, q, idx, 3, sp, sf) ||
      oracle_direct_k(pos, n, q, phi + 0, f + 0, 1))
    return fail("direct");
  for (int s = 0; s < 3; ++s)
    if (sp[s] != phi[idx[s]] || memcmp(sf + 3 * s, f + 3 * idx[s], 3 * sizeof(double)))
      return fail("sampled direct differs from the full sum");
  if (oracle_direct_sampled_k(pos, n, q, idx, 3, sp, sf, 2)) return fail("direct 1/r^2");

  /* trees: several heights, a one-level tree equal to the direct sum */
  if (run_tree(pos, n, q, 4, 5) || run_tree(pos, n, q, 3, 3) || run_tree(pos, n, q, 1, 2))
    return 1;
  oracle_tree* t1 = oracle_tree_build(pos, n, 1);
  double* phi1 = malloc(sizeof(double) * n);
  double* fo = malloc(sizeof(double) * 3 * n);
  if (!t1 || oracle_fmm(t1, 3, q, NULL, n, phi1, fo, NULL, NULL, NULL, NULL))
    return fail("one-level fmm");
  if (memcmp(phi1, phi, sizeof(double) * n) || memcmp(fo, f, 3 * sizeof(double) * n))
    return fail("one-level fmm differs from the direct sum");
  oracle_tree_free(t1);

  /* coincident points: every pair at distance zero */
  for (int64_t i = 0; i < 3 * 40; ++i) pos[i] = 0.25;
  if (run_tree(pos, 40, q, 3, 3)) return 1;

  /* rejected arguments */
  if (oracle_tree_build(pos, 0, 3) != NULL || oracle_cheb_nodes(0, xi) == 0)
    return fail("bad arguments accepted");

  free(pos), free(q), free(W), free(Wp), free(K), free(phi), free(f), free(phi1), free(fo);
  printf("asan_check: ok\n");
  return 0;
}
