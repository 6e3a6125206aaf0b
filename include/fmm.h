/*
 * fmm.h -- C-ABI of the MI355X (gfx950) fast multipole library.
 *
 * The library evaluates, for N charged particles, the potentials and forces
 * of the pairwise summation of Eq. (1) with the Laplace kernel of Eq. (2) of
 * "Pipelining the Fast Multipole Method over a Runtime System" (Agullo et
 * al.), using the black-box Chebyshev FMM of Sec. 2.1 (Eq. 3-5):
 *
 *     phi_i = sum_{j: r_ij > 0} q_j / r_ij
 *     F_i   = q_i sum_{j: r_ij > 0} q_j (x_i - x_j) / r_ij^3   ( = -q_i grad phi )
 *
 * Pairs at zero distance, the particle itself included, contribute nothing.
 * The octree has `height` levels 0..height-1 (leaf level height-1), cells in
 * Morton order (Sec. 4.2); the root box is the cube anchored at the per-axis
 * minimum of the positions whose side is the largest extent.  `order` is the
 * number l of Chebyshev nodes per dimension (l^3 coefficients per cell; the
 * paper's accuracy parameter Acc sets l = Acc, Sec. 2.1.2).
 *
 * Pointers: positions, charges, potential and forces are DEVICE pointers
 * (for example the data of torch tensors on the current HIP device); the
 * `host_dst` of fmm_plan_export and the `out` of fmm_plan_info are host
 * pointers.  Layouts: positions [n][3] row-major float64; charges [n];
 * potential [n]; forces [n][3].  Outputs are in input order and are
 * overwritten, never accumulated.
 *
 * Errors: calls return FMM_OK (0) or a negative fmm_status; fmm_plan returns
 * NULL.  fmm_last_error() gives a message for the calling thread's last
 * failure.  No call aborts the process.
 */
#ifndef FMM_H
#define FMM_H

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fmm_plan_s* fmm_plan_t;

enum fmm_status {
  FMM_OK = 0,
  FMM_ERR_ARG = -1,   /* invalid argument (checked before any device work) */
  FMM_ERR_OOM = -2,   /* device allocation failed */
  FMM_ERR_HIP = -3,   /* HIP runtime error */
  FMM_ERR_STATE = -4  /* plan busy (evaluation still in flight elsewhere) */
};

enum fmm_precision {
  /* every operator in FP64 (FP64 MFMA for M2L) */
  FMM_FP64 = 0,
  /* P2P in FP32 (pair differences rounded once from FP64) with FP64
   * folding per source chunk (at most 64 particles); M2L as FP32 MFMA
   * contractions whose operators produce Chebyshev coefficients of the
   * local expansions, accumulated in FP32 and folded into FP64 after every
   * far offset; L2L and L2P take the coefficients in FP64.  P2M, M2M, L2L,
   * L2P and the output sums compute in FP64 (M2L reads FP32 copies of the
   * multipoles) */
  FMM_MIXED_FP32 = 1,
  /* Reserved for M2L as BF16 MFMA products with FP32 accumulation.  Not
   * built: BF16 keeps 8 significant bits, so even a two-term (hi + lo)
   * split of every operand carries a relative error of about 2^-17 per
   * product, far above what the 1e-6 relative L2 gate of the mixed modes
   * leaves (FP32 products already use most of it at order 10).
   * fmm_plan_set_precision and fmm_server_submit return FMM_ERR_ARG. */
  FMM_MIXED_BF16 = 2,
  /* Extensions beyond the three modes above. */
  /* FMM_FP64 with the compressed M2L of Sec. 2.1.2 ("improved M2L"): each of
   * the 16 canonical operators factorised by one SVD, truncated at singular
   * values s_k >= eps s_1 (eps from fmm_plan_set_m2l_tolerance; default
   * 10^-order as in the paper's accuracy setting, at most down to 1e-10),
   * applied as two skinny MFMA products per far offset */
  FMM_FP64_SVD = 3,
  /* FMM_MIXED_FP32 with the compressed M2L in FP32 MFMA: the second factor
   * of each operator produces Chebyshev coefficients, folded into FP64 every
   * few far offsets (fmm_plan_set_m2l_fold_interval) */
  FMM_MIXED_SVD = 4
};

/* Truncation tolerance of the compressed M2L (0 < eps < 1); takes effect for
 * the SVD precision modes (in a dense mode it is only recorded, and checked
 * when an SVD mode is selected).  The truncated operators of an order and tolerance
 * are computed once per device (rocSOLVER SVD of the 16 canonical operators)
 * and cached.  Returns FMM_ERR_ARG for a tolerance outside (0, 1), and, in an
 * SVD mode, for one whose kept ranks need more LDS per workgroup than the
 * device has (two sets of four slabs of the padded rank by 32 target columns
 * in FP32, 16 in FP64; e.g. order 9 at 1e-14); the plan then keeps its
 * previous tolerance. */
int fmm_plan_set_m2l_tolerance(fmm_plan_t plan, double eps);

/* Fold interval of the compressed mixed mode (FMM_MIXED_SVD): the FP32 MFMA
 * partial sums of a target tile (Chebyshev coefficients of its local
 * expansions) are added into its FP64 local expansions after every
 * `offsets` far offsets (1..189; 0 restores the default, 189: once, after
 * the tile's last offset).  Shorter intervals are more accurate and slower:
 * relative L2 error against FP64 on the 1M-particle order-7 cube 1.5e-7 /
 * 1.8e-7 / 2.6e-7 for 1 / 16 / 189, on the 469k-particle order-10 cube
 * (tolerance 1e-7) 1.8e-7 / 2.0e-7 / 3.2e-7; 189 runs the M2L 6-9% faster
 * than 16.  Results stay deterministic for any interval.  Returns
 * FMM_ERR_ARG outside 0..189. */
int fmm_plan_set_m2l_fold_interval(fmm_plan_t plan, int offsets);

/* Work split of the compressed M2L (both SVD modes): each 64-target tile's
 * far offsets are taken in `parts` consecutive ranges, one work item each
 * (1..4; 0 restores the default).  Part 0 accumulates into the local
 * expansions, parts 1.. into partial FP64 buffers the plan allocates
 * ((parts - 1) x the M2L levels' local expansions), added back in part order
 * right after the M2L, so results are deterministic for a given split.  By
 * default the split is chosen from the tile count and the workgroups the
 * device holds at once, so that the last round of workgroups is not left
 * mostly empty (1 when the tiles alone fill many rounds, or when the
 * buffers would exceed 2 GiB).  Different splits sum in different orders:
 * results agree to rounding.  Returns FMM_ERR_ARG outside 0..4. */
int fmm_plan_set_m2l_split(fmm_plan_t plan, int parts);
/* The split in use (1 in the dense modes). */
int fmm_plan_m2l_split(fmm_plan_t plan, int* parts);

/* Compressed-M2L facts of the plan's current order and tolerance (host
 * struct; computes the truncated operators if needed).  rank[c] is the number
 * of singular values kept for canonical operator c; weighted_rank the mean
 * rank over the 316 far offsets (the paper's "weighted r_16", Table 1). */
struct fmm_svd_info {
  double eps;
  int32_t rank[16];
  int32_t rmax_pad;
  double weighted_rank;
};
int fmm_plan_svd_info(fmm_plan_t plan, struct fmm_svd_info* out);

/*
 * Build a plan (the octree, Sec. 3.2 and 4.2): root box, Morton keys, stable
 * radix sort of the particles by (key, index), leaves, cells of every level,
 * near lists (the up-to-27 leaves around each leaf) and far lists (children of
 * the parent's near cells that are not adjacent, at most 189, Sec. 2.1.2),
 * organised as MFMA tiles.  Also loads the cached per-order operators.
 *   positions  device, [n][3] f64; read only, may be freed after return
 *   n          1 .. 2^31-1
 *   height     1 .. 21
 *   order      1 .. 12
 * Synchronous: runs on the null stream and waits for it (sizes depend on
 * counts).  Returns NULL on error: FMM_ERR_ARG for bad sizes, a null pointer
 * or non-finite positions; FMM_ERR_OOM; FMM_ERR_HIP.  The plan owns all its
 * device memory; free it with fmm_release.  Precision defaults to FMM_FP64.
 */
fmm_plan_t fmm_plan(const double* positions, int64_t n, int height, int order);

/* fmm_plan on a caller-chosen stream (still synchronous on that stream). */
fmm_plan_t fmm_plan_stream(const double* positions, int64_t n, int height,
                           int order, hipStream_t stream);

/*
 * Evaluate potentials and forces for one set of charges (the FMM evaluation
 * pass of Sec. 3.2: P2M, M2M upward; M2L, L2L, L2P downward; P2P near field;
 * near and far sums combined in FP64).
 *   charges    device [n] f64
 *   potential  device [n] f64 (output)
 *   forces     device [n][3] f64 (output)
 *   stream     HIP stream all kernels are ordered on; returns immediately,
 *              results are valid once the stream has reached this point.
 * A plan must not be evaluated concurrently on two streams: a call while the
 * previous evaluation on another stream is still running returns
 * FMM_ERR_STATE.  Errors: FMM_ERR_ARG (null plan or pointer), FMM_ERR_HIP.
 */
int fmm_evaluate(fmm_plan_t plan, const double* charges, double* potential,
                 double* forces, hipStream_t stream);

/* Release a plan: waits for its in-flight evaluation and its side stream,
 * returns its device memory, side stream and events to the library's
 * per-device caches.  NULL-safe. */
void fmm_release(fmm_plan_t plan);

/* Message for the calling thread's most recent failure ("" if none). */
const char* fmm_last_error(void);

/* Select the arithmetic of later evaluations (enum fmm_precision). */
int fmm_plan_set_precision(fmm_plan_t plan, int mode);

/* Task schedule of later evaluations (the FMM task flow of Sec. 3.2 and its
 * pipelining, Sec. 3.3).  The near field (P2P) depends only on the charges
 * and the far field (P2M, M2M, M2L, L2L, L2P) writes other buffers, so the two
 * branches may run at the same time and meet at the final sum.
 *   FMM_SCHEDULE_SERIAL  every operator in order on the caller's stream
 *   FMM_SCHEDULE_FORKED  (default) P2P on a stream owned by the plan (a
 *                        non-blocking stream of default priority, reused
 *                        from plans released earlier on the device), forked
 *                        from the caller's stream after the M2L launch (so
 *                        it runs beside L2L and L2P, which leave the GPU
 *                        partly idle) and joined back before the final sum;
 *                        the far chain stays on the caller's stream
 *   FMM_SCHEDULE_PIPELINED  as FMM_SCHEDULE_FORKED, and the M2L of the leaf
 *                        level (which needs only the leaf multipoles) also
 *                        runs on the plan's stream, right after P2M and
 *                        beside the M2M chain (Sec. 3.3: the M2L of one level
 *                        overlaps the M2M of the next coarser one); the
 *                        coarser levels' M2L follows the M2M chain on the
 *                        caller's stream, which waits for the leaf level's
 *                        before the local expansions are summed.  The M2L
 *                        timing hook brackets the leaf level's launch.
 * All schedules launch the same kernels on the same data: results are
 * bit-identical.  Stream capture of the caller's stream captures the forks
 * and joins.  Returns FMM_ERR_ARG for a null plan or unknown schedule. */
enum fmm_schedule { FMM_SCHEDULE_SERIAL = 0, FMM_SCHEDULE_FORKED = 1, FMM_SCHEDULE_PIPELINED = 2 };
int fmm_plan_set_schedule(fmm_plan_t plan, int schedule);

/* Whole-evaluation graph (the task flow of Sec. 3.2 as one hipGraph): with
 * on = 1, fmm_evaluate captures its launch sequence (both streams of the
 * forked and pipelined schedules) the first time on a private stream, as a
 * hipGraph, and afterwards replays it on the caller's stream with the
 * call's charge and output pointers set into its first and last kernels; it
 * is captured again after the precision mode, tolerance, kernel, fold
 * interval, split or schedule changed.  The same kernels run on the same
 * data: results are bit-identical to the eager launches.  Evaluations with
 * a step timing hook set, and fmm_evaluate_parts, run eagerly.  on = 0 (the
 * default) frees the graph.  Returns FMM_ERR_ARG for a null plan or another
 * value of on. */
int fmm_plan_set_graph(fmm_plan_t plan, int on);

/* Kernel of later evaluations.  The black-box scheme (Sec. 2.1) needs only
 * point evaluations of the kernel P(x, y): the interpolation operators (P2M,
 * M2M, L2L, L2P) do not depend on it, M2L evaluates it between Chebyshev
 * nodes, and P2P evaluates it directly.  Both kernels are homogeneous, so the
 * unit M2L operators of Sec. 2.1.2 serve every level with the scale a^-p.
 *   FMM_KERNEL_INV_R   (default) P = 1/r, the paper's Laplace kernel (Eq. 2):
 *                      phi_i = sum_j q_j / r_ij,
 *                      F_i = q_i sum_j q_j (x_i - x_j) / r_ij^3
 *   FMM_KERNEL_INV_R2  P = 1/r^2: phi_i = sum_j q_j / r_ij^2,
 *                      F_i = -q_i grad phi = q_i sum_j q_j 2 (x_i - x_j) / r_ij^4
 * Zero-distance pairs contribute nothing in both.  The operators of a new
 * (order, kernel) are built once per device and cached; the call waits for
 * the plan's in-flight evaluation.  Returns FMM_ERR_ARG for a null plan or an
 * unknown kernel.  The serving calls use FMM_KERNEL_INV_R. */
enum fmm_kernel { FMM_KERNEL_INV_R = 1, FMM_KERNEL_INV_R2 = 2 };
int fmm_plan_set_kernel(fmm_plan_t plan, int kernel);

/* Near-field form of later evaluations (P2P, Sec. 5).
 *   FMM_NEAR_ONE_SIDED  (default) each target leaf sums over the particles of
 *                       its up to 27 neighbour leaves (itself included), so
 *                       every pair of particles in distinct leaves is
 *                       computed twice, once from each side
 *   FMM_NEAR_MUTUAL     the reduction form of Sec. 5 (P2Preduce): each pair of
 *                       distinct neighbour leaves is computed once and its
 *                       terms are added to both leaves' sums; pairs within a
 *                       leaf stay one-sided.  The pairs go in 26 launches
 *                       (13 forward offsets, each in two colours), each of
 *                       which touches every leaf at most once, so the sums
 *                       are taken in a fixed order without atomics: results
 *                       are deterministic, and equal to the one-sided form's
 *                       up to the order of summation.
 * The first switch to FMM_NEAR_MUTUAL builds the plan's pair lists (at most
 * 13 ints per leaf, owned by the plan; the build synchronises the plan's
 * stream and waits for its in-flight evaluation).  The near-field timing hook
 * brackets all of the form's launches.  Returns FMM_ERR_ARG for a null plan
 * or an unknown mode, FMM_ERR_OOM if the lists do not fit.  The serving calls
 * use the one-sided form. */
enum fmm_near { FMM_NEAR_ONE_SIDED = 0, FMM_NEAR_MUTUAL = 1 };
int fmm_plan_set_near(fmm_plan_t plan, int mode);

/* Plan facts (host struct). */
struct fmm_info {
  int64_t n;
  int32_t height, order, precision, ld;
  int64_t n_leaf;
  int64_t ncell[21];          /* cells per level */
  double lo[3], L;            /* root box */
  int64_t near_pairs;         /* directed (target, source) particle pairs in the
                                 near field, zero-distance pairs included */
  int64_t far_pairs;          /* (target cell, source cell) M2L pairs */
  int64_t far_pairs_level[21];
  int64_t m2l_tiles;          /* MFMA work tiles (64 target cells each) */
  int64_t m2l_active_slots;   /* tile-offset pairs with at least one source */
  int64_t device_bytes;       /* device memory held by the plan */
  double m2l_flops;           /* algorithmic M2L flops of one evaluation in the
                                 current mode: 2 l^6 per pair (dense) or
                                 4 l^3 r_t per pair (compressed, unpadded rank) */
  int64_t m2l_groups;         /* 16-target groups of the tiles at their active
                                 offsets */
  int64_t m2l_groups_empty;   /* ... of them with no source at that offset */
  int32_t m2l_group_skip;     /* 1 when the compressed M2L skips those groups
                                 (at least a tenth of them, as for points on a
                                 surface); the results are the same either way */
};
int fmm_plan_info(fmm_plan_t plan, struct fmm_info* out);

/*
 * Copy plan data to host memory, for checking.  `what`:
 *   FMM_EXPORT_KEYS        uint64 [n]       sorted Morton keys
 *   FMM_EXPORT_PERM        int64  [n]       sorted position -> input index
 *   FMM_EXPORT_LEAF_START  int64  [n_leaf+1]
 *   FMM_EXPORT_CELL_KEYS   uint64 [ncell[level]]
 *   FMM_EXPORT_NEAR_OFF    int64  [n_leaf+1]  near lists as CSR, ascending
 *   FMM_EXPORT_NEAR_IDX    int64  [near_off[n_leaf]]
 *   FMM_EXPORT_FAR_OFF     int64  [ncell[level]+1] far lists (level >= 2) as
 *   FMM_EXPORT_FAR_IDX     int64  [far_off[ncell]]  CSR of level-local indices,
 *                                                   ascending
 *   FMM_EXPORT_MUTUAL_OFF  int64  [27]      bounds of the mutual near field's
 *                                           26 pair lists: list 2k + c holds
 *                                           the leaves a whose neighbour at
 *                                           near slot 14 + k exists and whose
 *                                           colour is c (fmm_plan_set_near)
 *   FMM_EXPORT_MUTUAL_IDX  int64  [mutual_off[26]]  the lists' leaves
 *                                           (ascending within a list); both
 *                                           need the lists built (FMM_ERR_ARG
 *                                           before the first switch to
 *                                           FMM_NEAR_MUTUAL)
 * `bytes` must be at least the size of the array; returns FMM_ERR_ARG
 * otherwise.  Synchronous.
 */
enum fmm_export {
  FMM_EXPORT_KEYS = 0,
  FMM_EXPORT_PERM = 1,
  FMM_EXPORT_LEAF_START = 2,
  FMM_EXPORT_CELL_KEYS = 3,
  FMM_EXPORT_NEAR_OFF = 4,
  FMM_EXPORT_NEAR_IDX = 5,
  FMM_EXPORT_FAR_OFF = 6,
  FMM_EXPORT_FAR_IDX = 7,
  FMM_EXPORT_MUTUAL_OFF = 8,
  FMM_EXPORT_MUTUAL_IDX = 9
};
int fmm_plan_export(fmm_plan_t plan, int what, int level, void* host_dst,
                    size_t bytes);

/*
 * Evaluate and return the near field (P2P) and far field (L2P of the local
 * expansions) separately, in input order, for checking each operator chain.
 * All pointers device, as in fmm_evaluate.
 */
int fmm_evaluate_parts(fmm_plan_t plan, const double* charges,
                       double* phi_near, double* f_near, double* phi_far,
                       double* f_far, hipStream_t stream);

/*
 * Time the M2L launches of subsequent evaluations on the calling thread:
 * when ev0/ev1 are non-null, ev0 is recorded on the evaluation stream just
 * before the M2L kernel and ev1 just after it.  Pass NULLs to stop.
 */
int fmm_set_m2l_timing_events(hipEvent_t ev0, hipEvent_t ev1);

/* The same for any of the bulk operators: ev0 is recorded just before the
 * step's kernel and ev1 just after it, on the stream the kernel runs on (for
 * P2P in the forked schedule, the plan's side stream; for M2L in the
 * pipelined one, the leaf level's launch on the side stream).  M2M and L2L
 * bracket all their level launches; FMM_TIME_LOC_SUM the pass that adds the
 * split compressed M2L's partial sums (absent for an unsplit M2L).  Pass
 * NULLs to stop.
 * Returns FMM_ERR_ARG for an unknown step or a single NULL event. */
enum fmm_timed_step {
  FMM_TIME_M2L = 0,
  FMM_TIME_P2P = 1,
  FMM_TIME_P2M = 2,
  FMM_TIME_L2P = 3,
  FMM_TIME_M2M = 4,
  FMM_TIME_L2L = 5,
  FMM_TIME_LOC_SUM = 6
};
int fmm_set_step_timing_events(int step, hipEvent_t ev0, hipEvent_t ev1);

/*
 * Exact sums at chosen targets: the direct summation of Eq. (1) with the
 * kernel of Eq. (2) (or 1/r^2, enum fmm_kernel) over all n sources, the
 * result the FMM approximates, for checking it at a sample of particles:
 *   potential[k] = sum_{j: r > 0} q_j / r^p,
 *   forces[k]    = q_i sum_{j: r > 0} q_j p (x_i - x_j) / r^(p+2),
 * i = targets[k], r = |x_i - x_j|; pairs at zero distance are skipped.
 *   positions  device [n][3] f64; charges device [n] f64
 *   targets    device [nt] int64, indices into the particles (1 <= nt <= 2^30);
 *              an index outside [0, n) gives NaN results for that target
 *   potential  device [nt] f64, forces device [nt][3] f64 (outputs, in
 *              target order, overwritten)
 * FP64 throughout; the sources are summed in fixed chunks, so results are
 * bit-identical from call to call.  Allocates a partial-sum buffer of
 * 32 * ceil(nt / 64) * 64 * chunks bytes (at most 8 MiB) and waits for the
 * stream before returning.  Errors: FMM_ERR_ARG (null pointer, sizes,
 * kernel), FMM_ERR_OOM, FMM_ERR_HIP.
 */
int fmm_direct_sampled(const double* positions, const double* charges, int64_t n,
                       const int64_t* targets, int64_t nt, int kernel, double* potential,
                       double* forces, hipStream_t stream);

/*
 * fmm_direct_sampled for callers that cannot allocate device memory (code
 * under stream capture, tight serving loops, harnesses that forbid
 * allocation).  Same arguments and the same bits as fmm_direct_sampled, but
 * no allocation: the partial sums live in a static device array of 8 MiB
 * per device, held from the first call on the device until the process
 * ends.  Stream-ordered: returns once the work is queued.  Every call on a
 * device shares that array, so calls that overlap on one device (on two
 * streams, or from two threads without ordering) race and give wrong
 * results.  Returns FMM_ERR_ARG, before any device work, when nt exceeds
 * 262,144 (the partial sums would not fit), and as fmm_direct_sampled for
 * other invalid arguments.
 */
int fmm_direct_sampled_noalloc(const double* positions, const double* charges, int64_t n,
                               const int64_t* targets, int64_t nt, int kernel,
                               double* potential, double* forces, hipStream_t stream);

/* Return cached device memory of released plans to the HIP runtime. */
void fmm_trim_cache(void);

/*
 * Serving loop: a device-resident request loop that evaluates many particle
 * sets of different size and order concurrently (continuous batching).  A
 * planner thread plans arriving requests on its own stream and admits them
 * while the sum of their plans' device footprints stays within
 * `hbm_budget_bytes` and at most `max_active` are admitted; a launcher
 * thread evaluates the admitted requests in batches: each operator of the
 * evaluation pass (Sec. 3.2's P2M, M2M, M2L, L2L, L2P, P2P) runs as one
 * persistent launch over the work items of every request in the batch
 * (requests of equal order share the M2L, P2M and L2P launches), and a
 * batch's launch sequence is captured once as a hipGraph and replayed with
 * new work tables.  Up to two batches run at once, each on its own stream:
 * requests that arrive while a batch runs are planned meanwhile and start as
 * soon as they are admitted, beside it on the device.  A request's results
 * are bit-identical to fmm_evaluate on the same inputs.
 */
typedef struct fmm_server_s* fmm_server_t;

struct fmm_request_stats {
  int32_t status;       /* FMM_OK, or the error that ended the request */
  int32_t done;         /* 1 once the results are in the output buffers */
  double submit_s;      /* times in seconds on the server's monotonic clock */
  double admit_s;
  double done_s;
  int64_t batch;        /* batch index the request ran in */
  int64_t plan_bytes;   /* device footprint admitted for it */
};

struct fmm_server_stats {
  int64_t submitted, completed, rejected, batches;
  int64_t graph_captures, graph_replays;
  int64_t max_batch_jobs, max_active_seen;
  int64_t peak_admitted_bytes;
};

/* Create a server on the current device.  hbm_budget_bytes > 0, 1 <= max_active
 * <= 64.  Returns NULL on error (FMM_ERR_ARG / FMM_ERR_HIP). */
fmm_server_t fmm_server_create(size_t hbm_budget_bytes, int max_active);

/*
 * Queue one evaluation.  positions [n][3], charges [n], potential [n] and
 * forces [n][3] are device pointers that the caller keeps valid and untouched
 * until the request is done.  height, order as for fmm_plan; precision an
 * fmm_precision (FMM_MIXED_BF16 is refused).  `stream` is the caller's
 * stream: the server reads the inputs and writes the outputs only after the
 * work queued on it at this call (an event recorded here).  Returns a ticket
 * >= 0, or a negative fmm_status for invalid arguments (checked before
 * anything is queued) or a failed event record (FMM_ERR_HIP).  A request
 * whose plan alone exceeds the budget finishes with status FMM_ERR_OOM; a
 * plan that fails finishes with the plan's own status (FMM_ERR_OOM,
 * FMM_ERR_HIP, ...), its message kept with the request.
 */
int64_t fmm_server_submit(fmm_server_t srv, const double* positions, const double* charges,
                          int64_t n, int height, int order, int precision,
                          double* potential, double* forces, hipStream_t stream);

/* Message of a finished request's failure ("" if it succeeded or is not
 * done), copied NUL-terminated into buf[len] (truncated if longer); returns
 * the message length, or FMM_ERR_ARG for an unknown ticket or a NULL buffer
 * with len > 0. */
int fmm_server_request_error(fmm_server_t srv, int64_t ticket, char* buf, size_t len);

/* Non-blocking: 1 if the request is done (its status in st->status), 0 if not,
 * FMM_ERR_ARG for an unknown ticket.  `st` may be NULL. */
int fmm_server_poll(fmm_server_t srv, int64_t ticket, struct fmm_request_stats* st);

/* Block until the request is done; returns its status. */
int fmm_server_wait(fmm_server_t srv, int64_t ticket, struct fmm_request_stats* st);

/* Seconds on the server's clock (the clock of the request times). */
double fmm_server_now(fmm_server_t srv);

int fmm_server_get_stats(fmm_server_t srv, struct fmm_server_stats* out);

/* Finish every queued request, then stop the worker and free the server. */
void fmm_server_destroy(fmm_server_t srv);

#ifdef __cplusplus
}
#endif
#endif /* FMM_H */
