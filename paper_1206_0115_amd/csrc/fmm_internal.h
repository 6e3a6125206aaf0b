// Internal declarations of the MI355X FMM library (not part of the C-ABI).
//
// Data layout in HBM (all device arrays, one plan):
//   particles   sorted by (Morton key, input index); SoA px/py/pz (f64),
//               prel (float4: leaf-local x,y,z + charge) for the FP32 near field
//   cells       level-major "global cell ids": gid = lev_off[l] + i, i the
//               Morton rank within level l; one extra all-zero row at
//               gid = ncell_total stands in for absent M2L sources
//   W, Loc      [ncell_total + 1][ld] f64, ld = 16 * ceil(l^3 / 16), the
//               coefficient index (m1*l + m2)*l + m3, m1 along x
//   near        [n_leaf][27] leaf ids (-1 if empty), fixed offset order
//   M2L tiles   64 target cells of one level and one child parity; per tile
//               [189][64] source gids (zero row if absent) and the list of
//               slots with at least one source
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fmm.h"
#include "jobs.h"

namespace fmm {

constexpr int kMaxHeight = 21;
constexpr int kMaxOrder = 12;
// Plans with at most this many particles per leaf on average evaluate their
// local expansions with one wavefront per leaf spread over the l^3 terms
// (l2p_sparse_kernel); denser ones with lanes over particles (l2p_kernel).
// Per leaf of np particles the first costs about 20 np instructions per lane
// per 64 terms, the second one pass of about 3 l^2 + 2 l^3 per 32 particles:
// even near np = 7 at orders 7 to 10.
constexpr int kL2PSparseMax = 6;
constexpr int kTileN = 64;     // target cells per M2L tile
constexpr int kSlots = 189;    // far offsets per child parity
constexpr int kOffsets = 316;  // distinct far offsets

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
// status code of the calling thread's last failure (FMM_OK if none since
// the last fmm_plan call on the thread)
void set_error_code(int code);
int last_error_code();
struct FmmError {
  int code;
  std::string msg;
};
#define FMM_HIP_CHECK(expr)                                                  \
  do {                                                                       \
    hipError_t e_ = (expr);                                                  \
    if (e_ != hipSuccess)                                                    \
      throw ::fmm::FmmError{e_ == hipErrorOutOfMemory ? FMM_ERR_OOM : FMM_ERR_HIP, \
                            std::string(#expr) + ": " + hipGetErrorString(e_)}; \
  } while (0)

// ---------------------------------------------------------- device memory
// Caching allocator: blocks are kept in per-device free lists by size class
// and reused by later plans; hipMalloc only on a miss.
void* dev_alloc(size_t bytes);
void dev_free(void* p);
size_t dev_cached_bytes();
void dev_trim();
// A plan's side stream (non-blocking, default priority) and its events,
// recycled per device: creating and destroying them costs more host time
// than a plan's whole build.  put_* waits for the stream's work first.
hipStream_t side_stream_get(int device);
void side_stream_put(int device, hipStream_t s);
hipEvent_t event_get(int device);
void event_put(int device, hipEvent_t e);
// The calling thread's pinned host staging buffer, at least `bytes` long.
// Growing it frees the previous one: callers finish every transfer through
// it (a stream synchronisation) before asking for more.
void* pinned_staging(size_t bytes);

// ------------------------------------------------------ operator tables
// Per-order tables shared by all plans on a device (built once, cached).
struct OpSet {
  int order = 0, l3 = 0, ld = 0, mt = 0, kc = 0;
  double* cheb = nullptr;     // [l][l]: C[m][n] = (n==0 ? 1 : 2 T_n(xb_m)) / l
  // [2][l][l]: R_s[n][k], the coefficient of T_n in T_k((s + x)/2), s = -1, +1:
  // a parent's Chebyshev coefficients re-expanded on a child's interval
  double* child_modal = nullptr;
  double* child = nullptr;    // [2][l][l]: S(xb_m; (s + xb_m')/2), s = -1, +1
  double* kpack64 = nullptr;  // [316][mt][kc][64][4] unit M2L operators, MFMA order
  float* kpack32 = nullptr;   // FP32, rows in the Chebyshev-coefficient basis (see m2l.hip)
  int* slot_kid = nullptr;    // [8][189] packed-operator index of each slot
  signed char* slot_t = nullptr;  // [8][189][3] offset (tx, ty, tz) of each slot
};
// operators of an order for the kernel |x - y|^-kernel (1 or 2), cached per device
const OpSet* get_opset(int order, int kernel, hipStream_t stream);

// Compressed M2L operators (Sec. 2.1.2): one SVD per canonical operator,
// truncated at s_k >= eps s_1, shared by its 316-offset orbit through the
// signed permutations; cached per (device, order, eps).
struct SvdOps {
  int order = 0;
  double eps = 0.0;
  int rank[16] = {0};       // kept singular values per canonical operator
  int rmax_pad = 0;         // largest padded rank (multiple of 16)
  double weighted_rank = 0; // sum over the 316 offsets of the rank / 316
  int64_t flops_per_pair_weighted = 0;  // sum_t 4 l^3 rpad_t / 316, rounded
  int* rpad = nullptr;      // [316] padded rank per packed operator
  int* rk = nullptr;        // [316] kept rank per packed operator
  int64_t* off = nullptr;   // [316] element offset of its factors
  std::vector<int> rpad_h;
  double* p1_64 = nullptr;  // S V^T factors in fragment order
  float* p1_32 = nullptr;
  double* p2_64 = nullptr;  // U factors in fragment order
  float* p2_32 = nullptr;
};
const SvdOps* get_svd_ops(int order, double eps, int kernel, hipStream_t stream);
int kid_canon(int kid);  // canonical class (0..15) of packed operator kid

// ------------------------------------------- exact sums at sampled targets
// (direct.hip) The sources are cut into direct_chunks(n, nt) chunks, each
// summed by its own workgroups into a partial-sum buffer of
// direct_partial_doubles(nt, chunks) <= kDirectPartialMax doubles, which
// launch_direct then adds in chunk order.
constexpr int64_t kDirectPartialMax = int64_t(1) << 20;
int direct_chunks(int64_t n, int64_t nt);
size_t direct_partial_doubles(int64_t nt, int chunks);
void launch_direct(const double* pos, const double* q, int64_t n, const int64_t* targets,
                   int64_t nt, int p, double* phi, double* f, double* part, int chunks,
                   hipStream_t s);
int direct_check_args(const double* pos, const double* q, int64_t n, const int64_t* targets,
                      int64_t nt, int kernel, const double* phi, const double* f);

// ------------------------------------------------------------- the plan
struct M2LTile {
  int level;
  int parity;
  int first;  // index into tgt[] of the first target
  int count;  // targets in this tile (<= kTileN)
};

struct LevelView {
  int64_t ncell = 0;
  int64_t off = 0;                // global id of the level's first cell
  uint64_t* keys = nullptr;       // [ncell]
  int* child_start = nullptr;     // [ncell+1], indices in level+1
  int* parent = nullptr;          // [ncell], index in level-1
  int* lookup = nullptr;          // dense table over keys (8^l entries) or null
};

// Step tables a plan keeps for its own evaluations (one job each).
enum {
  kTabLeaf = 0,  // P2M, L2L, L2P, P2P: one item per leaf
  kTabCast = 1,  // FP32 copy of the multipoles: one item per row of levels >= 2
  kTabM2L = 2,   // one item per (M2L tile, M-block)
  kTabM2M = 3,   // + step s: parents at level h-2-s
  kTabL2L = 3 + kMaxHeight,  // + step s: children at level 3+s
  kTabLocSum = 3 + 2 * kMaxHeight,  // M2L parts: one item per row of levels >= 2
  kTabM2LLeaf = 4 + 2 * kMaxHeight,    // kTabM2L's items of the leaf-level tiles
  kTabM2LCoarse = 5 + 2 * kMaxHeight,  // kTabM2L's items of the coarser levels
  kTabCount = 6 + 2 * kMaxHeight
};

int m2l_nmb(int mt);      // M-blocks per M2L tile for mt 16-row tiles (dense)
// Compressed M2L for mt 16-row tiles and a slab stride of xs values (the
// kernel's shape depends on both): work items per tile, and 16-column
// N-tiles per item (launches of one order and precision that batch several
// plans group them by the latter)
int m2l_svd_nmb(int mt, bool fp32, int xs);
int m2l_svd_nt(int order, bool fp32, int xs);
int m2l_svd_slots(int order, bool fp32, int xs);  // compressed M2L workgroups resident at once
bool m2l_svd_splits(bool fp32);          // whether the compressed kernel takes m2l_parts
// LDS bytes of one compressed-M2L workgroup of nt N-tiles, and of the shape
// the kernel takes at this order
size_t m2l_svd_lds_bytes(int xs, bool fp32, int nt);
size_t m2l_svd_lds_need(int order, bool fp32, int xs);
int m2l_svd_xs(int rmax_pad, bool fp32);  // the slab stride for a padded rank

}  // namespace fmm

namespace fmm {
// mutual near field: the forward near-list slots 14..26 (plan.hip)
constexpr int kMutualSlots = 13;
constexpr int kMutualFirstSlot = 14;
}  // namespace fmm

struct fmm_plan_s {
  int device = 0;
  int64_t n = 0;
  int height = 0, order = 0, precision = FMM_FP64;
  double lo[3] = {0, 0, 0}, L = 1.0;
  const fmm::OpSet* ops = nullptr;
  double m2l_eps = 1e-8;              // truncation of the compressed M2L (set per order)
  const fmm::SvdOps* svd = nullptr;   // set when the precision mode compresses

  // particles
  double *px = nullptr, *py = nullptr, *pz = nullptr;
  float4* prel = nullptr;
  int* perm = nullptr;
  uint64_t* keys = nullptr;
  int64_t nleaf = 0;
  int* leaf_start = nullptr;
  int* near = nullptr;

  // cells
  fmm::LevelView lev[fmm::kMaxHeight];
  int64_t ncell_total = 0;

  // M2L work
  int64_t ntiles = 0;
  fmm::M2LTile* tiles = nullptr;
  int* tgt = nullptr;              // global ids of targets, grouped by (level, parity)
  int* tile_src = nullptr;         // [ntiles][189][64]
  unsigned char* tile_act = nullptr;  // [ntiles][189]
  unsigned char* tile_gmask = nullptr;  // [ntiles][189] 16-target groups with a source
  int* tile_nact = nullptr;        // [ntiles]
  std::vector<fmm::M2LTile> tiles_host;

  // statistics (exact counts)
  int64_t near_pairs = 0;          // directed near interactions, self pairs included
  int64_t far_pairs = 0;           // M2L (target, source) cell pairs
  int64_t far_pairs_level[fmm::kMaxHeight] = {0};
  int64_t active_slots = 0;        // sum over tiles of slots with a source
  int64_t m2l_groups = 0;          // 16-target groups at active slots
  int64_t m2l_groups_empty = 0;    // ... of them without a source
  bool m2l_gskip = false;          // the compressed M2L skips the empty groups
  const unsigned long long* stats_stage = nullptr;  // unread statistics (plan_stats)
  int64_t pairs_by_kid[fmm::kOffsets] = {0};  // far pairs per packed operator

  // evaluation buffers
  double *qs = nullptr, *W = nullptr, *Loc = nullptr;
  float* W32 = nullptr;
  double *phi_n = nullptr, *f_n = nullptr, *phi_f = nullptr, *f_f = nullptr;

  // kernel-side description of this plan and its step tables
  fmm::JobDev job_h{};
  fmm::JobDev* job_d = nullptr;
  fmm::StepTab tab_h[fmm::kTabCount];
  fmm::StepTab* tab_d = nullptr;

  hipEvent_t done = nullptr;       // recorded after each evaluation
  int schedule = FMM_SCHEDULE_FORKED;
  int kernel = FMM_KERNEL_INV_R;   // exponent p of the kernel |x - y|^-p
  int64_t w64_rows = 0;            // rows allocated in W (all cells + 1, or levels < h-1)
  bool w32_leaf = false;           // mixed modes: leaf multipoles only in W32
  int m2l_fold = 0;                // compressed FP32 fold interval (0: by order)
  int m2l_split = 0;               // compressed M2L offset ranges per tile (0: auto)
  int near_mode = FMM_NEAR_ONE_SIDED;  // fmm_plan_set_near
  int* mutual_list = nullptr;      // leaves of the mutual pair lists (built on first use)
  int64_t mutual_off[2 * fmm::kMutualSlots + 1] = {0};  // list (slot 14 + k, colour c) at 2k + c
  int m2l_parts = 1;               // the split in use
  double* LocX = nullptr;          // partial local expansions of parts 1..
  size_t locx_bytes = 0;
  hipStream_t side = nullptr;      // the near-field branch of the forked schedule
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  bool in_flight = false;
  hipStream_t last_stream = nullptr;  // stream of the last evaluation
  // whole-evaluation graph (fmm_plan_set_graph): the captured launch
  // sequence, its gather and combine nodes (which take each call's
  // pointers), and what it was captured for
  bool graph_on = false;
  int64_t job_version = 0;         // bumped by every upload_job
  int64_t graph_version = -1;      // job_version and schedule of the capture
  int graph_schedule = -1;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  hipGraphNode_t graph_gather = nullptr, graph_combine = nullptr;
  hipStream_t capture = nullptr;   // the private stream graphs are captured on
  std::vector<std::pair<void*, size_t>> blocks;  // every device block this plan owns
  size_t bytes = 0;
  std::mutex mu;

  void* alloc(size_t b);
  void free_block(void* ptr);      // return one block of this plan to the cache
  ~fmm_plan_s();
};

namespace fmm {
// plan construction (plan.hip)
void build_plan(fmm_plan_s* p, const double* positions, hipStream_t stream);
// The plan's statistics (pair counts), copied to the calling thread's
// pinned staging by build_plan without a wait: read them once the stream
// has been synchronised, before that staging is used again.
void plan_stats(fmm_plan_s* p);
// evaluation (eval.hip)
void evaluate(fmm_plan_s* p, const double* q, double* phi, double* f,
              double* phi_n, double* f_n, double* phi_f, double* f_f,
              hipStream_t stream);
// The same launches replayed from the plan's captured graph (captured on
// first use, and again after the job or the schedule changed).
void evaluate_graph(fmm_plan_s* p, const double* q, double* phi, double* f,
                    hipStream_t stream);
// the mutual near field's pair lists of the plan (plan.hip); synchronises s
void build_mutual_lists(fmm_plan_s* p, hipStream_t s);
// the 26 pair-list launches of the mutual near field (p2p_mutual.hip)
void launch_p2p_mutual(const fmm_plan_s* p, bool fp32, hipStream_t s);
// whether any step timing hook is set on the calling thread
bool timing_hooks_set();
void release_graph(fmm_plan_s* p);
// fill the plan's JobDev and step tables and copy them to the device (api.cpp)
void upload_job(fmm_plan_s* p, hipStream_t stream);
// Step timing hooks (enum fmm_timed_step): the step's launch in later
// evaluations on this thread is bracketed by these events when they are set.
constexpr int kTimedSteps = FMM_TIME_LOC_SUM + 1;
extern thread_local hipEvent_t g_time_ev[kTimedSteps][2];
}  // namespace fmm
