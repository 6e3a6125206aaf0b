// Job tables: how one kernel launch covers the work of one or many plans.
//
// Every evaluation kernel walks a flat item range (leaves, cells of a level,
// M2L tile blocks, particle chunks).  A StepTab lists the plans (jobs) taking
// part in one launch and the prefix sums of their item counts; a block finds
// its job by binary search and works on that job's item with that job's
// arrays.  A single evaluation is a one-job table built at plan time; the
// serving loop builds many-job tables per batch.  The per-item code is the
// same in both cases, so a plan's results do not depend on what else shares
// the launch.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fmm {

constexpr int kMaxJobs = 64;
constexpr int kMaxHeightJ = 21;

struct LeafGeom {
  double lo0, lo1, lo2, w;  // leaf width w, centre lo + (k + 1/2) w
  int bits;
};

struct M2LTile;

// Everything a kernel needs to know about one plan (device-resident copy).
struct JobDev {
  const double* px;
  const double* py;
  const double* pz;
  float4* prel;
  double* qs;
  const int* perm;
  const int* leaf_start;
  const uint64_t* leaf_keys;
  const int* near;
  int n, nleaf, height, order, ld, mt, kc, nmb, ntiles, has_far;
  int kernel;  // p of the kernel |x - y|^-p (1 or 2)
  int w32_leaf;  // leaf multipoles live in W32 only (W holds levels < h-1)
  int fold_every;  // compressed FP32 M2L: far offsets between FP64 folds
  // FP32 M2L (mixed modes): the local expansions of levels >= 2 leave M2L
  // as Chebyshev coefficients, and L2L and L2P take them as such
  int modal;
  // leaves hold few particles on average: L2P spreads each particle's l^3
  // terms over a wavefront's lanes (l2p_sparse_kernel)
  int l2p_sparse;
  // compressed M2L split: each tile's far offsets in m2l_parts consecutive
  // ranges, one work item each; part 0 writes Loc, part p > 0 the rows
  // (p - 1) * locx_rows + (target row - locx_first) of LocX
  int m2l_parts;
  int64_t locx_first, locx_rows;
  double* LocX;
  LeafGeom geo;
  double* W;
  float* W32;
  double* Loc;
  int64_t lev_off[kMaxHeightJ];
  int ncell[kMaxHeightJ];
  const int* child_start[kMaxHeightJ];
  const int* parent[kMaxHeightJ];
  const uint64_t* keys[kMaxHeightJ];
  const M2LTile* tiles;
  const int* tgt;
  const int* tile_src;
  const unsigned char* tile_act;
  const unsigned char* tile_gmask;  // per active slot: 16-target groups with a source
  const int* tile_nact;
  double scale[kMaxHeightJ];  // a_l^-p, the M2L level factor
  const double* kp64;
  const float* kp32;
  // compressed M2L (svd != 0): per packed operator kid, the padded rank, the
  // kept rank and the element offset of its two factors in the packs below
  int svd, xs;
  const int* svd_rpad;
  const int* svd_rank;
  const int64_t* svd_off;
  const double* p1_64;  // S V^T (rank x l^3) in MFMA fragment order
  const float* p1_32;
  const double* p2_64;  // U (l^3 x rank) in MFMA fragment order
  const float* p2_32;
  const int* slot_kid;
  const double* cheb;
  const double* child_modal;  // [2][l][l] coefficient re-expansion (OpSet)
  const double* child;
  double* phi_n;  // near/far partial results in sorted order
  double* f_n;
  double* phi_f;
  double* f_f;
};

// Per-evaluation pointers (input order), for the gather and combine steps.
struct CallDev {
  const double* q;
  double* phi;
  double* f;
  double* pn;
  double* fn;
  double* pf;
  double* ff;
};

struct StepTab {
  int njobs;
  int job[kMaxJobs];    // index into the job array
  int level[kMaxJobs];  // per-job level argument (M2M: parent level; L2L: child level)
  int start[kMaxJobs + 1];
  int first[kMaxJobs];  // M2L: the job's first item (a launch may take a range of its tiles)
};

__device__ inline int step_total(const StepTab& t) { return t.start[t.njobs]; }

// k with t.start[k] <= item < t.start[k+1]
__device__ inline int step_find(const StepTab& t, int item) {
  int lo = 0, hi = t.njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (t.start[mid] <= item) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Host-side launchers (eval.hip / m2l.hip).  `grid` <= 0 means one block per
// item (the total must then be given); a positive grid makes every block loop
// over items with that stride (persistent launch).
// kStepM2LSvd is the compressed M2L; `xs` is then the LDS row stride (the
// largest padded rank of the launch's jobs + 4).
enum StepKind { kStepGather, kStepP2M, kStepM2M, kStepCast, kStepM2L, kStepL2L, kStepL2P,
                kStepP2P, kStepCombine, kStepM2LSvd, kStepLocSum, kStepL2PSparse,
                kStepP2PSelf };
// gskip: the compressed M2L skips the 16-target groups without a source at
// an offset (plans whose tiles have many, fmm_info.m2l_group_skip).
void launch_step(StepKind kind, int order, bool fp32, const JobDev* jobs, const StepTab* tab,
                 const CallDev* calls, int grid, hipStream_t s, int xs = 0, bool gskip = false);

}  // namespace fmm
