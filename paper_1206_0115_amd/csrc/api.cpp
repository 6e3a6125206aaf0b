// C-ABI of the library: argument checks, plan lifecycle, export and errors.
// Every argument check happens before the first HIP call, so invalid calls
// fail the same way with or without a GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "fmm_internal.h"

namespace fmm {
namespace {
thread_local std::string g_last_error;
thread_local int g_last_code = FMM_OK;

StepTab one_job(int items, int level = 0) {
  StepTab t;
  std::memset(&t, 0, sizeof(t));
  t.njobs = 1;
  t.job[0] = 0;
  t.level[0] = level;
  t.start[0] = 0;
  t.start[1] = items;
  return t;
}
}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }
void set_error_code(int code) { g_last_code = code; }
int last_error_code() { return g_last_code; }

// Offset ranges per compressed-M2L tile.  Every tile's item runs all of its
// far offsets, so with few items the last round of resident workgroups is
// mostly empty (1M particles at order 7: 1184 items on 512 slots, the last
// 30% of the launch at 30% occupancy).  K ranges per tile make K times as
// many items of 1/K the length; K minimises the rounds ceil(items K / slots)
// / K (in tile lengths), among K whose partial buffers fit the budget.
static int auto_parts(int64_t items, int64_t slots, size_t part_bytes) {
  if (items <= 0 || items >= 6 * slots) return 1;
  constexpr size_t kBudget = size_t(2) << 30;
  int best = 1;
  double best_cost = double((items + slots - 1) / slots);
  for (int k = 2; k <= 4; ++k) {
    if (size_t(k - 1) * part_bytes > kBudget) break;
    const double cost = double((items * k + slots - 1) / slots) / k;
    if (cost < 0.98 * best_cost) {
      best = k;
      best_cost = cost;
    }
  }
  return best;
}

void upload_job(fmm_plan_s* p, hipStream_t s) {
  const int h = p->height;
  const OpSet* op = p->ops;
  JobDev& J = p->job_h;
  std::memset(&J, 0, sizeof(J));
  J.px = p->px;
  J.py = p->py;
  J.pz = p->pz;
  J.prel = p->prel;
  J.qs = p->qs;
  J.perm = p->perm;
  J.leaf_start = p->leaf_start;
  J.leaf_keys = p->lev[h - 1].keys;
  J.near = p->near;
  J.n = int(p->n);
  J.nleaf = int(p->nleaf);
  J.height = h;
  J.order = p->order;
  J.ld = op->ld;
  J.mt = op->mt;
  J.kc = op->kc;
  const bool fp32 = p->precision == FMM_MIXED_FP32 || p->precision == FMM_MIXED_SVD;
  J.kernel = p->kernel;
  J.w32_leaf = p->w32_leaf ? 1 : 0;
  // The FP32 partial sums are Chebyshev coefficients, whose rounding stays
  // relative to each coefficient, so by default they are folded into FP64
  // only once, after the item's last far offset: against FP64, 2.6e-7 at
  // order 7 (1M cube) and 3.2e-7 at order 10 (the 469k twin of the 30M
  // cube, eps 1e-7), for an M2L 6-9% faster than folding every 16 offsets
  // (1.8e-7, 2.0e-7) and far faster than every offset (1.5e-7, 1.8e-7)
  J.fold_every = p->m2l_fold > 0 ? p->m2l_fold : kSlots;
  J.svd = p->svd ? 1 : 0;
  if (p->svd) J.xs = m2l_svd_xs(p->svd->rmax_pad, fp32);
  J.nmb = p->svd ? m2l_svd_nmb(op->mt, fp32, J.xs) : m2l_nmb(op->mt);
  if (p->svd) {
    J.svd_rpad = p->svd->rpad;
    J.svd_rank = p->svd->rk;
    J.svd_off = p->svd->off;
    J.p1_64 = p->svd->p1_64;
    J.p1_32 = p->svd->p1_32;
    J.p2_64 = p->svd->p2_64;
    J.p2_32 = p->svd->p2_32;
  }
  J.ntiles = int(p->ntiles);
  J.has_far = h >= 3;
  J.modal = fp32 && h >= 3 ? 1 : 0;
  J.l2p_sparse = p->nleaf > 0 && p->n <= int64_t(kL2PSparseMax) * int64_t(p->nleaf) ? 1 : 0;
  // compressed M2L split (targets are the cells of levels 2 .. h-1)
  int parts = 1;
  const int64_t lrows = h >= 3 ? int64_t(p->ncell_total) - int64_t(p->lev[2].off) : 0;
  const size_t part_bytes = sizeof(double) * size_t(lrows) * op->ld;
  if (p->svd && h >= 3 && m2l_svd_splits(fp32)) {
    parts = p->m2l_split > 0 ? p->m2l_split
                             : auto_parts(int64_t(p->ntiles) * J.nmb,
                                          m2l_svd_slots(p->order, fp32, J.xs), part_bytes);
  }
  const size_t want = size_t(parts - 1) * part_bytes;
  bool split_oom = false;  // reported once the job below is consistent
  if (p->locx_bytes != want) {
    if (p->LocX) p->free_block(p->LocX);
    p->LocX = nullptr;
    p->locx_bytes = 0;
    if (want) {
      try {
        p->LocX = static_cast<double*>(p->alloc(want));
        p->locx_bytes = want;
      } catch (const FmmError&) {
        parts = 1;
        split_oom = p->m2l_split > 1;
      }
    }
  }
  p->m2l_parts = parts;
  J.m2l_parts = parts;
  J.locx_first = h >= 3 ? int64_t(p->lev[2].off) : 0;
  J.locx_rows = lrows;
  J.LocX = p->LocX;
  J.geo = {p->lo[0], p->lo[1], p->lo[2], p->L / double(int64_t(1) << (h - 1)), h - 1};
  J.W = p->W;
  J.W32 = p->W32;
  J.Loc = p->Loc;
  for (int l = 0; l < h; ++l) {
    J.lev_off[l] = p->lev[l].off;
    J.ncell[l] = int(p->lev[l].ncell);
    J.child_start[l] = p->lev[l].child_start;
    J.parent[l] = p->lev[l].parent;
    J.keys[l] = p->lev[l].keys;
  }
  // a_l = L / 2^(l+1); the unit operators are scaled by a_l^-p
  for (int l = 0; l < kMaxHeight; ++l) {
    const double inv_a = double(int64_t(1) << std::min(l + 1, 62)) / p->L;
    J.scale[l] = p->kernel == FMM_KERNEL_INV_R2 ? inv_a * inv_a : inv_a;
  }
  J.tiles = p->tiles;
  J.tgt = p->tgt;
  J.tile_src = p->tile_src;
  J.tile_act = p->tile_act;
  J.tile_gmask = p->tile_gmask;
  J.tile_nact = p->tile_nact;
  J.kp64 = op->kpack64;
  J.kp32 = op->kpack32;
  J.slot_kid = op->slot_kid;
  J.cheb = op->cheb;
  J.child_modal = op->child_modal;
  J.child = op->child;
  J.phi_n = p->phi_n;
  J.f_n = p->f_n;
  J.phi_f = p->phi_f;
  J.f_f = p->f_f;

  std::memset(p->tab_h, 0, sizeof(p->tab_h));
  p->tab_h[kTabLeaf] = one_job(int(p->nleaf));
  if (h >= 3) {
    // rows cast to FP32: levels 2 .. h-2 when P2M writes the leaves in FP32
    p->tab_h[kTabCast] = one_job(int((p->w32_leaf ? p->lev[h - 1].off : p->ncell_total + 1) -
                                     p->lev[2].off));
    p->tab_h[kTabM2L] = one_job(int(p->ntiles) * J.nmb * parts);
    // tiles are stored finest level first: the leaf level's, then the rest
    int64_t leaf_tiles = 0;
    while (leaf_tiles < p->ntiles && p->tiles_host[leaf_tiles].level == h - 1) ++leaf_tiles;
    const int leaf_items = int(leaf_tiles) * J.nmb * parts;
    p->tab_h[kTabM2LLeaf] = one_job(leaf_items);
    p->tab_h[kTabM2LCoarse] = one_job(int(p->ntiles) * J.nmb * parts - leaf_items);
    p->tab_h[kTabM2LCoarse].first[0] = leaf_items;
    p->tab_h[kTabLocSum] = one_job(parts > 1 ? int(lrows) : 0);
    for (int st = 0; st + 4 <= h; ++st) {
      p->tab_h[kTabM2M + st] = one_job(int(p->lev[h - 2 - st].ncell), h - 2 - st);
      // L2L items are the parents (level 2 + st) of the cells it updates
      p->tab_h[kTabL2L + st] = one_job(int(p->lev[2 + st].ncell), 3 + st);
    }
  }
  ++p->job_version;  // a captured evaluation graph no longer matches
  if (!p->job_d) p->job_d = static_cast<JobDev*>(p->alloc(sizeof(JobDev)));
  if (!p->tab_d) p->tab_d = static_cast<StepTab*>(p->alloc(sizeof(StepTab) * kTabCount));
  FMM_HIP_CHECK(hipMemcpyAsync(p->job_d, &p->job_h, sizeof(JobDev), hipMemcpyHostToDevice, s));
  FMM_HIP_CHECK(hipMemcpyAsync(p->tab_d, p->tab_h, sizeof(p->tab_h), hipMemcpyHostToDevice, s));
  FMM_HIP_CHECK(hipStreamSynchronize(s));
  if (split_oom)
    throw FmmError{FMM_ERR_OOM, "no device memory for the partial buffers of the M2L split; "
                                "the plan runs unsplit"};
}
}  // namespace fmm

void* fmm_plan_s::alloc(size_t b) {
  void* p = fmm::dev_alloc(b);
  blocks.push_back({p, b});
  bytes += b;
  return p;
}

void fmm_plan_s::free_block(void* ptr) {
  for (size_t i = 0; i < blocks.size(); ++i)
    if (blocks[i].first == ptr) {
      bytes -= blocks[i].second;
      fmm::dev_free(ptr);
      blocks.erase(blocks.begin() + i);
      return;
    }
}

fmm_plan_s::~fmm_plan_s() {
  // the evaluation's last work first: done, then the side stream
  fmm::event_put(device, done);
  fmm::release_graph(this);
  if (capture) fmm::side_stream_put(device, capture);
  fmm::side_stream_put(device, side);
  fmm::event_put(device, ev_fork);
  fmm::event_put(device, ev_join);
  for (auto& b : blocks) fmm::dev_free(b.first);
}

namespace {

int fail(int code, const std::string& msg) {
  fmm::set_error(msg);
  fmm::set_error_code(code);
  return code;
}

template <typename F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const fmm::FmmError& e) {
    return fail(e.code, e.msg);
  } catch (const std::bad_alloc&) {
    return fail(FMM_ERR_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(FMM_ERR_HIP, e.what());
  }
}

// A plan is busy while an evaluation enqueued on another stream has not
// finished; evaluations queued on the same stream are ordered by it.
int check_idle(fmm_plan_s* p, hipStream_t s) {
  if (p->in_flight && p->done && s != p->last_stream) {
    hipError_t e = hipEventQuery(p->done);
    if (e == hipErrorNotReady) return FMM_ERR_STATE;
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return FMM_ERR_HIP;
    }
    p->in_flight = false;
  }
  return FMM_OK;
}

}  // namespace

extern "C" {

const char* fmm_last_error(void) { return fmm::g_last_error.c_str(); }

fmm_plan_t fmm_plan_stream(const double* positions, int64_t n, int height, int order,
                           hipStream_t stream) {
  fmm::set_error("");
  fmm::set_error_code(FMM_OK);
  if (!positions) {
    fail(FMM_ERR_ARG, "positions is NULL");
    return nullptr;
  }
  if (n < 1 || n > int64_t(2147483646)) {
    fail(FMM_ERR_ARG, "n must be in [1, 2^31-2], got " + std::to_string(n));
    return nullptr;
  }
  if (height < 1 || height > fmm::kMaxHeight) {
    fail(FMM_ERR_ARG, "height must be in [1, 21], got " + std::to_string(height));
    return nullptr;
  }
  if (order < 1 || order > fmm::kMaxOrder) {
    fail(FMM_ERR_ARG, "order must be in [1, 12], got " + std::to_string(order));
    return nullptr;
  }
  fmm_plan_s* p = nullptr;
  int rc = guarded([&]() -> int {
    p = new fmm_plan_s();
    FMM_HIP_CHECK(hipGetDevice(&p->device));
    p->n = n;
    p->height = height;
    p->order = order;
    // the paper's accuracy setting ties the tolerance to the order,
    // eps = 10^-order (Sec. 2.1.2, Table 1); below 1e-10 the ranks would
    // outgrow the compressed kernel's LDS
    p->m2l_eps = std::pow(10.0, -double(std::min(order, 10)));
    p->ops = fmm::get_opset(order, p->kernel, stream);
    fmm::build_plan(p, positions, stream);
    const int ld = p->ops->ld;
    const size_t rows = size_t(p->ncell_total + 1);
    p->qs = static_cast<double*>(p->alloc(sizeof(double) * n));
    p->phi_n = static_cast<double*>(p->alloc(sizeof(double) * n));
    p->f_n = static_cast<double*>(p->alloc(sizeof(double) * 3 * n));
    if (height >= 3) {
      p->phi_f = static_cast<double*>(p->alloc(sizeof(double) * n));
      p->f_f = static_cast<double*>(p->alloc(sizeof(double) * 3 * n));
      p->Loc = static_cast<double*>(p->alloc(sizeof(double) * rows * ld));
      // the multipole buffers depend on the precision mode: ensure_w
    }
    fmm::upload_job(p, stream);  // ends with a synchronisation of the stream
    fmm::plan_stats(p);
    p->done = fmm::event_get(p->device);
    p->ev_fork = fmm::event_get(p->device);
    p->ev_join = fmm::event_get(p->device);
    p->side = fmm::side_stream_get(p->device);
    return FMM_OK;
  });
  if (rc != FMM_OK) {
    delete p;
    return nullptr;
  }
  return p;
}

fmm_plan_t fmm_plan(const double* positions, int64_t n, int height, int order) {
  return fmm_plan_stream(positions, n, height, order, nullptr);
}

void fmm_release(fmm_plan_t plan) {
  if (!plan) return;
  delete plan;
}

static bool is_mixed(int mode) { return mode == FMM_MIXED_FP32 || mode == FMM_MIXED_SVD; }

// Multipole storage for the plan's precision mode.  FP64 modes: W (FP64) for
// every cell.  Mixed modes: W32 (FP32) for every cell, written directly by P2M
// at the leaf level and cast from W above it, and W (FP64) only for the
// levels above the leaves, where M2M runs in FP64; this halves the largest
// buffer at the 288 GB scale.  The row past the last cell is the zero source
// of absent M2L slots.  Returns whether a buffer changed.
static bool ensure_w(fmm_plan_s* p, hipStream_t s) {
  if (p->height < 3) return false;
  const bool mixed = is_mixed(p->precision);
  const int ld = p->ops->ld;
  const int64_t rows = p->ncell_total + 1;
  const int64_t want64 = mixed ? p->lev[p->height - 1].off : rows;
  bool changed = false;
  if (p->w64_rows != want64 || !p->W) {
    if (p->W) p->free_block(p->W);
    p->W = nullptr;  // a failed allocation below leaves no stale pointer
    p->w64_rows = 0;
    p->W = static_cast<double*>(p->alloc(sizeof(double) * size_t(want64) * ld));
    if (!mixed)
      FMM_HIP_CHECK(hipMemsetAsync(p->W + (rows - 1) * ld, 0, sizeof(double) * ld, s));
    p->w64_rows = want64;
    changed = true;
  }
  if (mixed && !p->W32) {
    p->w32_leaf = false;
    p->W32 = static_cast<float*>(p->alloc(sizeof(float) * size_t(rows) * ld));
    FMM_HIP_CHECK(hipMemsetAsync(p->W32 + (rows - 1) * ld, 0, sizeof(float) * ld, s));
    changed = true;
  } else if (!mixed && p->W32) {
    p->free_block(p->W32);
    p->W32 = nullptr;
    changed = true;
  }
  if (p->w32_leaf != mixed) {
    p->w32_leaf = mixed;
    changed = true;
  }
  return changed;
}

// Apply the precision mode and M2L tolerance: size the multipole buffers for
// the mode, fetch the compressed operators of the SVD modes, and refresh the
// device-side job description.
static void apply_mode(fmm_plan_s* p, int mode) {
  if (p->in_flight) FMM_HIP_CHECK(hipEventSynchronize(p->done));
  const bool mixed = mode == FMM_MIXED_FP32 || mode == FMM_MIXED_SVD;
  const bool svd = mode == FMM_FP64_SVD || mode == FMM_MIXED_SVD;
  const fmm::SvdOps* sv = svd && p->height >= 3
                             ? fmm::get_svd_ops(p->order, p->m2l_eps, p->kernel, p->last_stream)
                             : nullptr;
  if (sv) {
    // the compressed kernel keeps two sets of four rank x 16*NT slabs in LDS
    const size_t need =
        fmm::m2l_svd_lds_need(p->order, mixed, fmm::m2l_svd_xs(sv->rmax_pad, mixed));
    int have = 0;
    FMM_HIP_CHECK(hipDeviceGetAttribute(&have, hipDeviceAttributeMaxSharedMemoryPerBlock,
                                        p->device));
    char tol[32];
    std::snprintf(tol, sizeof(tol), "%g", p->m2l_eps);
    if (need > size_t(have))
      throw fmm::FmmError{FMM_ERR_ARG,
                          "compressed M2L at order " + std::to_string(p->order) +
                              " and tolerance " + tol + " keeps rank " +
                              std::to_string(sv->rmax_pad) + " and needs " +
                              std::to_string(need) + " B of LDS (device: " +
                              std::to_string(have) +
                              "); use a larger tolerance or the dense mode"};
  }
  p->svd = sv;
  p->precision = mode;
  ensure_w(p, p->last_stream);
  fmm::upload_job(p, p->last_stream);
}

int fmm_plan_set_precision(fmm_plan_t p, int mode) {
  if (!p) return fail(FMM_ERR_ARG, "plan is NULL");
  if (mode == FMM_MIXED_BF16)
    return fail(FMM_ERR_ARG, "FMM_MIXED_BF16 is not built (BF16 products cannot meet the "
                             "1e-6 gate of the mixed modes); use FMM_MIXED_FP32 or FMM_MIXED_SVD");
  if (mode < FMM_FP64 || mode > FMM_MIXED_SVD)
    return fail(FMM_ERR_ARG, "unknown precision mode " + std::to_string(mode));
  return guarded([&]() -> int {
    std::lock_guard<std::mutex> lk(p->mu);
    apply_mode(p, mode);
    return FMM_OK;
  });
}

int fmm_plan_set_graph(fmm_plan_t p, int on) {
  if (!p) return fail(FMM_ERR_ARG, "plan is NULL");
  if (on != 0 && on != 1) return fail(FMM_ERR_ARG, "graph switch must be 0 or 1");
  return guarded([&]() -> int {
    std::lock_guard<std::mutex> lk(p->mu);
    if (p->in_flight) FMM_HIP_CHECK(hipEventSynchronize(p->done));
    p->graph_on = on != 0;
    if (!p->graph_on) fmm::release_graph(p);
    return FMM_OK;
  });
}

int fmm_plan_set_schedule(fmm_plan_t p, int schedule) {
  if (!p) return fail(FMM_ERR_ARG, "plan is NULL");
  if (schedule != FMM_SCHEDULE_SERIAL && schedule != FMM_SCHEDULE_FORKED &&
      schedule != FMM_SCHEDULE_PIPELINED)
    return fail(FMM_ERR_ARG, "unknown schedule " + std::to_string(schedule));
  return guarded([&]() -> int {
    std::lock_guard<std::mutex> lk(p->mu);
    p->schedule = schedule;
    return FMM_OK;
  });
}

int fmm_plan_set_near(fmm_plan_t p, int mode) {
  if (!p) return fail(FMM_ERR_ARG, "plan is NULL");
  if (mode != FMM_NEAR_ONE_SIDED && mode != FMM_NEAR_MUTUAL)
    return fail(FMM_ERR_ARG, "unknown near-field mode " + std::to_string(mode));
  return guarded([&]() -> int {
    std::lock_guard<std::mutex> lk(p->mu);
    if (p->in_flight) FMM_HIP_CHECK(hipEventSynchronize(p->done));
    if (mode == FMM_NEAR_MUTUAL && !p->mutual_list) fmm::build_mutual_lists(p, p->last_stream);
    if (mode != p->near_mode) fmm::release_graph(p);
    p->near_mode = mode;
    return FMM_OK;
  });
}

int fmm_plan_set_kernel(fmm_plan_t p, int kernel) {
  if (!p) return fail(FMM_ERR_ARG, "plan is NULL");
  if (kernel != FMM_KERNEL_INV_R && kernel != FMM_KERNEL_INV_R2)
    return fail(FMM_ERR_ARG, "unknown kernel " + std::to_string(kernel));
  return guarded([&]() -> int {
    std::lock_guard<std::mutex> lk(p->mu);
    if (p->in_flight) FMM_HIP_CHECK(hipEventSynchronize(p->done));
    const int prev = p->kernel;
    const fmm::OpSet* prev_ops = p->ops;
    p->kernel = kernel;
    try {
      p->ops = fmm::get_opset(p->order, kernel, p->last_stream);
      apply_mode(p, p->precision);
    } catch (...) {
      p->kernel = prev;
      p->ops = prev_ops;
      throw;
    }
    return FMM_OK;
  });
}

int fmm_plan_set_m2l_fold_interval(fmm_plan_t p, int offsets) {
  if (!p) return fail(FMM_ERR_ARG, "plan is NULL");
  if (offsets < 0 || offsets > fmm::kSlots)
    return fail(FMM_ERR_ARG, "fold interval must be in [0, 189], got " + std::to_string(offsets));
  return guarded([&]() -> int {
    std::lock_guard<std::mutex> lk(p->mu);
    if (p->in_flight) FMM_HIP_CHECK(hipEventSynchronize(p->done));
    p->m2l_fold = offsets;
    fmm::upload_job(p, p->last_stream);
    return FMM_OK;
  });
}

int fmm_plan_set_m2l_split(fmm_plan_t p, int parts) {
  if (!p) return fail(FMM_ERR_ARG, "plan is NULL");
  if (parts < 0 || parts > 4)
    return fail(FMM_ERR_ARG, "M2L split must be in [0, 4], got " + std::to_string(parts));
  return guarded([&]() -> int {
    std::lock_guard<std::mutex> lk(p->mu);
    if (p->in_flight) FMM_HIP_CHECK(hipEventSynchronize(p->done));
    const int prev = p->m2l_split;
    p->m2l_split = parts;
    try {
      fmm::upload_job(p, p->last_stream);
    } catch (...) {
      p->m2l_split = prev;
      throw;
    }
    return FMM_OK;
  });
}

int fmm_plan_m2l_split(fmm_plan_t p, int* parts) {
  if (!p) return fail(FMM_ERR_ARG, "plan is NULL");
  if (!parts) return fail(FMM_ERR_ARG, "parts is NULL");
  *parts = p->m2l_parts;
  return FMM_OK;
}

int fmm_plan_set_m2l_tolerance(fmm_plan_t p, double eps) {
  if (!p) return fail(FMM_ERR_ARG, "plan is NULL");
  if (!(eps > 0.0 && eps < 1.0)) return fail(FMM_ERR_ARG, "tolerance must be in (0, 1)");
  return guarded([&]() -> int {
    std::lock_guard<std::mutex> lk(p->mu);
    const double prev = p->m2l_eps;
    p->m2l_eps = eps;
    // the dense modes only record it: the operators (and, for a plan not
    // evaluated yet, the multipole buffers) are set up when a compressed
    // mode is selected
    if (p->precision != FMM_FP64_SVD && p->precision != FMM_MIXED_SVD) return FMM_OK;
    try {
      apply_mode(p, p->precision);
    } catch (...) {
      p->m2l_eps = prev;
      throw;
    }
    return FMM_OK;
  });
}

int fmm_plan_svd_info(fmm_plan_t p, struct fmm_svd_info* out) {
  if (!p || !out) return fail(FMM_ERR_ARG, "NULL argument");
  return guarded([&]() -> int {
    std::lock_guard<std::mutex> lk(p->mu);
    const fmm::SvdOps* sv = fmm::get_svd_ops(p->order, p->m2l_eps, p->kernel, p->last_stream);
    std::memset(out, 0, sizeof(*out));
    out->eps = sv->eps;
    for (int c = 0; c < 16; ++c) out->rank[c] = sv->rank[c];
    out->rmax_pad = sv->rmax_pad;
    out->weighted_rank = sv->weighted_rank;
    return FMM_OK;
  });
}

static int eval_common(fmm_plan_t p, const double* q, double* phi, double* f, double* pn,
                       double* fn, double* pf, double* ff, hipStream_t s) {
  if (!p) return fail(FMM_ERR_ARG, "plan is NULL");
  if (!q) return fail(FMM_ERR_ARG, "charges is NULL");
  if (phi == nullptr && pn == nullptr) return fail(FMM_ERR_ARG, "output is NULL");
  if ((phi && !f) || (pn && (!fn || !pf || !ff))) return fail(FMM_ERR_ARG, "output is NULL");
  return guarded([&]() -> int {
    std::lock_guard<std::mutex> lk(p->mu);
    int st = check_idle(p, s);
    if (st == FMM_ERR_STATE) return fail(st, "plan is still evaluating on another stream");
    if (st != FMM_OK) return fail(st, "event query failed");
    int dev = 0;
    FMM_HIP_CHECK(hipGetDevice(&dev));
    if (dev != p->device) return fail(FMM_ERR_ARG, "plan belongs to another device");
    // the first evaluation of a plan whose mode was never set allocates here
    if (ensure_w(p, s)) fmm::upload_job(p, s);
    if (p->graph_on && phi && !fmm::timing_hooks_set())
      fmm::evaluate_graph(p, q, phi, f, s);
    else
      fmm::evaluate(p, q, phi, f, pn, fn, pf, ff, s);
    FMM_HIP_CHECK(hipEventRecord(p->done, s));
    p->in_flight = true;
    p->last_stream = s;
    return FMM_OK;
  });
}

int fmm_evaluate(fmm_plan_t plan, const double* charges, double* potential, double* forces,
                 hipStream_t stream) {
  if (!potential || !forces) return fail(FMM_ERR_ARG, "output is NULL");
  return eval_common(plan, charges, potential, forces, nullptr, nullptr, nullptr, nullptr,
                     stream);
}

int fmm_evaluate_parts(fmm_plan_t plan, const double* charges, double* phi_near,
                       double* f_near, double* phi_far, double* f_far, hipStream_t stream) {
  if (!phi_near || !f_near || !phi_far || !f_far) return fail(FMM_ERR_ARG, "output is NULL");
  return eval_common(plan, charges, nullptr, nullptr, phi_near, f_near, phi_far, f_far,
                     stream);
}

int fmm_plan_info(fmm_plan_t p, struct fmm_info* out) {
  if (!p || !out) return fail(FMM_ERR_ARG, "NULL argument");
  std::memset(out, 0, sizeof(*out));
  out->n = p->n;
  out->height = p->height;
  out->order = p->order;
  out->precision = p->precision;
  out->ld = p->ops ? p->ops->ld : 0;
  out->n_leaf = p->nleaf;
  for (int l = 0; l < p->height; ++l) out->ncell[l] = p->lev[l].ncell;
  for (int d = 0; d < 3; ++d) out->lo[d] = p->lo[d];
  out->L = p->L;
  out->near_pairs = p->near_pairs;
  out->far_pairs = p->far_pairs;
  for (int l = 0; l < fmm::kMaxHeight; ++l) out->far_pairs_level[l] = p->far_pairs_level[l];
  out->m2l_tiles = p->ntiles;
  out->m2l_active_slots = p->active_slots;
  out->m2l_groups = p->m2l_groups;
  out->m2l_groups_empty = p->m2l_groups_empty;
  out->m2l_group_skip = p->m2l_gskip ? 1 : 0;
  out->device_bytes = int64_t(p->bytes);
  // algorithmic M2L flops of one evaluation in the current mode
  const double l3 = double(p->order) * p->order * p->order;
  if (p->svd) {
    double fl = 0.0;
    for (int k = 0; k < fmm::kOffsets; ++k)
      fl += double(p->pairs_by_kid[k]) * 4.0 * l3 *
            double(p->svd->rank[fmm::kid_canon(k)]);
    out->m2l_flops = fl;
  } else {
    out->m2l_flops = 2.0 * l3 * l3 * double(p->far_pairs);
  }
  return FMM_OK;
}

int fmm_plan_export(fmm_plan_t p, int what, int level, void* dst, size_t bytes) {
  if (!p || !dst) return fail(FMM_ERR_ARG, "NULL argument");
  auto need = [&](size_t b) { return bytes >= b; };
  return guarded([&]() -> int {
    std::lock_guard<std::mutex> lk(p->mu);
    const int64_t n = p->n, nl = p->nleaf;
    switch (what) {
      case FMM_EXPORT_KEYS:
        if (!need(sizeof(uint64_t) * n)) return fail(FMM_ERR_ARG, "buffer too small");
        FMM_HIP_CHECK(hipMemcpy(dst, p->keys, sizeof(uint64_t) * n, hipMemcpyDeviceToHost));
        return FMM_OK;
      case FMM_EXPORT_PERM: {
        if (!need(sizeof(int64_t) * n)) return fail(FMM_ERR_ARG, "buffer too small");
        std::vector<int> v(n);
        FMM_HIP_CHECK(hipMemcpy(v.data(), p->perm, sizeof(int) * n, hipMemcpyDeviceToHost));
        int64_t* o = static_cast<int64_t*>(dst);
        for (int64_t i = 0; i < n; ++i) o[i] = v[i];
        return FMM_OK;
      }
      case FMM_EXPORT_LEAF_START: {
        if (!need(sizeof(int64_t) * (nl + 1))) return fail(FMM_ERR_ARG, "buffer too small");
        std::vector<int> v(nl + 1);
        FMM_HIP_CHECK(hipMemcpy(v.data(), p->leaf_start, sizeof(int) * (nl + 1),
                                hipMemcpyDeviceToHost));
        int64_t* o = static_cast<int64_t*>(dst);
        for (int64_t i = 0; i <= nl; ++i) o[i] = v[i];
        return FMM_OK;
      }
      case FMM_EXPORT_CELL_KEYS: {
        if (level < 0 || level >= p->height) return fail(FMM_ERR_ARG, "bad level");
        const int64_t c = p->lev[level].ncell;
        if (!need(sizeof(uint64_t) * c)) return fail(FMM_ERR_ARG, "buffer too small");
        FMM_HIP_CHECK(hipMemcpy(dst, p->lev[level].keys, sizeof(uint64_t) * c,
                                hipMemcpyDeviceToHost));
        return FMM_OK;
      }
      case FMM_EXPORT_NEAR_OFF:
      case FMM_EXPORT_NEAR_IDX: {
        std::vector<int> nr(27 * nl);
        FMM_HIP_CHECK(hipMemcpy(nr.data(), p->near, sizeof(int) * 27 * nl,
                                hipMemcpyDeviceToHost));
        std::vector<int64_t> off(nl + 1, 0), idx;
        for (int64_t a = 0; a < nl; ++a) {
          std::vector<int64_t> row;
          for (int s = 0; s < 27; ++s)
            if (nr[27 * a + s] >= 0) row.push_back(nr[27 * a + s]);
          std::sort(row.begin(), row.end());
          idx.insert(idx.end(), row.begin(), row.end());
          off[a + 1] = int64_t(idx.size());
        }
        const std::vector<int64_t>& v = what == FMM_EXPORT_NEAR_OFF ? off : idx;
        if (!need(sizeof(int64_t) * v.size())) return fail(FMM_ERR_ARG, "buffer too small");
        std::memcpy(dst, v.data(), sizeof(int64_t) * v.size());
        return FMM_OK;
      }
      case FMM_EXPORT_FAR_OFF:
      case FMM_EXPORT_FAR_IDX: {
        if (level < 2 || level >= p->height) return fail(FMM_ERR_ARG, "bad level");
        const int64_t nc = p->lev[level].ncell, off0 = p->lev[level].off;
        std::vector<std::vector<int64_t>> rows(nc);
        if (p->ntiles > 0) {
          int64_t ntgt = 0;
          for (int l = 2; l < p->height; ++l) ntgt += p->lev[l].ncell;
          std::vector<int> tgt(ntgt), src(size_t(p->ntiles) * fmm::kSlots * fmm::kTileN);
          FMM_HIP_CHECK(hipMemcpy(tgt.data(), p->tgt, sizeof(int) * ntgt, hipMemcpyDeviceToHost));
          FMM_HIP_CHECK(hipMemcpy(src.data(), p->tile_src, sizeof(int) * src.size(),
                                  hipMemcpyDeviceToHost));
          for (int64_t t = 0; t < p->ntiles; ++t) {
            const fmm::M2LTile& tl = p->tiles_host[t];
            if (tl.level != level) continue;
            for (int j = 0; j < tl.count; ++j) {
              const int64_t c = tgt[tl.first + j] - off0;
              for (int s = 0; s < fmm::kSlots; ++s) {
                const int b = src[(t * fmm::kSlots + s) * fmm::kTileN + j];
                if (b != int(p->ncell_total)) rows[c].push_back(b - off0);
              }
            }
          }
        }
        std::vector<int64_t> off(nc + 1, 0), idx;
        for (int64_t c = 0; c < nc; ++c) {
          std::sort(rows[c].begin(), rows[c].end());
          idx.insert(idx.end(), rows[c].begin(), rows[c].end());
          off[c + 1] = int64_t(idx.size());
        }
        const std::vector<int64_t>& v = what == FMM_EXPORT_FAR_OFF ? off : idx;
        if (!need(sizeof(int64_t) * v.size())) return fail(FMM_ERR_ARG, "buffer too small");
        std::memcpy(dst, v.data(), sizeof(int64_t) * v.size());
        return FMM_OK;
      }
      case FMM_EXPORT_MUTUAL_OFF:
      case FMM_EXPORT_MUTUAL_IDX: {
        if (!p->mutual_list) return fail(FMM_ERR_ARG, "the mutual pair lists are not built");
        constexpr int kLists = 2 * fmm::kMutualSlots;
        const int64_t total = p->mutual_off[kLists];
        if (what == FMM_EXPORT_MUTUAL_OFF) {
          if (!need(sizeof(int64_t) * (kLists + 1))) return fail(FMM_ERR_ARG, "buffer too small");
          std::memcpy(dst, p->mutual_off, sizeof(int64_t) * (kLists + 1));
          return FMM_OK;
        }
        if (!need(sizeof(int64_t) * total)) return fail(FMM_ERR_ARG, "buffer too small");
        std::vector<int> v(total);
        if (total > 0)
          FMM_HIP_CHECK(hipMemcpy(v.data(), p->mutual_list, sizeof(int) * total,
                                  hipMemcpyDeviceToHost));
        int64_t* o = static_cast<int64_t*>(dst);
        for (int64_t i = 0; i < total; ++i) o[i] = v[i];
        return FMM_OK;
      }
      default:
        return fail(FMM_ERR_ARG, "unknown export item");
    }
  });
}

int fmm_set_step_timing_events(int step, hipEvent_t ev0, hipEvent_t ev1) {
  if (step < FMM_TIME_M2L || step > FMM_TIME_LOC_SUM)
    return fail(FMM_ERR_ARG, "unknown timed step " + std::to_string(step));
  if ((ev0 == nullptr) != (ev1 == nullptr)) return fail(FMM_ERR_ARG, "pass both events or none");
  fmm::g_time_ev[step][0] = ev0;
  fmm::g_time_ev[step][1] = ev1;
  return FMM_OK;
}

int fmm_set_m2l_timing_events(hipEvent_t ev0, hipEvent_t ev1) {
  return fmm_set_step_timing_events(FMM_TIME_M2L, ev0, ev1);
}

void fmm_trim_cache(void) { fmm::dev_trim(); }

}  // extern "C"
