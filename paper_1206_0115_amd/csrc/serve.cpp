// Serving loop: continuous batching of FMM evaluations on one GPU.
//
// Two threads.  The planner builds the plans of arriving requests on its
// own stream (root box, sort, lists: the synchronous part, after the
// caller's inputs are ready) and admits them while the admitted plans'
// device bytes stay within the budget.  The launcher evaluates batches: all
// admitted requests that are not yet running form one batch whose operators
// run as persistent launches over one shared work table (jobs.h), the whole
// launch sequence captured once per shape as a hipGraph and replayed with
// new tables.  The table travels inside the graph as a copy from a pinned
// host buffer.  Each of the two table buffers has its own execution stream,
// so a batch formed while another runs is launched at once and runs beside
// it on the device; batches retire in whatever order they finish.  Planning
// overlaps the running batches, and never holds up a launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "fmm_internal.h"
#include "jobs.h"

namespace fmm {
namespace {

// Launches per batch: up to 53 per order present (two per tree level for
// M2M and L2L, fourteen M2L forms, P2M, two L2P forms) and six more.
constexpr int kMaxSteps = 704;
constexpr int kBuffers = 2;
// Batching window: admitted requests wait for the planner to finish the
// requests that arrived with them, but no longer than this, so that a burst
// shares launches and a lone request starts almost at once.
constexpr double kBatchWindowS = 0.002;

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// code and message of the exception being handled
void current_failure(int& code, std::string& msg) {
  code = FMM_ERR_HIP;
  msg = "serving loop failure";
  try {
    throw;
  } catch (const FmmError& e) {
    code = e.code;
    msg = e.msg;
  } catch (const std::bad_alloc&) {
    code = FMM_ERR_OOM;
    msg = "host allocation failed";
  } catch (...) {
  }
}

// Blocks per persistent launch, by kernel (sized to keep every CU busy; a
// block loops over the items of the batch with this stride).
int persistent_grid(StepKind k) {
  switch (k) {
    case kStepM2L:
    case kStepM2LSvd: return 512;
    case kStepP2P:
    case kStepP2M:
    case kStepL2P: return 4096;
    default: return 1024;
  }
}

struct Request {
  int64_t id = 0;
  const double* pos = nullptr;
  const double* q = nullptr;
  int64_t n = 0;
  int h = 0, order = 0, prec = 0;
  double* phi = nullptr;
  double* f = nullptr;
  fmm_plan_s* plan = nullptr;
  int status = FMM_OK;
  bool done = false;
  double t_submit = 0, t_admit = 0, t_done = 0;
  int64_t batch = -1;
  int64_t bytes = 0;        // admitted footprint (known after the first plan)
  hipEvent_t inputs = nullptr;  // recorded on the caller's stream at submit
  std::string err;          // message of a failed request
};

struct Launch {
  StepKind kind;
  int order;
  bool fp32;
  int xs;  // LDS row stride of the compressed M2L
  bool gskip;  // compressed M2L: skip the 16-target groups without a source
};

struct TableBuf {
  void* pinned = nullptr;
  void* dev = nullptr;
  hipStream_t stream = nullptr;  // the batches of this buffer run here
  hipEvent_t last = nullptr;  // completion of the batch that last read it
  bool busy = false;
};

struct Batch {
  std::vector<Request*> reqs;
  hipEvent_t ev = nullptr;
  int buf = 0;
  int64_t index = 0;
};

const size_t kJobsOff = 0;
const size_t kCallsOff = align256(sizeof(JobDev) * kMaxJobs);
const size_t kTabsOff = kCallsOff + align256(sizeof(CallDev) * kMaxJobs);
const size_t kTableBytes = kTabsOff + sizeof(StepTab) * kMaxSteps;

}  // namespace
}  // namespace fmm

struct fmm_server_s {
  int device = 0;
  size_t budget = 0;
  int max_active = 0;
  hipStream_t plan_stream = nullptr;
  fmm::TableBuf buf[fmm::kBuffers];
  std::map<std::pair<int, std::string>, hipGraphExec_t> graphs;

  std::mutex mu;
  // cv_work wakes the planner (a submit, freed memory or slots), cv_launch
  // the launcher (a request admitted), cv_done the callers of wait
  std::condition_variable cv_work, cv_launch, cv_done;
  std::deque<fmm::Request*> pending;          // submitted, not yet admitted
  std::vector<fmm::Request*> ready;           // admitted, not yet launched
  std::deque<fmm::Batch> inflight;
  std::unordered_map<int64_t, fmm::Request*> all;
  int64_t next_id = 0;
  size_t used = 0;
  int active = 0;
  int planning = 0;  // requests taken from `pending` whose plans are being built
  bool stop = false;
  bool planner_done = false;
  struct fmm_server_stats st{};
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  std::thread planner, launcher;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  void plan_loop();
  void launch_loop();
  bool retire();
  bool admit();
  bool launch_batch();
  void launch_on(int bi, const std::vector<fmm::Request*>& reqs);
  void finish(fmm::Request* r, int status, const std::string& err = std::string());
};

using namespace fmm;

void fmm_server_s::finish(Request* r, int status, const std::string& err) {
  // called with mu held
  r->status = status;
  r->err = err;
  r->done = true;
  r->t_done = now();
  if (r->inputs) {
    (void)hipEventDestroy(r->inputs);
    r->inputs = nullptr;
  }
  if (status == FMM_OK) ++st.completed;
  else ++st.rejected;
  cv_done.notify_all();
}

// Retire every finished batch, in whatever order the streams finish them.
bool fmm_server_s::retire() {
  bool any = false;
  while (true) {
    Batch b;
    bool found = false;
    {
      std::lock_guard<std::mutex> lk(mu);
      for (auto it = inflight.begin(); it != inflight.end(); ++it) {
        hipError_t e = hipEventQuery(it->ev);
        if (e == hipErrorNotReady) continue;
        b = *it;
        inflight.erase(it);
        found = true;
        const int status = e == hipSuccess ? FMM_OK : FMM_ERR_HIP;
        if (e != hipSuccess) (void)hipGetLastError();
        for (Request* r : b.reqs) {
          used -= size_t(r->bytes);
          --active;
          finish(r, status, status == FMM_OK ? "" : hipGetErrorString(e));
        }
        break;
      }
    }
    if (!found) return any;
    any = true;
    buf[b.buf].busy = false;
    (void)hipEventDestroy(b.ev);
    for (Request* r : b.reqs) {
      fmm_release(r->plan);
      r->plan = nullptr;
    }
    cv_work.notify_all();
  }
}

// Plan pending requests in arrival order while slots and memory allow.
bool fmm_server_s::admit() {
  bool any = false;
  while (true) {
    Request* r = nullptr;
    {
      std::lock_guard<std::mutex> lk(mu);
      if (pending.empty() || active >= max_active) return any;
      r = pending.front();
      // footprint known from an earlier attempt and still too large for now
      if (r->bytes > 0 && used + size_t(r->bytes) > budget) return any;
      pending.pop_front();
      ++planning;
    }
    // the caller's inputs are ready on the device before the plan reads them
    FMM_HIP_CHECK(hipStreamWaitEvent(plan_stream, r->inputs, 0));
    fmm_plan_s* p = fmm_plan_stream(r->pos, r->n, r->h, r->order, plan_stream);
    int rc = p ? fmm_plan_set_precision(p, r->prec) : last_error_code();
    if (rc == FMM_OK && !p) rc = FMM_ERR_HIP;
    const std::string err = rc == FMM_OK ? std::string() : std::string(fmm_last_error());
    std::lock_guard<std::mutex> lk(mu);
    --planning;
    cv_launch.notify_all();
    if (!p || rc != FMM_OK) {
      if (p) fmm_release(p);
      finish(r, rc, err);
      any = true;
      continue;
    }
    r->bytes = int64_t(p->bytes);
    if (size_t(r->bytes) > budget) {
      fmm_release(p);
      finish(r, FMM_ERR_OOM, "the request's plan (" + std::to_string(r->bytes) +
                                 " bytes) exceeds the server's memory budget");
      any = true;
      continue;
    }
    if (used + size_t(r->bytes) > budget) {
      // wait for running batches to free memory; re-plan then
      fmm_release(p);
      pending.push_front(r);
      return any;
    }
    r->plan = p;
    r->t_admit = now();
    used += size_t(r->bytes);
    ++active;
    st.max_active_seen = std::max<int64_t>(st.max_active_seen, active);
    st.peak_admitted_bytes = std::max<int64_t>(st.peak_admitted_bytes, int64_t(used));
    ready.push_back(r);
    cv_launch.notify_all();
    any = true;
  }
}

// Build the batch's work table and launch sequence, then run it as a graph.
bool fmm_server_s::launch_batch() {
  int bi = -1;
  for (int i = 0; i < kBuffers; ++i)
    if (!buf[i].busy) {
      bi = i;
      break;
    }
  std::vector<Request*> reqs;
  {
    std::lock_guard<std::mutex> lk(mu);
    if (ready.empty() || bi < 0) return false;
    // wait for the rest of a burst, within the batching window
    const bool burst_planned = pending.empty() && planning == 0;
    if (!burst_planned && ready.size() < size_t(kMaxJobs) &&
        now() - ready.front()->t_admit < kBatchWindowS)
      return false;
    const size_t take = std::min<size_t>(ready.size(), kMaxJobs);
    reqs.assign(ready.begin(), ready.begin() + take);
    ready.erase(ready.begin(), ready.begin() + take);
  }
  try {
    launch_on(bi, reqs);
  } catch (...) {
    // the batch never ran: its requests end with the failure
    int code;
    std::string msg;
    current_failure(code, msg);
    std::lock_guard<std::mutex> lk(mu);
    for (Request* r : reqs) {
      used -= size_t(r->bytes);
      --active;
      fmm_release(r->plan);
      r->plan = nullptr;
      finish(r, code, msg);
    }
    cv_work.notify_all();
  }
  return true;
}

void fmm_server_s::launch_on(int bi, const std::vector<Request*>& reqs) {
  TableBuf& B = buf[bi];
  hipStream_t exec_stream = B.stream;
  if (B.last) FMM_HIP_CHECK(hipEventSynchronize(B.last));  // its copy has been consumed
  // the batch reads the callers' charges and writes their outputs: after
  // everything each caller's stream had queued at submit
  for (Request* r : reqs) FMM_HIP_CHECK(hipStreamWaitEvent(exec_stream, r->inputs, 0));
  char* host = static_cast<char*>(B.pinned);
  JobDev* jobs = reinterpret_cast<JobDev*>(host + kJobsOff);
  CallDev* calls = reinterpret_cast<CallDev*>(host + kCallsOff);
  StepTab* tabs = reinterpret_cast<StepTab*>(host + kTabsOff);
  const int nj = int(reqs.size());
  for (int j = 0; j < nj; ++j) {
    jobs[j] = reqs[j]->plan->job_h;
    calls[j] = CallDev{reqs[j]->q, reqs[j]->phi, reqs[j]->f, nullptr, nullptr, nullptr, nullptr};
  }

  std::vector<Launch> seq;
  std::string key;
  auto add = [&](StepKind kind, int order, bool fp32, auto want, auto items, auto level,
                 bool gskip = false) {
    StepTab& t = tabs[seq.size()];
    std::memset(&t, 0, sizeof(t));
    int tot = 0, xs = 0;
    for (int j = 0; j < nj; ++j) {
      if (!want(reqs[j])) continue;
      const int it = items(reqs[j]);
      if (it <= 0) continue;
      t.job[t.njobs] = j;
      t.level[t.njobs] = level(reqs[j]);
      t.start[t.njobs] = tot;
      tot += it;
      xs = std::max(xs, reqs[j]->plan->job_h.xs);
      ++t.njobs;
    }
    t.start[t.njobs] = tot;
    if (t.njobs == 0) return;
    if (seq.size() + 1 >= size_t(kMaxSteps)) throw FmmError{FMM_ERR_HIP, "batch step table full"};
    if (kind != kStepM2LSvd) xs = 0;
    seq.push_back({kind, order, fp32, xs, gskip});
    key += std::to_string(int(kind)) + ":" + std::to_string(order) + (fp32 ? "f" : "d") + ":" +
           std::to_string(xs) + (gskip ? "g" : "") + ";";
  };
  auto all_ = [](Request*) { return true; };
  auto lvl0 = [](Request*) { return 0; };
  auto chunks = [](Request* r) { return int((r->n + 255) / 256); };
  auto far = [](Request* r) { return r->h >= 3; };
  auto mixed = [](Request* r) {
    return r->prec == FMM_MIXED_FP32 || r->prec == FMM_MIXED_SVD;
  };
  auto svd = [](Request* r) { return r->plan->svd != nullptr; };

  std::vector<int> orders;
  for (Request* r : reqs)
    if (r->h >= 3 && std::find(orders.begin(), orders.end(), r->order) == orders.end())
      orders.push_back(r->order);
  std::sort(orders.begin(), orders.end());
  int steps = 0;
  for (Request* r : reqs) steps = std::max(steps, r->h - 3);

  add(kStepGather, 0, false, all_, chunks, lvl0);
  for (int L : orders)
    add(kStepP2M, L, false, [&](Request* r) { return far(r) && r->order == L; },
        [](Request* r) { return int(r->plan->nleaf); }, lvl0);
  // M2M and L2L are compiled per order: one launch per order present at
  // each level
  for (int s = 0; s < steps; ++s)
    for (int L : orders)
      add(kStepM2M, L, false, [&](Request* r) { return r->h - 4 >= s && r->order == L; },
          [&](Request* r) { return int(r->plan->lev[r->h - 2 - s].ncell); },
          [&](Request* r) { return r->h - 2 - s; });
  add(kStepCast, 0, true, [&](Request* r) { return far(r) && mixed(r); },
      [](Request* r) { return int(r->plan->tab_h[kTabCast].start[1]); }, lvl0);
  // dense, then compressed by the kernel's N-tiles per item (1, 2, 4): one
  // launch decodes every plan's items alike; the compressed plans that skip
  // empty 16-target groups (points on surfaces) in launches of their own
  auto svd_nt = [&](Request* r) { return m2l_svd_nt(r->order, mixed(r), r->plan->job_h.xs); };
  for (int L : orders)
    for (int f32 = 0; f32 < 2; ++f32)
      for (int cmp = 0; cmp < 4; ++cmp)
        for (int gs = 0; gs < (cmp ? 2 : 1); ++gs)
          add(cmp ? kStepM2LSvd : kStepM2L, L, f32 != 0,
              [&](Request* r) {
                return far(r) && r->order == L && mixed(r) == (f32 != 0) &&
                       svd(r) == (cmp != 0) &&
                       (cmp == 0 || (svd_nt(r) == 1 << (cmp - 1) &&
                                     r->plan->m2l_gskip == (gs != 0)));
              },
              [](Request* r) {
                return int(r->plan->ntiles) * r->plan->job_h.nmb * r->plan->job_h.m2l_parts;
              },
              lvl0, gs != 0);
  // partial sums of plans that split their compressed M2L back into Loc, and
  // the FP32 M2L's Chebyshev-coefficient rows back to node values
  add(kStepLocSum, 0, false, [&](Request* r) { return far(r) && r->plan->job_h.m2l_parts > 1; },
      [](Request* r) { return int(r->plan->job_h.locx_rows); }, lvl0);
  for (int s = 0; s < steps; ++s)
    for (int L : orders)
      add(kStepL2L, L, false, [&](Request* r) { return r->h - 4 >= s && r->order == L; },
          [&](Request* r) { return int(r->plan->lev[2 + s].ncell); },
          [&](Request*) { return 3 + s; });
  for (int L : orders)
    for (int sp = 0; sp < 2; ++sp)
      add(sp ? kStepL2PSparse : kStepL2P, L, false,
          [&](Request* r) {
            return far(r) && r->order == L && (r->plan->job_h.l2p_sparse != 0) == (sp != 0);
          },
          [](Request* r) { return int(r->plan->nleaf); }, lvl0);
  for (int f32 = 0; f32 < 2; ++f32)
    add(kStepP2P, 0, f32 != 0, [&](Request* r) { return mixed(r) == (f32 != 0); },
        [](Request* r) { return int(r->plan->nleaf); }, lvl0);
  add(kStepCombine, 0, false, all_, chunks, lvl0);

  // the graph for this launch sequence and buffer, captured on first use
  const JobDev* jobs_d = reinterpret_cast<const JobDev*>(static_cast<char*>(B.dev) + kJobsOff);
  const CallDev* calls_d = reinterpret_cast<const CallDev*>(static_cast<char*>(B.dev) + kCallsOff);
  const StepTab* tabs_d = reinterpret_cast<const StepTab*>(static_cast<char*>(B.dev) + kTabsOff);
  auto gk = std::make_pair(bi, key);
  auto it = graphs.find(gk);
  if (it == graphs.end()) {
    hipGraph_t g = nullptr;
    FMM_HIP_CHECK(hipStreamBeginCapture(exec_stream, hipStreamCaptureModeThreadLocal));
    FMM_HIP_CHECK(hipMemcpyAsync(B.dev, B.pinned, kTableBytes, hipMemcpyHostToDevice, exec_stream));
    for (size_t i = 0; i < seq.size(); ++i)
      launch_step(seq[i].kind, seq[i].order, seq[i].fp32, jobs_d, tabs_d + i, calls_d,
                  persistent_grid(seq[i].kind), exec_stream, seq[i].xs, seq[i].gskip);
    FMM_HIP_CHECK(hipStreamEndCapture(exec_stream, &g));
    hipGraphExec_t ge = nullptr;
    FMM_HIP_CHECK(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
    FMM_HIP_CHECK(hipGraphDestroy(g));
    it = graphs.emplace(gk, ge).first;
    ++st.graph_captures;
  }
  FMM_HIP_CHECK(hipGraphLaunch(it->second, exec_stream));
  Batch b;
  b.reqs = reqs;
  b.buf = bi;
  FMM_HIP_CHECK(hipEventCreateWithFlags(&b.ev, hipEventDisableTiming));
  FMM_HIP_CHECK(hipEventRecord(b.ev, exec_stream));
  if (B.last) FMM_HIP_CHECK(hipEventDestroy(B.last));
  FMM_HIP_CHECK(hipEventCreateWithFlags(&B.last, hipEventDisableTiming));
  FMM_HIP_CHECK(hipEventRecord(B.last, exec_stream));
  B.busy = true;
  {
    std::lock_guard<std::mutex> lk(mu);
    b.index = st.batches++;
    ++st.graph_replays;
    st.max_batch_jobs = std::max<int64_t>(st.max_batch_jobs, nj);
    for (Request* r : reqs) r->batch = b.index;
    inflight.push_back(b);
  }
}

// The planner: plans and admits arriving requests.
void fmm_server_s::plan_loop() {
  (void)hipSetDevice(device);
  while (true) {
    bool progress = false;
    try {
      progress = admit();
    } catch (...) {
      // a runtime failure ends every request not yet admitted
      int code;
      std::string msg;
      current_failure(code, msg);
      std::lock_guard<std::mutex> lk(mu);
      set_error(msg);
      for (Request* r : pending) finish(r, code, msg);
      pending.clear();
    }
    std::unique_lock<std::mutex> lk(mu);
    if (stop && pending.empty()) {
      planner_done = true;
      cv_launch.notify_all();
      break;
    }
    if (progress) continue;
    cv_work.wait_for(lk, std::chrono::milliseconds(5));
  }
}

// The launcher: retires finished batches and launches admitted requests.
void fmm_server_s::launch_loop() {
  (void)hipSetDevice(device);
  while (true) {
    bool progress = false;
    try {
      progress |= retire();
      progress |= launch_batch();
    } catch (...) {
      // a runtime failure ends every admitted request that is not running
      int code;
      std::string msg;
      current_failure(code, msg);
      std::lock_guard<std::mutex> lk(mu);
      set_error(msg);
      for (Request* r : ready) {
        if (r->plan) {
          used -= size_t(r->bytes);
          --active;
          fmm_release(r->plan);
          r->plan = nullptr;
        }
        finish(r, code, msg);
      }
      ready.clear();
      cv_work.notify_all();
    }
    std::unique_lock<std::mutex> lk(mu);
    if (stop && planner_done && ready.empty() && inflight.empty()) break;
    if (progress) continue;
    if (!inflight.empty()) {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
    } else {
      // admitted requests inside their batching window: look again soon
      cv_launch.wait_for(lk, ready.empty() ? std::chrono::microseconds(5000)
                                           : std::chrono::microseconds(200));
    }
  }
  // release the graphs
  for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
  graphs.clear();
}

extern "C" {

fmm_server_t fmm_server_create(size_t hbm_budget_bytes, int max_active) {
  set_error("");
  if (hbm_budget_bytes == 0) {
    set_error("hbm_budget_bytes must be > 0");
    return nullptr;
  }
  if (max_active < 1 || max_active > kMaxJobs) {
    set_error("max_active must be in [1, 64]");
    return nullptr;
  }
  fmm_server_s* s = new fmm_server_s();
  try {
    FMM_HIP_CHECK(hipGetDevice(&s->device));
    s->budget = hbm_budget_bytes;
    s->max_active = max_active;
    FMM_HIP_CHECK(hipStreamCreateWithFlags(&s->plan_stream, hipStreamNonBlocking));
    for (int i = 0; i < kBuffers; ++i) {
      FMM_HIP_CHECK(hipStreamCreateWithFlags(&s->buf[i].stream, hipStreamNonBlocking));
      FMM_HIP_CHECK(hipHostMalloc(&s->buf[i].pinned, kTableBytes, hipHostMallocDefault));
      std::memset(s->buf[i].pinned, 0, kTableBytes);
      FMM_HIP_CHECK(hipMalloc(&s->buf[i].dev, kTableBytes));
    }
  } catch (const FmmError& e) {
    set_error(e.msg);
    for (int i = 0; i < kBuffers; ++i) {
      if (s->buf[i].pinned) (void)hipHostFree(s->buf[i].pinned);
      if (s->buf[i].dev) (void)hipFree(s->buf[i].dev);
      if (s->buf[i].stream) (void)hipStreamDestroy(s->buf[i].stream);
    }
    if (s->plan_stream) (void)hipStreamDestroy(s->plan_stream);
    delete s;
    return nullptr;
  }
  s->planner = std::thread([s] { s->plan_loop(); });
  s->launcher = std::thread([s] { s->launch_loop(); });
  return s;
}

int64_t fmm_server_submit(fmm_server_t s, const double* positions, const double* charges,
                          int64_t n, int height, int order, int precision, double* potential,
                          double* forces, hipStream_t stream) {
  if (!s) {
    set_error("server is NULL");
    return FMM_ERR_ARG;
  }
  if (!positions || !charges || !potential || !forces) {
    set_error("NULL pointer argument");
    return FMM_ERR_ARG;
  }
  if (n < 1 || n > int64_t(2147483646) || height < 1 || height > kMaxHeight || order < 1 ||
      order > kMaxOrder || precision < FMM_FP64 || precision > FMM_MIXED_SVD ||
      precision == FMM_MIXED_BF16) {
    set_error("invalid n, height, order or precision");
    return FMM_ERR_ARG;
  }
  hipEvent_t inputs = nullptr;
  hipError_t e = hipEventCreateWithFlags(&inputs, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(inputs, stream);
  if (e != hipSuccess) {
    if (inputs) (void)hipEventDestroy(inputs);
    (void)hipGetLastError();
    set_error(std::string("recording the caller's stream failed: ") + hipGetErrorString(e));
    return FMM_ERR_HIP;
  }
  Request* r = new Request();
  r->inputs = inputs;
  r->pos = positions;
  r->q = charges;
  r->n = n;
  r->h = height;
  r->order = order;
  r->prec = precision;
  r->phi = potential;
  r->f = forces;
  std::lock_guard<std::mutex> lk(s->mu);
  r->id = s->next_id++;
  r->t_submit = s->now();
  s->all[r->id] = r;
  s->pending.push_back(r);
  ++s->st.submitted;
  s->cv_work.notify_all();
  return r->id;
}

static void fill_stats(const Request* r, fmm_request_stats* out) {
  if (!out) return;
  out->status = r->status;
  out->done = r->done ? 1 : 0;
  out->submit_s = r->t_submit;
  out->admit_s = r->t_admit;
  out->done_s = r->t_done;
  out->batch = r->batch;
  out->plan_bytes = r->bytes;
}

int fmm_server_poll(fmm_server_t s, int64_t ticket, fmm_request_stats* out) {
  if (!s) return FMM_ERR_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) {
    set_error("unknown ticket");
    return FMM_ERR_ARG;
  }
  fill_stats(it->second, out);
  return it->second->done ? 1 : 0;
}

int fmm_server_request_error(fmm_server_t s, int64_t ticket, char* buf, size_t len) {
  if (!s || (!buf && len > 0)) {
    set_error("server or buffer is NULL");
    return FMM_ERR_ARG;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) {
    set_error("unknown ticket");
    return FMM_ERR_ARG;
  }
  const std::string& m = it->second->err;
  if (len > 0) {
    const size_t k = std::min(len - 1, m.size());
    std::memcpy(buf, m.data(), k);
    buf[k] = '\0';
  }
  return int(m.size());
}

int fmm_server_wait(fmm_server_t s, int64_t ticket, fmm_request_stats* out) {
  if (!s) return FMM_ERR_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) {
    set_error("unknown ticket");
    return FMM_ERR_ARG;
  }
  Request* r = it->second;
  s->cv_done.wait(lk, [&] { return r->done; });
  fill_stats(r, out);
  return r->status;
}

double fmm_server_now(fmm_server_t s) { return s ? s->now() : 0.0; }

int fmm_server_get_stats(fmm_server_t s, struct fmm_server_stats* out) {
  if (!s || !out) return FMM_ERR_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->st;
  return FMM_OK;
}

void fmm_server_destroy(fmm_server_t s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
    s->cv_launch.notify_all();
  }
  if (s->planner.joinable()) s->planner.join();
  if (s->launcher.joinable()) s->launcher.join();
  for (auto& kv : s->all) {
    if (kv.second->plan) fmm_release(kv.second->plan);
    delete kv.second;
  }
  for (int i = 0; i < kBuffers; ++i) {
    if (s->buf[i].last) (void)hipEventDestroy(s->buf[i].last);
    (void)hipHostFree(s->buf[i].pinned);
    (void)hipFree(s->buf[i].dev);
    (void)hipStreamDestroy(s->buf[i].stream);
  }
  (void)hipStreamDestroy(s->plan_stream);
  delete s;
}

}  // extern "C"
