// Batched solves and the continuous-batching server, on fused launches.
//
// A FusedBatch advances several independent solves together.  One outer
// iteration of all of them is: one tile launch per set edge present (the
// tiles of every lattice with that edge), one boundary-block launch and one
// block-inverse launch over the sets of all lattices, and one persistent
// upper-level launch in which each lattice owns a range of workgroups and
// runs its own grid sums (the launch may exceed what fits the device at
// once: workgroups take their places in start order).  Every kernel reads its lattice's
// iteration counter and stop flag from device memory, so the launches of a
// chunk of iterations have fixed arguments: tl_solve_batch captures one
// chunk in a hipGraph and replays it.  Finished lattices' workgroups return
// at once.  After each chunk a small kernel gathers every lattice's control
// block into one array that is copied to the host in one transfer.
//
// The server keeps one FusedBatch of the admitted requests and rebuilds its
// tables whenever a request is admitted or retired, so requests that arrive
// while others run join at the next chunk boundary (continuous batching).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "tl.h"
#include "tl_internal.h"
#include "tl_runtime.h"

namespace tl {

namespace {

using Clock = std::chrono::steady_clock;

tl_status hip_status(hipError_t e) {
  return e == hipSuccess ? TL_OK : e == hipErrorOutOfMemory ? TL_E_NOMEM : TL_E_DEVICE;
}

#define TB_TRY(expr)                             \
  do {                                           \
    hipError_t e_ = (expr);                      \
    if (e_ != hipSuccess) return hip_status(e_); \
  } while (0)

struct Job {
  tl_lattice* L = nullptr;
  const double* f = nullptr;
  double* u = nullptr;
  Opts o{};
  Work* w = nullptr;
  bool own_work = true;
  tl_status status = TL_OK;
  tl_info info{};
  uint64_t ticket = 0;
  Clock::time_point t_submit, t_done;
  Clock::time_point t_seen;  // when the host first saw the solve stopped
  bool seen = false;
  bool finished = false;
  bool lock_lattice = true;  // false when the caller already holds the lattice lock
  hipEvent_t ready = nullptr;  // tl_submit: recorded on the caller's stream

  Job() = default;
  Job(const Job&) = delete;
  Job& operator=(const Job&) = delete;
  ~Job() {
    if (ready) (void)hipEventDestroy(ready);
  }
};

// Workgroup plan of a fused upper-level launch.  Each lattice gets the
// workgroup count of its single-lattice shape, which depends on the lattice
// alone, so its grid-sum order, and with it every rounding, is the same alone
// and in any batch.  The fused kernel hands out its workgroup indices in the
// order the workgroups start (see k_coarse_batch), so the launch may exceed
// the device's co-resident capacity when every lattice's own workgroups fit
// one XCD's share of it (not under TL_COARSE_BATCH_WG, for tool runs);
// otherwise all of the launch's workgroups must fit at once.  The plan picks an LDS size class (64 KB: two workgroups per CU
// beside the static arrays; else 152 KB: one) that every lattice's unstaged
// slice fits and at which one of those two conditions holds, and enables LDS
// staging per lattice where it still fits the class.  Returns false when no
// class qualifies.
constexpr int kXcdCount = 8;   // XCDs the workgroups of a launch are dealt over

bool plan_coarse(const std::vector<const Geo*>& gs, std::vector<int>* nw_out,
                 std::vector<CoarseShape>* shape_out, size_t* lds_out) {
  const int n = (int)gs.size();
  std::vector<CoarseShape> shape(n);
  std::vector<int> nw(n);
  int largest = 0;
  long used = 0;
  for (int b = 0; b < n; ++b) {
    shape[b] = coarse_shape(*gs[b]);
    nw[b] = shape[b].nwg;
    largest = std::max(largest, nw[b]);
    used += nw[b];
  }
  static const size_t classes[2] = {64 * 1024, COARSE_DYN_LDS_MAX};
  for (size_t cap : classes) {
    bool ok = true;
    for (int b = 0; b < n && ok; ++b) ok = coarse_lds_bytes(*gs[b], nw[b], 0, 0, shape[b].two_level) <= cap;
    const int fit = coarse_batch_capacity(cap);   // workgroups resident at once
    if (!ok || !(used <= fit || (coarse_batch_oversubscribe() && largest <= fit / kXcdCount))) continue;
    size_t lds = 0;
    for (int b = 0; b < n; ++b) {
      const int vec = shape[b].vec_lds && coarse_lds_bytes(*gs[b], nw[b], 1, 0, shape[b].two_level) <= cap;
      const int blk = vec && shape[b].blk_lds &&
                      coarse_lds_bytes(*gs[b], nw[b], 1, 1, shape[b].two_level) <= cap;
      shape[b].vec_lds = vec;
      shape[b].blk_lds = blk;
      lds = std::max(lds, coarse_lds_bytes(*gs[b], nw[b], vec, blk, shape[b].two_level));
    }
    *nw_out = nw;
    *shape_out = shape;
    *lds_out = lds;
    return true;
  }
  return false;
}

// True when every job's own upper-level workgroups can be resident at once.
bool coresident(const std::vector<Job*>& jobs) {
  std::vector<const Geo*> gs;
  for (Job* j : jobs) gs.push_back(&j->L->g);
  std::vector<int> nw;
  std::vector<CoarseShape> shape;
  size_t lds = 0;
  return plan_coarse(gs, &nw, &shape, &lds);
}

// Device tables of one fused batch.
struct FusedBatch {
  std::vector<Job*> jobs;
  std::vector<BatchEntry> h;
  BatchEntry* d_entries = nullptr;
  // tile launches: one per (set edge, overlap) present
  static constexpr int kEdges[3] = {16, 32, 64};
  static constexpr int kOverlaps[4] = {0, 1, 2, 4};
  static constexpr int kGroups = 12;
  int* d_tile_lat[kGroups] = {};
  int ntiles[kGroups] = {};
  bool any_band[kGroups] = {};   // a lattice of the group solves its regions exactly
  int* d_set_lat = nullptr;
  int nsets = 0;
  int* d_wg_lat = nullptr;
  int nwg = 0;
  int max_nwg = 0;              // the most upper-level workgroups of one lattice
  unsigned* d_ticket = nullptr; // workgroup ticket counter of the fused upper-level kernel
  size_t lds = 0;
  Ctrl* d_ctrl = nullptr;       // gathered control blocks
  Ctrl* h_ctrl = nullptr;       // pinned
  int cap = 0;                  // entries the ctrl buffers can hold
  bool mixed = false;

  void release_tables() {
    for (int k = 0; k < kGroups; ++k) {
      if (d_tile_lat[k]) (void)hipFree(d_tile_lat[k]);
      d_tile_lat[k] = nullptr;
    }
    for (void* p : {(void*)d_entries, (void*)d_set_lat, (void*)d_wg_lat, (void*)d_ticket})
      if (p) (void)hipFree(p);
    d_entries = nullptr;
    d_set_lat = d_wg_lat = nullptr;
    d_ticket = nullptr;
  }
  void release() {
    release_tables();
    if (d_ctrl) (void)hipFree(d_ctrl);
    if (h_ctrl) (void)hipHostFree(h_ctrl);
    d_ctrl = nullptr;
    h_ctrl = nullptr;
    cap = 0;
  }

  static int group_slot(int E, int ov) {
    return (E == 16 ? 0 : E == 32 ? 1 : 2) * 4 + (ov == 0 ? 0 : ov == 1 ? 1 : ov == 2 ? 2 : 3);
  }

  // Build the entry and lookup tables for the current jobs (all of whose
  // work spaces exist and were initialised).
  tl_status build(hipStream_t st) {
    release_tables();
    const int n = (int)jobs.size();
    if (n == 0) return TL_OK;
    mixed = jobs[0]->o.mixed;
    h.assign(n, BatchEntry{});
    for (bool& a : any_band) a = false;
    std::vector<int> tl[kGroups], sl;
    std::vector<const Geo*> gs(n);
    for (int b = 0; b < n; ++b) gs[b] = &jobs[b]->L->g;
    std::vector<int> nw;
    std::vector<CoarseShape> shape;
    if (!plan_coarse(gs, &nw, &shape, &lds)) return TL_E_BUDGET;
    std::vector<int> wl;
    nsets = 0;
    for (int b = 0; b < n; ++b) {
      Job* j = jobs[b];
      const Geo& g = j->L->g;
      BatchEntry& e = h[b];
      e.g = g;
      e.ea = j->L->ea;
      e.mask = j->L->mask;
      make_iteration_args(j->L, j->w, j->o, j->f, &e.ta, &e.oa, &e.ba, &e.ca);
      e.ca.nwg = nw[b];
      e.ca.vec_lds = shape[b].vec_lds;
      e.ca.blk_lds = shape[b].blk_lds;
      const int slot = group_slot(g.E, j->o.overlap);
      if (e.ta.band) any_band[slot] = true;
      e.tile0 = (int)tl[slot].size();
      for (int t = 0; t < g.M; ++t) tl[slot].push_back(b);
      e.set0 = nsets;
      for (int s = 0; s < g.M; ++s) sl.push_back(b);
      nsets += g.M;
      e.wg0 = (int)wl.size();
      e.nwg = nw[b];
      for (int w = 0; w < nw[b]; ++w) wl.push_back(b);
    }
    nwg = (int)wl.size();
    max_nwg = nw.empty() ? 0 : *std::max_element(nw.begin(), nw.end());
    auto up = [&](const void* src, size_t bytes, void** dst) -> hipError_t {
      hipError_t e = hipMalloc(dst, std::max<size_t>(bytes, 16));
      if (e == hipSuccess && bytes) e = hipMemcpyAsync(*dst, src, bytes, hipMemcpyHostToDevice, st);
      return e;
    };
    void* p;
    TB_TRY(up(h.data(), n * sizeof(BatchEntry), &p)); d_entries = (BatchEntry*)p;
    for (int k = 0; k < kGroups; ++k) {
      ntiles[k] = (int)tl[k].size();
      TB_TRY(up(tl[k].data(), tl[k].size() * sizeof(int), &p)); d_tile_lat[k] = (int*)p;
    }
    TB_TRY(up(sl.data(), sl.size() * sizeof(int), &p)); d_set_lat = (int*)p;
    TB_TRY(up(wl.data(), wl.size() * sizeof(int), &p)); d_wg_lat = (int*)p;
    TB_TRY(hipMalloc(&p, sizeof(unsigned))); d_ticket = (unsigned*)p;
    TB_TRY(hipMemsetAsync(d_ticket, 0, sizeof(unsigned), st));
    if (cap < n) {
      if (d_ctrl) (void)hipFree(d_ctrl);
      if (h_ctrl) (void)hipHostFree(h_ctrl);
      d_ctrl = nullptr;
      h_ctrl = nullptr;
      TB_TRY(hipMalloc((void**)&d_ctrl, n * sizeof(Ctrl)));
      TB_TRY(hipHostMalloc((void**)&h_ctrl, n * sizeof(Ctrl), hipHostMallocDefault));
      cap = n;
    }
    TB_TRY(hipStreamSynchronize(st));   // the host tables are reused by the next build
    return TL_OK;
  }

  // One outer iteration of every lattice in the batch.  ev (optional, kEvents
  // entries): recorded before the first launch, after each tile group, after
  // the boundary-block and block-inverse launches and after the upper level.
  static constexpr int kEvents = kGroups + 3;
  tl_status enqueue_iteration(hipStream_t st, hipEvent_t* ev = nullptr) const {
    if (ev) TB_TRY(hipEventRecord(ev[0], st));
    for (int k = 0; k < kGroups; ++k) {
      TB_TRY(launch_tile_batch(mixed, kEdges[k / 4], kOverlaps[k % 4], d_entries, d_tile_lat[k],
                               ntiles[k], any_band[k], st));
      if (ev) TB_TRY(hipEventRecord(ev[1 + k], st));
    }
    TB_TRY(launch_offdiag_batch(mixed, d_entries, d_set_lat, nsets, st));
    TB_TRY(launch_blockinv_batch(d_entries, d_set_lat, nsets, st));
    if (ev) TB_TRY(hipEventRecord(ev[kGroups + 1], st));
    TB_TRY(launch_coarse_batch(d_entries, d_wg_lat, d_ticket, nwg, max_nwg, lds, st));
    if (ev) TB_TRY(hipEventRecord(ev[kGroups + 2], st));
    return TL_OK;
  }

  tl_status read_ctrl(hipStream_t st) {
    const int n = (int)jobs.size();
    TB_TRY(launch_gather_ctrl(d_entries, n, d_ctrl, st));
    TB_TRY(hipMemcpyAsync(h_ctrl, d_ctrl, n * sizeof(Ctrl), hipMemcpyDeviceToHost, st));
    TB_TRY(hipStreamSynchronize(st));
    return TL_OK;
  }
};

tl_status alloc_and_start(Job* j, hipStream_t st) {
  if (tl_status s = ensure_band(j->L, j->o, st); s != TL_OK) return s;
  if (!j->w) {
    j->w = new (std::nothrow) Work();
    if (!j->w) return TL_E_NOMEM;
    j->own_work = true;
    tl_status s = j->w->alloc(j->L->g, j->o.mixed, j->o.max_iters + 1);
    if (s != TL_OK) return s;
  }
  tl_status s = hip_status(launch_init_state(j->L->g, j->L->mask, j->L->ufix, (const double2*)j->u,
                                             j->o.warm, j->w->u[0], j->w->u[1], j->w->d[0],
                                             j->w->d[1], j->o.mixed, j->w->a, j->w->flags,
                                             j->w->ctrl, st));
  if (s == TL_OK) s = ensure_coarse_space(j->L, j->w, j->o, j->f, st);
  return s;
}

// Retire a job whose control block says it stopped: copy out u and certify.
void finish_job(Job* j, const Ctrl& c, hipStream_t st) {
  if (c.err) {
    j->status = TL_E_DEVICE;
  } else {
    const int kf = c.iters;
    hipError_t e = launch_copy_out(j->L->g, j->w->u[(kf + 1) & 1], (double2*)j->u, st);
    double out3[3] = {0, 0, 0};
    tl_status cs = e == hipSuccess ? TL_OK : hip_status(e);
    if (cs == TL_OK) {
      if (j->lock_lattice) {
        std::lock_guard<std::mutex> lock(j->L->mu);
        cs = certify(j->L, j->f, j->u, nullptr, out3, st);
      } else {
        cs = certify(j->L, j->f, j->u, nullptr, out3, st);
      }
    }
    j->info.iters = kf;
    j->info.rel_res_l1 = out3[0];
    j->info.rel_res_l2 = out3[1];
    j->info.energy = out3[2];
    j->info.coarse_iters = c.coarse_iters;
    j->status = cs != TL_OK ? cs : (tl_status)c.status;
  }
  j->info.status = j->status;
  j->t_done = Clock::now();
}

void drop_work(Job* j) {
  if (j->w && j->own_work) {
    j->w->release();
    delete j->w;
  }
  j->w = nullptr;
}

// Kernel times of a profiled tl_solve_batch call.
struct BatchProfile {
  double tile_ms[3] = {0.0, 0.0, 0.0};   // by set edge 16, 32, 64
  int tile_launches[3] = {0, 0, 0};
  double offdiag_ms = 0.0, coarse_ms = 0.0;
};

int edge_slot(int E) { return E == 16 ? 0 : E == 32 ? 1 : 2; }

// Run one group of a tl_solve_batch call to completion: start
// every solve, build the fused tables, capture one chunk of iterations in a
// hipGraph and replay it until every lattice of the group has stopped, then
// copy out and certify each result (marking its job finished).  With a
// profile, iterations are enqueued one at a time with timing events and the
// control blocks read after each.
tl_status run_group(std::vector<Job*>& group, const std::map<tl_lattice*, int>& seen,
                    const Opts& o, hipStream_t st, BatchProfile* prof) {
  tl_status first = TL_OK;
  FusedBatch fb;
  for (Job* j : group) {
    if (seen.at(j->L) == 1) {   // a lattice that appears once uses its cached work space
      tl_status err = TL_OK;
      j->w = lattice_work(j->L, o.mixed, o.max_iters + 1, &err);
      j->own_work = false;
      if (!j->w) { first = err; break; }
    }
    first = alloc_and_start(j, st);
    if (first != TL_OK) break;
    fb.jobs.push_back(j);
  }
  if (first == TL_OK) first = fb.build(st);
  std::vector<hipEvent_t> ev;
  if (first == TL_OK && prof) {
    ev.resize(FusedBatch::kEvents, nullptr);
    for (hipEvent_t& e : ev)
      if (hipEventCreate(&e) != hipSuccess) { first = TL_E_DEVICE; break; }
  }
  if (first == TL_OK) {
    const int chunk = prof ? 1 : 8;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool use_graph = !prof && hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (use_graph) {
      tl_status s = TL_OK;
      for (int c = 0; c < chunk && s == TL_OK; ++c) s = fb.enqueue_iteration(st);
      const bool ended = hipStreamEndCapture(st, &graph) == hipSuccess;
      use_graph = s == TL_OK && ended &&
                  hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
      if (!use_graph) (void)hipGetLastError();
    }
    int rounds = 0;
    const int max_rounds = o.max_iters / chunk + 2;
    const int n = (int)group.size();
    std::vector<char> live(n, 1);
    for (;;) {
      tl_status s = TL_OK;
      {
        PersistentGuard guard(fb.nwg, st);
        if (use_graph) {
          s = hipGraphLaunch(exec, st) == hipSuccess ? TL_OK : TL_E_DEVICE;
        } else {
          for (int c = 0; c < chunk && s == TL_OK; ++c) s = fb.enqueue_iteration(st, prof ? ev.data() : nullptr);
        }
        if (s == TL_OK) s = fb.read_ctrl(st);
      }
      if (s != TL_OK) { first = s; break; }
      if (prof) {
        // the iteration just run: its tile groups with a lattice still iterating
        bool edge_live[3] = {false, false, false};
        for (int b = 0; b < n; ++b)
          if (live[b]) edge_live[edge_slot(group[b]->L->g.E)] = true;
        float ms[FusedBatch::kEvents] = {};
        for (int k = 1; k < FusedBatch::kEvents && s == TL_OK; ++k)
          if (hipEventElapsedTime(&ms[k], ev[k - 1], ev[k]) != hipSuccess) s = TL_E_DEVICE;
        if (s != TL_OK) { first = s; break; }
        bool launched[3] = {false, false, false};
        for (int k = 0; k < FusedBatch::kGroups; ++k) {
          const int slot = k / 4;
          if (!edge_live[slot] || fb.ntiles[k] == 0) continue;
          prof->tile_ms[slot] += ms[1 + k];
          launched[slot] = true;
        }
        for (int e = 0; e < 3; ++e) prof->tile_launches[e] += launched[e];
        prof->offdiag_ms += ms[FusedBatch::kGroups + 1];
        prof->coarse_ms += ms[FusedBatch::kGroups + 2];
      }
      const auto now = Clock::now();
      bool all = true;
      for (int b = 0; b < n; ++b) {
        const bool stopped = fb.h_ctrl[b].done || fb.h_ctrl[b].err;
        if (stopped && !group[b]->seen) {
          group[b]->seen = true;
          group[b]->t_seen = now;
        }
        live[b] = !stopped;
        all = all && stopped;
      }
      if (all) break;
      if (++rounds > max_rounds) { first = TL_E_DEVICE; break; }
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (first == TL_OK) {
      for (int b = 0; b < n; ++b) {
        finish_job(group[b], fb.h_ctrl[b], st);
        group[b]->finished = true;
      }
    }
  }
  for (hipEvent_t e : ev)
    if (e) (void)hipEventDestroy(e);
  fb.release();
  return first;
}

}  // namespace

}  // namespace tl

using namespace tl;

struct tl_server {
  size_t budget = 0;
  int max_slots = 1;
  size_t used = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Job*> queue;
  std::map<uint64_t, Job*> jobs;
  uint64_t next_ticket = 1;
  bool stopping = false;
  std::thread worker;
};

namespace {

size_t job_bytes(const Job* j) { return work_bytes(j->L->g, j->o.mixed, j->o.max_iters + 1); }

// Requests are grouped by precision: one fused batch per precision.
void server_loop(tl_server* S) {
  (void)hipSetDevice(S->device);
  FusedBatch fb[2];
  std::vector<Job*> live[2];
  bool dirty[2] = {false, false};
  const int chunk = 8;
  for (;;) {
    std::vector<Job*> admitted;
    {
      std::unique_lock<std::mutex> lock(S->mu);
      S->cv.wait(lock, [&] {
        return S->stopping || !S->queue.empty() || !live[0].empty() || !live[1].empty();
      });
      if (S->stopping && S->queue.empty() && live[0].empty() && live[1].empty()) break;
      while (!S->queue.empty() &&
             (int)(live[0].size() + live[1].size() + admitted.size()) < S->max_slots) {
        Job* j = S->queue.front();
        const size_t b = job_bytes(j);
        if (S->used + b > S->budget) break;
        // every lattice of the fused batch of the job's precision must keep
        // its own upper-level workgroups resident at once
        std::vector<Job*> group;
        for (Job* k : live[j->o.mixed ? 1 : 0]) group.push_back(k);
        for (Job* k : admitted)
          if (k->o.mixed == j->o.mixed) group.push_back(k);
        group.push_back(j);
        if (group.size() > 1 && !coresident(group)) break;
        S->queue.pop_front();
        S->used += b;
        admitted.push_back(j);
      }
    }
    for (Job* j : admitted) {
      // the request's load may still be in production on the caller's stream
      tl_status s = j->ready && hipStreamWaitEvent(S->stream, j->ready, 0) != hipSuccess
                        ? TL_E_DEVICE : TL_OK;
      if (s == TL_OK) s = alloc_and_start(j, S->stream);
      if (s != TL_OK) {
        drop_work(j);
        std::lock_guard<std::mutex> lock(S->mu);
        j->status = s;
        j->info.status = s;
        j->t_done = Clock::now();
        j->finished = true;
        S->used -= job_bytes(j);
        continue;
      }
      const int m = j->o.mixed ? 1 : 0;
      live[m].push_back(j);
      dirty[m] = true;
    }
    for (int m = 0; m < 2; ++m) {
      if (live[m].empty()) continue;
      tl_status s = TL_OK;
      if (dirty[m]) {
        fb[m].jobs = live[m];
        s = fb[m].build(S->stream);
        dirty[m] = false;
      }
      if (s == TL_OK) {
        PersistentGuard guard(fb[m].nwg, S->stream);
        for (int c = 0; c < chunk && s == TL_OK; ++c) s = fb[m].enqueue_iteration(S->stream);
        if (s == TL_OK) s = fb[m].read_ctrl(S->stream);
      }
      std::vector<Job*> still;
      for (size_t b = 0; b < live[m].size(); ++b) {
        Job* j = live[m][b];
        if (s != TL_OK) {
          j->status = s;
          j->info.status = s;
          j->t_done = Clock::now();
        } else if (fb[m].h_ctrl[b].done || fb[m].h_ctrl[b].err) {
          finish_job(j, fb[m].h_ctrl[b], S->stream);
        } else {
          still.push_back(j);
          continue;
        }
        (void)hipStreamSynchronize(S->stream);
        drop_work(j);
        std::lock_guard<std::mutex> lock(S->mu);
        j->finished = true;      // published under the lock that tl_poll takes
        S->used -= job_bytes(j);
        dirty[m] = true;
      }
      live[m].swap(still);
    }
  }
  fb[0].release();
  fb[1].release();
}

}  // namespace

extern "C" {

tl_status tl_solve_batch(int32_t n, tl_lattice* const* lats, const double* const* f_dev,
                         double* const* u_dev, const tl_opts* opts, tl_info* infos,
                         void* hip_stream) {
  if (n < 0 || (n > 0 && (!lats || !f_dev || !u_dev || !infos))) return TL_E_INVAL;
  for (int i = 0; i < n; ++i)
    if (!lats[i] || !f_dev[i] || !u_dev[i]) return TL_E_INVAL;
  if (n == 0) return TL_OK;
  Opts o;
  if (resolve_opts(opts, &o) != TL_OK) return TL_E_INVAL;
  o.trace = nullptr;
  BatchProfile prof;
  BatchProfile* pp = o.profile ? &prof : nullptr;
  o.profile = 0;
  hipStream_t user = (hipStream_t)hip_stream;
  const auto t_call = Clock::now();
  std::vector<Job> jobs(n);
  std::map<tl_lattice*, int> seen;
  for (int i = 0; i < n; ++i) seen[lats[i]]++;
  std::vector<std::unique_lock<std::mutex>> locks;
  for (auto& kv : seen) locks.emplace_back(kv.first->mu);
  // a private stream, so that the chunk can be captured even when the
  // caller passes the null stream; ordered after the caller's prior work
  hipStream_t st;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return TL_E_DEVICE;
  hipEvent_t ev_in, ev_out, e0, e1;
  (void)hipEventCreate(&ev_in);
  (void)hipEventCreate(&ev_out);
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  (void)hipEventRecord(ev_in, user);
  (void)hipStreamWaitEvent(st, ev_in, 0);
  (void)hipEventRecord(e0, st);
  // Lattices are taken in order into groups (one, unless adding a lattice
  // moves the group to an LDS class at which some lattice's upper-level
  // workgroups no longer fit at once); the groups run one after another.
  tl_status first = TL_OK;
  std::vector<Job*> pending;
  for (int i = 0; i < n; ++i) {
    Job& j = jobs[i];
    j.L = lats[i];
    j.f = f_dev[i];
    j.u = u_dev[i];
    j.o = o;
    apply_tuned(j.L, &j.o);
    j.lock_lattice = false;
    pending.push_back(&j);
  }
  size_t next = 0;
  while (next < pending.size() && first == TL_OK) {
    std::vector<Job*> group;
    while (next < pending.size()) {
      group.push_back(pending[next]);
      if (group.size() > 1 && !coresident(group)) { group.pop_back(); break; }
      ++next;
    }
    if (group.empty()) { first = TL_E_BUDGET; break; }   // one lattice that never fits
    first = run_group(group, seen, o, st, pp);
  }
  (void)hipEventRecord(e1, st);
  (void)hipEventSynchronize(e1);
  const auto t_end = Clock::now();
  for (int i = 0; i < n; ++i) {
    Job& j = jobs[i];
    if (!j.finished) j.status = first != TL_OK ? first : TL_E_DEVICE;
    j.info.status = j.status;
    j.info.ms = std::chrono::duration<double, std::milli>((j.seen ? j.t_seen : t_end) - t_call).count();
    if (pp) {
      const int e = edge_slot(j.L->g.E);
      j.info.tile_ms = prof.tile_ms[e];
      j.info.tile_launches = prof.tile_launches[e];
      j.info.offdiag_ms = prof.offdiag_ms;
      j.info.coarse_ms = prof.coarse_ms;
    }
    infos[i] = j.info;
    if (j.status != TL_OK && first == TL_OK) first = j.status;
    drop_work(&j);
  }
  (void)hipEventRecord(ev_out, st);
  (void)hipStreamWaitEvent(user, ev_out, 0);
  (void)hipStreamSynchronize(st);
  (void)hipStreamDestroy(st);
  for (hipEvent_t e : {ev_in, ev_out, e0, e1}) (void)hipEventDestroy(e);
  return first;
}

tl_status tl_server_create(size_t hbm_budget_bytes, int32_t max_slots, tl_server** out) {
  if (!out || max_slots < 1 || hbm_budget_bytes == 0) return TL_E_INVAL;
  *out = nullptr;
  tl_server* S = new (std::nothrow) tl_server();
  if (!S) return TL_E_NOMEM;
  S->budget = hbm_budget_bytes;
  S->max_slots = max_slots;
  if (hipGetDevice(&S->device) != hipSuccess ||
      hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess) {
    delete S;
    return TL_E_DEVICE;
  }
  S->worker = std::thread(server_loop, S);
  *out = S;
  return TL_OK;
}

tl_status tl_submit(tl_server* S, tl_lattice* L, const double* f_dev, double* u_dev,
                    const tl_opts* opts, void* hip_stream, uint64_t* ticket) {
  if (!S || !L || !f_dev || !u_dev || !ticket) return TL_E_INVAL;
  Job* j = new (std::nothrow) Job();
  if (!j) return TL_E_NOMEM;
  j->L = L;
  j->f = f_dev;
  j->u = u_dev;
  if (resolve_opts(opts, &j->o) != TL_OK) { delete j; return TL_E_INVAL; }
  apply_tuned(L, &j->o);
  j->o.trace = nullptr;
  j->o.profile = 0;
  if (job_bytes(j) > S->budget || !coresident({j})) { delete j; return TL_E_BUDGET; }
  // order the request after the caller's work on its stream (the load may be
  // produced there); the worker's stream waits on this event
  if (hipEventCreateWithFlags(&j->ready, hipEventDisableTiming) != hipSuccess) {
    j->ready = nullptr;
    delete j;
    return TL_E_DEVICE;
  }
  if (hipEventRecord(j->ready, (hipStream_t)hip_stream) != hipSuccess) { delete j; return TL_E_DEVICE; }
  j->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> lock(S->mu);
    j->ticket = S->next_ticket++;
    S->jobs[j->ticket] = j;
    S->queue.push_back(j);
  }
  S->cv.notify_one();
  *ticket = j->ticket;
  return TL_OK;
}

tl_status tl_poll(tl_server* S, uint64_t ticket, tl_info* out) {
  if (!S) return TL_E_INVAL;
  std::lock_guard<std::mutex> lock(S->mu);
  auto it = S->jobs.find(ticket);
  if (it == S->jobs.end()) return TL_E_INVAL;
  Job* j = it->second;
  if (!j->finished) return TL_PENDING;
  j->info.ms = std::chrono::duration<double, std::milli>(j->t_done - j->t_submit).count();
  if (out) *out = j->info;
  const tl_status s = j->status;
  S->jobs.erase(it);
  delete j;
  return s;
}

void tl_server_destroy(tl_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lock(S->mu);
    S->stopping = true;
  }
  S->cv.notify_all();
  if (S->worker.joinable()) S->worker.join();
  (void)hipStreamSynchronize(S->stream);
  (void)hipStreamDestroy(S->stream);
  for (auto& kv : S->jobs) delete kv.second;
  delete S;
}

}  // extern "C"
