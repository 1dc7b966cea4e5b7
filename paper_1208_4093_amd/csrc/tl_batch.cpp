// Batched solves and the continuous-batching server.
//
// Both advance a set of independent solves together, a round of outer
// iterations at a time, on one stream: every live solve enqueues its next
// iterations, one device-to-host copy per solve reads the stop flags, and
// finished solves are retired (their result copied out and certified).  The
// server admits queued requests between rounds while the device state of the
// admitted requests fits the HBM budget, so requests that arrive while
// others run join the next round.
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

struct Job {
  tl_lattice* L = nullptr;
  const double* f = nullptr;
  double* u = nullptr;
  Opts o{};
  Work* w = nullptr;
  bool own_work = false;
  int k = 0;                 // next outer iteration to enqueue
  bool live = false;
  tl_status status = TL_OK;
  tl_info info{};
  uint64_t ticket = 0;
  Clock::time_point t_submit, t_done;
  bool finished = false;
  bool lock_lattice = true;  // false when the caller already holds the lattice lock
};

tl_status hip_status(hipError_t e) {
  return e == hipSuccess ? TL_OK : e == hipErrorOutOfMemory ? TL_E_NOMEM : TL_E_DEVICE;
}

tl_status start_job(Job* j, hipStream_t st) {
  hipError_t e = launch_init_state(j->L->g, j->L->mask, j->L->ufix, (const double2*)j->u,
                                   j->o.warm, j->w->u[0], j->w->u[1], j->w->d[0], j->w->d[1],
                                   j->o.mixed, j->w->a, j->w->flags, j->w->ctrl, st);
  if (e != hipSuccess) return hip_status(e);
  j->k = 0;
  j->live = true;
  return TL_OK;
}

// Retire a job whose device flag is set: copy out u and certify it.
void finish_job(Job* j, hipStream_t st) {
  const Ctrl c = *j->w->ctrl_host;
  j->live = false;
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
    j->info.status = (tl_status)c.status;
    j->info.iters = kf;
    j->info.rel_res_l1 = out3[0];
    j->info.rel_res_l2 = out3[1];
    j->info.energy = out3[2];
    j->info.coarse_iters = c.coarse_iters;
    j->status = cs != TL_OK ? cs : (tl_status)c.status;
  }
  j->info.status = j->status;
  j->finished = true;
  j->t_done = Clock::now();
}

// One round: enqueue up to `chunk` iterations of every live job, read the
// flags, retire the finished jobs.  Returns a HIP failure, if any.
tl_status run_round(std::vector<Job*>& live, int chunk, hipStream_t st) {
  for (Job* j : live) {
    for (int c = 0; c < chunk && j->k <= j->o.max_iters; ++c, ++j->k) {
      tl_status s = enqueue_iteration(j->L, j->w, j->o, j->f, j->k, st);
      if (s != TL_OK) return s;
    }
    hipError_t e = hipMemcpyAsync(j->w->ctrl_host, j->w->ctrl, sizeof(Ctrl),
                                  hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return hip_status(e);
  }
  hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_status(e);
  std::vector<Job*> keep;
  for (Job* j : live) {
    const Ctrl& c = *j->w->ctrl_host;
    if (c.done || c.err || j->k > j->o.max_iters) finish_job(j, st);
    else keep.push_back(j);
  }
  live.swap(keep);
  return TL_OK;
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
  std::vector<Job*> live;
  std::map<uint64_t, Job*> jobs;
  uint64_t next_ticket = 1;
  bool stopping = false;
  std::thread worker;
};

namespace {

size_t job_bytes(const Job* j) { return work_bytes(j->L->g, j->o.mixed, j->o.max_iters + 1); }

void server_loop(tl_server* S) {
  (void)hipSetDevice(S->device);
  for (;;) {
    std::vector<Job*> admitted;
    {
      std::unique_lock<std::mutex> lock(S->mu);
      S->cv.wait(lock, [&] { return S->stopping || !S->queue.empty() || !S->live.empty(); });
      if (S->stopping && S->queue.empty() && S->live.empty()) return;
      while (!S->queue.empty() && (int)S->live.size() + (int)admitted.size() < S->max_slots) {
        Job* j = S->queue.front();
        const size_t b = job_bytes(j);
        if (S->used + b > S->budget) break;
        S->queue.pop_front();
        S->used += b;
        admitted.push_back(j);
      }
    }
    for (Job* j : admitted) {
      j->w = new (std::nothrow) Work();
      tl_status s = j->w ? j->w->alloc(j->L->g, j->o.mixed, j->o.max_iters + 1) : TL_E_NOMEM;
      if (s == TL_OK) s = start_job(j, S->stream);
      if (s != TL_OK) {
        j->status = s;
        j->info.status = s;
        j->finished = true;
        j->t_done = Clock::now();
        std::lock_guard<std::mutex> lock(S->mu);
        if (j->w) { j->w->release(); delete j->w; j->w = nullptr; }
        S->used -= job_bytes(j);
        continue;
      }
      std::lock_guard<std::mutex> lock(S->mu);
      S->live.push_back(j);
    }
    std::vector<Job*> live;
    {
      std::lock_guard<std::mutex> lock(S->mu);
      live = S->live;
    }
    if (live.empty()) continue;
    tl_status s = run_round(live, 8, S->stream);
    std::lock_guard<std::mutex> lock(S->mu);
    std::vector<Job*> still;
    for (Job* j : S->live) {
      if (s != TL_OK && !j->finished) {
        j->status = s;
        j->info.status = s;
        j->finished = true;
        j->t_done = Clock::now();
        j->live = false;
      }
      if (j->finished) {
        if (j->w) {
          (void)hipStreamSynchronize(S->stream);
          j->w->release();
          delete j->w;
          j->w = nullptr;
        }
        S->used -= job_bytes(j);
      } else {
        still.push_back(j);
      }
    }
    S->live.swap(still);
  }
}

}  // namespace

extern "C" {

tl_status tl_solve_batch(int32_t n, tl_lattice* const* lats, const double* const* f_dev,
                         double* const* u_dev, const tl_opts* opts, tl_info* infos,
                         void* hip_stream) {
  if (n < 0 || (n > 0 && (!lats || !f_dev || !u_dev || !infos))) return TL_E_INVAL;
  for (int i = 0; i < n; ++i)
    if (!lats[i] || !f_dev[i] || !u_dev[i]) return TL_E_INVAL;
  Opts o;
  resolve_opts(opts, &o);
  o.trace = nullptr;
  hipStream_t st = (hipStream_t)hip_stream;
  std::vector<Job> jobs(n);
  std::vector<Job*> live;
  tl_status first = TL_OK;
  // a lattice that appears once uses its cached work space; repeats get their own
  std::map<tl_lattice*, int> seen;
  for (int i = 0; i < n; ++i) seen[lats[i]]++;
  std::vector<std::unique_lock<std::mutex>> locks;
  for (auto& kv : seen) locks.emplace_back(kv.first->mu);
  for (int i = 0; i < n; ++i) {
    Job& j = jobs[i];
    j.L = lats[i];
    j.f = f_dev[i];
    j.u = u_dev[i];
    j.o = o;
    j.lock_lattice = false;
    tl_status s = TL_OK;
    if (seen[j.L] == 1) {
      Work*& w = j.L->work[o.mixed ? 1 : 0];
      if (!w || w->hist_cap < o.max_iters + 1) {
        if (w) { w->release(); delete w; }
        w = new (std::nothrow) Work();
        s = w ? w->alloc(j.L->g, o.mixed, o.max_iters + 1) : TL_E_NOMEM;
        if (s != TL_OK && w) { w->release(); delete w; w = nullptr; }
      }
      j.w = w;
    } else {
      j.w = new (std::nothrow) Work();
      j.own_work = true;
      s = j.w ? j.w->alloc(j.L->g, o.mixed, o.max_iters + 1) : TL_E_NOMEM;
    }
    if (s == TL_OK) s = start_job(&j, st);
    if (s != TL_OK) {
      j.status = s;
      j.info.status = s;
      j.finished = true;
      if (first == TL_OK) first = s;
    } else {
      live.push_back(&j);
    }
  }
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  (void)hipEventRecord(e0, st);
  int chunk = 4;
  while (!live.empty()) {
    tl_status s = run_round(live, chunk, st);
    if (s != TL_OK) {
      for (Job* j : live) { j->status = s; j->info.status = s; j->finished = true; }
      live.clear();
      if (first == TL_OK) first = s;
    }
    chunk = std::min(chunk * 2, 64);
  }
  (void)hipEventRecord(e1, st);
  (void)hipEventSynchronize(e1);
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  for (int i = 0; i < n; ++i) {
    Job& j = jobs[i];
    j.info.ms = ms;
    infos[i] = j.info;
    if (j.status != TL_OK && first == TL_OK) first = j.status;
    if (j.own_work && j.w) { j.w->release(); delete j.w; }
  }
  return first;
}

tl_status tl_server_create(size_t hbm_budget_bytes, int32_t max_slots, tl_server** out) {
  if (!out || max_slots < 1 || hbm_budget_bytes == 0) return TL_E_INVAL;
  *out = nullptr;
  tl_server* S = new (std::nothrow) tl_server();
  if (!S) return TL_E_NOMEM;
  S->budget = hbm_budget_bytes;
  S->max_slots = max_slots;
  if (hipGetDevice(&S->device) != hipSuccess || hipStreamCreate(&S->stream) != hipSuccess) {
    delete S;
    return TL_E_DEVICE;
  }
  S->worker = std::thread(server_loop, S);
  *out = S;
  return TL_OK;
}

tl_status tl_submit(tl_server* S, tl_lattice* L, const double* f_dev, double* u_dev,
                    const tl_opts* opts, uint64_t* ticket) {
  if (!S || !L || !f_dev || !u_dev || !ticket) return TL_E_INVAL;
  Job* j = new (std::nothrow) Job();
  if (!j) return TL_E_NOMEM;
  j->L = L;
  j->f = f_dev;
  j->u = u_dev;
  resolve_opts(opts, &j->o);
  j->o.trace = nullptr;
  if (job_bytes(j) > S->budget) { delete j; return TL_E_BUDGET; }
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
