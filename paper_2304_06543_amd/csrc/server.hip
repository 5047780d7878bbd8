// server.hip -- LBDD request server with continuous batching on one GPU.
//
// Clients submit instances at any time.  A host thread admits them in arrival
// order as HBM budget and job slots allow (AdmissionQueue), builds each
// admitted instance on the device (copy of CM, setup step of Algorithm 2) on
// its own stream while the resident service kernel keeps solving earlier
// jobs, then publishes the job.  Service workers (one workgroup each) pick up
// published jobs as they free up, so requests that arrive while others are
// running overlap with them on the device.  Completion is seen by polling
// flags in pinned host memory; results are copied out and the device memory
// is returned to the budget.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/lbdd.h"
#include "instance.hpp"
#include "lbdd_dev.hpp"
#include "sched.hpp"

namespace {


double wall() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

constexpr int64_t IDLE_TICKS = 20'000'000;   // workers leave after ~0.2 s idle (100 MHz timer)

struct Job {
  uint64_t id = 0;
  int32_t k = 0;
  int64_t n = 0;
  const int32_t *cm = nullptr;                 // borrowed until the job is done
  std::vector<int32_t> cap, pen;
  size_t footprint = 0;
  int state = LBDD_JOB_QUEUED;                 // or an LBDD_E_* code
  int64_t seq = -1;                            // publication number
  lbdd_instance *inst = nullptr;
  int64_t objective = 0;
  std::vector<int32_t> assign;
  double t_submit = 0, t_admit = 0, t_done = 0;
  double t_dev0 = 0, t_dev1 = 0;               // device clock: first and last iteration
};

}  // namespace

struct lbdd_server {
  size_t budget = 0;
  int32_t ring_size = 0;
  int workers = 0;
  double t0 = 0;
  hipStream_t run_st = nullptr, adm_st = nullptr;
  lbdd::ServiceCtl *ctl = nullptr;   // pinned (host view)
  lbdd::ServiceJob *ring = nullptr;  // pinned
  int64_t *done = nullptr;           // pinned [ring_size]
  lbdd::ServiceCtl *ctl_d = nullptr; // the same three, device view
  lbdd::ServiceJob *ring_d = nullptr;
  int64_t *done_d = nullptr;
  lbdd::ServiceDev *dev = nullptr;   // device: claim counter and control mirrors
  hipEvent_t kernel_end = nullptr;
  bool kernel_launched = false;

  std::mutex mu;
  std::condition_variable cv;
  std::thread th;
  bool stop = false;
  lbdd::AdmissionQueue queue;
  std::map<uint64_t, Job> jobs;
  std::vector<uint64_t> running;     // ids of published, not yet finished jobs
  std::vector<char> slot_busy;
  uint64_t next_id = 1;
  int64_t published = 0;
  size_t in_use = 0;
  int64_t stats[10] = {0};           // submitted, admitted, finished, failed, launches, peak jobs,
                                     // peak bytes, (unused), cancelled, timed out
  double queue_timeout = 0;          // seconds a job may wait for admission (0: no limit)

  int ensure_kernel() {
    if (kernel_launched && hipEventQuery(kernel_end) == hipErrorNotReady) return LBDD_OK;
    hipError_t e = lbdd::launch_service(ctl_d, ring_d, ring_size, done_d, dev, IDLE_TICKS, workers, run_st);
    if (e == hipSuccess) e = hipEventRecord(kernel_end, run_st);
    if (e != hipSuccess) return lbdd::fail(LBDD_E_DEVICE, "service kernel launch: %s", hipGetErrorString(e));
    kernel_launched = true;
    stats[4] += 1;
    return LBDD_OK;
  }

  void loop();
};

void lbdd_server::loop() {
  std::unique_lock<std::mutex> lk(mu);
  while (true) {
    // 0. jobs that waited longer than the queue timeout leave the queue
    if (queue_timeout > 0 && !queue.empty()) {
      const double now = wall() - t0;
      const size_t m = queue.erase_if(
          [&](uint64_t id) { return now - jobs[id].t_submit > queue_timeout; },
          [&](uint64_t id) { jobs[id].state = LBDD_E_TIMEOUT; jobs[id].cm = nullptr; });
      if (m) {
        stats[9] += (int64_t)m;
        cv.notify_all();
      }
    }
    // 1. admission
    for (;;) {
      const int64_t seq = published;
      const bool slot_free = !slot_busy[(size_t)(seq % ring_size)];
      uint64_t id;
      const size_t free_bytes = budget > in_use ? budget - in_use : 0;
      if (stop || !queue.next(free_bytes, (int)running.size(), slot_free, &id)) break;
      Job &j = jobs[id];
      lk.unlock();
      lbdd_instance *inst = nullptr;
      const int rc = lbdd_create(j.k, j.n, j.cm, j.cap.data(), j.pen.data(), 0, adm_st, &inst);
      lk.lock();
      if (rc != LBDD_OK) {
        j.state = rc;
        stats[3] += 1;
        cv.notify_all();
        continue;
      }
      j.inst = inst;
      j.seq = seq;
      j.t_admit = wall() - t0;
      j.state = LBDD_JOB_RUNNING;
      const int32_t slot = (int32_t)(seq % ring_size);
      slot_busy[slot] = 1;
      ring[slot].inst = inst->view();
      in_use += j.footprint;
      running.push_back(id);
      published = seq + 1;
      std::atomic_thread_fence(std::memory_order_seq_cst);
      __atomic_store_n(&ctl->published, published, __ATOMIC_RELEASE);
      stats[1] += 1;
      if ((int64_t)running.size() > stats[5]) stats[5] = (int64_t)running.size();
      if ((int64_t)in_use > stats[6]) stats[6] = (int64_t)in_use;
      if (ensure_kernel() != LBDD_OK) break;   // handled below
    }
    // 2. completions
    for (size_t i = 0; i < running.size();) {
      Job &j = jobs[running[i]];
      const int32_t slot = (int32_t)(j.seq % ring_size);
      if (__atomic_load_n(&done[slot], __ATOMIC_ACQUIRE) != j.seq + 1) { ++i; continue; }
      j.t_done = wall() - t0;
      lbdd_instance *inst = j.inst;
      lk.unlock();
      int64_t obj = 0;
      std::vector<int32_t> a((size_t)j.n);
      int rc = lbdd_objective(inst, &obj);
      if (rc == LBDD_OK) rc = lbdd_assignment(inst, a.data(), 0);
      // the counters of lbdd_stats, then the device timer's rate (kHz)
      constexpr int NST = lbdd::SC_NSTATS + 1;
      int64_t st[NST] = {0};
      if (rc == LBDD_OK && lbdd_stats(inst, st, NST) == NST && st[lbdd::SC_NSTATS] > 0) {
        const double hz = (double)st[lbdd::SC_NSTATS] * 1e3;
        j.t_dev0 = (double)st[lbdd::ST_T_FIRST] / hz;
        j.t_dev1 = (double)st[lbdd::ST_T_LAST] / hz;
      }
      lbdd_destroy(inst);
      lk.lock();
      j.inst = nullptr;
      j.objective = obj;
      j.assign.swap(a);
      j.state = rc == LBDD_OK ? LBDD_JOB_DONE : rc;
      stats[rc == LBDD_OK ? 2 : 3] += 1;
      slot_busy[slot] = 0;
      in_use -= j.footprint;
      running[i] = running.back();
      running.pop_back();
      cv.notify_all();
    }
    // 3. keep the workers alive while published work is unfinished (also
    //    while stopping: published jobs always run to completion)
    if (!running.empty() && ensure_kernel() != LBDD_OK) {
      for (uint64_t id : running) jobs[id].state = LBDD_E_DEVICE;   // cannot run them
      running.clear();
      stop = true;
      cv.notify_all();
    }
    if (stop && running.empty()) break;
    if (running.empty() && queue.empty()) {
      cv.wait(lk, [&] { return stop || !queue.empty(); });
    } else {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(50));
      lk.lock();
    }
  }
}

extern "C" {

int lbdd_server_create(size_t hbm_budget, int32_t max_jobs, int32_t reserve_cus, lbdd_server **out) {
  lbdd::g_err.clear();
  if (!out) return lbdd::fail(LBDD_E_INVAL, "out is NULL");
  *out = nullptr;
  if (hbm_budget == 0 || max_jobs < 1 || reserve_cus < 0)
    return lbdd::fail(LBDD_E_INVAL, "budget must be > 0, max_jobs >= 1, reserve_cus >= 0");
  lbdd_server *s = new (std::nothrow) lbdd_server;
  if (!s) return lbdd::fail(LBDD_E_NOMEM, "host allocation");
  s->budget = hbm_budget;
  s->ring_size = max_jobs;
  const int cus = lbdd::device_cus();
  s->workers = cus - reserve_cus > 0 ? cus - reserve_cus : 1;
  s->t0 = wall();
  s->slot_busy.assign((size_t)max_jobs, 0);
  hipError_t e = hipStreamCreateWithFlags(&s->run_st, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->adm_st, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&s->kernel_end, hipEventDisableTiming);
  // fine-grained, coherent pinned memory: host stores are seen by polling
  // workers and the workers' system-scope stores by the host
  const unsigned hf = hipHostMallocMapped | hipHostMallocCoherent;
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&s->ctl), sizeof(lbdd::ServiceCtl), hf);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&s->ring), sizeof(lbdd::ServiceJob) * (size_t)max_jobs, hf);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&s->done), sizeof(int64_t) * (size_t)max_jobs, hf);
  if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void **>(&s->ctl_d), s->ctl, 0);
  if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void **>(&s->ring_d), s->ring, 0);
  if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void **>(&s->done_d), s->done, 0);
  if (e == hipSuccess) e = hipMallocAsync(reinterpret_cast<void **>(&s->dev), sizeof(lbdd::ServiceDev), s->adm_st);
  const lbdd::ServiceDev zero{};
  if (e == hipSuccess) e = hipMemcpyAsync(s->dev, &zero, sizeof zero, hipMemcpyHostToDevice, s->adm_st);
  if (e == hipSuccess) e = hipStreamSynchronize(s->adm_st);
  if (e != hipSuccess) {
    lbdd_server_destroy(s);
    return lbdd::fail(e == hipErrorOutOfMemory ? LBDD_E_NOMEM : LBDD_E_DEVICE, "server setup: %s", hipGetErrorString(e));
  }
  memset(s->ctl, 0, sizeof(lbdd::ServiceCtl));
  memset(s->ring, 0, sizeof(lbdd::ServiceJob) * (size_t)max_jobs);
  for (int32_t i = 0; i < max_jobs; ++i) s->done[i] = 0;
  std::atomic_thread_fence(std::memory_order_seq_cst);
  s->th = std::thread([s] { s->loop(); });
  *out = s;
  return LBDD_OK;
}

int lbdd_server_submit(lbdd_server *s, int32_t k, int64_t n, const int32_t *cm, const int32_t *capacity,
                       const int32_t *penalty, uint64_t *ticket) {
  lbdd::g_err.clear();
  if (!s || !cm || !capacity || !penalty || !ticket) return lbdd::fail(LBDD_E_INVAL, "NULL argument");
  if (k < 1 || k > LBDD_MAX_K || n < 1 || n > LBDD_MAX_N) return lbdd::fail(LBDD_E_INVAL, "k or n out of range");
  Job j;
  j.k = k;
  j.n = n;
  j.cm = cm;
  j.cap.assign(capacity, capacity + k);
  j.pen.assign(penalty, penalty + k);
  j.footprint = lbdd::instance_footprint(k, n);
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return lbdd::fail(LBDD_E_STATE, "server is shutting down");
  j.id = s->next_id++;
  j.t_submit = wall() - s->t0;
  *ticket = j.id;
  s->queue.push(j.id, j.footprint);
  s->jobs.emplace(j.id, std::move(j));
  s->stats[0] += 1;
  s->cv.notify_all();
  return LBDD_OK;
}

int lbdd_server_poll(lbdd_server *s, uint64_t ticket, int32_t *state, int64_t *objective) {
  if (!s || !state) return lbdd::fail(LBDD_E_INVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return lbdd::fail(LBDD_E_INVAL, "unknown ticket %llu", (unsigned long long)ticket);
  *state = it->second.state;
  if (objective && it->second.state == LBDD_JOB_DONE) *objective = it->second.objective;
  return LBDD_OK;
}

int lbdd_server_wait(lbdd_server *s, uint64_t ticket, int64_t *objective) {
  if (!s) return lbdd::fail(LBDD_E_INVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return lbdd::fail(LBDD_E_INVAL, "unknown ticket %llu", (unsigned long long)ticket);
  s->cv.wait(lk, [&] { return it->second.state != LBDD_JOB_QUEUED && it->second.state != LBDD_JOB_RUNNING; });
  if (it->second.state != LBDD_JOB_DONE) return lbdd::fail(it->second.state, "job %llu failed", (unsigned long long)ticket);
  if (objective) *objective = it->second.objective;
  return LBDD_OK;
}

int lbdd_server_result(lbdd_server *s, uint64_t ticket, int32_t *assign, double *times) {
  if (!s) return lbdd::fail(LBDD_E_INVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return lbdd::fail(LBDD_E_INVAL, "unknown ticket %llu", (unsigned long long)ticket);
  Job &j = it->second;
  if (j.state == LBDD_JOB_QUEUED || j.state == LBDD_JOB_RUNNING) return lbdd::fail(LBDD_E_STATE, "job not finished");
  const int st = j.state;
  if (st == LBDD_JOB_DONE && assign) memcpy(assign, j.assign.data(), sizeof(int32_t) * (size_t)j.n);
  if (times) {
    times[0] = j.t_submit; times[1] = j.t_admit; times[2] = j.t_done;
    times[3] = j.t_dev0; times[4] = j.t_dev1;
  }
  s->jobs.erase(it);
  return st == LBDD_JOB_DONE ? LBDD_OK : lbdd::fail(st, "job failed");
}

int lbdd_server_cancel(lbdd_server *s, uint64_t ticket) {
  if (!s) return lbdd::fail(LBDD_E_INVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return lbdd::fail(LBDD_E_INVAL, "unknown ticket %llu", (unsigned long long)ticket);
  if (it->second.state != LBDD_JOB_QUEUED || !s->queue.erase(ticket))
    return lbdd::fail(LBDD_E_STATE, "job %llu is not waiting", (unsigned long long)ticket);
  it->second.state = LBDD_E_CANCELLED;
  it->second.cm = nullptr;
  s->stats[8] += 1;
  s->cv.notify_all();
  return LBDD_OK;
}

int lbdd_server_set_queue_timeout(lbdd_server *s, double seconds) {
  if (!s) return lbdd::fail(LBDD_E_INVAL, "NULL argument");
  if (!(seconds >= 0) || seconds > 1e9) return lbdd::fail(LBDD_E_INVAL, "timeout must be finite and >= 0");
  std::lock_guard<std::mutex> lk(s->mu);
  s->queue_timeout = seconds;
  s->cv.notify_all();
  return LBDD_OK;
}

int lbdd_server_stats(lbdd_server *s, int64_t *out, int32_t count) {
  if (!s || count < 0 || (count > 0 && !out)) return lbdd::fail(LBDD_E_INVAL, "bad argument");
  std::lock_guard<std::mutex> lk(s->mu);
  int64_t all[11] = {s->stats[0], s->stats[1], s->stats[2], s->stats[3], s->stats[4], s->stats[5],
                     s->stats[6], (int64_t)s->in_use, (int64_t)s->workers, s->stats[8], s->stats[9]};
  const int m = count < 11 ? count : 11;
  for (int i = 0; i < m; ++i) out[i] = all[i];
  return m;
}

void lbdd_server_destroy(lbdd_server *s) {
  if (!s) return;
  if (s->th.joinable()) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stop = true;                    // waiting jobs are dropped, running ones finish
      while (!s->queue.empty()) {
        uint64_t id;
        if (!s->queue.next((size_t)-1, 1, true, &id)) break;
        s->jobs[id].state = LBDD_E_STATE;
      }
      s->cv.notify_all();
    }
    s->th.join();
  }
  if (s->ctl) __atomic_store_n(&s->ctl->shutdown, 1, __ATOMIC_RELEASE);
  if (s->run_st) (void)hipStreamSynchronize(s->run_st);
  if (s->dev) (void)hipFreeAsync(s->dev, s->adm_st);
  if (s->adm_st) (void)hipStreamSynchronize(s->adm_st);
  if (s->ctl) (void)hipHostFree(s->ctl);
  if (s->ring) (void)hipHostFree(s->ring);
  if (s->done) (void)hipHostFree(s->done);
  if (s->kernel_end) (void)hipEventDestroy(s->kernel_end);
  if (s->run_st) (void)hipStreamDestroy(s->run_st);
  if (s->adm_st) (void)hipStreamDestroy(s->adm_st);
  delete s;
}

}  // extern "C"
