// Serving loop: NNCP jobs of uneven order, shape, rank and storage type arrive
// at any time. Two native threads share the GPU:
//  * the loader admits queued jobs in arrival order while fewer than
//    max_active are admitted and their device footprint fits the HBM budget
//    next to the others; it allocates the job's buffers (stream-ordered, so no
//    device-wide synchronisation), uploads the tensor and starting factors and
//    builds the job's plan (||X||^2, starting Grams) on its own stream, while
//    the running jobs keep computing;
//  * the worker advances every running job by one outer iteration per tick
//    through one batch, moves jobs whose upload has finished into the batch
//    between ticks, and retires finished jobs (results to host, buffers freed
//    on the loader's stream).
// This is continuous batching: jobs join and leave between ticks while others
// keep running, and the batch rewrites its device work lists in place rather
// than capturing its graph again. A job's arithmetic is that of its
// stand-alone plan, so its result does not depend on the mix. Not part of the
// paper, which runs one decomposition at a time; this is the serving layer
// around its method.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "nncp.h"
#include "nncp_internal.hpp"

namespace {

using Clock = std::chrono::steady_clock;

size_t elem_bytes(int dtype) { return dtype == NNCP_F32 ? 4 : 2; }

struct Job {
  uint64_t id = 0;
  // request
  const void* X = nullptr;  // caller's host tensor (valid until the job is done)
  int dtype = 0, N = 0, R = 0, update = 0, iters = 0, split = 0;
  int64_t dims[NNCP_MAX_MODES] = {};
  int64_t I = 0;
  std::vector<std::vector<float>> H0;  // copied at submit
  size_t footprint = 0;
  // device state while admitted
  void* Xd = nullptr;
  float* Hd[NNCP_MAX_MODES] = {};
  void* ws = nullptr;
  nncp_plan* plan = nullptr;
  int done_iters = 0;
  // timeline (seconds on the server clock) and outcome
  double t_submit = 0, t_admit = 0, t_start = 0, t_done = 0;
  int status = NNCP_EBUSY;  // EBUSY while queued/admitted, then OK or an error
  std::vector<std::vector<float>> H;  // results
  std::vector<double> lam, fit;
};

}  // namespace

struct nncp_server {
  size_t budget = 0;
  int max_active = 0;
  bool simulate = false;
  int device = 0;
  Clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_load, cv_work, cv_done;
  std::deque<uint64_t> queue;              // submitted, not yet admitted
  std::map<uint64_t, std::unique_ptr<Job>> jobs;
  std::vector<Job*> ready;                 // uploaded, waiting to join the batch
  std::vector<Job*> active;                // in the batch
  int admitted = 0;                        // loading + ready + active
  uint64_t next_id = 1;
  size_t used = 0, peak_used = 0;
  int64_t ticks = 0, completed = 0, rejected = 0;
  int peak_active = 0;
  double busy_s = 0;
  bool stop = false, loader_done = false;
  hipStream_t st = nullptr;    // worker: batch ticks, results to host
  hipStream_t up = nullptr;    // loader: allocation, upload, plan set-up, frees
  nncp_batch* batch = nullptr;
  std::thread loader, worker;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

size_t job_footprint(const Job& j) {
  size_t b = (size_t)j.I * elem_bytes(j.dtype);
  for (int n = 0; n < j.N; ++n) b += (size_t)j.dims[n] * j.R * sizeof(float) + 256;
  nncp_options o{};
  o.split = j.split;
  b += nncp_workspace_bytes(j.N, j.dims, j.R, j.dtype, &o) + 256;
  return b;
}

bool hip_failed(hipError_t e, int line) {
  if (e == hipSuccess) return false;
  nncpk::note_device_error((int)e, 200000 + line);
  return true;
}

// Frees the job's device buffers in stream order on the loader's stream (no
// device-wide synchronisation; the caller has finished using them).
void release_device(nncp_server* S, Job* j) {
  if (j->plan) nncp_plan_destroy(j->plan);
  j->plan = nullptr;
  for (int n = 0; n < j->N; ++n)
    if (j->Hd[n]) (void)hipFreeAsync(j->Hd[n], S->up);
  if (j->Xd) (void)hipFreeAsync(j->Xd, S->up);
  if (j->ws) (void)hipFreeAsync(j->ws, S->up);
  j->Xd = nullptr;
  j->ws = nullptr;
  for (auto& h : j->Hd) h = nullptr;
}

// Loader thread: allocate, upload the tensor and starting factors, and build
// the job's plan, all on the loader's stream.
int load_device(nncp_server* S, Job* j) {
  hipStream_t s = S->up;
  const size_t xb = (size_t)j->I * elem_bytes(j->dtype);
  if (hipMallocAsync(&j->Xd, xb, s) != hipSuccess) return NNCP_ENOMEM;
  if (hip_failed(hipMemcpyAsync(j->Xd, j->X, xb, hipMemcpyHostToDevice, s), __LINE__)) return NNCP_EDEVICE;
  for (int n = 0; n < j->N; ++n) {
    const size_t hb = (size_t)j->dims[n] * j->R * sizeof(float);
    if (hipMallocAsync((void**)&j->Hd[n], hb, s) != hipSuccess) return NNCP_ENOMEM;
    if (hip_failed(hipMemcpyAsync(j->Hd[n], j->H0[n].data(), hb, hipMemcpyHostToDevice, s), __LINE__))
      return NNCP_EDEVICE;
  }
  nncp_options o{};
  o.split = j->split;
  o.no_graph = 1;  // advanced by the batch's graph only
  const size_t wsb = nncp_workspace_bytes(j->N, j->dims, j->R, j->dtype, &o);
  if (wsb == 0) return NNCP_EINVAL;
  if (hipMallocAsync(&j->ws, wsb, s) != hipSuccess) return NNCP_ENOMEM;
  // plan set-up runs on the loader's stream and synchronises it; the plan's
  // later calls (finish, fits) are the worker's
  int r = nncp_plan_create(&j->plan, j->Xd, j->dtype, j->N, j->dims, j->R, j->update, j->Hd, nullptr, j->ws, wsb,
                           &o, s);
  if (r != NNCP_OK) return r;
  return nncp_plan_set_stream(j->plan, S->st);
}

// Worker thread, job finished: normalised factors, lambda and fits to host,
// then the device buffers are released.
int retire_device(nncp_server* S, Job* j) {
  int r = nncp_batch_remove(S->batch, j->plan);
  j->lam.assign(j->R, 0.0);
  if (r == NNCP_OK) r = nncp_plan_finish(j->plan, j->lam.data());
  if (r == NNCP_OK) {
    j->fit.assign(std::min(j->iters, 1024), 0.0);
    int cnt = 0;
    r = nncp_plan_fits(j->plan, j->fit.data(), (int)j->fit.size(), &cnt);
    j->fit.resize(std::min<size_t>(j->fit.size(), (size_t)std::max(cnt, 0)));
  }
  j->H.resize(j->N);
  for (int n = 0; r == NNCP_OK && n < j->N; ++n) {
    j->H[n].resize((size_t)j->dims[n] * j->R);
    if (hip_failed(hipMemcpyAsync(j->H[n].data(), j->Hd[n], j->H[n].size() * sizeof(float),
                                  hipMemcpyDeviceToHost, S->st),
                   __LINE__))
      r = NNCP_EDEVICE;
  }
  if (hip_failed(hipStreamSynchronize(S->st), __LINE__) && r == NNCP_OK) r = NNCP_EDEVICE;
  release_device(S, j);
  return r;
}

void finish_job(nncp_server* S, Job* j, int status) {  // with S->mu held
  j->status = status;
  j->t_done = S->now();
  S->used -= j->footprint;
  --S->admitted;
  S->cv_load.notify_all();
  S->cv_done.notify_all();
}

void loader_loop(nncp_server* S) {
  if (!S->simulate) (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  while (true) {
    if (S->queue.empty()) {
      if (S->stop) break;
      S->cv_load.wait(lk);
      continue;
    }
    Job* j = S->jobs[S->queue.front()].get();
    if (j->footprint > S->budget) {  // can never fit
      S->queue.pop_front();
      j->status = NNCP_ENOMEM;
      j->t_done = S->now();
      ++S->rejected;
      S->cv_done.notify_all();
      continue;
    }
    // arrival order: the head waits for a slot and for memory
    if (S->admitted >= S->max_active || S->used + j->footprint > S->budget) {
      S->cv_load.wait(lk);
      continue;
    }
    S->queue.pop_front();
    S->used += j->footprint;
    S->peak_used = std::max(S->peak_used, S->used);
    ++S->admitted;
    j->t_admit = S->now();
    lk.unlock();
    int r = NNCP_OK;
    if (S->simulate) {
      std::this_thread::sleep_for(std::chrono::microseconds(20));
    } else {
      r = load_device(S, j);
      if (r != NNCP_OK) release_device(S, j);
    }
    lk.lock();
    if (r != NNCP_OK) {
      ++S->rejected;
      finish_job(S, j, r);
      continue;
    }
    S->ready.push_back(j);
    S->cv_work.notify_all();
  }
  S->loader_done = true;
  S->cv_work.notify_all();
}

void worker_loop(nncp_server* S) {
  if (!S->simulate) (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  while (true) {
    // jobs whose upload has finished join the batch
    if (!S->ready.empty()) {
      std::vector<Job*> joining;
      joining.swap(S->ready);
      const double t = S->now();
      lk.unlock();
      std::vector<int> codes(joining.size(), NNCP_OK);
      if (!S->simulate)
        for (size_t k = 0; k < joining.size(); ++k) codes[k] = nncp_batch_add(S->batch, joining[k]->plan);
      lk.lock();
      for (size_t k = 0; k < joining.size(); ++k) {
        Job* j = joining[k];
        if (codes[k] != NNCP_OK) {
          lk.unlock();
          if (!S->simulate) release_device(S, j);
          lk.lock();
          ++S->rejected;
          finish_job(S, j, codes[k]);
          continue;
        }
        j->t_start = t;
        S->active.push_back(j);
      }
      S->peak_active = std::max(S->peak_active, (int)S->active.size());
    }
    if (S->active.empty()) {
      if (S->loader_done && S->ready.empty()) break;
      S->cv_work.wait(lk);
      continue;
    }
    // one tick: every running job advances one outer iteration
    std::vector<Job*> act = S->active;
    lk.unlock();
    const double tb = S->now();
    int r = NNCP_OK;
    if (S->simulate) {
      int64_t e = 0;
      for (Job* j : act) e += j->I;
      std::this_thread::sleep_for(std::chrono::microseconds(50 + e / 1000000));
    } else {
      r = nncp_batch_run(S->batch, 1);
    }
    const double te = S->now();
    lk.lock();
    S->busy_s += te - tb;
    ++S->ticks;
    std::vector<Job*> finished;
    for (Job* j : act) {
      ++j->done_iters;
      if (r != NNCP_OK || j->done_iters >= j->iters) finished.push_back(j);
    }
    for (Job* j : finished) S->active.erase(std::find(S->active.begin(), S->active.end(), j));
    lk.unlock();
    std::vector<int> codes(finished.size(), r);
    if (!S->simulate)
      for (size_t k = 0; k < finished.size(); ++k) {
        if (r == NNCP_OK) {
          codes[k] = retire_device(S, finished[k]);
        } else {
          nncp_batch_remove(S->batch, finished[k]->plan);
          release_device(S, finished[k]);
        }
      }
    lk.lock();
    for (size_t k = 0; k < finished.size(); ++k) {
      ++S->completed;
      finish_job(S, finished[k], codes[k]);
    }
  }
}

}  // namespace

extern "C" {

int nncp_server_create(nncp_server** out, size_t hbm_budget_bytes, int max_active, int flags) {
  if (!out || hbm_budget_bytes == 0 || max_active < 1) return NNCP_EINVAL;
  *out = nullptr;
  nncp_server* S = new (std::nothrow) nncp_server();
  if (!S) return NNCP_ENOMEM;
  S->budget = hbm_budget_bytes;
  S->max_active = max_active;
  S->simulate = (flags & NNCP_SERVER_SIMULATE) != 0;
  S->t0 = Clock::now();
  if (!S->simulate) {
    if (hipGetDevice(&S->device) != hipSuccess || hipStreamCreateWithFlags(&S->st, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&S->up, hipStreamNonBlocking) != hipSuccess) {
      if (S->st) hipStreamDestroy(S->st);
      delete S;
      return NNCP_EDEVICE;
    }
    int r = nncp_batch_create(&S->batch, S->st);
    if (r != NNCP_OK) {
      hipStreamDestroy(S->st);
      hipStreamDestroy(S->up);
      delete S;
      return r;
    }
  }
  try {
    S->loader = std::thread(loader_loop, S);
    S->worker = std::thread(worker_loop, S);
  } catch (...) {
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->stop = true;
    }
    S->cv_load.notify_all();
    if (S->loader.joinable()) S->loader.join();
    if (S->worker.joinable()) S->worker.join();
    if (S->batch) nncp_batch_destroy(S->batch);
    if (S->st) hipStreamDestroy(S->st);
    if (S->up) hipStreamDestroy(S->up);
    delete S;
    return NNCP_ENOMEM;
  }
  *out = S;
  return NNCP_OK;
}

int nncp_server_submit(nncp_server* S, const nncp_job_request* q, uint64_t* id) {
  if (!S || !q || !id || !q->X || !q->dims || !q->H0 || q->iters < 1) return NNCP_EINVAL;
  if (q->N < 2 || q->N > NNCP_MAX_MODES || q->R < 1 || q->R > 64) return NNCP_EINVAL;
  if (q->dtype != NNCP_F32 && q->dtype != NNCP_BF16 && q->dtype != NNCP_F16) return NNCP_EINVAL;
  if (q->update != NNCP_HALS && q->update != NNCP_MU) return NNCP_EINVAL;
  std::unique_ptr<Job> j(new (std::nothrow) Job());
  if (!j) return NNCP_ENOMEM;
  j->X = q->X;
  j->dtype = q->dtype;
  j->N = q->N;
  j->R = q->R;
  j->update = q->update;
  j->iters = q->iters;
  j->split = q->split;
  j->I = 1;
  for (int n = 0; n < q->N; ++n) {
    if (q->dims[n] < 1 || !q->H0[n]) return NNCP_EINVAL;
    j->dims[n] = q->dims[n];
    j->I *= q->dims[n];
  }
  nncp_options o{};
  o.split = q->split;
  if (nncp_workspace_bytes(j->N, j->dims, j->R, j->dtype, &o) == 0) return NNCP_EINVAL;
  try {
    j->H0.resize(q->N);
    for (int n = 0; n < q->N; ++n) j->H0[n].assign(q->H0[n], q->H0[n] + (size_t)q->dims[n] * q->R);
  } catch (...) {
    return NNCP_ENOMEM;
  }
  j->footprint = job_footprint(*j);
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->stop) return NNCP_ECANCELED;
  j->id = S->next_id++;
  j->t_submit = S->now();
  *id = j->id;
  S->queue.push_back(j->id);
  S->jobs[j->id] = std::move(j);
  S->cv_load.notify_all();
  return NNCP_OK;
}

int nncp_server_poll(nncp_server* S, uint64_t id, nncp_job_result* res) {
  if (!S) return NNCP_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->jobs.find(id);
  if (it == S->jobs.end()) return NNCP_ENOTFOUND;
  const Job* j = it->second.get();
  if (res) {
    res->status = j->status;
    res->iters_done = j->done_iters;
    res->submit_s = j->t_submit;
    res->admit_s = j->t_admit;
    res->start_s = j->t_start;
    res->done_s = j->t_done;
    res->footprint_bytes = j->footprint;
  }
  return j->status == NNCP_EBUSY ? NNCP_EBUSY : NNCP_OK;
}

int nncp_server_fetch(nncp_server* S, uint64_t id, float* const* H, double* lambda, double* fit, int fit_cap,
                      int* fit_count) {
  if (!S) return NNCP_EINVAL;
  std::unique_ptr<Job> j;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->jobs.find(id);
    if (it == S->jobs.end()) return NNCP_ENOTFOUND;
    if (it->second->status == NNCP_EBUSY) return NNCP_EBUSY;
    j = std::move(it->second);
    S->jobs.erase(it);
  }
  if (j->status != NNCP_OK) return j->status;
  // (a simulated server computes nothing: its jobs finish with empty results)
  for (int n = 0; H && n < (int)j->H.size(); ++n)
    if (H[n]) std::memcpy(H[n], j->H[n].data(), j->H[n].size() * sizeof(float));
  if (lambda && !j->lam.empty()) std::memcpy(lambda, j->lam.data(), j->lam.size() * sizeof(double));
  const int nf = std::min<int>((int)j->fit.size(), std::max(fit_cap, 0));
  if (fit && nf > 0) std::memcpy(fit, j->fit.data(), nf * sizeof(double));
  if (fit_count) *fit_count = (int)j->fit.size();
  return NNCP_OK;
}

int nncp_server_wait(nncp_server* S, uint64_t id, double timeout_s) {
  if (!S) return NNCP_EINVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  auto done = [&] {
    auto it = S->jobs.find(id);
    return it == S->jobs.end() || it->second->status != NNCP_EBUSY;
  };
  if (timeout_s < 0) S->cv_done.wait(lk, done);
  else if (!S->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done)) return NNCP_EBUSY;
  return S->jobs.count(id) ? NNCP_OK : NNCP_ENOTFOUND;
}

int nncp_server_get_stats(nncp_server* S, nncp_server_stats* out) {
  if (!S || !out) return NNCP_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  out->queued = (int)S->queue.size();
  out->active = (int)S->active.size();
  out->peak_active = S->peak_active;
  out->ticks = S->ticks;
  out->completed = S->completed;
  out->rejected = S->rejected;
  out->bytes_in_use = S->used;
  out->peak_bytes = S->peak_used;
  out->budget_bytes = S->budget;
  out->busy_s = S->busy_s;
  out->now_s = S->now();
  out->graph_captures = 0;
  out->list_updates = 0;
  out->rebuild_s = 0.0;
  out->graph_s = 0.0;
  if (S->batch) {
    int64_t c = 0, u = 0;
    nncp_batch_captures(S->batch, &c, &u);
    out->graph_captures = c;
    out->list_updates = u;
    nncp_batch_build_time(S->batch, &out->rebuild_s, &out->graph_s);
  }
  return NNCP_OK;
}

int nncp_server_destroy(nncp_server* S) {
  if (!S) return NNCP_EINVAL;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    // queued jobs that never started are cancelled; admitted ones finish
    for (uint64_t id : S->queue) {
      Job* j = S->jobs[id].get();
      j->status = NNCP_ECANCELED;
      j->t_done = S->now();
    }
    S->queue.clear();
  }
  S->cv_load.notify_all();
  S->cv_done.notify_all();
  if (S->loader.joinable()) S->loader.join();
  if (S->worker.joinable()) S->worker.join();
  if (S->batch) nncp_batch_destroy(S->batch);
  if (S->up) {
    (void)hipStreamSynchronize(S->up);
    hipStreamDestroy(S->up);
  }
  if (S->st) hipStreamDestroy(S->st);
  delete S;
  return NNCP_OK;
}

}  // extern "C"
