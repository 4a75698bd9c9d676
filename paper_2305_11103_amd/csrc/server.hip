// Continuous-batching inversion server (binv_server_*; declared in binv.h).
//
// Requests of any order arrive through binv_submit from any host thread and
// wait in a FIFO queue (in host staging memory).  A scheduler thread admits
// them in order while the server's HBM budget and in-flight limit allow, and
// gives each admitted request its own device state (A, X and, for large
// orders, the working panels of a context).  Work then proceeds in two ways:
//  - requests of order <= kSmallMax are grouped: every scheduling round packs
//    all admitted small requests into one buffer and inverts them with the
//    register-resident batched kernels (one launch per size tier);
//  - larger requests go to a pool of worker threads, each owning a library
//    context and its own stream, so several sweeps overlap on the device.
// A request that arrives while others are running is admitted as soon as
// memory and slots free up.  binv_poll returns BINV_E_BUSY until the request
// is done, then copies X out and releases the request's device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "binv_internal.h"

namespace {

constexpr int kSmallMax = 128;     // orders batched into shared launches
constexpr int kWorkers = 3;        // concurrent large requests
constexpr int kMaxRoundSmall = 65536;

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

binv_status sfail(binv_status st, const std::string& msg) {
  binv::set_error(msg);
  return st;
}

enum ReqState { Q_QUEUED = 0, Q_ADMITTED, Q_RUNNING, Q_DONE, Q_FAILED };

struct Request {
  uint64_t id = 0;
  int64_t n = 0;
  int prec = BINV_PREC_FP64;
  double target = 1e-10;
  std::vector<double> hostA;  // staging until admission
  double* dA = nullptr;       // device copy of A (server-owned)
  double* dX = nullptr;       // device result
  size_t bytes = 0;           // device bytes charged to the budget
  ReqState state = Q_QUEUED;
  binv_status status = BINV_OK;
  std::string error;
  binv_info info;
  double t_submit = 0, t_admit = 0, t_done = 0;
};

// device bytes a request needs while in flight
size_t request_bytes(int64_t n, int prec) {
  const size_t nn = (size_t)n * (size_t)n;
  size_t b = 16 * nn;                                       // A and X
  if (n > kSmallMax) {
    const int64_t blk = std::min<int64_t>(512, n);
    b += 4 * 8 * (size_t)blk * (size_t)n + 8 * (size_t)blk * blk * 2;  // panels (two sets) + pivots
    if (prec == BINV_PREC_MIXED_F32) b += 20 * nn;          // FP32 copy, residual, next iterate
  }
  return b;
}

}  // namespace

struct binv_server {
  int device = 0;
  size_t budget = 0;
  int max_inflight = 0;
  std::mutex mu;
  std::condition_variable cv;      // wakes the scheduler
  std::condition_variable wcv;     // wakes the workers
  std::deque<Request*> queue;      // submitted, not admitted
  std::deque<Request*> large_ready;
  std::vector<Request*> small_ready;
  std::unordered_map<uint64_t, Request*> all;
  size_t used = 0;
  int inflight = 0;
  uint64_t next_id = 1;
  bool stop = false;
  std::thread sched;
  std::vector<std::thread> workers;
  binv_ctx* wctx[kWorkers] = {nullptr};
  // round buffers of the small-request path
  hipStream_t rstream = nullptr;
  binv::DevBuf rA, rX, rmats, rorder, rbounds, rinfo;
  // statistics
  std::atomic<int64_t> completed{0};
};

namespace {

void finish(binv_server* s, Request* r, binv_status st, const std::string& err) {
  std::lock_guard<std::mutex> g(s->mu);
  r->status = st;
  r->error = err;
  r->state = (st == BINV_OK) ? Q_DONE : Q_FAILED;
  r->t_done = now_s();
  s->inflight--;
  s->completed++;
  s->cv.notify_all();
}

// Admit queued requests in order while memory and slots allow (mu held).
void admit_locked(binv_server* s) {
  while (!s->queue.empty() && s->inflight < s->max_inflight) {
    Request* r = s->queue.front();
    if (s->used + r->bytes > s->budget) break;  // wait until results are collected
    const size_t nn = (size_t)r->n * (size_t)r->n;
    if (hipMalloc(&r->dA, sizeof(double) * std::max<size_t>(nn, 1)) != hipSuccess) {
      r->dA = nullptr;
      (void)hipGetLastError();
      break;
    }
    if (hipMalloc(&r->dX, sizeof(double) * std::max<size_t>(nn, 1)) != hipSuccess) {
      (void)hipFree(r->dA);
      r->dA = nullptr;
      r->dX = nullptr;
      (void)hipGetLastError();
      break;
    }
    if (nn) (void)hipMemcpy(r->dA, r->hostA.data(), sizeof(double) * nn, hipMemcpyHostToDevice);
    std::vector<double>().swap(r->hostA);
    s->queue.pop_front();
    s->used += r->bytes;
    s->inflight++;
    r->state = Q_ADMITTED;
    r->t_admit = now_s();
    if (r->n <= kSmallMax) s->small_ready.push_back(r);
    else {
      s->large_ready.push_back(r);
      s->wcv.notify_one();
    }
  }
}

// One scheduling round of the small path: pack, invert, unpack.
void run_small_round(binv_server* s, std::vector<Request*>& reqs) {
  const int64_t cnt = (int64_t)reqs.size();
  std::vector<binv::SmallMat> mats(cnt);
  std::vector<int32_t> bounds;
  std::vector<std::vector<int32_t>> tiers(5);
  int64_t off = 0;
  for (int64_t i = 0; i < cnt; ++i) {
    const int m = (int)reqs[i]->n;
    mats[i].off = off;
    mats[i].m = m;
    mats[i].nb = 1;  // one diagonal block: pivoting over the whole matrix
    mats[i].bnd = (int32_t)bounds.size();
    mats[i].id = (int32_t)i;
    bounds.push_back(0);
    bounds.push_back(m);
    int t = 0;
    while (m > binv::small_tier_limit(t)) ++t;
    tiers[t].push_back((int32_t)i);
    off += (int64_t)m * m;
  }
  std::vector<int32_t> order;
  int64_t first[5], count[5];
  for (int t = 0; t < 5; ++t) {
    first[t] = (int64_t)order.size();
    count[t] = (int64_t)tiers[t].size();
    order.insert(order.end(), tiers[t].begin(), tiers[t].end());
  }
  hipStream_t st = s->rstream;
  binv_status e = BINV_OK;
  std::string err;
  if ((e = s->rA.ensure(sizeof(double) * std::max<int64_t>(off, 1))) != BINV_OK ||
      (e = s->rX.ensure(sizeof(double) * std::max<int64_t>(off, 1))) != BINV_OK ||
      (e = s->rmats.ensure(sizeof(binv::SmallMat) * cnt)) != BINV_OK ||
      (e = s->rorder.ensure(sizeof(int32_t) * cnt)) != BINV_OK ||
      (e = s->rbounds.ensure(sizeof(int32_t) * bounds.size())) != BINV_OK ||
      (e = s->rinfo.ensure(sizeof(int32_t) * cnt)) != BINV_OK) {
    err = "round buffers: out of device memory";
  }
  std::vector<int32_t> hinfo(cnt, 0);
  if (e == BINV_OK) {
    hipError_t he = hipSuccess;
    double* A = (double*)s->rA.p;
    double* X = (double*)s->rX.p;
    for (int64_t i = 0; i < cnt && he == hipSuccess; ++i)
      he = hipMemcpyAsync(A + mats[i].off, reqs[i]->dA, sizeof(double) * mats[i].m * mats[i].m,
                          hipMemcpyDeviceToDevice, st);
    if (he == hipSuccess) he = hipMemcpyAsync(s->rmats.p, mats.data(), sizeof(binv::SmallMat) * cnt, hipMemcpyHostToDevice, st);
    if (he == hipSuccess) he = hipMemcpyAsync(s->rorder.p, order.data(), sizeof(int32_t) * cnt, hipMemcpyHostToDevice, st);
    if (he == hipSuccess)
      he = hipMemcpyAsync(s->rbounds.p, bounds.data(), sizeof(int32_t) * bounds.size(), hipMemcpyHostToDevice, st);
    for (int t = 0; t < 5 && he == hipSuccess; ++t)
      he = binv::launch_small_tier(t, A, X, (const binv::SmallMat*)s->rmats.p, (const int32_t*)s->rorder.p + first[t],
                                   count[t], (const int32_t*)s->rbounds.p, (int32_t*)s->rinfo.p, st);
    for (int64_t i = 0; i < cnt && he == hipSuccess; ++i)
      he = hipMemcpyAsync(reqs[i]->dX, X + mats[i].off, sizeof(double) * mats[i].m * mats[i].m,
                          hipMemcpyDeviceToDevice, st);
    if (he == hipSuccess) he = hipMemcpyAsync(hinfo.data(), s->rinfo.p, sizeof(int32_t) * cnt, hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    if (he != hipSuccess) {
      e = BINV_E_HIP;
      err = std::string("small round: ") + hipGetErrorString(he);
    }
  }
  for (int64_t i = 0; i < cnt; ++i) {
    std::memset(&reqs[i]->info, 0, sizeof(binv_info));
    reqs[i]->info.converged = 1;
    if (e != BINV_OK) finish(s, reqs[i], e, err);
    else if (hinfo[i] != 0)
      finish(s, reqs[i], BINV_E_SINGULAR, "exactly-zero pivot at row " + std::to_string(hinfo[i]));
    else finish(s, reqs[i], BINV_OK, "");
  }
}

void scheduler_main(binv_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (!s->stop) {
    admit_locked(s);
    if (!s->small_ready.empty()) {
      std::vector<Request*> round;
      round.swap(s->small_ready);
      if ((int)round.size() > kMaxRoundSmall) {
        s->small_ready.assign(round.begin() + kMaxRoundSmall, round.end());
        round.resize(kMaxRoundSmall);
      }
      for (Request* r : round) r->state = Q_RUNNING;
      lk.unlock();
      run_small_round(s, round);
      lk.lock();
      continue;
    }
    s->cv.wait_for(lk, std::chrono::microseconds(200));
  }
}

void worker_main(binv_server* s, int w) {
  (void)hipSetDevice(s->device);
  hipStream_t st = nullptr;
  (void)hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  for (;;) {
    Request* r = nullptr;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->wcv.wait(lk, [&] { return s->stop || !s->large_ready.empty(); });
      if (s->stop && s->large_ready.empty()) break;
      r = s->large_ready.front();
      s->large_ready.pop_front();
      r->state = Q_RUNNING;
    }
    binv_status e;
    std::memset(&r->info, 0, sizeof(binv_info));
    binv_opts o;
    std::memset(&o, 0, sizeof(o));
    o.block = r->n >= 2048 ? 512 : (r->n >= 512 ? 256 : 128);
    o.flags = BINV_F_SYNC | (r->n < 4096 ? BINV_F_NO_LOOKAHEAD : 0u);
    if (r->prec == BINV_PREC_MIXED_F32) {
      e = binv_invert_mixed(s->wctx[w], r->n, r->dA, r->n, r->dX, r->n, &o, r->target, -1, st, &r->info);
    } else {
      e = binv_invert(s->wctx[w], r->n, r->dA, r->n, r->dX, r->n, &o, st, nullptr);
      r->info.converged = 1;
    }
    finish(s, r, e, e == BINV_OK ? "" : binv_last_error());
  }
  if (st) (void)hipStreamDestroy(st);
}

}  // namespace

extern "C" {

binv_status binv_server_create(int device, size_t hbm_budget_bytes, int32_t max_inflight, binv_server** out) {
  if (!out) return sfail(BINV_E_INVALID, "out is NULL");
  *out = nullptr;
  if (hbm_budget_bytes == 0) return sfail(BINV_E_INVALID, "zero HBM budget");
  binv_server* s = new (std::nothrow) binv_server();
  if (!s) return sfail(BINV_E_NOMEM, "out of host memory");
  s->device = device;
  s->budget = hbm_budget_bytes;
  s->max_inflight = max_inflight > 0 ? max_inflight : 1 << 20;
  if (hipSetDevice(device) != hipSuccess || hipStreamCreateWithFlags(&s->rstream, hipStreamNonBlocking) != hipSuccess) {
    delete s;
    return sfail(BINV_E_HIP, "cannot use the device");
  }
  for (int w = 0; w < kWorkers; ++w) {
    binv_status st = binv_create(&s->wctx[w], device);
    if (st != BINV_OK) {
      for (int v = 0; v < w; ++v) binv_destroy(s->wctx[v]);
      (void)hipStreamDestroy(s->rstream);
      delete s;
      return st;
    }
  }
  s->sched = std::thread(scheduler_main, s);
  for (int w = 0; w < kWorkers; ++w) s->workers.emplace_back(worker_main, s, w);
  *out = s;
  return BINV_OK;
}

binv_status binv_submit(binv_server* s, int64_t n, const double* A, int a_is_device, int32_t prec, double target,
                        uint64_t* ticket) {
  if (!s || !ticket) return sfail(BINV_E_INVALID, "NULL argument");
  if (n < 1 || (!A)) return sfail(BINV_E_INVALID, "n must be positive and A non-NULL");
  if (prec != BINV_PREC_FP64 && prec != BINV_PREC_MIXED_F32) return sfail(BINV_E_INVALID, "unknown precision");
  Request* r = new (std::nothrow) Request();
  if (!r) return sfail(BINV_E_NOMEM, "out of host memory");
  r->n = n;
  r->prec = prec;
  r->target = target > 0 ? target : 1e-10;
  r->bytes = request_bytes(n, prec);
  if (r->bytes > s->budget) {
    delete r;
    return sfail(BINV_E_NOMEM, "request alone exceeds the server's HBM budget");
  }
  const size_t nn = (size_t)n * (size_t)n;
  try {
    r->hostA.resize(nn);
  } catch (...) {
    delete r;
    return sfail(BINV_E_NOMEM, "out of host memory for staging");
  }
  hipError_t e = a_is_device ? hipMemcpy(r->hostA.data(), A, sizeof(double) * nn, hipMemcpyDeviceToHost)
                             : hipSuccess;
  if (!a_is_device) std::memcpy(r->hostA.data(), A, sizeof(double) * nn);
  if (e != hipSuccess) {
    delete r;
    return sfail(BINV_E_HIP, std::string("copy of A: ") + hipGetErrorString(e));
  }
  r->t_submit = now_s();
  {
    std::lock_guard<std::mutex> g(s->mu);
    r->id = s->next_id++;
    s->all[r->id] = r;
    s->queue.push_back(r);
    s->cv.notify_all();
  }
  *ticket = r->id;
  return BINV_OK;
}

binv_status binv_poll(binv_server* s, uint64_t ticket, double* X, int x_is_device, binv_info* info,
                      binv_request_times* times) {
  if (!s) return sfail(BINV_E_INVALID, "server is NULL");
  Request* r = nullptr;
  {
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return sfail(BINV_E_NOTFOUND, "unknown ticket");
    r = it->second;
    if (r->state != Q_DONE && r->state != Q_FAILED) return BINV_E_BUSY;
    s->all.erase(it);
  }
  binv_status st = r->status;
  if (st == BINV_OK && X) {
    const size_t nn = (size_t)r->n * (size_t)r->n;
    hipError_t e = hipMemcpy(X, r->dX, sizeof(double) * nn, x_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost);
    if (e != hipSuccess) st = sfail(BINV_E_HIP, std::string("copy of X: ") + hipGetErrorString(e));
  } else if (st != BINV_OK) {
    binv::set_error(r->error);
  }
  if (info) *info = r->info;
  if (times) {
    times->queue_ms = (r->t_admit - r->t_submit) * 1e3;
    times->total_ms = (r->t_done - r->t_submit) * 1e3;
  }
  if (r->dA) (void)hipFree(r->dA);
  if (r->dX) (void)hipFree(r->dX);
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->used -= r->bytes;
    s->cv.notify_all();
  }
  delete r;
  return st;
}

binv_status binv_server_destroy(binv_server* s) {
  if (!s) return BINV_OK;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    s->cv.notify_all();
    s->wcv.notify_all();
  }
  if (s->sched.joinable()) s->sched.join();
  for (auto& t : s->workers)
    if (t.joinable()) t.join();
  for (auto& kv : s->all) {
    Request* r = kv.second;
    if (r->dA) (void)hipFree(r->dA);
    if (r->dX) (void)hipFree(r->dX);
    delete r;
  }
  for (int w = 0; w < kWorkers; ++w) binv_destroy(s->wctx[w]);
  for (binv::DevBuf* d : {&s->rA, &s->rX, &s->rmats, &s->rorder, &s->rbounds, &s->rinfo}) d->release();
  if (s->rstream) (void)hipStreamDestroy(s->rstream);
  delete s;
  return BINV_OK;
}

}  // extern "C"
