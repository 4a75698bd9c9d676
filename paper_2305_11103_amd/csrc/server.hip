// Continuous-batching inversion server (binv_server_*; declared in binv.h).
//
// Requests of any order arrive through binv_submit from any host thread and
// wait in a FIFO queue (in host staging memory).  A scheduler thread admits
// them in order while the server's HBM budget and in-flight limit allow, and
// gives each admitted request its own device state (A, X and, for large
// orders, the working panels of a context).  Work then proceeds in two ways:
//  - requests of order <= kRoundMax are grouped: every scheduling round packs
//    all admitted small requests into one buffer and inverts them with the
//    batched kernels: the register-resident tiers up to kSmallMax (one launch
//    per size tier), the swept step above (one launch per block step);
//  - larger requests go to a pool of worker threads, each owning a library
//    context and its own stream, so several sweeps overlap on the device.
// A request that arrives while others are running is admitted as soon as
// memory and slots free up.  binv_poll returns BINV_E_BUSY until the request
// is done, then copies X out and releases the request's device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdlib>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "binv_internal.h"

namespace {

constexpr int kSmallMax = binv::kSmallMaxOrder;  // orders inverted by the register tiers of a round
constexpr int kRoundMax = 256;     // orders grouped into rounds (above kSmallMax: swept steps)
constexpr int kSweptBlock = 128;   // largest diagonal block of a swept step
constexpr int kMaxWorkers = 8;     // concurrent large requests (BINV_SERVER_WORKERS, default 2)
constexpr int kMaxRoundSmall = 65536;
constexpr int64_t kBigN = 4096;    // orders served one at a time on worker 0
constexpr double kFp32Reach = 1e-6;  // rho the FP32 sweep can meet without refinement
// The device's check (an FP64 residual, or its random-probe estimate) carries
// its own rounding error, and the estimate a spread, of the order of the rho
// it measures near 1e-10, so a request is refined until that check reads half
// its target.
constexpr double kCheckMargin = 0.5;

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
  size_t blk = 0;             // bytes of the request's device block (A then X)
  size_t ws = 0;              // workspace reserved for it until it finishes
  bool on_device = false;     // dA/dX already allocated and charged at submit
  bool fp32_start = false;    // the sweep ran in FP32 (mixed request)
  ReqState state = Q_QUEUED;
  binv_status status = BINV_OK;
  std::string error;
  binv_info info;
  double t_submit = 0, t_admit = 0, t_done = 0;
};

// Allocation class of a request block: 1/8-octave steps, at least 64 KiB.
size_t size_class(size_t bytes) {
  size_t c = 64 << 10;
  if (bytes <= c) return c;
  int e = 63 - __builtin_clzll((unsigned long long)bytes);  // 2^e <= bytes < 2^(e+1)
  const size_t step = (size_t)1 << (e - 3);
  return (bytes + step - 1) / step * step;
}

// Device bytes of a request's block (A then X).
size_t block_bytes(int64_t n) { return size_class(2 * sizeof(double) * std::max<size_t>((size_t)n * (size_t)n, 1)); }

// Diagonal-block order the workers use for a request of order n.
int worker_block(int64_t n) { return n >= 2048 ? 512 : (n >= 512 ? 256 : 128); }

// Does a request run in a round (shared launches) rather than on a worker?
// Orders up to kSmallMax always do; kSmallMax < n <= kRoundMax unless the
// request starts from the FP32 sweep, which only the workers run.
bool in_round(int64_t n, bool fp32_start) { return n <= kSmallMax || (n <= kRoundMax && !fp32_start); }

// Upper bound of the workspace a request makes the server hold while it runs:
// in a round its share of the round's buffers (packed copies of A and X, two
// m x m refinement buffers, the tables, and for a swept order the pivot
// inverse and the two panels of its steps); otherwise what a worker
// context's binv_invert_mixed can grow to for it: the sweep's panels (two
// sets under the lookahead) and the nested pivot sweep's, the residual and
// next iterate, the compensated residual's split operands, and the FP32
// working copy and panels when it starts from the FP32 sweep.
size_t workspace_bytes(int64_t n, bool fp32_start) {
  const size_t nn = (size_t)n * (size_t)n, d = sizeof(double);
  if (in_round(n, fp32_start)) {
    size_t w = 4 * d * nn + 64;
    if (n > kSmallMax) w += d * (kSweptBlock * kSweptBlock + 2 * kSweptBlock * (size_t)n) + 4 * sizeof(binv::SweptJob);
    return w;
  }
  const size_t b = (size_t)worker_block(n), sets = n >= kBigN ? 2 : 1;
  size_t w = sets * d * (2 * b * (size_t)n + b * b);  // level-0 panels and pivot inverse
  w += 2 * d * (2 * 64 * b + 64 * 64);               // the nested pivot sweep's panels
  w += d * (nn + nn + 1025) + 2 * d * (2 * nn) + 2 * sizeof(int) * (size_t)n + d;  // res, xn, parts, splits, info
  if (fp32_start) w += sizeof(float) * (nn + 2 * b * (size_t)n + b * b) + 2 * d * b * b;
  return w + (1 << 20);  // allocation granularity
}

}  // namespace

struct binv_server {
  int device = 0;
  size_t budget = 0;
  int max_inflight = 0;
  uint32_t flags = 0;              // BINV_SERVER_*
  std::mutex mu;
  std::condition_variable cv;      // wakes the scheduler
  std::condition_variable wcv;     // wakes the workers
  std::deque<Request*> queue;      // submitted, not admitted
  std::deque<Request*> big_ready;   // order >= kBigN: worker 0 only, one at a time
  std::deque<Request*> mid_ready;   // other orders below kBigN: any worker
  std::vector<Request*> small_ready;
  std::unordered_map<uint64_t, Request*> all;
  std::deque<uint64_t> done_q;     // finished tickets in completion order
  std::condition_variable dcv;     // wakes binv_next_done
  size_t used = 0;
  size_t peak = 0;
  int inflight = 0;
  uint64_t next_id = 1;
  bool stop = false;
  std::thread sched;
  std::thread rounds;                // runs the rounds, apart from admission
  std::condition_variable rcv;       // wakes the round thread
  bool round_running = false;        // the round thread is using the round buffers
  std::vector<std::thread> workers;
  int nworkers = 2;
  binv_ctx* wctx[kMaxWorkers] = {nullptr};
  // Device blocks of finished requests, kept for reuse by size class so that
  // collecting a result never calls hipFree (which waits for the whole
  // device and would stall the other requests' work).
  std::mutex pool_mu;
  std::multimap<size_t, void*> pool;
  size_t pooled = 0;
  // round buffers of the small-request path
  hipStream_t rstream = nullptr;
  // copies in and out of request state; every copy is waited for, so a
  // worker stream never reads a block before its input has landed
  hipStream_t cstream = nullptr;
  binv::DevBuf rA, rX, rmats, rorder, rbounds, rinfo, rwork, rtarget, rrho, rsteps, rsw, rjobs;
  // Accounting: `used` counts every byte the server holds on the device or
  // has promised: blocks of admitted requests, blocks kept in the cache,
  // workspace held by the worker contexts (ws_held) and by the round buffers
  // (round_held), and the workspace reserved for requests still running.
  size_t ws_held[kMaxWorkers] = {0};
  bool worker_busy[kMaxWorkers] = {false};
  size_t round_held = 0;
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
  s->done_q.push_back(r->id);
  s->cv.notify_all();
  s->dcv.notify_all();
}

hipError_t copy_sync(binv_server* s, void* dst, const void* src, size_t bytes, hipMemcpyKind kind) {
  if (bytes == 0) return hipSuccess;
  hipError_t e = hipMemcpyAsync(dst, src, bytes, kind, s->cstream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->cstream);
  return e;
}

// Whether the cache holds a block of class c.
bool pool_has(binv_server* s, size_t c) {
  std::lock_guard<std::mutex> g(s->pool_mu);
  return s->pool.find(c) != s->pool.end();
}

// A block of class c from the cache (already counted in `used`), or NULL.
void* pool_take(binv_server* s, size_t c) {
  std::lock_guard<std::mutex> g(s->pool_mu);
  auto it = s->pool.find(c);
  if (it == s->pool.end()) return nullptr;
  void* p = it->second;
  s->pool.erase(it);
  s->pooled -= c;
  return p;
}

// Free one cached block of a class other than `keep` (mu held); false if
// none is left.  hipFree waits for the device, so this runs only when a
// request could not be admitted otherwise.
bool pool_evict_locked(binv_server* s, size_t keep) {
  void* p = nullptr;
  size_t c = 0;
  {
    std::lock_guard<std::mutex> g(s->pool_mu);
    for (auto it = s->pool.begin(); it != s->pool.end(); ++it)
      if (it->first != keep) {
        p = it->second;
        c = it->first;
        s->pool.erase(it);
        s->pooled -= c;
        break;
      }
  }
  if (!p) return false;
  (void)hipFree(p);
  s->used -= c;
  return true;
}

// Release the workspace of idle worker contexts (mu held), the largest
// first, until `need` more bytes fit; false if that is not enough.
bool trim_workers_locked(binv_server* s, size_t need) {
  while (s->used + need > s->budget) {
    int best = -1;
    for (int w = 0; w < s->nworkers; ++w)
      if (!s->worker_busy[w] && s->ws_held[w] > 0 && (best < 0 || s->ws_held[w] > s->ws_held[best])) best = w;
    if (best < 0) return false;
    binv_ctx* c = s->wctx[best];
    for (auto& L : c->lv)
      for (int h = 0; h < 2; ++h) {
        L.ct[h].release();
        L.r[h].release();
        L.p[h].release();
      }
    c->info.release();
    c->piv.release();
    for (binv::DevBuf* d : {&c->mx_w32, &c->mx_ct32, &c->mx_r32, &c->mx_p32, &c->mx_p64a, &c->mx_p64b, &c->mx_res,
                            &c->mx_xn, &c->mx_part, &c->mx_split_a, &c->mx_split_x, &c->mx_exps})
      d->release();
    s->used -= s->ws_held[best];
    s->ws_held[best] = binv::ctx_device_bytes(c);  // 0
    s->used += s->ws_held[best];
  }
  return true;
}

// Make room for a request (mu held): its workspace reservation and, unless
// the cache has a block of its class, a new block; cached blocks of other
// classes and idle workers' workspace are released when that is the only way,
// and, called from the scheduler thread (the only one that uses them), the
// small-request round buffers too, while no round is using them.
bool make_room_locked(binv_server* s, Request* r) {
  const size_t need = r->ws + (pool_has(s, r->blk) ? 0 : r->blk);
  while (s->used + need > s->budget)
    if (!pool_evict_locked(s, r->blk)) break;
  if (s->used + need > s->budget) (void)trim_workers_locked(s, need);
  if (s->used + need > s->budget && !s->round_running && s->round_held > 0) {
    for (binv::DevBuf* d : {&s->rA, &s->rX, &s->rmats, &s->rorder, &s->rbounds, &s->rinfo, &s->rwork, &s->rtarget,
                            &s->rrho, &s->rsteps, &s->rsw, &s->rjobs})
      d->release();
    s->used -= s->round_held;
    s->round_held = 0;
  }
  return s->used + need <= s->budget;
}

// A and X of one request share one block: A first, X after it.  Charges
// the block (unless it comes from the cache, where it is already counted)
// and the workspace reservation (mu held).
bool request_alloc_locked(binv_server* s, Request* r) {
  const size_t nn = std::max<size_t>((size_t)r->n * (size_t)r->n, 1);
  double* p = (double*)pool_take(s, r->blk);
  if (!p) {
    if (hipMalloc((void**)&p, r->blk) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    s->used += r->blk;
  }
  s->used += r->ws;
  s->peak = std::max(s->peak, s->used);
  r->dA = p;
  r->dX = p + nn;
  return true;
}

// The request's block back to the cache, which keeps at most a quarter of the
// budget in blocks (still counted in `used`); otherwise it is freed.  Any
// workspace reservation left is released (mu held).
void request_release_locked(binv_server* s, Request* r) {
  if (r->dA) {
    bool kept = false;
    {
      std::lock_guard<std::mutex> g(s->pool_mu);
      if (s->pooled + r->blk <= s->budget / 4) {
        s->pool.emplace(r->blk, (void*)r->dA);
        s->pooled += r->blk;
        kept = true;
      }
    }
    if (!kept) {
      (void)hipFree(r->dA);
      s->used -= r->blk;
    }
  }
  s->used -= r->ws;
  r->ws = 0;
  r->dA = r->dX = nullptr;
}

// Does the request start from the FP32 sweep (a mixed request whose target
// is within that sweep's reach, or any mixed request under strict precision)?
bool fp32_start_of(const binv_server* s, const Request* r) {
  return r->prec == BINV_PREC_MIXED_F32 && ((s->flags & BINV_SERVER_STRICT_PRECISION) || r->target >= kFp32Reach);
}

// Queue an admitted request for its lane (mu held).  Large orders run one at
// a time on worker 0, with the lookahead schedule: one sweep of that size
// already keeps the device busy, and two of them side by side were measured
// slower than one after the other.  Mid orders are latency-bound sweeps that
// the other workers overlap with it and with each other.
void route_locked(binv_server* s, Request* r) {
  if (in_round(r->n, fp32_start_of(s, r))) {
    s->small_ready.push_back(r);
    s->rcv.notify_one();
    return;
  }
  if (r->n >= kBigN) s->big_ready.push_back(r);
  else s->mid_ready.push_back(r);
  s->wcv.notify_all();
}

// Admit queued requests in order while memory and slots allow (mu held).
void admit_locked(binv_server* s) {
  while (!s->queue.empty() && s->inflight < s->max_inflight) {
    Request* r = s->queue.front();
    if (r->on_device) {
      s->queue.pop_front();
      s->inflight++;
      r->state = Q_ADMITTED;
      r->t_admit = now_s();
      route_locked(s, r);
      continue;
    }
    if (!make_room_locked(s, r)) break;  // wait until results are collected
    const size_t nn = (size_t)r->n * (size_t)r->n;
    if (!request_alloc_locked(s, r)) break;
    if (copy_sync(s, r->dA, r->hostA.data(), sizeof(double) * nn, hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipGetLastError();
      request_release_locked(s, r);
      break;
    }
    std::vector<double>().swap(r->hostA);
    s->queue.pop_front();
    s->inflight++;
    r->state = Q_ADMITTED;
    r->t_admit = now_s();
    route_locked(s, r);
  }
}

// Block orders of a swept request: m split into ceil(m / kSweptBlock) near-equal
// blocks, the larger ones last.
std::vector<int> swept_blocks(int m) {
  const int pieces = (m + kSweptBlock - 1) / kSweptBlock;
  std::vector<int> ord(pieces);
  for (int q = 0; q < pieces; ++q) ord[q] = m / pieces + (q >= pieces - m % pieces ? 1 : 0);
  return ord;
}

// One scheduling round: pack, invert, check and refine, unpack.  Orders up to
// kSmallMax are inverted by the register tiers (one diagonal block, pivoting
// over the whole matrix).  Larger orders are swept block by block (Eq. (a)
// unrolled): the requests' matrices are the round's device-resident state, and
// block step p of every request that has one runs in one shared launch
// (k_swept_step, one workgroup per request: pivot leaf, row panel, column-panel
// copy, Schur update), so each step index is one launch for the whole round.
void run_small_round(binv_server* s, std::vector<Request*>& reqs) {
  const int64_t cnt = (int64_t)reqs.size();
  std::vector<binv::SmallMat> mats(cnt);
  std::vector<int32_t> bounds;
  std::vector<std::vector<int32_t>> tiers(binv::kSmallTierCount);
  std::vector<int32_t> swept;  // request indices of the swept orders
  std::vector<int64_t> sw_off;  // their workspace offsets (elements)
  int64_t off = 0, sw_elems = 0;
  for (int64_t i = 0; i < cnt; ++i) {
    const int m = (int)reqs[i]->n;
    mats[i].off = off;
    mats[i].m = m;
    mats[i].nb = 1;  // one diagonal block: pivoting over the whole matrix
    mats[i].bnd = (int32_t)bounds.size();
    mats[i].id = (int32_t)i;
    bounds.push_back(0);
    bounds.push_back(m);
    if (m > kSmallMax) {
      swept.push_back((int32_t)i);
      sw_off.push_back(sw_elems);
      sw_elems += (int64_t)kSweptBlock * kSweptBlock + 2LL * kSweptBlock * m;
    } else {
      int t = 0;
      while (m > binv::small_tier_limit(t)) ++t;
      tiers[t].push_back((int32_t)i);
    }
    off += (int64_t)m * m;
  }
  std::vector<int32_t> order;
  int64_t first[binv::kSmallTierCount], count[binv::kSmallTierCount];
  for (int t = 0; t < binv::kSmallTierCount; ++t) {
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
      (e = s->rinfo.ensure(sizeof(int32_t) * cnt)) != BINV_OK ||
      (e = s->rwork.ensure(sizeof(double) * 2 * std::max<int64_t>(off, 1))) != BINV_OK ||
      (e = s->rtarget.ensure(sizeof(double) * cnt)) != BINV_OK ||
      (e = s->rrho.ensure(sizeof(double) * cnt)) != BINV_OK ||
      (e = s->rsteps.ensure(sizeof(int32_t) * cnt)) != BINV_OK ||
      (e = s->rsw.ensure(sizeof(double) * std::max<int64_t>(sw_elems, 1))) != BINV_OK) {
    err = "round buffers: out of device memory";
  }
  // the swept steps' jobs: step p of request i reads its matrix as left by
  // step p - 1 (A itself for p = 0) and writes X; P, Ct and R live in the
  // request's slice of the round workspace
  std::vector<binv::SweptJob> jobs;
  std::vector<std::pair<int64_t, int64_t>> step_jobs;  // (first job, jobs with a block > 64) per step
  std::vector<int64_t> step_count;
  if (e == BINV_OK && !swept.empty()) {
    const double* A = (const double*)s->rA.p;
    double* X = (double*)s->rX.p;
    double* ws = (double*)s->rsw.p;
    std::vector<std::vector<int>> blocks;
    size_t steps = 0;
    for (int32_t i : swept) {
      blocks.push_back(swept_blocks(mats[i].m));
      steps = std::max(steps, blocks.back().size());
    }
    for (size_t p = 0; p < steps; ++p) {
      const int64_t first = (int64_t)jobs.size();
      for (size_t t = 0; t < swept.size(); ++t) {
        const int i = swept[t];
        if (p >= blocks[t].size()) continue;
        const int m = mats[i].m;
        int o = 0;
        for (size_t q = 0; q < p; ++q) o += blocks[t][q];
        const int bs = blocks[t][p];
        const double* Win = (p == 0 ? A : (const double*)X) + mats[i].off;
        double* Wout = X + mats[i].off;
        double* P = ws + sw_off[t];
        double* Ct = P + kSweptBlock * kSweptBlock;
        double* R = Ct + (int64_t)kSweptBlock * m;
        binv::SweptJob j;
        std::memset(&j, 0, sizeof(j));
        j.leaf.A = Win + (int64_t)o * m + o; j.leaf.lda = m; j.leaf.P = P; j.leaf.ldp = bs; j.leaf.b = bs;
        j.leaf.row0 = o; j.leaf.info = (int32_t*)s->rinfo.p + i;
        binv::StepArgs& ra = j.row;
        ra.A = P; ra.lda = bs; ra.B = Win + (int64_t)o * m; ra.ldb = m; ra.W = R; ra.ldw = m;
        ra.R = P; ra.ldr = bs; ra.M = bs; ra.N = m; ra.K = bs; ra.o = o; ra.b = bs; ra.oc = o;
        binv::StepArgs& sa = j.schur;
        sa.A = Ct; sa.lda = bs; sa.B = R; sa.ldb = m; sa.W = Wout; sa.ldw = m; sa.Win = Win; sa.ldwin = m;
        sa.R = R; sa.ldr = m; sa.M = m; sa.N = m; sa.K = bs; sa.o = o; sa.b = bs; sa.oc = o;
        jobs.push_back(j);
      }
      std::stable_sort(jobs.begin() + first, jobs.end(),
                       [](const binv::SweptJob& x, const binv::SweptJob& y) { return x.leaf.b > y.leaf.b; });
      int64_t big = 0;
      for (int64_t q = first; q < (int64_t)jobs.size(); ++q) big += jobs[q].leaf.b > 64;
      step_jobs.emplace_back(first, big);
      step_count.push_back((int64_t)jobs.size() - first);
    }
    if ((e = s->rjobs.ensure(sizeof(binv::SweptJob) * jobs.size())) != BINV_OK)
      err = "round buffers: out of device memory";
  }
  std::vector<int32_t> hinfo(cnt, 0), hsteps(cnt, 0);
  std::vector<double> htarget(cnt), hrho(cnt, 0.0);
  for (int64_t i = 0; i < cnt; ++i) htarget[i] = kCheckMargin * reqs[i]->target;
  if (e == BINV_OK) {
    hipError_t he = hipSuccess;
    double* A = (double*)s->rA.p;
    double* X = (double*)s->rX.p;
    for (int64_t i = 0; i < cnt && he == hipSuccess; ++i)
      he = hipMemcpyAsync(A + mats[i].off, reqs[i]->dA, sizeof(double) * mats[i].m * mats[i].m,
                          hipMemcpyDeviceToDevice, st);
    if (he == hipSuccess) he = hipMemcpyAsync(s->rmats.p, mats.data(), sizeof(binv::SmallMat) * cnt, hipMemcpyHostToDevice, st);
    // (the register tiers' members only: the swept orders are not in it)
    if (he == hipSuccess && !order.empty())
      he = hipMemcpyAsync(s->rorder.p, order.data(), sizeof(int32_t) * order.size(), hipMemcpyHostToDevice, st);
    if (he == hipSuccess)
      he = hipMemcpyAsync(s->rbounds.p, bounds.data(), sizeof(int32_t) * bounds.size(), hipMemcpyHostToDevice, st);
    if (he == hipSuccess && !jobs.empty()) {
      he = hipMemcpyAsync(s->rjobs.p, jobs.data(), sizeof(binv::SweptJob) * jobs.size(), hipMemcpyHostToDevice, st);
      // the leaves record a zero pivot with a compare-and-swap on a zeroed word
      if (he == hipSuccess) he = hipMemsetAsync(s->rinfo.p, 0, sizeof(int32_t) * cnt, st);
    }
    for (int t = 0; t < binv::kSmallTierCount && he == hipSuccess; ++t)
      he = binv::launch_small_tier(t, A, X, (const binv::SmallMat*)s->rmats.p, (const int32_t*)s->rorder.p + first[t],
                                   count[t], (const int32_t*)s->rbounds.p, (int32_t*)s->rinfo.p, st);
    for (size_t p = 0; p < step_jobs.size() && he == hipSuccess; ++p) {
      const binv::SweptJob* dj = (const binv::SweptJob*)s->rjobs.p + step_jobs[p].first;
      he = binv::launch_swept_step(dj, step_jobs[p].second, 128, st);
      if (he == hipSuccess)
        he = binv::launch_swept_step(dj + step_jobs[p].second, step_count[p] - step_jobs[p].second, 64, st);
    }
    // residual check of every matrix against its request's target, with up to
    // three Newton-Schulz steps where it misses (a singular member's X is not
    // used, so its refinement result does not matter)
    if (he == hipSuccess)
      he = hipMemcpyAsync(s->rtarget.p, htarget.data(), sizeof(double) * cnt, hipMemcpyHostToDevice, st);
    if (he == hipSuccess)
      he = binv::launch_small_refine(A, X, (const binv::SmallMat*)s->rmats.p, nullptr, cnt, (double*)s->rwork.p,
                                     1e-10, (const double*)s->rtarget.p, 3, (double*)s->rrho.p,
                                     (int32_t*)s->rsteps.p, st);
    for (int64_t i = 0; i < cnt && he == hipSuccess; ++i)
      he = hipMemcpyAsync(reqs[i]->dX, X + mats[i].off, sizeof(double) * mats[i].m * mats[i].m,
                          hipMemcpyDeviceToDevice, st);
    if (he == hipSuccess) he = hipMemcpyAsync(hinfo.data(), s->rinfo.p, sizeof(int32_t) * cnt, hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipMemcpyAsync(hrho.data(), s->rrho.p, sizeof(double) * cnt, hipMemcpyDeviceToHost, st);
    if (he == hipSuccess)
      he = hipMemcpyAsync(hsteps.data(), s->rsteps.p, sizeof(int32_t) * cnt, hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    if (he != hipSuccess) {
      e = BINV_E_HIP;
      err = std::string("small round: ") + hipGetErrorString(he);
    }
  }
  {
    // the round buffers are charged as they grew; the requests' workspace
    // reservations end with the round
    size_t held = 0;
    for (const binv::DevBuf* d : {&s->rA, &s->rX, &s->rmats, &s->rorder, &s->rbounds, &s->rinfo, &s->rwork,
                                  &s->rtarget, &s->rrho, &s->rsteps, &s->rsw, &s->rjobs})
      held += d->bytes;
    std::lock_guard<std::mutex> g(s->mu);
    s->used += held;
    s->used -= s->round_held;
    s->round_held = held;
    for (int64_t i = 0; i < cnt; ++i) {
      s->used -= reqs[i]->ws;
      reqs[i]->ws = 0;
    }
    s->peak = std::max(s->peak, s->used);
  }
  for (int64_t i = 0; i < cnt; ++i) {
    std::memset(&reqs[i]->info, 0, sizeof(binv_info));
    reqs[i]->info.rho = hrho[i];
    reqs[i]->info.rho_steps[0] = hrho[i];
    reqs[i]->info.refine_steps = hsteps[i];
    reqs[i]->info.converged = hrho[i] <= reqs[i]->target;
    if (e != BINV_OK) finish(s, reqs[i], e, err);
    else if (hinfo[i] != 0)
      finish(s, reqs[i], BINV_E_SINGULAR, "exactly-zero pivot at row " + std::to_string(hinfo[i]));
    else if (!reqs[i]->info.converged)
      finish(s, reqs[i], BINV_E_NOCONVERGE, "rho " + std::to_string(hrho[i]) + " above the request's target");
    else finish(s, reqs[i], BINV_OK, "");
  }
}

// Admission runs on its own thread, so that a round waiting for the device
// (its launches queue behind the workers' full-device grids) never holds up
// the admission of the workers' next requests.
void scheduler_main(binv_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (!s->stop) {
    admit_locked(s);
    s->cv.wait_for(lk, std::chrono::microseconds(200));
  }
}

// Rounds: everything admitted for the shared launches since the last round.
void rounds_main(binv_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    s->rcv.wait(lk, [&] { return s->stop || !s->small_ready.empty(); });
    if (s->small_ready.empty()) break;  // stopping, nothing left
    std::vector<Request*> round;
    round.swap(s->small_ready);
    if ((int)round.size() > kMaxRoundSmall) {
      s->small_ready.assign(round.begin() + kMaxRoundSmall, round.end());
      round.resize(kMaxRoundSmall);
    }
    for (Request* r : round) r->state = Q_RUNNING;
    s->round_running = true;
    lk.unlock();
    run_small_round(s, round);
    lk.lock();
    s->round_running = false;
    s->cv.notify_all();  // the round's reservations are released: admission may proceed
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
      // worker 0 takes large orders first; every worker takes mid orders
      auto ready = [&] { return !s->mid_ready.empty() || (w == 0 && !s->big_ready.empty()); };
      s->wcv.wait(lk, [&] { return s->stop || ready(); });
      if (s->stop && !ready()) break;
      std::deque<Request*>& q = (w == 0 && !s->big_ready.empty()) ? s->big_ready : s->mid_ready;
      r = q.front();
      q.pop_front();
      r->state = Q_RUNNING;
      s->worker_busy[w] = true;
    }
    binv_status e;
    std::memset(&r->info, 0, sizeof(binv_info));
    binv_opts o;
    std::memset(&o, 0, sizeof(o));
    o.block = r->n >= 2048 ? 512 : (r->n >= 512 ? 256 : 128);
    // lookahead (the pivot chain on a side stream) for the large lane only;
    // mid-size sweeps overlap each other instead
    o.flags = BINV_F_SYNC | (r->n < kBigN ? BINV_F_NO_LOOKAHEAD : 0u);
    // Every request ends with the FP64 residual check against its target
    // (the random-probe estimate unless BINV_SERVER_FULL_CHECK) and is refined
    // only if the check fails.  An FP64 request starts from the FP64 sweep.  A mixed
    // request starts from the FP32 sweep when its target is within that
    // sweep's reach or the server honours tags strictly; otherwise one
    // Newton-Schulz step (two FP64 GEMMs of the sweep's size) would cost more
    // than the FP64 sweep it saves, so it starts from the FP64 sweep too.
    const bool fp32_start = r->prec == BINV_PREC_MIXED_F32 &&
                            ((s->flags & BINV_SERVER_STRICT_PRECISION) || r->target >= kFp32Reach);
    if (!fp32_start) o.flags |= BINV_F_REFINE_FROM_FP64;
    if (!(s->flags & BINV_SERVER_FULL_CHECK)) o.flags |= BINV_F_SAMPLED_CHECK;
    e = binv_invert_mixed(s->wctx[w], r->n, r->dA, r->n, r->dX, r->n, &o, kCheckMargin * r->target, -1, st,
                          &r->info);
    r->info.converged = r->info.rho <= r->target;
    // the check asked for a margin below the target; only a result above the
    // request's own target is reported as not converged
    if (e == BINV_E_NOCONVERGE && r->info.converged) e = BINV_OK;
    r->fp32_start = fp32_start;
    {
      // the context keeps the workspace it grew to: charged from now on in
      // place of the request's reservation
      const size_t held = binv::ctx_device_bytes(s->wctx[w]);
      std::lock_guard<std::mutex> g(s->mu);
      s->used += held;
      s->used -= s->ws_held[w] + r->ws;
      s->ws_held[w] = held;
      r->ws = 0;
      s->worker_busy[w] = false;
      s->peak = std::max(s->peak, s->used);
    }
    finish(s, r, e, e == BINV_OK ? "" : binv_last_error());
  }
  if (st) (void)hipStreamDestroy(st);
}

}  // namespace

extern "C" {

binv_status binv_server_create(int device, size_t hbm_budget_bytes, int32_t max_inflight, uint32_t flags,
                               binv_server** out) {
  if (!out) return sfail(BINV_E_INVALID, "out is NULL");
  *out = nullptr;
  if (hbm_budget_bytes == 0) return sfail(BINV_E_INVALID, "zero HBM budget");
  binv_server* s = new (std::nothrow) binv_server();
  if (!s) return sfail(BINV_E_NOMEM, "out of host memory");
  s->device = device;
  s->budget = hbm_budget_bytes;
  s->max_inflight = max_inflight > 0 ? max_inflight : 1 << 20;
  s->flags = flags;
  if (hipSetDevice(device) != hipSuccess || hipStreamCreateWithFlags(&s->rstream, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&s->cstream, hipStreamNonBlocking) != hipSuccess) {
    if (s->rstream) (void)hipStreamDestroy(s->rstream);
    delete s;
    return sfail(BINV_E_HIP, "cannot use the device");
  }
  if (const char* e = getenv("BINV_SERVER_WORKERS")) {
    const int v = atoi(e);
    if (v >= 1 && v <= kMaxWorkers) s->nworkers = v;
  }
  for (int w = 0; w < s->nworkers; ++w) {
    binv_status st = binv_create(&s->wctx[w], device);
    if (st != BINV_OK) {
      for (int v = 0; v < w; ++v) binv_destroy(s->wctx[v]);
      (void)hipStreamDestroy(s->rstream);
      (void)hipStreamDestroy(s->cstream);
      delete s;
      return st;
    }
    // the lookahead of the large lane runs on unmasked streams: the other
    // workers' requests fill every CU, so CUs reserved for one request's pivot
    // chain would only be taken from the mix (measured: 385 against 423
    // solves/s at saturation)
    s->wctx[w]->cu_mask = false;
  }
  s->sched = std::thread(scheduler_main, s);
  s->rounds = std::thread(rounds_main, s);
  for (int w = 0; w < s->nworkers; ++w) s->workers.emplace_back(worker_main, s, w);
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
  const bool fp32_start = prec == BINV_PREC_MIXED_F32 &&
                          ((s->flags & BINV_SERVER_STRICT_PRECISION) || r->target >= kFp32Reach);
  r->blk = block_bytes(n);
  r->ws = workspace_bytes(n, fp32_start);
  if (r->blk + r->ws > s->budget) {
    delete r;
    return sfail(BINV_E_NOMEM, "request alone exceeds the server's HBM budget");
  }
  const size_t nn = (size_t)n * (size_t)n;
  if (a_is_device) {
    // device input: copy it straight into the request's device state when the
    // budget has room now (charged at once), else stage it in host memory
    bool reserved = false;
    {
      std::lock_guard<std::mutex> g(s->mu);
      // only when the queue is empty: a device input must not overtake
      // requests waiting for room
      reserved = s->queue.empty() && make_room_locked(s, r) && request_alloc_locked(s, r);
    }
    if (reserved) {
      hipError_t e = copy_sync(s, r->dA, A, sizeof(double) * nn, hipMemcpyDeviceToDevice);
      if (e == hipSuccess) {
        r->on_device = true;
      } else {
        (void)hipGetLastError();
        std::lock_guard<std::mutex> g(s->mu);
        request_release_locked(s, r);
        const bool fp32 = prec == BINV_PREC_MIXED_F32 &&
                          ((s->flags & BINV_SERVER_STRICT_PRECISION) || r->target >= kFp32Reach);
        r->ws = workspace_bytes(n, fp32);
      }
    }
  }
  if (!r->on_device) {
    try {
      r->hostA.resize(nn);
    } catch (...) {
      delete r;
      return sfail(BINV_E_NOMEM, "out of host memory for staging");
    }
    hipError_t e = a_is_device ? copy_sync(s, r->hostA.data(), A, sizeof(double) * nn, hipMemcpyDeviceToHost)
                               : hipSuccess;
    if (!a_is_device) std::memcpy(r->hostA.data(), A, sizeof(double) * nn);
    if (e != hipSuccess) {
      delete r;
      return sfail(BINV_E_HIP, std::string("copy of A: ") + hipGetErrorString(e));
    }
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
  if (st != BINV_OK) binv::set_error(r->error);
  if ((st == BINV_OK || st == BINV_E_NOCONVERGE) && X) {
    const size_t nn = (size_t)r->n * (size_t)r->n;
    hipError_t e = copy_sync(s, X, r->dX, sizeof(double) * nn, x_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost);
    if (e != hipSuccess) st = sfail(BINV_E_HIP, std::string("copy of X: ") + hipGetErrorString(e));
  }
  if (info) *info = r->info;
  if (times) {
    times->queue_ms = (r->t_admit - r->t_submit) * 1e3;
    times->total_ms = (r->t_done - r->t_submit) * 1e3;
  }
  {
    std::lock_guard<std::mutex> g(s->mu);
    request_release_locked(s, r);
    s->cv.notify_all();
  }
  delete r;
  return st;
}

binv_status binv_next_done(binv_server* s, int64_t wait_us, uint64_t* ticket) {
  if (!s || !ticket) return sfail(BINV_E_INVALID, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  auto pop = [&]() -> bool {
    while (!s->done_q.empty()) {
      const uint64_t t = s->done_q.front();
      s->done_q.pop_front();
      if (s->all.count(t)) {  // not collected yet
        *ticket = t;
        return true;
      }
    }
    return false;
  };
  if (pop()) return BINV_OK;
  if (wait_us > 0) {
    const auto until = std::chrono::steady_clock::now() + std::chrono::microseconds(wait_us);
    while (!s->stop && std::chrono::steady_clock::now() < until) {
      s->dcv.wait_until(lk, until);
      if (pop()) return BINV_OK;
    }
  }
  return BINV_E_BUSY;
}

binv_status binv_server_stats(binv_server* s, size_t* used, size_t* peak, int64_t* completed) {
  if (!s) return sfail(BINV_E_INVALID, "server is NULL");
  std::lock_guard<std::mutex> g(s->mu);
  if (used) *used = s->used;
  if (peak) *peak = s->peak;
  if (completed) *completed = s->completed.load();
  return BINV_OK;
}

binv_status binv_server_destroy(binv_server* s) {
  if (!s) return BINV_OK;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    s->cv.notify_all();
    s->rcv.notify_all();
    s->wcv.notify_all();
    s->dcv.notify_all();
  }
  if (s->sched.joinable()) s->sched.join();
  if (s->rounds.joinable()) s->rounds.join();
  for (auto& t : s->workers)
    if (t.joinable()) t.join();
  for (auto& kv : s->all) {
    Request* r = kv.second;
    if (r->dA) (void)hipFree(r->dA);
    delete r;
  }
  for (auto& kv : s->pool) (void)hipFree(kv.second);
  for (int w = 0; w < s->nworkers; ++w) binv_destroy(s->wctx[w]);
  for (binv::DevBuf* d : {&s->rA, &s->rX, &s->rmats, &s->rorder, &s->rbounds, &s->rinfo, &s->rwork, &s->rtarget,
                          &s->rrho, &s->rsteps, &s->rsw, &s->rjobs})
    d->release();
  if (s->rstream) (void)hipStreamDestroy(s->rstream);
  if (s->cstream) (void)hipStreamDestroy(s->cstream);
  delete s;
  return BINV_OK;
}

}  // extern "C"
