// C ABI of the batched inversion (binv_batch_*; declared in include/binv.h).
//
// A plan fixes the orders and diagonal-block partitions of a batch of small
// matrices packed back to back.  Matrices of order <= 192 go to one of six
// register-resident tiers (k_small_inverse: one pass, pivoting restricted to
// each diagonal block); orders 193..256 are swept block by block, one launch
// per step and shape class with one workgroup per matrix doing the whole step
// (k_swept_step: pivot leaf, row panel, column-panel copy, Schur update), the
// same Eq. (a) step as the single-matrix path.  All
// job tables live on the device, so a run is a fixed sequence of launches that
// is captured once into a HIP graph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "binv_internal.h"

namespace {

constexpr int kSmallTiers = binv::kSmallTierCount;
constexpr int kBlockMax = 128;  // largest diagonal block of the swept tier

binv_status bfail(binv_status st, const std::string& msg) {
  binv::set_error(msg);
  return st;
}

#define BHIP(expr)                                                                      \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return bfail(BINV_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <class T>
binv_status upload(const std::vector<T>& h, void** d) {
  *d = nullptr;
  if (h.empty()) return BINV_OK;
  if (hipMalloc(d, sizeof(T) * h.size()) != hipSuccess) {
    *d = nullptr;
    return bfail(BINV_E_NOMEM, "hipMalloc for the batch plan failed");
  }
  BHIP(hipMemcpy(*d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice));
  return BINV_OK;
}

}  // namespace

// One step of the swept tier: the jobs of all matrices that have a block s.
struct SweptStep {
  int64_t first = 0, count = 0;  // range in the per-step job arrays
  int bmax = 0, mmax = 0;
  // jobs are ordered by pivot-block order, largest first, in two shape
  // classes: cls[0] with blocks > 64, cls[1] with blocks <= 64
  int64_t cls[2] = {0, 0};
  double row_flops = 0, schur_flops = 0;  // algorithmic flops of the step's GEMMs
  double leaf_flops = 0;                  // 2 b^3 per pivot block
};

struct binv_batch {
  binv_ctx* ctx = nullptr;
  int device = 0;
  int64_t count = 0;
  int64_t total = 0;      // packed elements
  double flops = 0;       // 2 sum m^3
  std::vector<int64_t> off;
  std::vector<int32_t> m;
  // small tiers
  int64_t tier_first[kSmallTiers] = {0}, tier_count[kSmallTiers] = {0};
  int variant[kSmallTiers] = {0};  // launch shape per tier (autotuned)
  double tier_flops[kSmallTiers] = {0};  // 2 sum m^3 per tier
  void* d_mats = nullptr;    // SmallMat per matrix (all matrices)
  void* d_order = nullptr;   // matrix indices grouped by tier
  void* d_bounds = nullptr;  // diagonal-block boundaries
  // swept tier (orders 193..256)
  std::vector<SweptStep> steps;
  std::vector<int32_t> swept;     // matrix indices
  std::vector<int64_t> ws_off;    // workspace offset (elements) per swept matrix
  int64_t ws_elems = 0;
  void* d_ws = nullptr;
  // job tables are built per (A, X, info) binding; rebuilt when they change
  const void* bound_A = nullptr;
  void* bound_X = nullptr;
  void* bound_info = nullptr;
  void* d_jobs = nullptr;  // SweptJob per (step, swept matrix)
  // graph of the whole run for the current binding
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;
  std::vector<int32_t> bounds_host;
  std::vector<int32_t> bnd_index;
  // the paper's level scheme (binv_invert_batched_levels): matrices grouped
  // by tier (orders <= 8, 16, 32, 64), formed on its first call
  bool lvl_ready = false;
  int64_t lvl_first[binv::kLevelClasses] = {0}, lvl_count[binv::kLevelClasses] = {0};
  size_t lvl_lds[binv::kLevelClasses] = {0};    // each class launch's dynamic LDS (doubles)
  double lvl_flops[binv::kLevelClasses] = {0};  // the scheme's own flops per class
  void* d_lvl_order = nullptr;
};

namespace {

void free_bindings(binv_batch* b) {
  if (b->d_jobs) (void)hipFree(b->d_jobs);
  b->d_jobs = nullptr;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->bound_A = nullptr;
  b->bound_X = nullptr;
  b->bound_info = nullptr;
}

// Build the per-step job table of the swept tier for buffers (A, X, info):
// one job per (step, matrix), each step's jobs ordered by pivot-block order,
// largest first, so that the two shape classes (> 64, <= 64) are contiguous.
binv_status bind(binv_batch* b, const double* A, double* X, int32_t* info) {
  free_bindings(b);
  std::vector<binv::SweptJob> jobs;
  double* ws = (double*)b->d_ws;
  for (size_t s = 0; s < b->steps.size(); ++s) {
    const size_t first = jobs.size();
    for (size_t t = 0; t < b->swept.size(); ++t) {
      const int i = b->swept[t];
      const int mi = b->m[i];
      const int bi = b->bnd_index[i];
      const int nb = b->bnd_index[i + 1] - bi - 1;
      if ((int)s >= nb) continue;
      const int o = b->bounds_host[bi + s];
      const int bs = b->bounds_host[bi + s + 1] - o;
      const double* Win = (s == 0 ? A : (const double*)X) + b->off[i];
      double* Wout = X + b->off[i];
      double* P = ws + b->ws_off[t];
      double* Ct = P + kBlockMax * kBlockMax;
      double* R = Ct + (int64_t)kBlockMax * mi;
      binv::SweptJob j;
      std::memset(&j, 0, sizeof(j));
      j.leaf.A = Win + (int64_t)o * mi + o; j.leaf.lda = mi; j.leaf.P = P; j.leaf.ldp = bs; j.leaf.b = bs;
      j.leaf.row0 = o; j.leaf.info = info + i;
      binv::StepArgs& ra = j.row;
      ra.A = P; ra.lda = bs; ra.B = Win + (int64_t)o * mi; ra.ldb = mi; ra.W = R; ra.ldw = mi;
      ra.R = P; ra.ldr = bs; ra.M = bs; ra.N = mi; ra.K = bs; ra.o = o; ra.b = bs; ra.oc = o;
      binv::StepArgs& sa = j.schur;
      // the old column panel goes to Ct (m-major, ld = b) before the update
      sa.A = Ct; sa.lda = bs; sa.B = R; sa.ldb = mi; sa.W = Wout; sa.ldw = mi; sa.Win = Win; sa.ldwin = mi;
      sa.R = R; sa.ldr = mi; sa.M = mi; sa.N = mi; sa.K = bs; sa.o = o; sa.b = bs; sa.oc = o;
      jobs.push_back(j);
    }
    std::stable_sort(jobs.begin() + first, jobs.end(),
                     [](const binv::SweptJob& x, const binv::SweptJob& y) { return x.leaf.b > y.leaf.b; });
  }
  binv_status st;
  if ((st = upload(jobs, &b->d_jobs)) != BINV_OK) return st;
  b->bound_A = A;
  b->bound_X = X;
  b->bound_info = info;
  return BINV_OK;
}

// Enqueue the whole batched inversion on stream s.  `timed`: bracket the
// launches with the context's phase timers (never inside a graph capture).
binv_status enqueue(binv_batch* b, const double* A, double* X, int32_t* info, hipStream_t s, bool timed) {
  binv_ctx* c = b->ctx;
  const int lvl = timed ? 0 : 1;  // level != 0 disables the timers
  // every matrix's info word starts at 0; the small tiers overwrite theirs
  BHIP(binv::launch_fill_i32(info, b->count, 0, s));
  for (int t = 0; t < kSmallTiers; ++t) {
    binv::PhaseTimer tm(c, lvl, BINV_PHASE_SMALL, s);
    if (tm.on()) tm.flops = b->tier_flops[t];
    BHIP(binv::launch_small_tier(t, b->variant[t], A, X, (const binv::SmallMat*)b->d_mats,
                                 (const int32_t*)b->d_order + b->tier_first[t], b->tier_count[t],
                                 (const int32_t*)b->d_bounds, info, s));
  }
  for (const SweptStep& st : b->steps) {
    // one workgroup per matrix does the whole step (leaf, row panel, Schur)
    binv::PhaseTimer tm(c, lvl, BINV_PHASE_SCHUR, s);
    if (tm.on()) tm.flops = st.leaf_flops + st.row_flops + st.schur_flops;
    const binv::SweptJob* jobs = (const binv::SweptJob*)b->d_jobs + st.first;
    BHIP(binv::launch_swept_step(jobs, st.cls[0], 128, s));
    BHIP(binv::launch_swept_step(jobs + st.cls[0], st.count - st.cls[0], 64, s));
  }
  return BINV_OK;
}

int count_bucket(int64_t count) {
  int k = 0;
  while (k < 39 && (int64_t(1) << (k + 1)) <= count) ++k;
  return k;
}

}  // namespace

extern "C" {

binv_status binv_batch_create(binv_ctx* ctx, int64_t count, const int32_t* m, const int32_t* k, const int32_t* part,
                              binv_batch** plan) {
  if (!plan) return bfail(BINV_E_INVALID, "plan is NULL");
  *plan = nullptr;
  if (!ctx) return bfail(BINV_E_INVALID, "ctx is NULL");
  if (count < 0 || (count > 0 && !m)) return bfail(BINV_E_INVALID, "bad count or NULL orders");
  binv_batch* b = new (std::nothrow) binv_batch();
  if (!b) return bfail(BINV_E_NOMEM, "out of host memory");
  b->ctx = ctx;
  (void)hipGetDevice(&b->device);
  b->count = count;
  b->off.resize(count);
  b->m.resize(count);
  b->bnd_index.resize(count + 1);
  std::vector<binv::SmallMat> mats(count);
  std::vector<std::vector<int32_t>> tiers(kSmallTiers);
  int64_t off = 0, poff = 0;
  int maxsteps = 0;
  for (int64_t i = 0; i < count; ++i) {
    const int mi = m[i];
    if (mi < 1 || mi > 256) {
      delete b;
      return bfail(BINV_E_INVALID, "matrix order outside 1..256 at index " + std::to_string(i));
    }
    const int ki = k ? k[i] : 1;
    if (ki < 1 || ki > mi) {
      delete b;
      return bfail(BINV_E_INVALID, "block count outside 1..m at index " + std::to_string(i));
    }
    b->off[i] = off;
    b->m[i] = mi;
    b->bnd_index[i] = (int32_t)b->bounds_host.size();
    // diagonal blocks: given orders, or floor(m/k) with the remainder on the last blocks
    std::vector<int> ord(ki);
    if (part) {
      int64_t sum = 0;
      for (int j = 0; j < ki; ++j) {
        ord[j] = part[poff + j];
        if (ord[j] < 1) {
          delete b;
          return bfail(BINV_E_INVALID, "non-positive block order at index " + std::to_string(i));
        }
        sum += ord[j];
      }
      poff += ki;
      if (sum != mi) {
        delete b;
        return bfail(BINV_E_INVALID, "block orders do not sum to m at index " + std::to_string(i));
      }
    } else {
      const int base = mi / ki, rem = mi - base * ki;
      for (int j = 0; j < ki; ++j) ord[j] = base + (j >= ki - rem ? 1 : 0);
    }
    // the swept tier needs blocks of at most 128: split larger ones in halves
    std::vector<int> fin;
    for (int x : ord) {
      if (mi > binv::kSmallMaxOrder && x > kBlockMax) {
        const int pieces = (x + kBlockMax - 1) / kBlockMax;
        for (int q = 0; q < pieces; ++q) fin.push_back(x / pieces + (q >= pieces - x % pieces ? 1 : 0));
      } else {
        fin.push_back(x);
      }
    }
    int acc = 0;
    b->bounds_host.push_back(0);
    for (int x : fin) {
      acc += x;
      b->bounds_host.push_back(acc);
    }
    mats[i].off = off;
    mats[i].m = mi;
    mats[i].nb = (int)fin.size();
    mats[i].bnd = b->bnd_index[i];
    mats[i].id = (int)i;
    if (mi <= binv::kSmallMaxOrder) {
      int t = 0;
      while (mi > binv::small_tier_limit(t)) ++t;
      tiers[t].push_back((int32_t)i);
      b->tier_flops[t] += 2.0 * mi * (double)mi * mi;
    } else {
      b->swept.push_back((int32_t)i);
      maxsteps = std::max(maxsteps, (int)fin.size());
    }
    off += (int64_t)mi * mi;
    b->flops += 2.0 * mi * (double)mi * mi;
  }
  b->bnd_index[count] = (int32_t)b->bounds_host.size();
  b->total = off;
  // largest matrices first within each tier
  std::vector<int32_t> order;
  for (int t = 0; t < kSmallTiers; ++t) {
    std::stable_sort(tiers[t].begin(), tiers[t].end(), [&](int32_t x, int32_t y) { return b->m[x] > b->m[y]; });
    b->tier_first[t] = (int64_t)order.size();
    b->tier_count[t] = (int64_t)tiers[t].size();
    const int8_t known = ctx->tuned_small[t][count_bucket(b->tier_count[t])];
    b->variant[t] = known >= 0 ? known : 0;
    order.insert(order.end(), tiers[t].begin(), tiers[t].end());
  }
  std::stable_sort(b->swept.begin(), b->swept.end(), [&](int32_t x, int32_t y) { return b->m[x] > b->m[y]; });
  int64_t ws = 0;
  for (int32_t i : b->swept) {
    b->ws_off.push_back(ws);
    ws += (int64_t)kBlockMax * kBlockMax + 2LL * kBlockMax * b->m[i];
  }
  b->ws_elems = ws;
  int64_t first = 0;
  for (int s = 0; s < maxsteps; ++s) {
    SweptStep st;
    st.first = first;
    for (int32_t i : b->swept) {
      const int bi = b->bnd_index[i];
      const int nb = b->bnd_index[i + 1] - bi - 1;
      if (s < nb) {
        ++st.count;
        const int bs = b->bounds_host[bi + s + 1] - b->bounds_host[bi + s];
        const double mi = b->m[i];
        st.bmax = std::max(st.bmax, bs);
        st.mmax = std::max(st.mmax, b->m[i]);
        st.cls[bs > 64 ? 0 : 1]++;
        st.row_flops += 2.0 * bs * (double)bs * (mi - bs);
        st.leaf_flops += 2.0 * bs * (double)bs * bs;
        st.schur_flops += 2.0 * bs * (mi - bs) * mi;
      }
    }
    first += st.count;
    b->steps.push_back(st);
  }
  binv_status st;
  if ((st = upload(mats, &b->d_mats)) != BINV_OK || (st = upload(order, &b->d_order)) != BINV_OK ||
      (st = upload(b->bounds_host, &b->d_bounds)) != BINV_OK) {
    binv_batch_destroy(b);
    return st;
  }
  if (ws > 0 && hipMalloc(&b->d_ws, sizeof(double) * (size_t)ws) != hipSuccess) {
    b->d_ws = nullptr;
    binv_batch_destroy(b);
    return bfail(BINV_E_NOMEM, "hipMalloc of the batch workspace failed");
  }
  *plan = b;
  return BINV_OK;
}

binv_status binv_batch_destroy(binv_batch* b) {
  if (!b) return BINV_OK;
  if (b->cap) (void)hipStreamSynchronize(b->cap);
  free_bindings(b);
  for (void* p : {b->d_mats, b->d_order, b->d_bounds, b->d_ws, b->d_lvl_order})
    if (p) (void)hipFree(p);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
  return BINV_OK;
}

binv_status binv_batch_query(const binv_batch* b, int64_t* count, int64_t* total_elems, double* flops) {
  if (!b) return bfail(BINV_E_INVALID, "plan is NULL");
  if (count) *count = b->count;
  if (total_elems) *total_elems = b->total;
  if (flops) *flops = b->flops;
  return BINV_OK;
}

binv_status binv_invert_batched(binv_batch* b, const double* A, double* X, int32_t* d_info, uint32_t flags,
                                void* stream) {
  if (!b) return bfail(BINV_E_INVALID, "plan is NULL");
  if (b->count == 0) return BINV_OK;
  if (!A || !X || !d_info) return bfail(BINV_E_INVALID, "A, X and d_info must be device pointers");
  if (A != X) {
    const char* a0 = (const char*)A;
    const char* a1 = (const char*)(A + b->total);
    const char* x0 = (const char*)X;
    const char* x1 = (const char*)(X + b->total);
    if (a0 < x1 && x0 < a1) return bfail(BINV_E_INVALID, "A and X overlap without being the same buffer");
  }
  hipStream_t s = (hipStream_t)stream;
  if (b->bound_A != A || b->bound_X != X || b->bound_info != d_info) {
    binv_status st = bind(b, A, X, d_info);
    if (st != BINV_OK) return st;
  }
  if (flags & BINV_F_GRAPH) {
    if (!b->exec) {
      if (!b->cap) BHIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
      BHIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
      binv_status st = enqueue(b, A, X, d_info, b->cap, false);
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(b->cap, &g);
      if (st != BINV_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
      }
      if (e != hipSuccess) return bfail(BINV_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
      b->graph = g;
      BHIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    }
    BHIP(hipGraphLaunch(b->exec, s));
  } else {
    binv_status st = enqueue(b, A, X, d_info, s, true);
    if (st != BINV_OK) return st;
  }
  if (flags & BINV_F_SYNC) BHIP(hipStreamSynchronize(s));
  return BINV_OK;
}

binv_status binv_level_partition(int32_t m, int32_t capacity, int32_t* k, int32_t* part) {
  if (m < 1 || !k) return bfail(BINV_E_INVALID, "order must be positive and k not NULL");
  int nk = 1;
  if (m >= 4) {
    int lg = 0;
    while ((2 << lg) <= m) ++lg;  // floor(log2 m)
    nk = 1 << (lg - 1);
  }
  *k = nk;
  if (!part) return BINV_OK;
  if (capacity < nk) return bfail(BINV_E_INVALID, "part holds fewer entries than the block count");
  const int q = m / nk, r = m - q * nk;
  for (int i = 0; i < nk; ++i) part[i] = q + (i >= nk - r ? 1 : 0);
  return BINV_OK;
}

binv_status binv_invert_batched_levels(binv_batch* b, const double* A, double* X, int32_t* d_info, uint32_t flags,
                                       void* stream) {
  if (!b) return bfail(BINV_E_INVALID, "plan is NULL");
  if (flags & ~(BINV_F_SYNC | BINV_F_GRAPH)) return bfail(BINV_E_INVALID, "unknown flags");
  if (b->count == 0) return BINV_OK;
  if (!A || !X || !d_info) return bfail(BINV_E_INVALID, "A, X and d_info must be device pointers");
  if (A != X) {
    const char* a0 = (const char*)A;
    const char* a1 = (const char*)(A + b->total);
    const char* x0 = (const char*)X;
    const char* x1 = (const char*)(X + b->total);
    if (a0 < x1 && x0 < a1) return bfail(BINV_E_INVALID, "A and X overlap without being the same buffer");
  }
  if (!b->lvl_ready) {
    constexpr int NC = binv::kLevelClasses;
    std::vector<int32_t> classes[NC];
    for (int64_t i = 0; i < b->count; ++i) {
      const int mi = b->m[i];
      const int bi = b->bnd_index[i];
      const int nk = b->bnd_index[i + 1] - bi - 1;
      const std::string at = " (matrix " + std::to_string(i) + ")";
      if (mi > binv::level_class_limit(NC - 1)) return bfail(BINV_E_INVALID, "the level scheme takes orders <= 64" + at);
      if (nk & (nk - 1)) return bfail(BINV_E_INVALID, "the block count must be a power of two" + at);
      for (int j = 0; j < nk; ++j)
        if (b->bounds_host[bi + j + 1] - b->bounds_host[bi + j] > 4)
          return bfail(BINV_E_INVALID, "the level scheme's diagonal blocks have orders <= 4" + at);
      int c = 0;
      while (mi > binv::level_class_limit(c)) ++c;
      // M_inv (its top-level diagonal squares where the class splits it)
      // and the provisional sets (every level-l unit's square)
      const int ha = (binv::level_class_split(c) && nk >= 2) ? b->bounds_host[bi + nk / 2] - b->bounds_host[bi] : mi;
      size_t need = (size_t)ha * ha + (size_t)(mi - ha) * (mi - ha);
      double fl = 0.0;
      for (int j = 0; j < nk; ++j) {
        const double bj = b->bounds_host[bi + j + 1] - b->bounds_host[bi + j];
        fl += 2.0 * bj * bj * bj * nk;  // one closed-form inverse per block and ◊ step (N_k of them)
      }
      for (int l = 1; (1 << l) <= nk; ++l)
        for (int v = 0; v < (nk >> l); ++v) {
          const int u0 = b->bounds_host[bi + (v << l)];
          const int uh = b->bounds_host[bi + (v << l) + (1 << (l - 1))];
          const int u1 = b->bounds_host[bi + ((v + 1) << l)];
          need += (size_t)(u1 - u0) * (u1 - u0);
          // per unit: →, ← and ∼ 4 na nd (na + nd), ↑↓ 2 na nd (na + nd),
          // once per inversion of the matrices containing the unit
          const double na = uh - u0, nd = u1 - uh;
          fl += 6.0 * na * nd * (na + nd) * (double)(nk >> l);
        }
      if (need > binv::kLevelLdsDoubles)
        return bfail(BINV_E_INVALID, "the inverse's diagonal squares and provisional sets exceed the on-chip store" + at);
      classes[c].push_back((int32_t)i);
      b->lvl_flops[c] += fl;
      b->lvl_lds[c] = std::max(b->lvl_lds[c], need);
    }
    std::vector<int32_t> order;
    for (int c = 0; c < NC; ++c) {
      b->lvl_first[c] = (int64_t)order.size();
      b->lvl_count[c] = (int64_t)classes[c].size();
      order.insert(order.end(), classes[c].begin(), classes[c].end());
    }
    binv_status st = upload(order, &b->d_lvl_order);
    if (st != BINV_OK) return st;
    b->lvl_ready = true;
  }
  hipStream_t s = (hipStream_t)stream;
  for (int c = 0; c < binv::kLevelClasses; ++c) {
    binv::PhaseTimer tm(b->ctx, 0, BINV_PHASE_SMALL, s);
    if (tm.on()) tm.flops = b->lvl_flops[c];
    BHIP(binv::launch_level_class(c, A, X, (const binv::SmallMat*)b->d_mats,
                                  (const int32_t*)b->d_lvl_order + b->lvl_first[c], b->lvl_count[c], b->lvl_lds[c],
                                  (const int32_t*)b->d_bounds, d_info, s));
  }
  if (flags & BINV_F_SYNC) BHIP(hipStreamSynchronize(s));
  return BINV_OK;
}

binv_status binv_batch_tune(binv_batch* b, const double* A, double* X, int32_t* d_info, int32_t reps, void* stream,
                            int32_t* chosen, double* ms) {
  if (!b) return bfail(BINV_E_INVALID, "plan is NULL");
  if (reps < 1) return bfail(BINV_E_INVALID, "reps must be at least 1");
  if (chosen)
    for (int t = 0; t < kSmallTiers; ++t) chosen[t] = -1;
  if (ms)
    for (int i = 0; i < kSmallTiers * binv::kSmallVariants; ++i) ms[i] = 0.0;
  if (b->count == 0) return BINV_OK;
  if (!A || !X || !d_info) return bfail(BINV_E_INVALID, "A, X and d_info must be device pointers");
  if (A == X) return bfail(BINV_E_INVALID, "tuning needs X separate from A (every shape reruns the batch)");
  {
    const char* a0 = (const char*)A;
    const char* a1 = (const char*)(A + b->total);
    const char* x0 = (const char*)X;
    const char* x1 = (const char*)(X + b->total);
    if (a0 < x1 && x0 < a1) return bfail(BINV_E_INVALID, "A and X overlap");
  }
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  BHIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return bfail(BINV_E_HIP, "hipEventCreate failed");
  }
  binv_status st = BINV_OK;
  for (int t = 0; t < kSmallTiers && st == BINV_OK; ++t) {
    if (b->tier_count[t] == 0) continue;
    int best = 0;
    double best_ms = 1e300;
    for (int v = 0; v < binv::small_variant_count(t) && st == BINV_OK; ++v) {
      double vbest = 1e300;
      for (int r = 0; r <= reps && st == BINV_OK; ++r) {  // launch 0 warms up
        hipError_t e = hipEventRecord(e0, s);
        if (e == hipSuccess)
          e = binv::launch_small_tier(t, v, A, X, (const binv::SmallMat*)b->d_mats,
                                      (const int32_t*)b->d_order + b->tier_first[t], b->tier_count[t],
                                      (const int32_t*)b->d_bounds, d_info, s);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float f = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&f, e0, e1);
        if (e != hipSuccess) {
          st = bfail(BINV_E_HIP, std::string("tuning launch: ") + hipGetErrorString(e));
          break;
        }
        if (r > 0) vbest = std::min(vbest, (double)f);
      }
      if (ms) ms[t * binv::kSmallVariants + v] = vbest;
      if (vbest < best_ms) {
        best_ms = vbest;
        best = v;
      }
    }
    if (st != BINV_OK) break;
    b->variant[t] = best;
    b->ctx->tuned_small[t][count_bucket(b->tier_count[t])] = (int8_t)best;
    if (chosen) chosen[t] = best;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != BINV_OK) return st;
  // the captured graph holds the old shapes
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  // leave X and d_info holding a complete inversion with the chosen shapes
  return binv_invert_batched(b, A, X, d_info, BINV_F_SYNC, stream);
}

binv_status binv_batch_residual(binv_batch* b, const double* A, const double* X, double* d_rho, void* stream) {
  if (!b) return bfail(BINV_E_INVALID, "plan is NULL");
  if (b->count == 0) return BINV_OK;
  if (!A || !X || !d_rho) return bfail(BINV_E_INVALID, "A, X and d_rho must be device pointers");
  // norm only: X is read, never written (no workspace)
  BHIP(binv::launch_small_refine(A, const_cast<double*>(X), (const binv::SmallMat*)b->d_mats, nullptr, b->count,
                                 nullptr, 0.0, nullptr, 0, d_rho, nullptr, (hipStream_t)stream));
  return BINV_OK;
}

binv_status binv_batch_shape(int32_t tier, int32_t shape, int32_t out[4]) {
  if (tier < 0 || tier >= kSmallTiers || shape < 0 || shape >= binv::small_variant_count(tier) || !out)
    return bfail(BINV_E_INVALID, "tier or shape out of range");
  int sh[4];
  binv::small_variant_shape(tier, shape, sh);
  for (int i = 0; i < 4; ++i) out[i] = sh[i];
  return BINV_OK;
}

}  // extern "C"
