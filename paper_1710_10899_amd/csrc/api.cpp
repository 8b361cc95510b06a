// C-ABI layer: plan cache, size buckets, chunked workspace, launch
// sequences, hipGraph capture and replay, status counters, phase timing.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstddef>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <tuple>
#include <vector>

#include "../../include/submat.h"
#include "autotune.hpp"
#include "kernels.hpp"
#include "krylov.hpp"

using namespace submat;

namespace {

// ------------------------------------------------------------------ options
struct Options {
  double kappa_max = 1e5;
  int use_graph = 1;
  int small_max = 0;       // one-wavefront bucket edge set by the caller (0: the tuning table's)
  double ws_bytes = 0.0;
  double cluster_tol = 1e-7;
  int deterministic = 0;   // adjoint assembled in a fixed order instead of by atomic adds
  int plain_stride = 1;    // the per-column path computes every plain_stride-th column only
  int xcd_queues = 1;      // unit launches take their work from one queue per XCD
  uint64_t tune_gen = 0;   // bumped whenever the tuning table is reloaded
};
Options g_opt;
std::mutex g_mu;

#define HIP_TRY(expr)                      \
  do {                                     \
    hipError_t _e = (expr);                \
    if (_e != hipSuccess) return SUBMAT_EHIP; \
  } while (0)

template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  ~DevBuf() { if (p) (void)hipFree(p); }
  int alloc(size_t count) {
    if (p) { (void)hipFree(p); p = nullptr; }
    n = count;
    if (count == 0) return SUBMAT_OK;
    if (hipMalloc((void**)&p, count * sizeof(T)) != hipSuccess) { p = nullptr; (void)hipGetLastError(); return SUBMAT_ENOMEM; }
    return SUBMAT_OK;
  }
};

// --------------------------------------------------------------- device ctx
struct DeviceCtx {
  int device = -1;
  int num_cus = 0;
  int lds_limit = 65536;
  // status counters (ST_NSLOTS int64 slots) per stream: a call resets and
  // fills the block of the stream it runs on
  std::map<uintptr_t, std::unique_ptr<DevBuf<int64_t>>> status;
  rocblas_handle blas = nullptr;  // dense products of the refinement, created on first use
  ~DeviceCtx() {
    if (blas) (void)rocblas_destroy_handle(blas);
  }
};
std::map<int, std::unique_ptr<DeviceCtx>> g_dev;

// Streams whose last call was the forward that allocates nothing: its
// status slots are in that entry point's scratch (device, stream -> address).
std::map<std::pair<int, uintptr_t>, int64_t*> g_noalloc_status;

// Status block of `stream` on this device, allocated (and zeroed) on first use.
int stream_status(DeviceCtx* ctx, hipStream_t stream, int64_t** out) {
  auto& slot = ctx->status[(uintptr_t)stream];
  if (!slot) {
    auto b = std::make_unique<DevBuf<int64_t>>();
    int rc = b->alloc(ST_NSLOTS);
    if (rc) return rc;
    HIP_TRY(hipMemset(b->p, 0, ST_NSLOTS * sizeof(int64_t)));
    slot = std::move(b);
  }
  *out = slot->p;
  return SUBMAT_OK;
}

int get_ctx(DeviceCtx** out);

// The status block a query on `stream` reads: the no-alloc entry point's
// scratch when that was the stream's last call, else the stream's own.
int status_for_query(DeviceCtx* ctx, hipStream_t stream, int64_t** out) {
  auto it = g_noalloc_status.find({ctx->device, (uintptr_t)stream});
  if (it != g_noalloc_status.end()) {
    *out = it->second;
    return SUBMAT_OK;
  }
  return stream_status(ctx, stream, out);
}

int get_ctx(DeviceCtx** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  auto it = g_dev.find(dev);
  if (it == g_dev.end()) {
    auto ctx = std::make_unique<DeviceCtx>();
    ctx->device = dev;
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    ctx->num_cus = prop.multiProcessorCount;
    ctx->lds_limit = (int)prop.sharedMemPerBlock;
    it = g_dev.emplace(dev, std::move(ctx)).first;
  }
  *out = it->second.get();
  return SUBMAT_OK;
}

// --------------------------------------------------------------------- plan
// Scratch bytes per large item: the eigensolver's two FP64 ld x ld arrays,
// or the back-transformation's blocks (sized in FP64 for both precisions).
int64_t scratch_bytes(int ld) {
  const int64_t eig = 2 * (int64_t)ld * ld, back = (int64_t)apply_scratch_elems(ld);
  return 8 * (eig > back ? eig : back);
}

struct Chunk {
  int start = 0, count = 0, max_m = 0;
  int64_t slab_bytes = 0;   // S (and Q, W) bytes for this chunk
  int64_t vec_bytes = 0;    // per vector array
  int64_t escr_bytes = 0;   // eigensolver scratch
};

struct GraphEntry {
  std::vector<uintptr_t> key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint64_t stamp = 0;
};

// Device memory one stream's calls on a plan work in: slabs, vectors and
// scratch of one chunk, per-item flags, work counters, and the graphs
// captured for that stream. Calls on different streams never share one.
struct Workspace {
  uint64_t last_use = 0;
  DevBuf<char> S, Q, W, dv, ev, tv, escr;
  DevBuf<int32_t> flags;
  DevBuf<int32_t> counters;
  DevBuf<double> dsmall;   // deterministic adjoint: D of the one-wavefront columns
  std::vector<GraphEntry> graphs;
  uint64_t stamp = 0;
  hipStream_t cap_stream = nullptr;
  ~Workspace() {
    for (auto& g : graphs) {
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
      if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
  }
  int64_t bytes() const {
    return (int64_t)(S.n + Q.n + W.n + dv.n + ev.n + tv.n + escr.n) + 4 * (int64_t)(flags.n + counters.n) +
           8 * (int64_t)dsmall.n;
  }
};

struct Plan {
  int device = 0;
  uint64_t last_use = 0;  // plan-cache clock at the last call with this pattern
  const int32_t* rowptr = nullptr;
  const int32_t* colind = nullptr;
  int32_t n = 0;
  int64_t nnz = 0;
  int small_max = 64;
  std::vector<int32_t> h_m;
  DevBuf<int32_t> d_m, d_c;
  DevBuf<int32_t> tpos;   // transpose position of every stored entry (the gather's symmetrisation)
  // buckets (columns, largest m first)
  std::vector<int32_t> small_items, large_items;
  DevBuf<int32_t> d_small, d_large;
  int small_mmax = 0, large_mmax = 0;
  // large-item layout
  DevBuf<int32_t> d_ldm;
  DevBuf<int64_t> d_off, d_voff, d_eoff, d_sqoff, d_sdoff;
  std::vector<int64_t> h_sqoff, h_sdoff;
  std::vector<Chunk> chunks;
  int64_t saved_q_bytes = 0, saved_bytes = 0;
  // workspace sizes (bytes / elements) of one stream
  int64_t ws_slab = 0, ws_vec = 0, ws_escr = 0;
  int max_count = 0;
  int ncounters = 0;
  int64_t small_d_elems = 0;          // sum of m^2 over the one-wavefront columns
  // deterministic adjoint: per column, the phase that computes its D (0 = the
  // one-wavefront launch, 1 + c = large-order chunk c) and where D lies
  // (element offset and leading dimension)
  DevBuf<int32_t> d_dphase, d_dld;
  DevBuf<int64_t> d_doff;
  std::map<uintptr_t, std::unique_ptr<Workspace>> ws;   // by stream
  int64_t bytes() const {
    int64_t b = 4 * (int64_t)(d_m.n + d_c.n + tpos.n + d_small.n + d_large.n + d_ldm.n + d_dphase.n + d_dld.n) +
                8 * (int64_t)(d_off.n + d_voff.n + d_eoff.n + d_sqoff.n + d_sdoff.n + d_doff.n);
    for (auto& w : ws) b += w.second->bytes();
    return b;
  }
};

using PlanKey = std::tuple<int, uintptr_t, uintptr_t, int32_t, int64_t>;
std::map<PlanKey, std::unique_ptr<Plan>> g_plans;

// Saved buffers filled by a forward call: the plan, value type and precision
// they were filled for. A backward call that names a buffer not recorded
// here for its own pattern, type and precision is rejected (SUBMAT_ESAVED).
struct SavedTag {
  PlanKey key;
  int32_t dtype = 0, precision = 0;
};
std::map<uintptr_t, SavedTag> g_saved;

void forget_saved(const PlanKey& key) {
  for (auto it = g_saved.begin(); it != g_saved.end();) {
    if (it->second.key == key) it = g_saved.erase(it);
    else ++it;
  }
}

int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// Plan cache bookkeeping: a use clock for least-recently-used eviction and
// the device bytes a plan and its workspaces hold.
uint64_t g_plan_clock = 0;

int64_t plan_bytes(const Plan& P) { return P.bytes(); }

// Workspaces kept per plan: calls on more streams than this drop the least
// recently used one (freeing waits for the device).
constexpr size_t kMaxWorkspaces = 4;

// Drop cached plans of this device, least recently used first, until the
// others hold at most `keep` bytes (all of them for keep < 0). Freeing
// synchronises the device, so no queued work still uses them.
void evict_plans(int device, int64_t keep) {
  for (;;) {
    int64_t held = 0;
    auto victim = g_plans.end();
    for (auto p = g_plans.begin(); p != g_plans.end(); ++p) {
      if (p->second->device != device) continue;
      held += plan_bytes(*p->second);
      if (victim == g_plans.end() || p->second->last_use < victim->second->last_use) victim = p;
    }
    if (victim == g_plans.end() || (keep >= 0 && held <= keep)) return;
    forget_saved(victim->first);
    g_plans.erase(victim);
  }
}

int build_plan_once(const int32_t* rowptr, const int32_t* colind, int32_t n, int64_t nnz, hipStream_t stream,
                    DeviceCtx* ctx, Plan** out);

// Cached plan for the pattern, built on first use. A new plan's workspace
// is sized from the free device memory after the other plans of the device
// have been trimmed (least recently used first) to a quarter of it; if the
// allocation still fails, every other plan is dropped and the build retried.
int build_plan(const int32_t* rowptr, const int32_t* colind, int32_t n, int64_t nnz, hipStream_t stream,
               DeviceCtx* ctx, Plan** out) {
  PlanKey key{ctx->device, (uintptr_t)rowptr, (uintptr_t)colind, n, nnz};
  auto it = g_plans.find(key);
  if (it != g_plans.end()) {
    it->second->last_use = ++g_plan_clock;
    *out = it->second.get();
    return SUBMAT_OK;
  }
  size_t free_b = 0, total_b = 0;
  HIP_TRY(hipMemGetInfo(&free_b, &total_b));
  evict_plans(ctx->device, (int64_t)(total_b / 4));
  int rc = build_plan_once(rowptr, colind, n, nnz, stream, ctx, out);
  if (rc == SUBMAT_ENOMEM) {
    (void)hipGetLastError();
    evict_plans(ctx->device, -1);
    rc = build_plan_once(rowptr, colind, n, nnz, stream, ctx, out);
  }
  return rc;
}

int build_plan_once(const int32_t* rowptr, const int32_t* colind, int32_t n, int64_t nnz, hipStream_t stream,
                    DeviceCtx* ctx, Plan** out) {
  PlanKey key{ctx->device, (uintptr_t)rowptr, (uintptr_t)colind, n, nnz};
  auto plan = std::make_unique<Plan>();
  Plan& P = *plan;
  P.device = ctx->device;
  P.rowptr = rowptr;
  P.colind = colind;
  P.n = n;
  P.nnz = nnz;
  P.small_max = std::min(64, std::max(1, g_opt.small_max > 0 ? g_opt.small_max : tuned_small_max()));
  int rc;
  if ((rc = P.d_m.alloc(n)) || (rc = P.d_c.alloc(n))) return rc;
  DevBuf<uint32_t> err;
  if ((rc = err.alloc(1))) return rc;
  HIP_TRY(hipMemsetAsync(err.p, 0, sizeof(uint32_t), stream));
  HIP_TRY(launch_plan_pattern(rowptr, colind, n, nnz, P.d_m.p, P.d_c.p, err.p, stream));
  P.h_m.resize(n);
  uint32_t h_err = 0;
  HIP_TRY(hipMemcpyAsync(P.h_m.data(), P.d_m.p, n * sizeof(int32_t), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipMemcpyAsync(&h_err, err.p, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  if (h_err & (PAT_ROWPTR | PAT_RANGE | PAT_ORDER | PAT_ASYM)) return SUBMAT_EPATTERN;
  if (h_err & PAT_NODIAG) return SUBMAT_ENODIAG;
  int maxm = 0;
  for (int j = 0; j < n; ++j) maxm = std::max(maxm, P.h_m[j]);
  if (maxm > SUBMAT_MAX_ORDER) return SUBMAT_ETOOBIG;
  if ((rc = P.tpos.alloc(nnz))) return rc;
  HIP_TRY(launch_transpose_positions(rowptr, colind, n, P.tpos.p, stream));

  // buckets in longest-processing-time order (largest m first)
  std::vector<int32_t> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return P.h_m[a] > P.h_m[b]; });
  for (int32_t j : order) (P.h_m[j] <= P.small_max ? P.small_items : P.large_items).push_back(j);
  P.small_mmax = P.small_items.empty() ? 0 : P.h_m[P.small_items.front()];
  P.large_mmax = P.large_items.empty() ? 0 : P.h_m[P.large_items.front()];

  // large-item layout: chunks bounded by the workspace budget
  const int nl = (int)P.large_items.size();
  std::vector<int32_t> ldm(nl);
  std::vector<int64_t> off(nl), voff(nl), eoff(nl);
  P.h_sqoff.resize(nl);
  P.h_sdoff.resize(nl);
  size_t free_b = 0, total_b = 0;
  HIP_TRY(hipMemGetInfo(&free_b, &total_b));
  double budget = g_opt.ws_bytes > 0 ? g_opt.ws_bytes : 0.5 * (double)free_b;
  // per item: S, Q, W slabs (8 ld^2 each), 4 vectors (8 ld each), scratch of the eigensolver (two FP64
  // ld^2 arrays) and of the back-transformation
  int64_t sq = 0, sd = 0;
  Chunk cur;
  auto item_bytes = [&](int m, int ld) {
    (void)m;
    return 3 * 8 * (int64_t)ld * ld + 4 * 8 * (int64_t)ld + scratch_bytes(ld);
  };
  double used = 0;
  for (int g = 0; g < nl; ++g) {
    const int m = P.h_m[P.large_items[g]];
    const int ld = (int)round_up(m, 16);
    ldm[g] = ld;
    const int64_t ib = item_bytes(m, ld);
    if (cur.count > 0 && used + ib > budget) {
      P.chunks.push_back(cur);
      cur = Chunk();
      used = 0;
    }
    if (cur.count == 0) cur.start = g;
    off[g] = cur.slab_bytes;
    voff[g] = cur.vec_bytes;
    eoff[g] = cur.escr_bytes;
    cur.slab_bytes += 8 * (int64_t)ld * ld;
    cur.vec_bytes += 8 * (int64_t)ld;
    cur.escr_bytes += scratch_bytes(ld);
    cur.max_m = std::max(cur.max_m, m);
    cur.count++;
    used += ib;
    P.h_sqoff[g] = sq;
    sq += 8 * (int64_t)ld * ld;
  }
  if (cur.count > 0) P.chunks.push_back(cur);
  for (int g = 0; g < nl; ++g) {
    P.h_sdoff[g] = sq + sd;
    sd += 8 * (int64_t)ldm[g];
  }
  P.saved_q_bytes = sq;
  P.saved_bytes = nl ? (sq + sd + 4 * (int64_t)nl) : 0;

  for (auto& c : P.chunks) {
    P.ws_slab = std::max(P.ws_slab, c.slab_bytes);
    P.ws_vec = std::max(P.ws_vec, c.vec_bytes);
    P.ws_escr = std::max(P.ws_escr, c.escr_bytes);
    P.max_count = std::max(P.max_count, c.count);
  }
  // where the deterministic adjoint finds each column's D: the one-wavefront
  // columns in a buffer of their own (leading dimension m), the large-order
  // columns in their chunk's S slab (leading dimension ldm)
  std::vector<int32_t> dphase(n, -1), dld(n, 0);
  std::vector<int64_t> doff(n, 0);
  for (int32_t j : P.small_items) {
    dphase[j] = 0;
    dld[j] = P.h_m[j];
    doff[j] = P.small_d_elems;
    P.small_d_elems += (int64_t)P.h_m[j] * P.h_m[j];
  }
  for (int ci = 0; ci < (int)P.chunks.size(); ++ci)
    for (int g = P.chunks[ci].start; g < P.chunks[ci].start + P.chunks[ci].count; ++g) {
      const int32_t j = P.large_items[g];
      dphase[j] = 1 + ci;
      dld[j] = ldm[g];
      doff[j] = off[g];   // bytes; the kernel divides by the element size
    }
  if ((rc = P.d_small.alloc(P.small_items.size())) || (rc = P.d_large.alloc(nl)) || (rc = P.d_ldm.alloc(nl)) ||
      (rc = P.d_off.alloc(nl)) || (rc = P.d_voff.alloc(nl)) || (rc = P.d_eoff.alloc(nl)) ||
      (rc = P.d_sqoff.alloc(nl)) || (rc = P.d_sdoff.alloc(nl)) || (rc = P.d_dphase.alloc(n)) ||
      (rc = P.d_dld.alloc(n)) || (rc = P.d_doff.alloc(n)))
    return rc;
  // one work counter per persistent launch of the longest sequence (the
  // per-column path launches up to 10 kernels per column)
  P.ncounters = 64 + 128 * (int)P.chunks.size() + 16 * n;
  auto up = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
    if (!bytes) return hipSuccess;
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, stream);
  };
  HIP_TRY(up(P.d_small.p, P.small_items.data(), P.small_items.size() * 4));
  HIP_TRY(up(P.d_large.p, P.large_items.data(), nl * 4));
  HIP_TRY(up(P.d_ldm.p, ldm.data(), nl * 4));
  HIP_TRY(up(P.d_off.p, off.data(), nl * 8));
  HIP_TRY(up(P.d_voff.p, voff.data(), nl * 8));
  HIP_TRY(up(P.d_eoff.p, eoff.data(), nl * 8));
  HIP_TRY(up(P.d_sqoff.p, P.h_sqoff.data(), nl * 8));
  HIP_TRY(up(P.d_sdoff.p, P.h_sdoff.data(), nl * 8));
  HIP_TRY(up(P.d_dphase.p, dphase.data(), (size_t)n * 4));
  HIP_TRY(up(P.d_dld.p, dld.data(), (size_t)n * 4));
  HIP_TRY(up(P.d_doff.p, doff.data(), (size_t)n * 8));
  HIP_TRY(hipStreamSynchronize(stream));
  P.last_use = ++g_plan_clock;
  *out = plan.get();
  g_plans.emplace(key, std::move(plan));
  return SUBMAT_OK;
}

int alloc_workspace(Plan& P, Workspace& W) {
  int rc;
  if ((rc = W.S.alloc(P.ws_slab)) || (rc = W.Q.alloc(P.ws_slab)) || (rc = W.W.alloc(P.ws_slab)) ||
      (rc = W.dv.alloc(P.ws_vec)) || (rc = W.ev.alloc(P.ws_vec)) || (rc = W.tv.alloc(P.ws_vec)) ||
      (rc = W.escr.alloc(P.ws_escr)) || (rc = W.flags.alloc(std::max(P.max_count, 1))) ||
      (rc = W.counters.alloc(P.ncounters)))
    return rc;
  HIP_TRY(hipStreamCreateWithFlags(&W.cap_stream, hipStreamNonBlocking));
  return SUBMAT_OK;
}

// The workspace of `stream` on plan P, allocated on the stream's first call.
// When it does not fit, the other plans of the device, then this plan's
// other workspaces, are dropped (least recently used first) and the
// allocation is retried.
int get_workspace(Plan& P, hipStream_t stream, Workspace** out) {
  const uintptr_t key = (uintptr_t)stream;
  auto it = P.ws.find(key);
  if (it == P.ws.end()) {
    if (P.ws.size() >= kMaxWorkspaces) {
      auto old = std::min_element(P.ws.begin(), P.ws.end(), [](const auto& a, const auto& b) {
        return a.second->last_use < b.second->last_use;
      });
      P.ws.erase(old);
    }
    auto w = std::make_unique<Workspace>();
    int rc = alloc_workspace(P, *w);
    if (rc == SUBMAT_ENOMEM) {
      (void)hipGetLastError();
      w.reset();
      for (auto p = g_plans.begin(); p != g_plans.end();) {
        if (p->second.get() != &P && p->second->device == P.device) {
          forget_saved(p->first);
          p = g_plans.erase(p);
        } else {
          ++p;
        }
      }
      P.ws.clear();
      w = std::make_unique<Workspace>();
      rc = alloc_workspace(P, *w);
    }
    if (rc) return rc;
    it = P.ws.emplace(key, std::move(w)).first;
  }
  it->second->last_use = ++g_plan_clock;
  *out = it->second.get();
  return SUBMAT_OK;
}

// Drops the cached plans (all workspaces and graphs) and Krylov data of one
// pattern on the current device; returns whether any existed.
bool release_pattern(int device, const int32_t* rowptr, const int32_t* colind, int32_t n, int64_t nnz);

// ------------------------------------------------------- Krylov patterns
// Validated pattern (same device check as the plan), the transpose position
// of every stored entry, and grow-only vectors for the sparse products and
// Krylov loops. Cached by (device, rowptr, colind, n, nnz), like plans.
struct KrylovPattern {
  int32_t n = 0;
  int64_t nnz = 0;
  int lanes = 64;
  DevBuf<int32_t> tpos;
  DevBuf<double> xt;        // transposed values of the preconditioner / root
  DevBuf<double> vec;       // work vectors
  DevBuf<double> small;     // Lanczos coefficients and reduction partials
  DevBuf<uint32_t> ticket;
  DevBuf<CgState> state;
  DevBuf<double> dense;     // refinement: dense A, T = A X, and the next iterate
};
std::map<PlanKey, std::unique_ptr<KrylovPattern>> g_kry;

int get_krylov(const int32_t* rowptr, const int32_t* colind, int32_t n, int64_t nnz, hipStream_t s,
               DeviceCtx* ctx, KrylovPattern** out) {
  PlanKey key{ctx->device, (uintptr_t)rowptr, (uintptr_t)colind, n, nnz};
  auto it = g_kry.find(key);
  if (it != g_kry.end()) {
    *out = it->second.get();
    return SUBMAT_OK;
  }
  auto kp = std::make_unique<KrylovPattern>();
  int rc;
  {
    DevBuf<int32_t> m, c;
    DevBuf<uint32_t> err;
    if ((rc = m.alloc(n)) || (rc = c.alloc(n)) || (rc = err.alloc(1))) return rc;
    HIP_TRY(hipMemsetAsync(err.p, 0, sizeof(uint32_t), s));
    HIP_TRY(launch_plan_pattern(rowptr, colind, n, nnz, m.p, c.p, err.p, s));
    uint32_t h_err = 0;
    HIP_TRY(hipMemcpyAsync(&h_err, err.p, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (h_err & (PAT_ROWPTR | PAT_RANGE | PAT_ORDER | PAT_ASYM)) return SUBMAT_EPATTERN;
    if (h_err & PAT_NODIAG) return SUBMAT_ENODIAG;
  }
  kp->n = n;
  kp->nnz = nnz;
  kp->lanes = spmv_lanes((double)nnz / n);
  if ((rc = kp->tpos.alloc(nnz)) || (rc = kp->ticket.alloc(1)) || (rc = kp->state.alloc(1))) return rc;
  HIP_TRY(launch_transpose_positions(rowptr, colind, n, kp->tpos.p, s));
  HIP_TRY(hipMemsetAsync(kp->ticket.p, 0, sizeof(uint32_t), s));
  *out = kp.get();
  g_kry.emplace(key, std::move(kp));
  return SUBMAT_OK;
}

template <class T>
int ensure(DevBuf<T>& b, size_t count) {
  return b.n >= count ? SUBMAT_OK : b.alloc(count);
}

// ----------------------------------------------------------- launch sequence
enum Phase { PH_RESET = 0, PH_SMALL, PH_GATHER, PH_TRIDIAG, PH_EIG, PH_ORTH, PH_BACK, PH_COLUMN, PH_ADJOINT, PH_FALLBACK, PH_N };

struct Call {
  const void* vals;
  int vdtype;
  SpecFn fn;
  int precision;
  void* x;          // forward output
  const void* gx;   // backward input
  void* ga;         // backward output
  char* saved;      // optional saved buffer
  bool bwd;
  int det = 0;      // backward: deterministic assembly
};

struct Timer {
  bool on = false;
  hipStream_t s = nullptr;
  double ms[PH_N] = {0};
  int launches[PH_N] = {0};
  hipEvent_t a = nullptr, b = nullptr;
  int start(int) {
    if (!on) return SUBMAT_OK;
    HIP_TRY(hipEventRecord(a, s));
    return SUBMAT_OK;
  }
  int stop(int ph) {
    if (!on) return SUBMAT_OK;
    HIP_TRY(hipEventRecord(b, s));
    HIP_TRY(hipEventSynchronize(b));
    float t = 0;
    HIP_TRY(hipEventElapsedTime(&t, a, b));
    ms[ph] += t;
    launches[ph] += 1;
    return SUBMAT_OK;
  }
};

#define SEQ_TRY(expr)                   \
  do {                                  \
    int _r = (expr);                    \
    if (_r != SUBMAT_OK) return _r;     \
  } while (0)
#define HIP_SEQ(ph, expr)                                  \
  do {                                                     \
    SEQ_TRY(tm.start(ph));                                 \
    if ((expr) != hipSuccess) return SUBMAT_EHIP;          \
    SEQ_TRY(tm.stop(ph));                                  \
  } while (0)

int persistent_grid(DeviceCtx* ctx, int n_items, int per_cu) {
  int g = ctx->num_cus * per_cu;
  if (g > n_items) g = n_items;
  return g < 1 ? 1 : g;
}

LargeArgs make_large(Plan& P, Workspace& W, const Call& c, int chunk, int g_first, int count, int max_m) {
  LargeArgs a{};
  a.rowptr = P.rowptr;
  a.colind = P.colind;
  a.tpos = P.tpos.p;
  a.vals = c.vals;
  a.vdtype = c.vdtype;
  a.items = P.d_large.p + g_first;
  a.cidx = P.d_c.p;
  a.ldm = P.d_ldm.p + g_first;
  a.off = P.d_off.p + g_first;
  a.voff = P.d_voff.p + g_first;
  a.eoff = P.d_eoff.p + g_first;
  if (c.saved) {
    a.qoff = P.d_sqoff.p + g_first;
    a.doff = P.d_sdoff.p + g_first;
    a.Q = c.saved;
    a.d = c.saved;
  } else {
    a.qoff = P.d_off.p + g_first;
    a.doff = P.d_voff.p + g_first;
    a.Q = W.Q.p;
    a.d = W.dv.p;
  }
  a.n_items = count;
  a.max_m = max_m;
  a.S = W.S.p;
  a.W = W.W.p;
  a.e = W.ev.p;
  a.tau = W.tv.p;
  a.escr = W.escr.p;
  a.flags = (c.saved ? (int32_t*)(c.saved + P.saved_bytes - 4 * (int64_t)P.large_items.size()) + g_first
                     : W.flags.p + (g_first - P.chunks[chunk].start));
  a.fn = c.fn;
  a.kappa_max = g_opt.kappa_max;
  a.cluster_tol = g_opt.cluster_tol;
  a.x = c.x;
  a.gx = c.gx;
  a.ga = c.ga;
  a.det = c.bwd ? c.det : 0;
  return a;
}

// One pass of the large-order pipeline over items [g_first, g_first+count)
// of `chunk`, in FP64 or FP32. `only_flagged` restricts it to the items the
// FP32 pass sent to FP64. With a saved buffer in the backward, only the
// adjoint runs.
int run_large(Plan& P, Workspace& W, DeviceCtx* ctx, const Call& c, int64_t* status, hipStream_t s, Timer& tm,
              int& ctr, int chunk, int g_first, int count, int max_m, int fp64, int only_flagged, bool per_column) {
  LargeArgs a = make_large(P, W, c, chunk, g_first, count, max_m);
  a.status = status;
  a.lds_limit = ctx->lds_limit;
  a.fp64 = fp64;
  a.only_flagged = only_flagged;
  const int tune_cu = per_column ? 0 : tuned_blocks_per_cu(max_m, fp64);
  a.grid = per_column ? 1 : persistent_grid(ctx, count, tune_cu);
  const int ph = only_flagged ? PH_FALLBACK : -1;
  auto next = [&]() { a.work_ctr = W.counters.p + (ctr++ % P.ncounters); };
  // unit launches: one counter, or one per XCD queue (consecutive; the
  // counter budget of a batched call leaves room for them without wrapping)
  const int queues = (!per_column && g_opt.xcd_queues) ? kXcdQueueCount : 1;
  auto next_units = [&](LargeArgs& b) {
    if (ctr % P.ncounters + queues > P.ncounters) ctr += P.ncounters - ctr % P.ncounters;
    b.work_ctr = W.counters.p + (ctr % P.ncounters);
    b.xcd_queues = queues > 1;
    ctr += queues;
  };
  // Kernels whose registers and LDS leave room for more workgroups per
  // compute unit than the tuned value get at least that many (measured on
  // the overlap workloads: the gather, the column and the
  // reorthogonalisation are latency-bound, and more resident workgroups
  // hide it); a workgroup that cannot be resident at once starts later and
  // finds the work counter exhausted.
  auto with_grid = [&](int min_per_cu) {
    LargeArgs o = a;
    if (!per_column) o.grid = persistent_grid(ctx, count, std::max(tune_cu, min_per_cu));
    return o;
  };
  const bool eig = !(c.bwd && c.saved);
  if (eig) {
    next(); HIP_SEQ(ph < 0 ? PH_GATHER : ph, launch_gather_large(with_grid(8), s));
    // the reduction: panel width and workgroups per compute unit from the
    // tuning table (its LDS panel copy is sized for that many)
    {
      LargeArgs r = with_grid(0);
      r.nb = tuned_reduction_nb(max_m, fp64);
      r.red_per_cu = reduction_fit_per_cu(max_m, r.nb, fp64, ctx->lds_limit, tuned_reduction_per_cu(max_m, fp64));
      if (!per_column) r.grid = persistent_grid(ctx, count, r.red_per_cu);
      next();
      r.work_ctr = a.work_ctr;
      HIP_SEQ(ph < 0 ? PH_TRIDIAG : ph, launch_tridiagonalise(r, s));
    }
    {
      // the eigensolver's workgroups share a compute unit's LDS
      LargeArgs b = a;
      const int fit = (int)(ctx->lds_limit / (int64_t)(eig_lds_bytes(max_m) + 2048));
      const int bpc = std::max(1, std::min(tuned_eig_blocks_per_cu(max_m), fit));
      b.grid = per_column ? 1 : persistent_grid(ctx, count, bpc);
      next();
      b.work_ctr = a.work_ctr;
      HIP_SEQ(ph < 0 ? PH_EIG : ph, launch_tridiag_eig(b, s));
    }
    next(); HIP_SEQ(ph < 0 ? PH_ORTH : ph, launch_eig_orth(with_grid(4), s));
    // the eigenvector matrix Q = Q1 Z is formed only where it is used: by the
    // adjoint, or kept in a saved buffer for a later adjoint
    if (c.bwd || c.saved) {
      next(); HIP_SEQ(ph < 0 ? PH_BACK : ph, launch_back_prep(with_grid(back_blocks_per_cu()), s));
      {
        // the column units: a grid over units rather than items
        LargeArgs b = with_grid(back_blocks_per_cu());
        if (!per_column) b.grid = persistent_grid(ctx, back_apply_units(count, max_m), back_blocks_per_cu());
        next_units(b);
        HIP_SEQ(ph < 0 ? PH_BACK : ph, launch_back_apply(b, s));
      }
    }
  }
  next();
  if (c.bwd) {
    HIP_SEQ(ph < 0 ? PH_ADJOINT : ph, launch_adjoint_prep(with_grid(adjoint_blocks_per_cu()), s));
    LargeArgs b = with_grid(adjoint_blocks_per_cu());
    if (!per_column) b.grid = persistent_grid(ctx, back_apply_units(count, max_m), adjoint_blocks_per_cu());
    for (int lower = 0; lower < 2; ++lower) {
      next_units(b);
      HIP_SEQ(ph < 0 ? PH_ADJOINT : ph, launch_adjoint_product(b, lower, s));
    }
    next();
    HIP_SEQ(ph < 0 ? PH_ADJOINT : ph, launch_adjoint_scatter(with_grid(adjoint_blocks_per_cu()), s));
  } else if (c.saved) HIP_SEQ(ph < 0 ? PH_COLUMN : ph, launch_apply_column(with_grid(8), s));
  else HIP_SEQ(ph < 0 ? PH_COLUMN : ph, launch_column_factored(with_grid(column_waves_per_cu()), s));
  return SUBMAT_OK;
}

DetReduceArgs det_args(const Plan& P, const Call& c, int phase, const void* base, int bytes_off) {
  DetReduceArgs d{};
  d.rowptr = P.rowptr;
  d.colind = P.colind;
  d.tpos = P.tpos.p;
  d.n = P.n;
  d.phase = phase;
  d.dphase = P.d_dphase.p;
  d.dld = P.d_dld.p;
  d.doff = P.d_doff.p;
  d.base = base;
  d.bytes_off = bytes_off;
  d.ga = c.ga;
  return d;
}

int run_sequence(Plan& P, Workspace& W, DeviceCtx* ctx, const Call& c, int64_t* status, hipStream_t s, Timer& tm) {
  int ctr = 0;
  HIP_SEQ(PH_RESET, launch_reset_status(status, W.counters.p, P.ncounters, s));
  if (c.bwd) HIP_SEQ(PH_RESET, launch_fill_zero(c.ga, P.nnz * (c.vdtype == 0 ? 8 : 4), s));
  const bool plain = c.precision == SUBMAT_PREC_F64_PLAIN;
  const int mixed = c.precision == SUBMAT_PREC_F32_MIXED;
  // small-order bucket
  if (!P.small_items.empty()) {
    SmallArgs sa{};
    sa.rowptr = P.rowptr;
    sa.colind = P.colind;
    sa.vals = c.vals;
    sa.vdtype = c.vdtype;
    sa.cidx = P.d_c.p;
    sa.fn = c.fn;
    sa.mixed = mixed;
    sa.kappa_max = g_opt.kappa_max;
    sa.x = c.bwd ? nullptr : c.x;
    sa.gx = c.bwd ? c.gx : nullptr;
    sa.ga = c.bwd ? c.ga : nullptr;
    sa.status = status;
    const bool det_small = c.bwd && c.det;
    if (det_small) {
      if (W.dsmall.n < (size_t)P.small_d_elems) return SUBMAT_EINVAL;  // sized by run_call
      sa.dout = W.dsmall.p;
      sa.doff = P.d_doff.p;
      sa.dld = P.d_dld.p;
    }
    if (!plain) {
      sa.items = P.d_small.p;
      sa.n_items = (int)P.small_items.size();
      sa.mmax = P.small_mmax;
      sa.grid = persistent_grid(ctx, sa.n_items, 8);
      sa.work_ctr = W.counters.p + (ctr++ % P.ncounters);
      HIP_SEQ(PH_SMALL, launch_small(sa, s));
    } else {
      for (size_t i = 0; i < P.small_items.size(); i += g_opt.plain_stride) {
        sa.items = P.d_small.p + i;
        sa.n_items = 1;
        sa.mmax = P.h_m[P.small_items[i]];
        sa.grid = 1;
        sa.work_ctr = W.counters.p + (ctr++ % P.ncounters);
        HIP_SEQ(PH_SMALL, launch_small(sa, s));
      }
    }
    if (det_small) HIP_SEQ(PH_ADJOINT, launch_adjoint_reduce(det_args(P, c, 0, W.dsmall.p, 0), c.vdtype,
                                                              ctx->num_cus, s));
  }
  // large-order bucket, chunk by chunk
  for (int ci = 0; ci < (int)P.chunks.size(); ++ci) {
    const Chunk& ch = P.chunks[ci];
    if (plain) {
      // large items are numbered across chunks in one order (largest first)
      for (int g = ch.start; g < ch.start + ch.count; ++g)
        if (g % g_opt.plain_stride == 0)
          SEQ_TRY(run_large(P, W, ctx, c, status, s, tm, ctr, ci, g, 1, P.h_m[P.large_items[g]], 1, 0, true));
    } else if (!mixed) {
      SEQ_TRY(run_large(P, W, ctx, c, status, s, tm, ctr, ci, ch.start, ch.count, ch.max_m, 1, 0, false));
    } else {
      SEQ_TRY(run_large(P, W, ctx, c, status, s, tm, ctr, ci, ch.start, ch.count, ch.max_m, 0, 0, false));
      SEQ_TRY(run_large(P, W, ctx, c, status, s, tm, ctr, ci, ch.start, ch.count, ch.max_m, 1, 1, false));
    }
    if (c.bwd && c.det)
      HIP_SEQ(PH_ADJOINT, launch_adjoint_reduce(det_args(P, c, 1 + ci, W.W.p, 1), c.vdtype, ctx->num_cus, s));
  }
  // the atomic scatter-adds fill the lower triangle; the upper one mirrors it
  if (c.bwd && !c.det)
    HIP_SEQ(PH_ADJOINT, launch_adjoint_mirror(P.rowptr, P.colind, P.tpos.p, P.n, c.ga, c.vdtype, ctx->num_cus, s));
  return SUBMAT_OK;
}

uintptr_t fn_alpha_bits(const SpecFn& f) {
  uint64_t b = 0;
  std::memcpy(&b, &f.alpha, sizeof(b));
  return (uintptr_t)b;
}

int launch_graph(Plan& P, Workspace& W, DeviceCtx* ctx, const Call& c, int64_t* status, hipStream_t s) {
  std::vector<uintptr_t> key = {(uintptr_t)c.vals, (uintptr_t)c.vdtype, (uintptr_t)c.fn.kind, (uintptr_t)c.fn.p,
                                fn_alpha_bits(c.fn), (uintptr_t)c.precision,
                                (uintptr_t)c.x, (uintptr_t)c.gx, (uintptr_t)c.ga, (uintptr_t)c.saved,
                                (uintptr_t)c.bwd, (uintptr_t)c.det, (uintptr_t)(g_opt.kappa_max * 1e3),
                                (uintptr_t)(g_opt.cluster_tol * 1e12),
                                (uintptr_t)g_opt.tune_gen};
  GraphEntry* hit = nullptr;
  for (auto& g : W.graphs)
    if (g.key == key) hit = &g;
  if (!hit) {
    if (W.graphs.size() >= 8) {
      auto old = std::min_element(W.graphs.begin(), W.graphs.end(),
                                  [](const GraphEntry& a, const GraphEntry& b) { return a.stamp < b.stamp; });
      if (old->exec) (void)hipGraphExecDestroy(old->exec);
      if (old->graph) (void)hipGraphDestroy(old->graph);
      W.graphs.erase(old);
    }
    GraphEntry ge;
    ge.key = key;
    Timer off;
    HIP_TRY(hipStreamBeginCapture(W.cap_stream, hipStreamCaptureModeThreadLocal));
    int rc = run_sequence(P, W, ctx, c, status, W.cap_stream, off);
    hipGraph_t graph = nullptr;
    hipError_t ec = hipStreamEndCapture(W.cap_stream, &graph);
    if (rc != SUBMAT_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (ec != hipSuccess) return SUBMAT_EHIP;
    ge.graph = graph;
    if (hipGraphInstantiate(&ge.exec, graph, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return SUBMAT_EHIP;
    }
    W.graphs.push_back(ge);
    hit = &W.graphs.back();
  }
  hit->stamp = ++W.stamp;
  HIP_TRY(hipGraphLaunch(hit->exec, s));
  return SUBMAT_OK;
}

int check_args(const int32_t* rowptr, const int32_t* colind, const void* vals, int32_t n, int64_t nnz,
               int32_t dtype, int32_t precision) {
  if (!rowptr || !colind || !vals) return SUBMAT_EINVAL;
  if (n < 1 || nnz < n) return SUBMAT_EINVAL;
  if (dtype != SUBMAT_F64 && dtype != SUBMAT_F32) return SUBMAT_EINVAL;
  if (precision < SUBMAT_PREC_F64 || precision > SUBMAT_PREC_F64_PLAIN) return SUBMAT_EINVAL;
  if (nnz > (int64_t)INT32_MAX) return SUBMAT_EINVAL;
  return SUBMAT_OK;
}

// Function code and parameter -> SpecFn; root orders are int32 integers
// >= 1, exponents finite.
int make_fn(int32_t kind, double param, SpecFn* out) {
  if (kind == SUBMAT_FN_INV_ROOT || kind == SUBMAT_FN_ROOT) {
    if (!(param >= 1.0 && param <= (double)INT32_MAX) || param != std::floor(param)) return SUBMAT_EINVAL;
    *out = SpecFn{kind, (int)param, 0.0};
    return SUBMAT_OK;
  }
  if (kind == SUBMAT_FN_POWER) {
    if (!std::isfinite(param)) return SUBMAT_EINVAL;
    *out = SpecFn{kind, 1, param};
    return SUBMAT_OK;
  }
  return SUBMAT_EINVAL;
}

int run_call(const int32_t* rowptr, const int32_t* colind, int32_t n, int64_t nnz, Call& c, void* stream,
             Timer* timer) {
  DeviceCtx* ctx = nullptr;
  SEQ_TRY(get_ctx(&ctx));
  hipStream_t s = (hipStream_t)stream;
  Plan* P = nullptr;
  SEQ_TRY(build_plan(rowptr, colind, n, nnz, s, ctx, &P));
  if (c.saved && c.precision == SUBMAT_PREC_F64_PLAIN) c.saved = nullptr;
  const PlanKey key{ctx->device, (uintptr_t)rowptr, (uintptr_t)colind, n, nnz};
  if (c.saved && c.bwd) {
    auto t = g_saved.find((uintptr_t)c.saved);
    if (t == g_saved.end() || !(t->second.key == key) || t->second.dtype != c.vdtype ||
        t->second.precision != c.precision)
      return SUBMAT_ESAVED;
  }
  Workspace* W = nullptr;
  SEQ_TRY(get_workspace(*P, s, &W));
  // buffers a call needs are allocated here, never while a graph is captured
  if (c.bwd && c.det && W->dsmall.n < (size_t)P->small_d_elems) SEQ_TRY(W->dsmall.alloc(P->small_d_elems));
  int64_t* status = nullptr;
  SEQ_TRY(stream_status(ctx, s, &status));
  g_noalloc_status.erase({ctx->device, (uintptr_t)s});
  int rc;
  if (timer) {
    timer->s = s;
    timer->on = true;
    HIP_TRY(hipEventCreate(&timer->a));
    HIP_TRY(hipEventCreate(&timer->b));
    rc = run_sequence(*P, *W, ctx, c, status, s, *timer);
    (void)hipEventDestroy(timer->a);
    (void)hipEventDestroy(timer->b);
  } else if (g_opt.use_graph && c.precision != SUBMAT_PREC_F64_PLAIN) {
    rc = launch_graph(*P, *W, ctx, c, status, s);
  } else {
    Timer off;
    rc = run_sequence(*P, *W, ctx, c, status, s, off);
  }
  if (rc == SUBMAT_OK && c.saved && !c.bwd) g_saved[(uintptr_t)c.saved] = SavedTag{key, c.vdtype, c.precision};
  return rc;
}

bool release_pattern(int device, const int32_t* rowptr, const int32_t* colind, int32_t n, int64_t nnz) {
  const PlanKey key{device, (uintptr_t)rowptr, (uintptr_t)colind, n, nnz};
  bool found = false;
  auto it = g_plans.find(key);
  if (it != g_plans.end()) {
    forget_saved(key);
    g_plans.erase(it);
    found = true;
  }
  auto kt = g_kry.find(key);
  if (kt != g_kry.end()) {
    g_kry.erase(kt);
    found = true;
  }
  return found;
}

// ------------------------------------------------------------- Krylov loops
constexpr uint64_t kLanczosSeed = 0x1710108995ull;

int check_krylov_args(const int32_t* rowptr, const int32_t* colind, int32_t n, int64_t nnz) {
  if (!rowptr || !colind || n < 1 || nnz < n || nnz > (int64_t)INT32_MAX) return SUBMAT_EINVAL;
  return SUBMAT_OK;
}

int residual_norm_impl(const int32_t* rowptr, const int32_t* colind, const double* a_vals, const double* x_vals,
                       int32_t n, int64_t nnz, int p, int kmax, double tol, double* norm, int32_t* iters,
                       hipStream_t s) {
  DeviceCtx* ctx = nullptr;
  KrylovPattern* K = nullptr;
  int rc;
  if ((rc = get_ctx(&ctx)) || (rc = get_krylov(rowptr, colind, n, nnz, s, ctx, &K))) return rc;
  const int64_t N = n;
  const int RB = reduction_blocks();
  if ((rc = ensure(K->vec, (size_t)(kmax + 5) * N)) || (rc = ensure(K->small, (size_t)3 * kmax + 4 + RB)) ||
      (rc = ensure(K->xt, (size_t)nnz)))
    return rc;
  double* V = K->vec.p;                       // (kmax + 1) columns
  double* a0 = V + (int64_t)(kmax + 1) * N;
  double* a1 = a0 + N;
  double* a2 = a1 + N;
  double* w = a2 + N;
  double* alpha = K->small.p;                 // kmax
  double* b2 = alpha + kmax;                  // kmax
  double* h = b2 + kmax;                      // kmax + 1
  double* lam_d = h + kmax + 1;               // 1
  double* tmp = lam_d + 1;                    // 1
  KrylovScratch ks{tmp + 2, K->ticket.p};
  HIP_TRY(launch_gather_transpose(K->tpos.p, x_vals, nnz, K->xt.p, s));
  const SpmvArgs A{rowptr, colind, a_vals, n, K->lanes};
  const SpmvArgs Xn{rowptr, colind, K->xt.p, n, K->lanes};  // X v (column-based values, transposed)
  const SpmvArgs Xt{rowptr, colind, x_vals, n, K->lanes};   // X^T v
  HIP_TRY(hipMemsetAsync(alpha, 0, sizeof(double) * kmax, s));
  HIP_TRY(launch_random_vector(a0, N, kLanczosSeed, s));
  HIP_TRY(launch_dot(a0, a0, N, ks, tmp, nullptr, s));
  HIP_TRY(launch_scale(a0, V, N, nullptr, tmp, 1, s));
  double lam = 0.0, lam_prev = -1.0;
  int j = 0;
  while (j < kmax) {
    const double* v = V + (int64_t)j * N;
    // R v = X^p (A v) - v
    HIP_TRY(launch_spmv(A, v, a0, 0.0, nullptr, nullptr, s));
    double* src = a0;
    for (int r = 0; r < p; ++r) {
      double* dst = src == a0 ? a1 : a0;
      HIP_TRY(launch_spmv(Xn, src, dst, -1.0, r == p - 1 ? v : nullptr, nullptr, s));
      src = dst;
    }
    double* rv = src;
    // R^T (R v) = A (X^T)^p (R v) - R v
    double* pp[2] = {rv == a0 ? a1 : a0, a2};
    const double* src2 = rv;
    for (int r = 0; r < p; ++r) {
      double* dst = pp[r & 1];
      HIP_TRY(launch_spmv(Xt, src2, dst, 0.0, nullptr, nullptr, s));
      src2 = dst;
    }
    HIP_TRY(launch_spmv(A, src2, w, -1.0, rv, nullptr, s));
    // full reorthogonalisation (twice) against v_0..v_j; the v_j components
    // are the Lanczos diagonal
    for (int pass = 0; pass < 2; ++pass) {
      HIP_TRY(launch_gemv_t(V, N, j + 1, w, h, s));
      HIP_TRY(launch_gemv_n_sub(V, N, j + 1, h, w, alpha, j, s));
    }
    HIP_TRY(launch_dot(w, w, N, ks, b2 + j, nullptr, s));
    HIP_TRY(launch_scale(w, V + (int64_t)(j + 1) * N, N, nullptr, b2 + j, 1, s));
    ++j;
    if (j % 4 == 0 || j == kmax) {
      HIP_TRY(launch_tridiag_max(alpha, b2, j, lam_d, s));
      HIP_TRY(hipMemcpyAsync(&lam, lam_d, sizeof(double), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      if (lam_prev >= 0.0 && std::fabs(lam - lam_prev) <= tol * std::fabs(lam)) break;
      lam_prev = lam;
    }
  }
  *norm = std::sqrt(lam > 0.0 ? lam : 0.0);
  if (iters) *iters = j;
  return SUBMAT_OK;
}

int pcg_impl(const int32_t* rowptr, const int32_t* colind, const double* a_vals, const double* k_vals, int32_t n,
             int64_t nnz, const double* b, double* x, double tol, int max_iter, int32_t* iters, double* relres,
             double* true_relres, hipStream_t s) {
  DeviceCtx* ctx = nullptr;
  KrylovPattern* K = nullptr;
  int rc;
  if ((rc = get_ctx(&ctx)) || (rc = get_krylov(rowptr, colind, n, nnz, s, ctx, &K))) return rc;
  const int64_t N = n;
  const int RB = reduction_blocks();
  if ((rc = ensure(K->vec, (size_t)6 * N)) || (rc = ensure(K->small, (size_t)4 + RB))) return rc;
  if (k_vals && (rc = ensure(K->xt, (size_t)nnz))) return rc;
  double* r = K->vec.p;
  double* pv = r + N;
  double* q = pv + N;
  double* t = q + N;
  double* u = t + N;
  double* y = k_vals ? u + N : x;   // without a preconditioner the iterate is x itself
  double* sc = K->small.p;          // 2 scalars
  KrylovScratch ks{sc + 2, K->ticket.p};
  CgState* st = K->state.p;
  const int32_t* done = (const int32_t*)((const char*)st + offsetof(CgState, done));
  CgState init{};
  init.tol = tol;
  HIP_TRY(hipMemcpyAsync(st, &init, sizeof(CgState), hipMemcpyHostToDevice, s));
  const SpmvArgs A{rowptr, colind, a_vals, n, K->lanes};
  SpmvArgs Kn{}, Kt{};
  if (k_vals) {
    HIP_TRY(launch_gather_transpose(K->tpos.p, k_vals, nnz, K->xt.p, s));
    Kn = SpmvArgs{rowptr, colind, K->xt.p, n, K->lanes};  // K v
    Kt = SpmvArgs{rowptr, colind, k_vals, n, K->lanes};   // K^T v
    HIP_TRY(launch_spmv(Kt, b, r, 0.0, nullptr, nullptr, s));
  } else {
    HIP_TRY(hipMemcpyAsync(r, b, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
  }
  HIP_TRY(launch_cg_start(y, r, pv, N, st, ks, s));
  CgState h{};
  HIP_TRY(hipMemcpyAsync(&h, st, sizeof(CgState), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  int launched = 0;
  constexpr int kBatch = 32;
  while (launched < max_iter && !h.done) {
    const int nb = std::min(kBatch, max_iter - launched);
    for (int i = 0; i < nb; ++i) {
      if (k_vals) {
        HIP_TRY(launch_spmv(Kn, pv, t, 0.0, nullptr, done, s));
        HIP_TRY(launch_spmv(A, t, u, 0.0, nullptr, done, s));
        HIP_TRY(launch_spmv(Kt, u, q, 0.0, nullptr, done, s));
      } else {
        HIP_TRY(launch_spmv(A, pv, q, 0.0, nullptr, done, s));
      }
      HIP_TRY(launch_dot(pv, q, N, ks, &st->pq, done, s));
      HIP_TRY(launch_cg_update(y, r, pv, q, N, st, ks, s));
      HIP_TRY(launch_cg_direction(pv, r, N, st, s));
    }
    launched += nb;
    HIP_TRY(hipMemcpyAsync(&h, st, sizeof(CgState), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (h.done) break;
  }
  if (k_vals) HIP_TRY(launch_spmv(Kn, y, x, 0.0, nullptr, nullptr, s));
  // true residual ||b - A x|| / ||b||
  HIP_TRY(launch_spmv(A, x, t, -1.0, b, nullptr, s));
  HIP_TRY(launch_dot(t, t, N, ks, sc, nullptr, s));
  HIP_TRY(launch_dot(b, b, N, ks, sc + 1, nullptr, s));
  double h2[2] = {0.0, 0.0};
  HIP_TRY(hipMemcpyAsync(h2, sc, sizeof(h2), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (iters) *iters = h.iters;
  if (relres) *relres = h.bnorm > 0.0 ? std::sqrt(h.rr) / h.bnorm : 0.0;
  if (true_relres) *true_relres = h2[1] > 0.0 ? std::sqrt(h2[0] / h2[1]) : 0.0;
  return h.breakdown ? SUBMAT_EBREAKDOWN : SUBMAT_OK;
}

int refine_inverse_impl(const int32_t* rowptr, const int32_t* colind, const double* a_vals, const double* x_vals,
                        int32_t n, int64_t nnz, double* xd, int max_iter, double tol, int32_t* iters,
                        double* residual, hipStream_t s) {
  DeviceCtx* ctx = nullptr;
  KrylovPattern* K = nullptr;
  int rc;
  if ((rc = get_ctx(&ctx)) || (rc = get_krylov(rowptr, colind, n, nnz, s, ctx, &K))) return rc;
  const size_t nn = (size_t)n * n;
  const int RB = reduction_blocks();
  if ((rc = ensure(K->dense, 3 * nn)) || (rc = ensure(K->small, (size_t)2 + RB))) return rc;
  if (!ctx->blas && rocblas_create_handle(&ctx->blas) != rocblas_status_success) {
    ctx->blas = nullptr;
    return SUBMAT_EHIP;
  }
  if (rocblas_set_stream(ctx->blas, s) != rocblas_status_success) return SUBMAT_EHIP;
  double* Ad = K->dense.p;
  double* T = Ad + nn;
  double* U = T + nn;
  double* fro2 = K->small.p;
  KrylovScratch ks{fro2 + 2, K->ticket.p};
  HIP_TRY(hipMemsetAsync(Ad, 0, nn * sizeof(double), s));
  HIP_TRY(hipMemsetAsync(xd, 0, nn * sizeof(double), s));
  HIP_TRY(launch_densify(rowptr, colind, a_vals, n, 0, Ad, s));
  HIP_TRY(launch_densify(rowptr, colind, x_vals, n, 1, xd, s));
  // Row-major M is column-major M^T: T = A X is T^T = X^T A^T, and
  // U = 2 X - X T is U^T = 2 X^T - T^T X^T.
  const double one = 1.0, zero = 0.0, minus_one = -1.0, two = 2.0;
  double* X = xd;
  double res = 0.0, res0 = -1.0;
  int k = 0;
  bool converged = false, diverged = false;
  for (;;) {
    if (rocblas_dgemm(ctx->blas, rocblas_operation_none, rocblas_operation_none, n, n, n, &one, X, n, Ad, n, &zero, T,
                      n) != rocblas_status_success)
      return SUBMAT_EHIP;
    HIP_TRY(launch_residual_fro2(T, n, ks, fro2, s));
    double h = 0.0;
    HIP_TRY(hipMemcpyAsync(&h, fro2, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    res = std::sqrt(h / n);
    if (res0 < 0.0) res0 = res;
    if (res <= tol) { converged = true; break; }
    if (!std::isfinite(res) || res > 1e3 * (res0 > 1.0 ? res0 : 1.0)) { diverged = true; break; }
    if (k >= max_iter) break;
    HIP_TRY(hipMemcpyAsync(U, X, nn * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (rocblas_dgemm(ctx->blas, rocblas_operation_none, rocblas_operation_none, n, n, n, &minus_one, T, n, X, n, &two,
                      U, n) != rocblas_status_success)
      return SUBMAT_EHIP;
    std::swap(X, U);
    ++k;
  }
  if (X != xd) HIP_TRY(hipMemcpyAsync(xd, X, nn * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  (void)K->dense.alloc(0);  // 3 n^2 doubles: not kept between calls
  if (iters) *iters = k;
  if (residual) *residual = res;
  return converged ? SUBMAT_OK : (diverged || k >= max_iter ? SUBMAT_ENOCONV : SUBMAT_OK);
}

}  // namespace

// ======================================================================= ABI
extern "C" {

int submat_matfun_fwd(const int32_t* rowptr, const int32_t* colind, const void* vals, int32_t n, int64_t nnz,
                      int32_t fn, double param, int32_t dtype, int32_t precision, void* x_vals, void* saved,
                      void* stream) {
  SpecFn f{};
  int rc = check_args(rowptr, colind, vals, n, nnz, dtype, precision);
  if (!rc) rc = make_fn(fn, param, &f);
  if (rc) return rc;
  if (!x_vals) return SUBMAT_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  Call c{vals, dtype, f, precision, x_vals, nullptr, nullptr, (char*)saved, false};
  return run_call(rowptr, colind, n, nnz, c, stream, nullptr);
}

int submat_matfun_bwd(const int32_t* rowptr, const int32_t* colind, const void* vals, int32_t n, int64_t nnz,
                      int32_t fn, double param, int32_t dtype, int32_t precision, const void* grad_x,
                      void* grad_a, const void* saved, void* stream) {
  SpecFn f{};
  int rc = check_args(rowptr, colind, vals, n, nnz, dtype, precision);
  if (!rc) rc = make_fn(fn, param, &f);
  if (rc) return rc;
  if (!grad_x || !grad_a) return SUBMAT_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  Call c{vals, dtype, f, precision, nullptr, grad_x, grad_a, (char*)saved, true, g_opt.deterministic};
  return run_call(rowptr, colind, n, nnz, c, stream, nullptr);
}

int submat_invroot_fwd(const int32_t* rowptr, const int32_t* colind, const void* vals, int32_t n, int64_t nnz,
                       int32_t p, int32_t dtype, int32_t precision, void* x_vals, void* saved, void* stream) {
  return submat_matfun_fwd(rowptr, colind, vals, n, nnz, SUBMAT_FN_INV_ROOT, (double)p, dtype, precision, x_vals,
                           saved, stream);
}

int submat_invroot_fwd_noalloc(const int32_t* rowptr, const int32_t* colind, const void* vals, int32_t n,
                               int64_t nnz, int32_t p, int32_t dtype, int32_t precision, void* x_vals,
                               void* stream) {
  SpecFn f{};
  int rc = check_args(rowptr, colind, vals, n, nnz, dtype, precision);
  if (!rc) rc = make_fn(SUBMAT_FN_INV_ROOT, (double)p, &f);
  if (rc) return rc;
  if (!x_vals || precision == SUBMAT_PREC_F64_PLAIN) return SUBMAT_EINVAL;
  if (n > kNoAllocMaxN) return SUBMAT_ETOOBIG;
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceCtx* ctx = nullptr;
  SEQ_TRY(get_ctx(&ctx));
  hipStream_t s = (hipStream_t)stream;
  int64_t* status = nullptr;
  rc = noalloc_forward(rowptr, colind, vals, n, nnz, f, dtype, precision == SUBMAT_PREC_F32_MIXED, g_opt.kappa_max,
                       x_vals, ctx->num_cus, s, &status);
  if (rc) return rc;
  g_noalloc_status[{ctx->device, (uintptr_t)s}] = status;
  return SUBMAT_OK;
}

int submat_invroot_bwd(const int32_t* rowptr, const int32_t* colind, const void* vals, int32_t n, int64_t nnz,
                       int32_t p, int32_t dtype, int32_t precision, const void* grad_x, void* grad_a,
                       const void* saved, void* stream) {
  return submat_matfun_bwd(rowptr, colind, vals, n, nnz, SUBMAT_FN_INV_ROOT, (double)p, dtype, precision, grad_x,
                           grad_a, saved, stream);
}

int64_t submat_saved_bytes(const int32_t* rowptr, const int32_t* colind, int32_t n, int64_t nnz, int32_t dtype,
                           int32_t precision) {
  if (!rowptr || !colind || n < 1 || nnz < n) return SUBMAT_EINVAL;
  if (dtype != SUBMAT_F64 && dtype != SUBMAT_F32) return SUBMAT_EINVAL;
  (void)precision;
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceCtx* ctx = nullptr;
  int rc = get_ctx(&ctx);
  if (rc) return rc;
  Plan* P = nullptr;
  rc = build_plan(rowptr, colind, n, nnz, nullptr, ctx, &P);
  if (rc) return rc;
  return P->saved_bytes;
}

int submat_query_status(void* stream, int64_t* n_nonpositive, int64_t* n_fallback, int64_t* n_unconverged) {
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceCtx* ctx = nullptr;
  int rc = get_ctx(&ctx);
  if (rc) return rc;
  int64_t* st = nullptr;
  if ((rc = status_for_query(ctx, (hipStream_t)stream, &st))) return rc;
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  int64_t h[ST_NSLOTS] = {0};
  HIP_TRY(hipMemcpy(h, st, sizeof(h), hipMemcpyDeviceToHost));
  if (n_nonpositive) *n_nonpositive = h[ST_NONPOS];
  if (n_fallback) *n_fallback = h[ST_FALLBACK];
  if (n_unconverged) *n_unconverged = h[ST_UNCONV];
  return SUBMAT_OK;
}

int submat_query_counters(void* stream, int64_t* out, int32_t n) {
  if (!out || n < 1 || n > 8) return SUBMAT_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceCtx* ctx = nullptr;
  int rc = get_ctx(&ctx);
  if (rc) return rc;
  int64_t* st = nullptr;
  if ((rc = status_for_query(ctx, (hipStream_t)stream, &st))) return rc;
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  HIP_TRY(hipMemcpy(out, st, (size_t)n * sizeof(int64_t), hipMemcpyDeviceToHost));
  return SUBMAT_OK;
}

int submat_set_option(int32_t key, double value) {
  std::lock_guard<std::mutex> lk(g_mu);
  switch (key) {
    case SUBMAT_OPT_KAPPA_MAX:
      if (!(value > 1.0)) return SUBMAT_EINVAL;
      g_opt.kappa_max = value;
      return SUBMAT_OK;
    case SUBMAT_OPT_USE_GRAPH:
      g_opt.use_graph = value != 0.0;
      return SUBMAT_OK;
    case SUBMAT_OPT_SMALL_MAX:
      if (value < 0 || value > 64 || value != std::floor(value)) return SUBMAT_EINVAL;
      g_opt.small_max = (int)value;  // 0: the tuning table's edge
      g_plans.clear();
      g_saved.clear();
      return SUBMAT_OK;
    case SUBMAT_OPT_WS_BYTES:
      if (value < 0) return SUBMAT_EINVAL;
      g_opt.ws_bytes = value;
      g_plans.clear();
      g_saved.clear();
      return SUBMAT_OK;
    case SUBMAT_OPT_CLUSTER_TOL:
      if (!(value >= 0.0 && value < 1.0)) return SUBMAT_EINVAL;
      g_opt.cluster_tol = value;
      return SUBMAT_OK;
    case SUBMAT_OPT_TUNE_FILE: {
      if (value != 0.0 && value != 1.0) return SUBMAT_EINVAL;
      const int edge = tuned_small_max();
      reload_tuning(value == 1.0);
      g_opt.tune_gen++;
      if (g_opt.small_max == 0 && tuned_small_max() != edge) {
        // the bucket edge is part of every plan
        g_plans.clear();
        g_saved.clear();
      }
      return SUBMAT_OK;
    }
    case SUBMAT_OPT_DETERMINISTIC:
      if (value != 0.0 && value != 1.0) return SUBMAT_EINVAL;
      g_opt.deterministic = (int)value;
      return SUBMAT_OK;
    case SUBMAT_OPT_PLAIN_STRIDE:
      if (!(value >= 1.0 && value <= 1e9) || value != std::floor(value)) return SUBMAT_EINVAL;
      g_opt.plain_stride = (int)value;
      return SUBMAT_OK;
    case SUBMAT_OPT_XCD_QUEUES:
      if (value != 0.0 && value != 1.0) return SUBMAT_EINVAL;
      g_opt.xcd_queues = (int)value;
      return SUBMAT_OK;
    default:
      return SUBMAT_EINVAL;
  }
}

double submat_get_option(int32_t key) {
  std::lock_guard<std::mutex> lk(g_mu);
  switch (key) {
    case SUBMAT_OPT_KAPPA_MAX: return g_opt.kappa_max;
    case SUBMAT_OPT_USE_GRAPH: return g_opt.use_graph;
    case SUBMAT_OPT_SMALL_MAX: return g_opt.small_max > 0 ? g_opt.small_max : tuned_small_max();
    case SUBMAT_OPT_WS_BYTES: return g_opt.ws_bytes;
    case SUBMAT_OPT_CLUSTER_TOL: return g_opt.cluster_tol;
    case SUBMAT_OPT_TUNE_FILE: return tuning_from_file() ? 1.0 : 0.0;
    case SUBMAT_OPT_DETERMINISTIC: return g_opt.deterministic;
    case SUBMAT_OPT_PLAIN_STRIDE: return g_opt.plain_stride;
    case SUBMAT_OPT_XCD_QUEUES: return g_opt.xcd_queues;
    default: return NAN;
  }
}

const char* submat_strerror(int32_t code) {
  switch (code) {
    case SUBMAT_OK: return "ok";
    case SUBMAT_EINVAL: return "invalid argument";
    case SUBMAT_EPATTERN: return "invalid or asymmetric sparsity pattern";
    case SUBMAT_ENODIAG: return "diagonal entry not stored";
    case SUBMAT_ENOMEM: return "device allocation failed";
    case SUBMAT_EHIP: return "HIP runtime error";
    case SUBMAT_ETOOBIG: return "submatrix order exceeds SUBMAT_MAX_ORDER";
    case SUBMAT_ESAVED: return "saved buffer does not match";
    case SUBMAT_EBREAKDOWN: return "CG breakdown (operator not positive definite)";
    case SUBMAT_ENOCONV: return "refinement did not converge";
    default: return "unknown status code";
  }
}

void submat_release(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  (void)hipDeviceSynchronize();
  g_plans.clear();
  g_kry.clear();
  g_saved.clear();
}

int submat_release_pattern(const int32_t* rowptr, const int32_t* colind, int32_t n, int64_t nnz) {
  if (!rowptr || !colind) return SUBMAT_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  (void)release_pattern(dev, rowptr, colind, n, nnz);
  return SUBMAT_OK;
}

int submat_spmv(const int32_t* rowptr, const int32_t* colind, const double* vals, int32_t n, int64_t nnz,
                int32_t trans, const double* x, double* y, void* stream) {
  int rc = check_krylov_args(rowptr, colind, n, nnz);
  if (rc) return rc;
  if (!vals || !x || !y || (trans != 0 && trans != 1)) return SUBMAT_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  hipStream_t s = (hipStream_t)stream;
  DeviceCtx* ctx = nullptr;
  KrylovPattern* K = nullptr;
  if ((rc = get_ctx(&ctx)) || (rc = get_krylov(rowptr, colind, n, nnz, s, ctx, &K))) return rc;
  const double* v = vals;
  if (trans) {
    if ((rc = ensure(K->xt, (size_t)nnz))) return rc;
    HIP_TRY(launch_gather_transpose(K->tpos.p, vals, nnz, K->xt.p, s));
    v = K->xt.p;
  }
  HIP_TRY(launch_spmv(SpmvArgs{rowptr, colind, v, n, K->lanes}, x, y, 0.0, nullptr, nullptr, s));
  return SUBMAT_OK;
}

int submat_residual_norm(const int32_t* rowptr, const int32_t* colind, const double* a_vals, const double* x_vals,
                         int32_t n, int64_t nnz, int32_t p, int32_t max_iter, double tol, double* norm,
                         int32_t* iters, void* stream) {
  int rc = check_krylov_args(rowptr, colind, n, nnz);
  if (rc) return rc;
  if (!a_vals || !x_vals || !norm || p < 1 || max_iter < 1 || max_iter > 4096 || !(tol >= 0.0)) return SUBMAT_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  return residual_norm_impl(rowptr, colind, a_vals, x_vals, n, nnz, p, max_iter, tol, norm, iters,
                            (hipStream_t)stream);
}

int submat_refine_inverse(const int32_t* rowptr, const int32_t* colind, const double* a_vals, const double* x_vals,
                          int32_t n, int64_t nnz, double* x_dense, int32_t max_iter, double tol, int32_t* iters,
                          double* residual, void* stream) {
  int rc = check_krylov_args(rowptr, colind, n, nnz);
  if (rc) return rc;
  if (!a_vals || !x_vals || !x_dense || max_iter < 0 || !(tol >= 0.0) || n > 65536) return SUBMAT_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  return refine_inverse_impl(rowptr, colind, a_vals, x_vals, n, nnz, x_dense, max_iter, tol, iters, residual,
                             (hipStream_t)stream);
}

int submat_pcg(const int32_t* rowptr, const int32_t* colind, const double* a_vals, const double* k_vals, int32_t n,
               int64_t nnz, const double* b, double* x, double tol, int32_t max_iter, int32_t* iters,
               double* relres, double* true_relres, void* stream) {
  int rc = check_krylov_args(rowptr, colind, n, nnz);
  if (rc) return rc;
  if (!a_vals || !b || !x || max_iter < 0 || !(tol > 0.0)) return SUBMAT_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  return pcg_impl(rowptr, colind, a_vals, k_vals, n, nnz, b, x, tol, max_iter, iters, relres, true_relres,
                  (hipStream_t)stream);
}

int32_t submat_version(void) { return 131; }

int submat_time_phases(const int32_t* rowptr, const int32_t* colind, const void* vals, int32_t n, int64_t nnz,
                       int32_t fn, double param, int32_t dtype, int32_t precision, void* x_vals,
                       const void* grad_x, void* grad_a, void* stream, double* phase_ms, int32_t* phase_launches) {
  SpecFn f{};
  int rc = check_args(rowptr, colind, vals, n, nnz, dtype, precision);
  if (!rc) rc = make_fn(fn, param, &f);
  if (rc) return rc;
  if (!x_vals || !phase_ms || !phase_launches) return SUBMAT_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  Timer tm;
  Call c{vals, dtype, f, precision, x_vals, nullptr, nullptr, nullptr, false};
  rc = run_call(rowptr, colind, n, nnz, c, stream, &tm);
  if (rc) return rc;
  if (grad_x && grad_a) {
    Call cb{vals, dtype, f, precision, nullptr, grad_x, grad_a, nullptr, true, g_opt.deterministic};
    rc = run_call(rowptr, colind, n, nnz, cb, stream, &tm);
    if (rc) return rc;
  }
  for (int i = 0; i < SUBMAT_NUM_PHASES; ++i) {
    phase_ms[i] = tm.ms[i];
    phase_launches[i] = tm.launches[i];
  }
  return SUBMAT_OK;
}

}  // extern "C"
