// runtime.hip -- host runtime and C ABI of libmcx (see include/mcx.h).
//
// The host validates input, tabulates the material, sizes the device memory
// and drives the event loop: each chunk of histories runs as repeated
// iterations {source, flight, knock, e+- steps, advance}; the host checks the
// device-side completion flag after every batch of iterations, then flushes
// the per-history tally of the chunk into Sum q / Sum q^2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "launch.h"
#include "mcx.h"
#include "mcx_internal.h"
#include "tables.h"

// tally table: 2^MCX_TALLY_LOG2 slots, a chunk of histories sized so that at
// most 1/MCX_TALLY_LOAD_DIV of them are occupied
#ifndef MCX_TALLY_LOG2
#define MCX_TALLY_LOG2 29
#endif
#ifndef MCX_TALLY_LOAD_DIV
#define MCX_TALLY_LOAD_DIV 4
#endif

using namespace mcx;

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool ext = false;  // carved from the caller's workspace: never freed here
};

struct mcx_ctx {
  int device = 0;
  int precision = MCX_FP64;
  std::string err;
  hipStream_t stream = nullptr;
  bool have_transport = false, have_material = false, have_phantom = false, have_sources = false;
  mcx_transport tr{};
  uint32_t grad_flags = 0;  // mcx_set_gradient
  mcx_material_desc mat{};
  BuiltTables tabs;
  DevBuf d_tab;
  // phantom
  int nx = 0, ny = 0, nz = 0;
  double vox[3] = {0, 0, 0}, org[3] = {0, 0, 0};
  DevBuf d_rho;
  DevBuf d_cube;  // same-density cube half-widths, one byte per voxel
  // several materials: tables per material, and the per-voxel index
  BuiltTables mtabs[kMaxMat];
  bool have_mat[kMaxMat] = {false, false, false, false};
  DevBuf d_vmat;
  int vmat_max = -1;  // largest material index of the phantom (-1: no material array)
  // sources
  std::vector<SourceDev> src;
  DevBuf d_src;
  uint64_t total_hist = 0;
  // tallies
  DevBuf d_sumq, d_sumq2;
  uint64_t n_done = 0;
  // event queues
  uint32_t cap = 1u << 25, block = 256, steps = 128;
  DevBuf d_queues;
  size_t queue_cap_built = 0;
  DevBuf d_cnt;
  Counters* h_cnt = nullptr;  // pinned
  // tally table
  uint64_t hslots = 1ull << MCX_TALLY_LOG2;  // keys and scores, 16 B a slot
  DevBuf d_htab;  // TSlot[hslots]
  double pairs_per_hist = 0.0;
  bool table_dirty = false;  // a failed run may have left entries behind
  // caller-owned workspace (mcx_set_workspace): queues, counters and tally
  // table are carved from it; ws_cap is the bank size of the current carve
  void* ws = nullptr;
  size_t ws_bytes = 0;
  uint32_t ws_cap = 0;
  // cancellation request (mcx_cancel may be called from another host thread)
  std::atomic<int> cancel{0};
  uint64_t next_history = 0;  // first history id not completed by the last run
  // per-source dose influence (mcx_set_influence): (source, voxel) keys,
  // Sum q and Sum q^2, overflow flag
  int influence = 0;
  uint64_t islots = 0;
  DevBuf d_ikeys, d_iq, d_iq2, d_iovf;
  // test mode
  int test_mode = 0;
  DevBuf d_hhash, d_hled;
  uint64_t last_n = 0;
  bool last_valid = false;
  // the last run, for the density-gradient replays
  uint32_t run_seed = 0;
  uint64_t run_first = 0, run_n = 0;
  bool run_known = false;
  DevBuf d_adj_w, d_adj_q, d_adj_grad, d_adj_dl, d_adj_out, d_adj_sum;
  double ms_backward = 0.0;
  // stats
  uint64_t iterations = 0, chunks = 0, tally_pairs = 0;
  double ms_transport = 0.0, ms_flush = 0.0;
  // replay batches of iterations as one captured HIP graph (timing off only)
  int use_graph = 1;
  // the instantiated batch graph of the last run of each mode (forward,
  // replay A, replay B): a later run with the same kernels only updates its
  // arguments (hipGraphExecUpdate) instead of instantiating a new one
  hipGraphExec_t gexec[3] = {nullptr, nullptr, nullptr};
  // per-kernel timing with HIP events on the run's stream
  int timing = 0;
  std::vector<hipEvent_t> events;  // kBatch iterations x (kTimedKernels + 1)
  double ms_kernel[kTimedKernels] = {0, 0, 0, 0};
  uint64_t timed_iterations = 0;
};

#ifndef MCX_BATCH
#define MCX_BATCH 8
#endif
#ifndef MCX_GRID_WAVES
#define MCX_GRID_WAVES 8192
#endif
static constexpr int kBatch = MCX_BATCH;  // iterations between completion checks
// wavefronts launched per transport kernel: the kernels loop over their queue
// (grid stride, or persistent lanes), so a grid that fills the chip twice
// over serves any queue length, and blocks that find no work cost launch time
static constexpr int kGridWaves = MCX_GRID_WAVES;

namespace {

int fail(mcx_ctx* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return code;
}

int hip_fail(mcx_ctx* c, hipError_t e, const char* what) {
  return fail(c, MCX_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

void dfree(DevBuf& b) {
  if (b.p && !b.ext) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
  b.ext = false;
}

int dalloc(mcx_ctx* c, DevBuf& b, size_t bytes, const char* what) {
  if (b.p && b.bytes >= bytes) return MCX_OK;
  dfree(b);
  if (bytes == 0) return MCX_OK;
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) {
    b.p = nullptr;
    (void)hipGetLastError();
    return fail(c, MCX_E_NOMEM, "hipMalloc of %zu bytes for %s failed: %s", bytes, what, hipGetErrorString(e));
  }
  b.bytes = bytes;
  return MCX_OK;
}

bool fp64(const mcx_ctx* c) { return c->precision == MCX_FP64; }
// interaction forcing on: a factor above 1 (0 and 1 mean analog)
bool forced(const mcx_transport& t) { return t.force_in > 1.0 || t.force_br > 1.0; }
// weighted particles: forcing or bremsstrahlung splitting
bool weighted_run(const mcx_transport& t) { return forced(t) || t.split_br == 2; }
size_t tsize(const mcx_ctx* c) { return fp64(c) ? sizeof(double) : sizeof(float); }
uint64_t nvox(const mcx_ctx* c) { return uint64_t(c->nx) * c->ny * c->nz; }

template <typename T>
void carve_banks(mcx_ctx* c, KArgs<T>& a) {
  char* p = static_cast<char*>(c->d_queues.p);
  const size_t n = c->cap;
  auto take = [&](size_t bytes) {
    char* r = p;
    p += (bytes + 255) & ~size_t(255);
    return r;
  };
  for (int q = 0; q < Q_NQ; ++q) {
    Bank<T>& b = a.q[q];
    for (int k = 0; k < kMaxChunks; ++k)
      b.c[k] = k < rec_chunks<T>() ? reinterpret_cast<Chunk*>(take(n * sizeof(Chunk))) : nullptr;
    b.hash = reinterpret_cast<uint64_t*>(take(n * sizeof(uint64_t)));
    b.w = reinterpret_cast<double*>(take(n * sizeof(double)));
    b.clk = q == Q_E0 || q == Q_E1 ? reinterpret_cast<T*>(take(n * sizeof(T))) : nullptr;
  }
}

size_t queue_bytes(const mcx_ctx* c) {
  const size_t n = c->cap;
  // records, event hashes, weights; the hard-event clocks of the two e+- queues
  const size_t per = ((n * sizeof(Chunk) + 255) / 256 * 256) * (fp64(c) ? 5 : 4) + 2 * ((n * 8 + 255) / 256 * 256);
  return per * Q_NQ + 2 * ((n * tsize(c) + 255) / 256 * 256);
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
constexpr uint64_t kTableSlots = 1ull << MCX_TALLY_LOG2;  // library-owned table
constexpr uint64_t kMinWsSlots = 1ull << 20;              // smallest table in a workspace
constexpr size_t kSlotBytes = sizeof(uint64_t) + sizeof(double);

// queues of a workspace carve (the table follows them)
size_t ws_fixed_bytes(const mcx_ctx* c) { return align256(queue_bytes(c)); }

// carve the queues and the largest power-of-two tally table that fits from
// the caller's workspace, and clear the table
int carve_workspace(mcx_ctx* c) {
  const size_t fixed = ws_fixed_bytes(c);
  if (c->ws_bytes < fixed + kMinWsSlots * kSlotBytes)
    return fail(c, MCX_E_RANGE, "workspace of %zu bytes is too small for a bank of %u records (needs >= %zu)", c->ws_bytes,
                c->cap, fixed + size_t(kMinWsSlots * kSlotBytes));
  uint64_t slots = kTableSlots;
  const uint64_t room = (c->ws_bytes - fixed) / kSlotBytes;
  while (slots > room) slots >>= 1;
  char* base = static_cast<char*>(c->ws);
  const size_t qb = align256(queue_bytes(c));
  c->d_queues = DevBuf{base, qb, true};
  c->d_htab = DevBuf{base + fixed, slots * kSlotBytes, true};
  c->hslots = slots;
  c->queue_cap_built = c->cap;
  c->ws_cap = c->cap;
  hipError_t e = launch_clear_table(static_cast<TSlot*>(c->d_htab.p), slots, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "clear workspace");
  c->table_dirty = false;
  return MCX_OK;
}

int ensure_workspace(mcx_ctx* c) {
  int rc;
  // a new bank size moves the table that follows the queues
  if (c->ws && c->ws_cap != c->cap && (rc = carve_workspace(c))) return rc;
  if (!c->ws && (c->queue_cap_built != c->cap || !c->d_queues.p)) {
    dfree(c->d_queues);
    if ((rc = dalloc(c, c->d_queues, queue_bytes(c), "event queues"))) return rc;
    c->queue_cap_built = c->cap;
  }
  // fresh allocations are cleared on the context's stream (non-blocking, so
  // it does not order against the null stream) and waited for: reused device
  // memory may still hold an earlier context's entries
  if (!c->d_htab.p) {
    if ((rc = dalloc(c, c->d_htab, c->hslots * kSlotBytes, "tally table"))) return rc;
    hipError_t e = launch_clear_table(static_cast<TSlot*>(c->d_htab.p), c->hslots, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "clear tally table");
  }
  return MCX_OK;
}

template <typename T>
void fill_args(mcx_ctx* c, KArgs<T>& a, uint32_t seed, int mode = 0, double qbar = 0.0) {
  std::memset(&a, 0, sizeof(a));
  const BuiltTables& b = c->tabs;
  a.tb.t = static_cast<const T*>(c->d_tab.p);
  a.tb.n = b.n;
  a.tb.lemin = T(b.lemin);
  a.tb.inv_dl = T(1.0 / b.dl);
  a.tb.dl = T(b.dl);
  a.tb.emin = T(c->tr.e_min);
  a.tb.thr_pp = T(b.thr_pp);
  a.tb.thr_in[0] = T(b.thr_in[0]);
  a.tb.thr_in[1] = T(b.thr_in[1]);
  a.tb.thr_br = T(b.thr_br);
  a.tb.k_coef = T(b.k_coef);
  a.tb.eta_a = T(b.eta_a);
  a.tb.eta_b = T(b.eta_b);
  a.tb.ray_a = T(b.ray_a);
  a.tb.strag_k = T(b.strag_k);
  a.tb.strag_b = T(b.strag_b);
  a.tb.wcc_soft = T(b.wcc_soft);
  a.tb.wcr_soft = T(b.wcr_soft);
  a.tb.annih_k = T(b.annih_k);
  a.tb.nmat = 1;
  for (int k = 0; k < kMaxMat; ++k) {
    const BuiltTables& bk = c->have_mat[k] ? c->mtabs[k] : b;
    if (c->have_mat[k]) a.tb.nmat = std::max(a.tb.nmat, k + 1);
    MatConst<T>& mc = a.tb.mc[k];
    mc.k_coef = T(bk.k_coef);
    mc.eta_a = T(bk.eta_a);
    mc.eta_b = T(bk.eta_b);
    mc.ray_a = T(bk.ray_a);
    mc.strag_k = T(bk.strag_k);
    mc.strag_b = T(bk.strag_b);
    mc.annih_k = T(bk.annih_k);
  }
  a.mat = static_cast<const uint8_t*>(c->d_vmat.p);
  a.nx = c->nx; a.ny = c->ny; a.nz = c->nz;
  a.dx = c->vox[0]; a.dy = c->vox[1]; a.dz = c->vox[2];
  a.ox = c->org[0]; a.oy = c->org[1]; a.oz = c->org[2];
  a.idx = 1.0 / c->vox[0]; a.idy = 1.0 / c->vox[1]; a.idz = 1.0 / c->vox[2];
  a.rho = static_cast<const T*>(c->d_rho.p);
  a.cube = static_cast<const uint8_t*>(c->d_cube.p);
  for (int i = 0; i < 3; ++i) a.eabs[i] = T(c->tr.eabs[i]);
  a.c2 = T(c->tr.c2);
  a.wcc = T(c->tr.wcc);
  a.wcr = T(c->tr.wcr);
  a.seed = seed;
  a.src = static_cast<const SourceDev*>(c->d_src.p);
  a.nsrc = int(c->src.size());
  a.htab = static_cast<TSlot*>(c->d_htab.p);
  a.hmask = c->hslots - 1;
  a.sum_q = static_cast<double*>(c->d_sumq.p);
  a.sum_q2 = static_cast<double*>(c->d_sumq2.p);
  a.test_mode = c->test_mode;
  a.hist_hash = static_cast<uint64_t*>(c->d_hhash.p);
  a.hist_led = static_cast<double*>(c->d_hled.p);
  a.cnt = static_cast<Counters*>(c->d_cnt.p);
  carve_banks(c, a);
  a.cap = c->cap;
  a.steps = c->steps;
  a.mode = mode;
  a.straggle = (c->tr.flags & MCX_STRAGGLING) ? 1 : 0;
  a.grad_e = (c->grad_flags & MCX_GRAD_DEFLECTION_ENERGY) ? 1 : 0;
  a.annih = (c->tr.flags & MCX_ANNIH_FLIGHT) ? 1 : 0;
  a.mm = c->d_vmat.p ? 1 : 0;
  a.vr = weighted_run(c->tr) ? 1 : 0;
  a.split_br = c->tr.split_br == 2 ? 2 : 1;
  a.f_in = c->tr.force_in > 1.0 ? c->tr.force_in : 1.0;
  a.f_br = c->tr.force_br > 1.0 ? c->tr.force_br : 1.0;
  if (mode) {
    a.test_mode = 0;
    a.adj_w = static_cast<const double*>(c->d_adj_w.p);
    a.adj_q = static_cast<double*>(c->d_adj_q.p);
    a.adj_grad = static_cast<double*>(c->d_adj_grad.p);
    a.adj_qbar = qbar;
  }
}

// Checkpoint: this header, then Sum q and Sum q^2 (nvox doubles each), then
// an FNV-1a hash of every byte before it.
struct CkptHeader {
  char magic[8];
  uint32_t version;
  int32_t precision;
  int32_t nx, ny, nz;
  uint32_t nstat;
  uint32_t run_seed;
  uint32_t run_known;
  uint32_t reserved;
  double voxel[3];
  uint64_t n_done, next_history, run_first, run_n;
  uint64_t iterations, chunks, tally_pairs;
  double ms_transport, ms_flush;
  uint64_t stat[S_NSTAT];
  double e_dep, e_esc;
};
constexpr char kCkptMagic[8] = {'M', 'C', 'X', 'C', 'K', 'P', 'T', '1'};
constexpr uint32_t kCkptVersion = 2;

size_t ckpt_bytes(const mcx_ctx* c) { return sizeof(CkptHeader) + 2 * nvox(c) * sizeof(double) + sizeof(uint64_t); }

// Histories [first, first + n) in chunks.  *completed receives the number of
// histories transported: n, or fewer when a forward run honours a
// cancellation request (then MCX_E_CANCELLED).
template <typename T>
int run_impl(mcx_ctx* c, uint32_t seed, uint64_t first, uint64_t n, hipStream_t s, int mode = 0,
             double qbar = 0.0, uint64_t* completed = nullptr, bool allow_graph = true) {
  if (completed) *completed = 0;
  KArgs<T> a;
  fill_args(c, a, seed, mode, qbar);
  const uint32_t target = c->cap / 4;
  int grid = int((std::min<uint64_t>(c->cap, 2ull * target) + c->block - 1) / c->block);
  grid = std::min(grid, int(uint64_t(kGridWaves) * 64 / c->block));
  grid = std::max(grid, 1);
  // The run's tally slots: a power-of-two prefix of the table that holds the
  // whole run at a quarter of the bounded load factor (the full table until
  // the pairs per history are known; the margin covers runs whose sources
  // leave more pairs per history than the estimate).  The flush scans only
  // these slots, so a small run does not pay for the full table; every slot
  // a run used is empty again after its flush.
  uint64_t slots = c->hslots;
  if (mode == 0 && c->pairs_per_hist > 0.0) {
    const double need = 4.0 * double(n) * 1.25 * c->pairs_per_hist * MCX_TALLY_LOAD_DIV;
    uint64_t sl = std::min<uint64_t>(1ull << 16, c->hslots);
    while (sl < c->hslots && double(sl) < need) sl <<= 1;
    slots = sl;
  }
  a.hmask = slots - 1;
  const uint64_t table_budget = slots / MCX_TALLY_LOAD_DIV;  // bounded load factor: few second probes
  uint64_t done = 0;
  auto t0 = std::chrono::steady_clock::now();
  double flush_ms = 0.0;
  int par = 0;
  // kBatch iterations (parities 0, 1, 0, ...) captured once per run: a batch
  // is then one graph launch; kBatch is even, so every batch starts at parity 0
  hipGraphExec_t gexec = nullptr;
  const bool use_graph = allow_graph && c->use_graph && !c->timing;
  if (use_graph) {
    // capture this run's batch (its kernels and arguments); the context keeps
    // the instantiated graph of the mode's last run and updates it in place
    // when the kernels are the same (only arguments changed), which is much
    // cheaper than instantiating
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    for (int k = 0; k < kBatch && e == hipSuccess; ++k) e = launch_iteration(a, k & 1, target, grid, int(c->block), s, nullptr);
    hipError_t e2 = hipStreamEndCapture(s, &graph);
    if (e == hipSuccess) e = e2;
    hipGraphExec_t& cached = c->gexec[mode];
    if (e == hipSuccess && cached) {
      hipGraphNode_t bad = nullptr;
      hipGraphExecUpdateResult res = hipGraphExecUpdateError;
      if (hipGraphExecUpdate(cached, graph, &bad, &res) == hipSuccess && res == hipGraphExecUpdateSuccess) {
        gexec = cached;
      } else {
        (void)hipGetLastError();
        (void)hipGraphExecDestroy(cached);
        cached = nullptr;
      }
    }
    if (e == hipSuccess && !gexec) {
      e = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
      if (e == hipSuccess) cached = gexec;
    }
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return hip_fail(c, e, "capture of the iteration graph");
    }
  }
  bool cancelled = false;
  while (done < n && !cancelled) {
    uint64_t chunk;
    if (c->pairs_per_hist > 0.0) chunk = uint64_t(double(table_budget) / (1.25 * c->pairs_per_hist));
    else chunk = std::min<uint64_t>(1ull << 16, table_budget / 64);  // first chunk: up to 64 pairs a history
    chunk = std::max<uint64_t>(chunk, 1024);
    chunk = std::min<uint64_t>(chunk, n - done);
    const uint64_t cf = first + done, ce = cf + chunk;
    hipError_t e = launch_chunk_init(a.cnt, cf, ce, first, uint32_t(std::min<uint64_t>(chunk, target)), s);
    if (e != hipSuccess) return hip_fail(c, e, "chunk init launch");
    for (;;) {
      if (use_graph) {
        e = hipGraphLaunch(gexec, s);
        if (e != hipSuccess) return hip_fail(c, e, "graph launch");
        c->iterations += kBatch;
      } else {
        for (int k = 0; k < kBatch; ++k) {
          hipEvent_t* ev = c->timing ? &c->events[size_t(k) * (kTimedKernels + 1)] : nullptr;
          e = launch_iteration(a, par, target, grid, int(c->block), s, ev);
          if (e != hipSuccess) return hip_fail(c, e, "iteration launch");
          par ^= 1;
          c->iterations++;
        }
      }
      e = hipMemcpyAsync(c->h_cnt, a.cnt, sizeof(Counters), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) return hip_fail(c, e, "transport iterations");
      if (c->timing) {
        for (int k = 0; k < kBatch; ++k) {
          const hipEvent_t* ev = &c->events[size_t(k) * (kTimedKernels + 1)];
          for (int j = 0; j < kTimedKernels; ++j) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, ev[j], ev[j + 1]) == hipSuccess) c->ms_kernel[j] += ms;
          }
        }
        c->timed_iterations += kBatch;
      }
      if (c->h_cnt->overflow & OVF_QUEUE)
        return fail(c, MCX_E_RANGE, "event queue overflow (capacity %u records); raise the bank size", c->cap);
      if (c->h_cnt->overflow & OVF_TALLY)
        return fail(c, MCX_E_RANGE, "tally table overflow (%llu slots)", (unsigned long long)slots);
      if (c->h_cnt->overflow & OVF_SOURCE) return fail(c, MCX_E_INVALID, "a source point lies outside the phantom");
      if (c->h_cnt->overflow & OVF_LOST) return fail(c, MCX_E_DEVICE, "a particle lost its direction (no exit face)");
      if (c->h_cnt->done) break;
      if (mode == 0 && !cancelled && c->cancel.exchange(0) != 0) {
        // close admission: the histories admitted so far, [cf, cursor), run
        // to completion and are flushed as usual; no later one starts
        cancelled = true;
        c->h_cnt->chunk_end = c->h_cnt->cursor;
        c->h_cnt->adm = 0u;
        char* dc = reinterpret_cast<char*>(a.cnt);
        e = hipMemcpyAsync(dc + offsetof(Counters, chunk_end), &c->h_cnt->chunk_end, sizeof(uint64_t),
                           hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
          e = hipMemcpyAsync(dc + offsetof(Counters, adm), &c->h_cnt->adm, sizeof(uint32_t), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_fail(c, e, "close admission");
      }
    }
    if (cancelled) chunk = c->h_cnt->chunk_end - cf;
    if (mode != 0) {  // replays leave the tally table untouched
      done += chunk;
      continue;
    }
    auto tf = std::chrono::steady_clock::now();
    uint32_t iovf = 0;
    if (c->influence) {
      e = launch_flush_influence(a.htab, slots, a.sum_q2, a.cnt, c->test_mode, a.hist_led, n, a.src, a.nsrc,
                                 static_cast<uint64_t*>(c->d_ikeys.p), static_cast<double*>(c->d_iq.p),
                                 static_cast<double*>(c->d_iq2.p), c->islots - 1, static_cast<uint32_t*>(c->d_iovf.p), s);
      if (e == hipSuccess) e = hipMemcpyAsync(&iovf, c->d_iovf.p, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    } else {
      e = launch_flush(a.htab, slots, a.sum_q, a.sum_q2, a.cnt, c->test_mode, a.hist_led, n, s);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(c->h_cnt, a.cnt, sizeof(Counters), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(c, e, "tally flush");
    if (iovf) return fail(c, MCX_E_RANGE, "influence table overflow (%llu slots)", (unsigned long long)c->islots);
    flush_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tf).count();
    const double pairs = double(c->h_cnt->occupied);
    c->tally_pairs += c->h_cnt->occupied;
    const double pph = chunk ? pairs / double(chunk) : 0.0;
    c->pairs_per_hist = std::max(c->pairs_per_hist * 0.5, pph);
    if (c->pairs_per_hist < 1.0) c->pairs_per_hist = 1.0;
    c->chunks++;
    done += chunk;
  }
  const double total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (completed) *completed = done;
  if (mode != 0) {
    c->ms_backward += total_ms;
    return MCX_OK;
  }
  c->ms_transport += total_ms - flush_ms;
  c->ms_flush += flush_ms;
  if (cancelled && done < n)  // (a request that came too late to stop any history is dropped)
    return fail(c, MCX_E_CANCELLED, "cancelled: histories [%llu, %llu) are complete", (unsigned long long)first,
                (unsigned long long)(first + done));
  return MCX_OK;
}

// ---------------------------------------------------------------------------
// Fixed device scratch of mcx_run_static, for callers that cannot allocate:
// the event queues and the (history, voxel) tally table of a run live in this
// file-scope array instead of memory the library or the caller allocates.
// Each device the library runs on holds its own copy until the process ends.
// Host code never passes `scratch` itself to a kernel (in host code the name
// is a stand-in, not a device address): mcx_create looks up the address of
// the current device's copy once per device, and only that address is used.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[MCX_STATIC_SCRATCH_BYTES];

constexpr uint32_t kStaticBank = 1u << 16;  // largest bank a static run uses
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices];  // device address of each device's copy
hipError_t g_scratch_rc[kMaxDevices];
bool g_scratch_done[kMaxDevices];

// once per device, with that device current
void static_scratch_init(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_done[dev]) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
  }
  g_scratch[dev] = p;
  g_scratch_rc[dev] = e;
  g_scratch_done[dev] = true;
}

void* static_scratch(int dev, hipError_t* rc) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (dev < 0 || dev >= kMaxDevices || !g_scratch_done[dev]) {
    *rc = hipErrorNotInitialized;
    return nullptr;
  }
  *rc = g_scratch_rc[dev];
  return g_scratch[dev];
}

// checks shared by mcx_run and mcx_run_static
int check_run(mcx_ctx* c, uint64_t seed, uint64_t first, uint64_t n) {
  if (!c->have_sources || !c->have_material || !c->have_phantom)
    return fail(c, MCX_E_STATE, "set transport, material, phantom and sources first");
  if (seed > 0xFFFFFFFFull) return fail(c, MCX_E_INVALID, "seed must be < 2^32");
  for (int k = 0; k <= c->vmat_max; ++k)
    if (!c->have_mat[k]) return fail(c, MCX_E_STATE, "the phantom uses material %d, which is not loaded", k);
  if (first + n > c->total_hist || first + n < first) return fail(c, MCX_E_RANGE, "history range exceeds the sources");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, MCX_E_DEVICE, "hipSetDevice");
  return MCX_OK;
}

// bookkeeping of a complete (or cancelled) forward run
void record_run(mcx_ctx* c, uint64_t seed, uint64_t first, uint64_t n, uint64_t completed) {
  c->n_done += completed;
  c->next_history = first + completed;
  c->run_seed = uint32_t(seed);
  c->run_first = first;
  c->run_n = completed;
  c->run_known = completed > 0 && c->n_done == completed;
  c->last_n = n;
  c->last_valid = c->test_mode != 0;
}

}  // namespace

extern "C" {

int mcx_create(mcx_ctx** out, int hip_device, int precision) {
  if (!out) return MCX_E_INVALID;
  *out = nullptr;
  if (precision != MCX_FP64 && precision != MCX_MIXED) return MCX_E_INVALID;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev) {
    (void)hipGetLastError();
    return MCX_E_DEVICE;
  }
  mcx_ctx* c = new (std::nothrow) mcx_ctx();
  if (!c) return MCX_E_NOMEM;
  c->device = hip_device;
  c->precision = precision;
  if (hipSetDevice(hip_device) != hipSuccess || hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    delete c;
    return MCX_E_DEVICE;
  }
  // the loop and statistics counters, on the device and pinned on the host
  hipError_t e = hipMalloc(&c->d_cnt.p, sizeof(Counters));
  if (e == hipSuccess) {
    c->d_cnt.bytes = sizeof(Counters);
    e = hipMemsetAsync(c->d_cnt.p, 0, sizeof(Counters), c->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&c->h_cnt), sizeof(Counters), hipHostMallocDefault);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    mcx_destroy(c);
    return MCX_E_NOMEM;
  }
  // this device's copy of the fixed scratch array (mcx_run_static)
  static_scratch_init(hip_device);
  *out = c;
  return MCX_OK;
}

void mcx_destroy(mcx_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (hipEvent_t ev : c->events) (void)hipEventDestroy(ev);
  for (DevBuf* b : {&c->d_tab, &c->d_rho, &c->d_cube, &c->d_src, &c->d_sumq, &c->d_sumq2, &c->d_queues, &c->d_cnt, &c->d_htab,
                    &c->d_ikeys, &c->d_iq, &c->d_iq2, &c->d_iovf, &c->d_vmat, &c->d_adj_w, &c->d_adj_q,
                    &c->d_adj_grad,
                    &c->d_adj_dl, &c->d_adj_out,
                    &c->d_adj_sum, &c->d_hhash, &c->d_hled})
    dfree(*b);
  if (c->h_cnt) (void)hipHostFree(c->h_cnt);
  for (hipGraphExec_t& g : c->gexec)
    if (g) (void)hipGraphExecDestroy(g);
  if (c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

const char* mcx_last_error(mcx_ctx* c) { return c ? c->err.c_str() : "null context"; }

int mcx_set_transport(mcx_ctx* c, const mcx_transport* t) {
  if (!c) return MCX_E_INVALID;
  if (!t) return fail(c, MCX_E_INVALID, "null transport");
  if (t->n_grid < 16 || t->n_grid > kMaxGrid) return fail(c, MCX_E_INVALID, "n_grid must be in [16, %d]", kMaxGrid);
  if (!(t->e_min > 0.0) || !(t->e_max > t->e_min)) return fail(c, MCX_E_INVALID, "need 0 < e_min < e_max");
  if (!(t->c1 > 0.0 && t->c1 <= 0.2 && t->c2 > 0.0 && t->c2 <= 0.2))
    return fail(c, MCX_E_INVALID, "C1 and C2 must lie in (0, 0.2]");
  if (!(t->wcc > 0.0) || !(t->wcr > 0.0)) return fail(c, MCX_E_INVALID, "Wcc and Wcr must be positive");
  for (int i = 0; i < 3; ++i)
    if (!(t->eabs[i] >= t->e_min)) return fail(c, MCX_E_INVALID, "Eabs must be >= e_min");
  for (double f : {t->force_in, t->force_br})
    if (!(f == 0.0 || (f >= 1.0 && f <= kMaxForce)))
      return fail(c, MCX_E_INVALID, "forcing factors must be 0 (none) or in [1, %g]", kMaxForce);
  if (t->split_br < 0 || t->split_br > 2) return fail(c, MCX_E_INVALID, "split_br must be 0, 1 or 2");
  c->tr = *t;
  c->have_transport = true;
  c->have_material = false;
  for (bool& h : c->have_mat) h = false;
  c->run_known = false;  // the gradient replays would run other physics
  return MCX_OK;
}

int mcx_load_material(mcx_ctx* c, int mat_id, const mcx_material_desc* m) {
  if (!c) return MCX_E_INVALID;
  if (!m) return fail(c, MCX_E_INVALID, "null material");
  if (mat_id < 0 || mat_id >= kMaxMat) return fail(c, MCX_E_UNSUPPORTED, "material ids are 0..%d", kMaxMat - 1);
  if (!c->have_transport) return fail(c, MCX_E_STATE, "set the transport parameters first");
  const double pos[] = {m->z_mol, m->a_mol, m->zz1_mol, m->z_screen, m->i_exc, m->pe_eref, m->ray_a};
  for (double v : pos)
    if (!(v > 0.0)) return fail(c, MCX_E_INVALID, "material parameters must be positive");
  if (!(m->pe_coef >= 0.0) || !(m->pp_coef >= 0.0) || !(m->ray_f0 >= 0.0) || !(m->brems_b >= 0.0))
    return fail(c, MCX_E_INVALID, "material coefficients must be non-negative");
  std::string err;
  BuiltTables b;
  if (!build_tables(*m, c->tr, &b, &err)) return fail(c, MCX_E_INVALID, "%s", err.c_str());
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, MCX_E_DEVICE, "hipSetDevice");
  c->run_known = false;  // the gradient replays would run other tables
  c->mtabs[mat_id] = std::move(b);
  c->have_mat[mat_id] = true;
  if (mat_id == 0) {
    c->tabs = c->mtabs[0];
    c->mat = *m;
    c->have_material = true;
  }
  if (!c->have_material) return MCX_OK;  // uploaded once material 0 is there
  // device block: material 0's channels, the soft-law table, then the
  // channels of materials 1, 2, ... (missing ones hold material 0's)
  const int n = c->tabs.n;
  const size_t ch = size_t(T_NCH) * n;
  int nm = 1;
  for (int k = 1; k < kMaxMat; ++k)
    if (c->have_mat[k]) nm = k + 1;
  std::vector<double> blk(c->tabs.block.begin(), c->tabs.block.end());
  for (int k = 1; k < nm; ++k) {
    const BuiltTables& bk = c->have_mat[k] ? c->mtabs[k] : c->tabs;
    blk.insert(blk.end(), bk.block.begin(), bk.block.begin() + ch);
  }
  int rc;
  const size_t bytes = blk.size() * tsize(c);
  if ((rc = dalloc(c, c->d_tab, bytes, "tables"))) return rc;
  hipError_t e;
  if (fp64(c)) {
    e = hipMemcpy(c->d_tab.p, blk.data(), bytes, hipMemcpyHostToDevice);
  } else {
    std::vector<float> f(blk.begin(), blk.end());
    e = hipMemcpy(c->d_tab.p, f.data(), bytes, hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) return hip_fail(c, e, "copy tables");
  e = configure_kernels(n, fp64(c));
  if (e != hipSuccess) return hip_fail(c, e, "configure kernels");
  return MCX_OK;
}

int mcx_reset_tallies(mcx_ctx* c) {
  if (!c) return MCX_E_INVALID;
  if (!c->have_phantom) return fail(c, MCX_E_STATE, "no phantom");
  (void)hipSetDevice(c->device);
  const size_t bytes = nvox(c) * sizeof(double);
  hipError_t e = hipMemsetAsync(c->d_sumq.p, 0, bytes, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->d_sumq2.p, 0, bytes, c->stream);
  if (e == hipSuccess && c->d_cnt.p) e = hipMemsetAsync(c->d_cnt.p, 0, sizeof(Counters), c->stream);
  if (e == hipSuccess && c->influence) {
    e = hipMemsetAsync(c->d_ikeys.p, 0xFF, c->islots * sizeof(uint64_t), c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->d_iq.p, 0, c->islots * sizeof(double), c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->d_iq2.p, 0, c->islots * sizeof(double), c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->d_iovf.p, 0, sizeof(uint32_t), c->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "reset tallies");
  c->n_done = 0;
  c->run_known = false;
  c->iterations = c->chunks = c->tally_pairs = 0;
  c->ms_transport = c->ms_flush = 0.0;
  for (double& m : c->ms_kernel) m = 0.0;
  c->ms_backward = 0.0;
  c->timed_iterations = 0;
  return MCX_OK;
}

int mcx_load_phantom(mcx_ctx* c, const mcx_phantom_desc* p) {
  if (!c) return MCX_E_INVALID;
  if (!p || !p->rho) return fail(c, MCX_E_INVALID, "null phantom");
  if (p->nx < 1 || p->ny < 1 || p->nz < 1 || p->nx > 1024 || p->ny > 1024 || p->nz > 1024)
    return fail(c, MCX_E_INVALID, "grid dimensions must be in [1, 1024]");
  for (int k = 0; k < 3; ++k)
    if (!(p->voxel_cm[k] > 0.0) || !std::isfinite(p->origin_cm[k]))
      return fail(c, MCX_E_INVALID, "voxel sizes must be positive and origins finite");
  (void)hipSetDevice(c->device);
  const uint64_t nv = uint64_t(p->nx) * p->ny * p->nz;
  // every check on the host before any device state changes
  std::vector<double> h(nv);
  hipError_t e = hipMemcpy(h.data(), p->rho, nv * sizeof(double),
                           p->rho_on_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost);
  if (e != hipSuccess) return hip_fail(c, e, "read densities");
  for (uint64_t v = 0; v < nv; ++v)
    if (!(h[v] > 0.0) || !std::isfinite(h[v])) return fail(c, MCX_E_INVALID, "density must be > 0 (voxel %llu)", (unsigned long long)v);
  int mx = -1;
  if (p->mat) {
    mx = 0;
    for (uint64_t v = 0; v < nv; ++v) {
      if (p->mat[v] >= kMaxMat) return fail(c, MCX_E_INVALID, "material index %d >= %d (voxel %llu)", int(p->mat[v]),
                                            kMaxMat, (unsigned long long)v);
      mx = std::max(mx, int(p->mat[v]));
    }
  }
  // from here on the old phantom is gone: a failure leaves none (MCX_E_STATE
  // for runs and gradients until a load succeeds)
  c->have_phantom = false;
  c->run_known = false;
  c->n_done = 0;
  int rc;
  if ((rc = dalloc(c, c->d_rho, nv * tsize(c), "densities"))) return rc;
  if (fp64(c)) {
    e = hipMemcpy(c->d_rho.p, h.data(), nv * sizeof(double), hipMemcpyHostToDevice);
  } else {
    std::vector<float> f(h.begin(), h.end());
    e = hipMemcpy(c->d_rho.p, f.data(), nv * sizeof(float), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) return hip_fail(c, e, "copy densities");
  // per-voxel materials (several-material kernels), else none
  c->vmat_max = -1;
  dfree(c->d_vmat);
  if (p->mat) {
    if ((rc = dalloc(c, c->d_vmat, nv, "voxel materials"))) return rc;
    e = hipMemcpy(c->d_vmat.p, p->mat, nv, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(c, e, "copy voxel materials");
    c->vmat_max = mx;
  }
  // same-density (and same-material) cubes for the photon walk (a scratch
  // byte per voxel while the map is built)
  if ((rc = dalloc(c, c->d_cube, nv, "same-density cube map"))) return rc;
  {
    DevBuf tmp;
    if ((rc = dalloc(c, tmp, nv, "cube map scratch"))) return rc;
    const uint8_t* vm = static_cast<const uint8_t*>(c->d_vmat.p);
    e = fp64(c) ? launch_cube_map(static_cast<const double*>(c->d_rho.p), vm, p->nx, p->ny, p->nz,
                                  static_cast<uint8_t*>(c->d_cube.p), static_cast<uint8_t*>(tmp.p), c->stream)
                : launch_cube_map(static_cast<const float*>(c->d_rho.p), vm, p->nx, p->ny, p->nz,
                                  static_cast<uint8_t*>(c->d_cube.p), static_cast<uint8_t*>(tmp.p), c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    dfree(tmp);
    if (e != hipSuccess) return hip_fail(c, e, "same-density cube map");
  }
  if ((rc = dalloc(c, c->d_sumq, nv * sizeof(double), "Sum q"))) return rc;
  if ((rc = dalloc(c, c->d_sumq2, nv * sizeof(double), "Sum q^2"))) return rc;
  c->nx = p->nx; c->ny = p->ny; c->nz = p->nz;
  for (int k = 0; k < 3; ++k) {
    c->vox[k] = p->voxel_cm[k];
    c->org[k] = p->origin_cm[k];
  }
  c->have_phantom = true;
  return mcx_reset_tallies(c);
}

static bool inside(const mcx_ctx* c, double x, double y, double z) {
  const double p[3] = {x, y, z};
  const int n[3] = {c->nx, c->ny, c->nz};
  for (int k = 0; k < 3; ++k) {
    const double f = std::floor((p[k] - c->org[k]) / c->vox[k]);
    if (!(f >= 0.0) || !(f < double(n[k]))) return false;
  }
  return true;
}

int mcx_set_sources(mcx_ctx* c, const mcx_source* s, int n) {
  if (!c) return MCX_E_INVALID;
  if (!s || n < 1) return fail(c, MCX_E_INVALID, "need at least one source");
  if (!c->have_phantom || !c->have_material) return fail(c, MCX_E_STATE, "load the material and phantom first");
  std::vector<SourceDev> v(n);
  uint64_t total = 0;
  for (int i = 0; i < n; ++i) {
    const mcx_source& q = s[i];
    if (q.particle < 0 || q.particle > 2) return fail(c, MCX_E_INVALID, "source %d: bad particle", i);
    if (q.kind != MCX_SRC_PENCIL && q.kind != MCX_SRC_RECT) return fail(c, MCX_E_INVALID, "source %d: bad kind", i);
    if (!(q.energy > c->tr.eabs[q.particle]) || !(q.energy <= c->tr.e_max))
      return fail(c, MCX_E_RANGE, "source %d: energy must lie in (Eabs, e_max]", i);
    const double nn = std::sqrt(q.dir[0] * q.dir[0] + q.dir[1] * q.dir[1] + q.dir[2] * q.dir[2]);
    if (!(std::fabs(nn - 1.0) < 1e-9)) return fail(c, MCX_E_INVALID, "source %d: direction is not a unit vector", i);
    if (q.kind == MCX_SRC_PENCIL) {
      if (!inside(c, q.pos[0], q.pos[1], q.pos[2])) return fail(c, MCX_E_INVALID, "source %d: start outside the phantom", i);
    } else {
      if (!(q.width[0] >= 0.0) || !(q.width[1] >= 0.0)) return fail(c, MCX_E_INVALID, "source %d: bad width", i);
      const double hx = 0.5 * q.width[0], hy = 0.5 * q.width[1];
      for (int sx = -1; sx <= 1; sx += 2)
        for (int sy = -1; sy <= 1; sy += 2)
          if (!inside(c, q.pos[0] + sx * hx, q.pos[1] + sy * hy, q.pos[2]))
            return fail(c, MCX_E_INVALID, "source %d: rectangle leaves the phantom", i);
    }
    SourceDev& d = v[i];
    d.particle = q.particle;
    d.kind = q.kind;
    d.energy = q.energy;
    for (int k = 0; k < 3; ++k) {
      d.pos[k] = q.pos[k];
      d.dir[k] = q.dir[k];
    }
    d.width[0] = q.width[0];
    d.width[1] = q.width[1];
    total += q.n_hist;
    d.end = total;
  }
  if (total > 0xFFFFFFFFull) return fail(c, MCX_E_RANGE, "more than 2^32 histories");
  (void)hipSetDevice(c->device);
  int rc;
  if ((rc = dalloc(c, c->d_src, v.size() * sizeof(SourceDev), "sources"))) return rc;
  hipError_t e = hipMemcpy(c->d_src.p, v.data(), v.size() * sizeof(SourceDev), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(c, e, "copy sources");
  c->src = std::move(v);
  c->total_hist = total;
  c->have_sources = true;
  c->run_known = false;  // the gradient replays would start other histories
  return MCX_OK;
}

int mcx_set_launch(mcx_ctx* c, uint32_t bank, uint32_t block, uint32_t steps) {
  if (!c) return MCX_E_INVALID;
  if (bank) {
    if (bank < 1024 || bank > (1u << 26)) return fail(c, MCX_E_INVALID, "bank must lie in [1024, 2^26]");
    c->cap = bank;
  }
  if (block) {
    if (block % 64 || block > uint32_t(kMaxBlock))
      return fail(c, MCX_E_INVALID, "block must be a multiple of 64, <= %d", kMaxBlock);
    c->block = block;
  }
  if (steps) {
    if (steps > 4096) return fail(c, MCX_E_INVALID, "steps must be <= 4096");
    c->steps = steps;
  }
  return MCX_OK;
}

int mcx_set_gradient(mcx_ctx* c, uint32_t flags) {
  if (!c) return MCX_E_INVALID;
  if (flags & ~uint32_t(MCX_GRAD_DEFLECTION_ENERGY)) return fail(c, MCX_E_INVALID, "unknown gradient flags 0x%x", flags);
  c->grad_flags = flags;
  return MCX_OK;
}

int mcx_set_timing(mcx_ctx* c, int on) {
  if (!c) return MCX_E_INVALID;
  if (on && c->events.empty()) {
    (void)hipSetDevice(c->device);
    c->events.resize(size_t(kBatch) * (kTimedKernels + 1));
    for (hipEvent_t& ev : c->events) {
      hipError_t e = hipEventCreate(&ev);
      if (e != hipSuccess) {
        c->events.clear();
        return hip_fail(c, e, "hipEventCreate");
      }
    }
  }
  c->timing = on ? 1 : 0;
  return MCX_OK;
}

int mcx_set_graph(mcx_ctx* c, int on) {
  if (!c) return MCX_E_INVALID;
  c->use_graph = on ? 1 : 0;
  return MCX_OK;
}

// FNV-1a over the bytes that shape the workload
static uint64_t fnv(uint64_t h, const void* p, size_t n) {
  const unsigned char* b = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
  return h;
}

int mcx_autotune(mcx_ctx* c, uint64_t n_sample, const char* cache_path, uint32_t* chosen) {
  if (!c) return MCX_E_INVALID;
  if (!c->have_sources) return fail(c, MCX_E_STATE, "set transport, material, phantom and sources first");
  if (n_sample == 0 || n_sample > c->total_hist) n_sample = std::min<uint64_t>(c->total_hist, 200000);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c->device) != hipSuccess) return fail(c, MCX_E_DEVICE, "device properties");
  uint64_t h = 1469598103934665603ull;
  h = fnv(h, prop.gcnArchName, std::strlen(prop.gcnArchName));
  h = fnv(h, &c->precision, sizeof(c->precision));
  const int dims[3] = {c->nx, c->ny, c->nz};
  h = fnv(h, dims, sizeof(dims));
  h = fnv(h, &c->tr, sizeof(c->tr));
  for (const SourceDev& sd : c->src) {
    h = fnv(h, &sd.particle, sizeof(sd.particle));
    h = fnv(h, &sd.energy, sizeof(sd.energy));
    h = fnv(h, &sd.end, sizeof(sd.end));
  }
  char key[32];
  std::snprintf(key, sizeof(key), "%016llx", (unsigned long long)h);
  if (cache_path) {
    if (FILE* f = std::fopen(cache_path, "r")) {
      char line[512];
      while (std::fgets(line, sizeof(line), f)) {
        char k[64];
        unsigned b = 0, bl = 0, st = 0;
        if (std::sscanf(line, "{\"key\": \"%63[0-9a-f]\", \"bank\": %u, \"block\": %u, \"steps\": %u", k, &b, &bl,
                        &st) == 4 &&
            std::strcmp(k, key) == 0) {
          std::fclose(f);
          int rc = mcx_set_launch(c, b, bl, st);
          if (!rc && chosen) { chosen[0] = b; chosen[1] = bl; chosen[2] = st; }
          return rc;
        }
      }
      std::fclose(f);
    }
  }
  // Bank size by rule, not by timing: its population target (a quarter of
  // it) should hold every history of the run at once, up to 2^24, within a
  // quarter of the device memory.  A sample small enough to time cannot show
  // the bank's effect (every candidate admits the whole sample at once).
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return fail(c, MCX_E_DEVICE, "device memory size");
  const uint32_t saved_cap = c->cap;
  uint32_t bank = 1u << 20;
  while (bank < (1u << 26) && uint64_t(bank / 4) < std::min<uint64_t>(c->total_hist, 1ull << 24)) bank <<= 1;
  for (;;) {
    c->cap = bank;
    const size_t qb = queue_bytes(c);
    if (bank <= (1u << 20) || qb <= total_b / 4) break;
    bank >>= 1;
  }
  c->cap = saved_cap;
  const uint32_t banks[] = {bank};
  const uint32_t blocks[] = {128u, 256u};
  const uint32_t steps[] = {32u, 128u, 512u};
  double best = 0.0;
  uint32_t bb = c->cap, bbl = c->block, bst = c->steps;
  const int test = c->test_mode;
  c->test_mode = 0;
  int rc = MCX_OK;
  for (uint32_t b : banks)
    for (uint32_t bl : blocks)
      for (uint32_t st : steps) {
        if ((rc = mcx_set_launch(c, b, bl, st))) break;
        if ((rc = mcx_reset_tallies(c))) break;
        auto t0 = std::chrono::steady_clock::now();
        if ((rc = mcx_run(c, 12345, 0, n_sample, nullptr))) break;
        const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        const double rate = double(n_sample) / dt;
        if (rate > best) { best = rate; bb = b; bbl = bl; bst = st; }
      }
  c->test_mode = test;
  if (rc) return rc;
  if ((rc = mcx_set_launch(c, bb, bbl, bst))) return rc;
  if ((rc = mcx_reset_tallies(c))) return rc;
  if (chosen) { chosen[0] = bb; chosen[1] = bbl; chosen[2] = bst; }
  if (cache_path) {
    if (FILE* f = std::fopen(cache_path, "a")) {
      std::fprintf(f, "{\"key\": \"%s\", \"bank\": %u, \"block\": %u, \"steps\": %u, \"hist_per_s\": %.6g, \"device\": \"%s\"}\n",
                   key, bb, bbl, bst, best, prop.gcnArchName);
      std::fclose(f);
    }
  }
  return MCX_OK;
}

int mcx_set_test_mode(mcx_ctx* c, int on) {
  if (!c) return MCX_E_INVALID;
  c->test_mode = on ? 1 : 0;
  return MCX_OK;
}

int mcx_run(mcx_ctx* c, uint64_t seed, uint64_t first, uint64_t n, void* stream) {
  if (!c) return MCX_E_INVALID;
  int rc = check_run(c, seed, first, n);
  if (rc) return rc;
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : c->stream;
  c->last_valid = false;
  if (n == 0) return MCX_OK;
  if ((rc = ensure_workspace(c))) return rc;
  if (c->table_dirty) {
    hipError_t e = launch_clear_table(static_cast<TSlot*>(c->d_htab.p), c->hslots, s);
    if (e != hipSuccess) return hip_fail(c, e, "clear tally table");
  }
  c->table_dirty = true;
  if (c->test_mode) {
    if ((rc = dalloc(c, c->d_hhash, n * sizeof(uint64_t), "history hashes"))) return rc;
    if ((rc = dalloc(c, c->d_hled, 3 * n * sizeof(double), "history ledger"))) return rc;
    hipError_t e = hipMemsetAsync(c->d_hhash.p, 0, n * sizeof(uint64_t), s);
    if (e == hipSuccess) e = hipMemsetAsync(c->d_hled.p, 0, 3 * n * sizeof(double), s);
    if (e != hipSuccess) return hip_fail(c, e, "clear history results");
  }
  uint64_t completed = 0;
  rc = fp64(c) ? run_impl<double>(c, uint32_t(seed), first, n, s, 0, 0.0, &completed)
               : run_impl<float>(c, uint32_t(seed), first, n, s, 0, 0.0, &completed);
  if (rc && rc != MCX_E_CANCELLED) return rc;
  // complete, or cancelled with [first, first + completed) done and flushed
  c->table_dirty = false;
  record_run(c, seed, first, n, completed);
  return rc;
}

int mcx_run_static(mcx_ctx* c, uint64_t seed, uint64_t first, uint64_t n, void* stream) {
  if (!c) return MCX_E_INVALID;
  int rc = check_run(c, seed, first, n);
  if (rc) return rc;
  if (c->test_mode)
    return fail(c, MCX_E_UNSUPPORTED, "test mode needs per-history buffers sized by the run: use mcx_run");
  hipError_t e;
  char* base = static_cast<char*>(static_scratch(c->device, &e));
  if (!base) return fail(c, MCX_E_DEVICE, "no static scratch on device %d: %s", c->device, hipGetErrorString(e));
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : c->stream;
  c->last_valid = false;
  if (n == 0) return MCX_OK;
  // the queues of the bank (the configured one, at most kStaticBank
  // records), then the largest power-of-two tally table that fits
  struct Saved {
    mcx_ctx* c;
    uint32_t cap;
    DevBuf q, t;
    uint64_t hslots;
    size_t built;
    ~Saved() {
      c->cap = cap;
      c->d_queues = q;
      c->d_htab = t;
      c->hslots = hslots;
      c->queue_cap_built = built;
    }
  } saved{c, c->cap, c->d_queues, c->d_htab, c->hslots, c->queue_cap_built};
  c->cap = std::min(c->cap, kStaticBank);
  const size_t qb = align256(queue_bytes(c));
  uint64_t slots = kTableSlots;
  while (slots > 1 && qb + slots * kSlotBytes > size_t(MCX_STATIC_SCRATCH_BYTES)) slots >>= 1;
  if (qb + slots * kSlotBytes > size_t(MCX_STATIC_SCRATCH_BYTES) || slots < kMinWsSlots)
    return fail(c, MCX_E_RANGE, "static scratch of %zu bytes holds no bank of %u records with a table of 2^20 slots",
                size_t(MCX_STATIC_SCRATCH_BYTES), c->cap);
  c->d_queues = DevBuf{base, qb, true};
  c->d_htab = DevBuf{base + qb, slots * kSlotBytes, true};
  c->hslots = slots;
  c->queue_cap_built = c->cap;
  // the array keeps the last call's contents: an empty table to start (a
  // kernel, not a memset: a caller may capture the work of a static run)
  e = launch_clear_table(static_cast<TSlot*>(c->d_htab.p), slots, s);
  if (e != hipSuccess) return hip_fail(c, e, "clear static tally table");
  uint64_t completed = 0;
  // no graph: instantiating one allocates
  rc = fp64(c) ? run_impl<double>(c, uint32_t(seed), first, n, s, 0, 0.0, &completed, false)
               : run_impl<float>(c, uint32_t(seed), first, n, s, 0, 0.0, &completed, false);
  if (rc && rc != MCX_E_CANCELLED) return rc;
  record_run(c, seed, first, n, completed);
  return rc;
}

int mcx_dose_backward(mcx_ctx* c, const double* dl_ddose, double* dl_drho, int on_device, void* stream) {
  if (!c) return MCX_E_INVALID;
  if (!dl_ddose || !dl_drho) return fail(c, MCX_E_INVALID, "null gradient array");
  if (!c->run_known || !c->have_sources || !c->have_material || !c->have_phantom ||
      c->run_first + c->run_n > c->total_hist)
    return fail(c, MCX_E_STATE, "the tallies must hold exactly one run since the last reset, with its setup unchanged");
  for (int k = 0; k <= c->vmat_max; ++k)
    if (!c->have_mat[k]) return fail(c, MCX_E_STATE, "the phantom uses material %d, which is not loaded", k);
  if (c->tr.flags & MCX_STRAGGLING)
    return fail(c, MCX_E_UNSUPPORTED, "the gradient has no term for a straggled soft loss");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, MCX_E_DEVICE, "hipSetDevice");
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : c->stream;
  const uint64_t nv = nvox(c), n = c->run_n;
  int rc;
  if ((rc = dalloc(c, c->d_adj_w, nv * sizeof(double), "gradient weights")) ||
      (rc = dalloc(c, c->d_adj_grad, nv * sizeof(double), "gradient accumulator")) ||
      (rc = dalloc(c, c->d_adj_q, n * sizeof(double), "history scores")) ||
      (rc = dalloc(c, c->d_adj_sum, sizeof(double), "score sum")))
    return rc;
  const double* dl = dl_ddose;
  double* out = dl_drho;
  if (!on_device) {
    if ((rc = dalloc(c, c->d_adj_dl, nv * sizeof(double), "loss gradient")) ||
        (rc = dalloc(c, c->d_adj_out, nv * sizeof(double), "density gradient")))
      return rc;
    hipError_t e = hipMemcpyAsync(c->d_adj_dl.p, dl_ddose, nv * sizeof(double), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(c, e, "copy loss gradient");
    dl = static_cast<const double*>(c->d_adj_dl.p);
    out = static_cast<double*>(c->d_adj_out.p);
  }
  // the statistics describe the forward run: keep them across the replays
  Counters saved;
  hipError_t e = hipMemcpyAsync(&saved, c->d_cnt.p, sizeof(Counters), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(c, e, "save statistics");
  const uint64_t iters = c->iterations, chunks = c->chunks;
  const double vol = c->vox[0] * c->vox[1] * c->vox[2];
  e = fp64(c) ? launch_adjoint_weights(dl, static_cast<const double*>(c->d_rho.p), nv, vol,
                                       static_cast<double*>(c->d_adj_w.p), s)
              : launch_adjoint_weights(dl, static_cast<const float*>(c->d_rho.p), nv, vol,
                                       static_cast<double*>(c->d_adj_w.p), s);
  if (e == hipSuccess) e = hipMemsetAsync(c->d_adj_grad.p, 0, nv * sizeof(double), s);
  if (e == hipSuccess) e = hipMemsetAsync(c->d_adj_q.p, 0, n * sizeof(double), s);
  if (e == hipSuccess) e = hipMemsetAsync(c->d_adj_sum.p, 0, sizeof(double), s);
  if (e != hipSuccess) return hip_fail(c, e, "prepare gradient");
  const int test = c->test_mode;
  c->test_mode = 0;
  // replay A: Q_h per history and the local soft-loss derivative
  rc = fp64(c) ? run_impl<double>(c, c->run_seed, c->run_first, n, s, 1)
               : run_impl<float>(c, c->run_seed, c->run_first, n, s, 1);
  double qsum = 0.0;
  if (!rc) {
    e = launch_sum(static_cast<const double*>(c->d_adj_q.p), n, static_cast<double*>(c->d_adj_sum.p), s);
    if (e == hipSuccess) e = hipMemcpyAsync(&qsum, c->d_adj_sum.p, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) rc = hip_fail(c, e, "score mean");
  }
  // replay B: (Q_h - Qbar) times the free-flight scores
  if (!rc)
    rc = fp64(c) ? run_impl<double>(c, c->run_seed, c->run_first, n, s, 2, qsum / double(n))
                 : run_impl<float>(c, c->run_seed, c->run_first, n, s, 2, qsum / double(n));
  c->test_mode = test;
  c->iterations = iters;
  c->chunks = chunks;
  if (rc) return rc;
  e = fp64(c) ? launch_adjoint_finalize(static_cast<const double*>(c->d_adj_grad.p), dl,
                                        static_cast<const double*>(c->d_sumq.p),
                                        static_cast<const double*>(c->d_rho.p), nv, vol, double(n), out, s)
              : launch_adjoint_finalize(static_cast<const double*>(c->d_adj_grad.p), dl,
                                        static_cast<const double*>(c->d_sumq.p),
                                        static_cast<const float*>(c->d_rho.p), nv, vol, double(n), out, s);
  if (e == hipSuccess && !on_device) e = hipMemcpyAsync(dl_drho, out, nv * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(c->d_cnt.p, &saved, sizeof(Counters), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(c, e, "finalize gradient");
  return MCX_OK;
}

int mcx_get_tally(mcx_ctx* c, double* sum_q, double* sum_q2, int dst_on_device, void* stream) {
  if (!c) return MCX_E_INVALID;
  if (!c->have_phantom) return fail(c, MCX_E_STATE, "no phantom");
  (void)hipSetDevice(c->device);
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : c->stream;
  const size_t bytes = nvox(c) * sizeof(double);
  const hipMemcpyKind k = dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  hipError_t e = hipSuccess;
  if (sum_q) e = hipMemcpyAsync(sum_q, c->d_sumq.p, bytes, k, s);
  if (e == hipSuccess && sum_q2) e = hipMemcpyAsync(sum_q2, c->d_sumq2.p, bytes, k, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(c, e, "copy tally");
  return MCX_OK;
}

int mcx_get_dose(mcx_ctx* c, double* dose, double* sigma, int dst_on_device, void* stream) {
  if (!c) return MCX_E_INVALID;
  if (!dose) return fail(c, MCX_E_INVALID, "null dose");
  if (!c->have_phantom) return fail(c, MCX_E_STATE, "no phantom");
  if (c->n_done == 0) return fail(c, MCX_E_STATE, "no histories have been run");
  (void)hipSetDevice(c->device);
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : c->stream;
  const uint64_t nv = nvox(c);
  double* dd = dose;
  double* ds = sigma;
  DevBuf tmp;
  if (!dst_on_device) {
    int rc = dalloc(c, tmp, 2 * nv * sizeof(double), "dose staging");
    if (rc) return rc;
    dd = static_cast<double*>(tmp.p);
    ds = sigma ? dd + nv : nullptr;
  }
  const double vol = c->vox[0] * c->vox[1] * c->vox[2];
  hipError_t e = fp64(c) ? launch_dose(static_cast<double*>(c->d_sumq.p), static_cast<double*>(c->d_sumq2.p),
                                       static_cast<const double*>(c->d_rho.p), nv, vol, double(c->n_done), dd, ds, s)
                         : launch_dose(static_cast<double*>(c->d_sumq.p), static_cast<double*>(c->d_sumq2.p),
                                       static_cast<const float*>(c->d_rho.p), nv, vol, double(c->n_done), dd, ds, s);
  if (e == hipSuccess && !dst_on_device) {
    e = hipMemcpyAsync(dose, dd, nv * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && sigma) e = hipMemcpyAsync(sigma, ds, nv * sizeof(double), hipMemcpyDeviceToHost, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  dfree(tmp);
  if (e != hipSuccess) return hip_fail(c, e, "dose");
  return MCX_OK;
}

int mcx_get_stats(mcx_ctx* c, mcx_stats* out) {
  if (!c || !out) return MCX_E_INVALID;
  std::memset(out, 0, sizeof(*out));
  out->histories = c->n_done;
  out->iterations = c->iterations;
  out->chunks = c->chunks;
  out->tally_pairs = c->tally_pairs;
  out->ms_transport = c->ms_transport;
  out->ms_flush = c->ms_flush;
  out->ms_source = c->ms_kernel[0];
  out->ms_flight = c->ms_kernel[1];
  out->ms_knock = c->ms_kernel[2];
  out->ms_estep = c->ms_kernel[3];
  out->timed_iterations = c->timed_iterations;
  out->ms_backward = c->ms_backward;
  out->next_history = c->next_history;
  if (!c->d_cnt.p) return MCX_OK;
  (void)hipSetDevice(c->device);
  Counters h;
  hipError_t e = hipMemcpy(&h, c->d_cnt.p, sizeof(Counters), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(c, e, "read statistics");
  out->flights = h.stat[S_FLIGHTS];
  out->compton = h.stat[S_COMPTON];
  out->photo = h.stat[S_PHOTO];
  out->rayleigh = h.stat[S_RAYLEIGH];
  out->pair = h.stat[S_PAIR];
  out->esteps = h.stat[S_ESTEPS];
  out->hard_el = h.stat[S_HARD_EL];
  out->hard_in = h.stat[S_HARD_IN];
  out->hard_br = h.stat[S_HARD_BR];
  out->delta = h.stat[S_DELTA];
  out->annih = h.stat[S_ANNIH];
  out->crossings = h.stat[S_CROSSINGS];
  out->secondaries = h.stat[S_SECONDARIES];
  out->deposits = h.stat[S_DEPOSITS];
  out->absorbed = h.stat[S_ABSORBED];
  out->escaped = h.stat[S_ESCAPED];
  out->pos_esc = h.stat[S_POSESC];
  out->evisits = h.stat[S_EVISITS];
  out->ewrites = h.stat[S_EWRITES];
  out->inserts = h.stat[S_INSERTS];
  out->annih_flight = h.stat[S_ANNIH_FLIGHT];
  out->e_dep = h.e_dep;
  out->e_esc = h.e_esc;
  return MCX_OK;
}

int mcx_get_history_results(mcx_ctx* c, uint64_t* hashes, double* ledger) {
  if (!c) return MCX_E_INVALID;
  if (!c->last_valid) return fail(c, MCX_E_STATE, "the last run was not in test mode");
  (void)hipSetDevice(c->device);
  hipError_t e = hipSuccess;
  if (hashes) e = hipMemcpy(hashes, c->d_hhash.p, c->last_n * sizeof(uint64_t), hipMemcpyDeviceToHost);
  if (e == hipSuccess && ledger) e = hipMemcpy(ledger, c->d_hled.p, 3 * c->last_n * sizeof(double), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(c, e, "read history results");
  return MCX_OK;
}

int mcx_checkpoint(mcx_ctx* c, void* buf, size_t* size) {
  if (!c || !size) return MCX_E_INVALID;
  if (!c->have_phantom) return fail(c, MCX_E_STATE, "no phantom");
  const size_t need = ckpt_bytes(c);
  if (!buf) {
    *size = need;
    return MCX_OK;
  }
  if (*size < need) {
    *size = need;
    return fail(c, MCX_E_RANGE, "checkpoint needs %zu bytes", need);
  }
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, MCX_E_DEVICE, "hipSetDevice");
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "synchronize");
  CkptHeader h;
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, kCkptMagic, sizeof(h.magic));
  h.version = kCkptVersion;
  h.precision = c->precision;
  h.nx = c->nx; h.ny = c->ny; h.nz = c->nz;
  h.nstat = S_NSTAT;
  h.run_seed = c->run_seed;
  h.run_known = c->run_known ? 1u : 0u;
  for (int k = 0; k < 3; ++k) h.voxel[k] = c->vox[k];
  h.n_done = c->n_done;
  h.next_history = c->next_history;
  h.run_first = c->run_first;
  h.run_n = c->run_n;
  h.iterations = c->iterations;
  h.chunks = c->chunks;
  h.tally_pairs = c->tally_pairs;
  h.ms_transport = c->ms_transport;
  h.ms_flush = c->ms_flush;
  if (c->d_cnt.p) {
    Counters k;
    e = hipMemcpy(&k, c->d_cnt.p, sizeof(Counters), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(c, e, "read statistics");
    std::memcpy(h.stat, k.stat, sizeof(h.stat));
    h.e_dep = k.e_dep;
    h.e_esc = k.e_esc;
  }
  char* out = static_cast<char*>(buf);
  std::memcpy(out, &h, sizeof(h));
  const size_t vb = nvox(c) * sizeof(double);
  e = hipMemcpy(out + sizeof(h), c->d_sumq.p, vb, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(out + sizeof(h) + vb, c->d_sumq2.p, vb, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(c, e, "read tallies");
  const uint64_t sum = fnv(1469598103934665603ull, out, need - sizeof(uint64_t));
  std::memcpy(out + need - sizeof(uint64_t), &sum, sizeof(sum));
  *size = need;
  return MCX_OK;
}

int mcx_restore(mcx_ctx* c, const void* buf, size_t size) {
  if (!c) return MCX_E_INVALID;
  if (!buf) return fail(c, MCX_E_INVALID, "null checkpoint");
  if (!c->have_phantom) return fail(c, MCX_E_STATE, "load the phantom first");
  const size_t need = ckpt_bytes(c);
  if (size != need) return fail(c, MCX_E_INVALID, "checkpoint of %zu bytes, this phantom needs %zu", size, need);
  const char* in = static_cast<const char*>(buf);
  CkptHeader h;
  std::memcpy(&h, in, sizeof(h));
  uint64_t sum;
  std::memcpy(&sum, in + need - sizeof(uint64_t), sizeof(sum));
  if (std::memcmp(h.magic, kCkptMagic, sizeof(h.magic)) != 0 || h.version != kCkptVersion || h.nstat != S_NSTAT)
    return fail(c, MCX_E_INVALID, "not a checkpoint of this library version");
  if (sum != fnv(1469598103934665603ull, in, need - sizeof(uint64_t)))
    return fail(c, MCX_E_INVALID, "checkpoint checksum mismatch");
  if (h.precision != c->precision) return fail(c, MCX_E_INVALID, "checkpoint precision differs from the context's");
  if (h.nx != c->nx || h.ny != c->ny || h.nz != c->nz || h.voxel[0] != c->vox[0] || h.voxel[1] != c->vox[1] ||
      h.voxel[2] != c->vox[2])
    return fail(c, MCX_E_INVALID, "checkpoint phantom grid differs from the context's");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, MCX_E_DEVICE, "hipSetDevice");
  int rc;
  if (!c->d_cnt.p) {
    if ((rc = dalloc(c, c->d_cnt, sizeof(Counters), "counters"))) return rc;
  }
  Counters k;
  std::memset(&k, 0, sizeof(k));
  std::memcpy(k.stat, h.stat, sizeof(k.stat));
  k.e_dep = h.e_dep;
  k.e_esc = h.e_esc;
  const size_t vb = nvox(c) * sizeof(double);
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess) e = hipMemcpy(c->d_cnt.p, &k, sizeof(Counters), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->d_sumq.p, in + sizeof(h), vb, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->d_sumq2.p, in + sizeof(h) + vb, vb, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(c, e, "write tallies");
  c->n_done = h.n_done;
  c->next_history = h.next_history;
  c->run_seed = h.run_seed;
  c->run_first = h.run_first;
  c->run_n = h.run_n;
  c->run_known = false;  // the replays need the run's own context
  c->iterations = h.iterations;
  c->chunks = h.chunks;
  c->tally_pairs = h.tally_pairs;
  c->ms_transport = h.ms_transport;
  c->ms_flush = h.ms_flush;
  c->last_valid = false;
  return MCX_OK;
}

int mcx_set_influence(mcx_ctx* c, int on, uint32_t log2_slots) {
  if (!c) return MCX_E_INVALID;
  if (!on) {
    for (DevBuf* b : {&c->d_ikeys, &c->d_iq, &c->d_iq2, &c->d_iovf}) dfree(*b);
    c->influence = 0;
    c->islots = 0;
    return MCX_OK;
  }
  if (log2_slots < 10 || log2_slots > 30) return fail(c, MCX_E_INVALID, "log2_slots must lie in [10, 30]");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, MCX_E_DEVICE, "hipSetDevice");
  const uint64_t slots = 1ull << log2_slots;
  int rc;
  if ((rc = dalloc(c, c->d_ikeys, slots * sizeof(uint64_t), "influence keys")) ||
      (rc = dalloc(c, c->d_iq, slots * sizeof(double), "influence Sum q")) ||
      (rc = dalloc(c, c->d_iq2, slots * sizeof(double), "influence Sum q^2")) ||
      (rc = dalloc(c, c->d_iovf, sizeof(uint32_t), "influence overflow flag"))) {
    for (DevBuf* b : {&c->d_ikeys, &c->d_iq, &c->d_iq2, &c->d_iovf}) dfree(*b);
    c->influence = 0;
    return rc;
  }
  hipError_t e = hipMemsetAsync(c->d_ikeys.p, 0xFF, slots * sizeof(uint64_t), c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->d_iq.p, 0, slots * sizeof(double), c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->d_iq2.p, 0, slots * sizeof(double), c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->d_iovf.p, 0, sizeof(uint32_t), c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "clear influence table");
  c->influence = 1;
  c->islots = slots;
  return MCX_OK;
}

int mcx_get_influence(mcx_ctx* c, uint32_t* source, uint32_t* voxel, double* sum_q, double* sum_q2, uint64_t capacity,
                      uint64_t* n) {
  if (!c || !n) return MCX_E_INVALID;
  if (!c->influence) return fail(c, MCX_E_STATE, "influence output is off (mcx_set_influence)");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, MCX_E_DEVICE, "hipSetDevice");
  hipStream_t s = c->stream;
  DevBuf cnt;
  int rc = dalloc(c, cnt, sizeof(unsigned long long), "influence count");
  if (rc) return rc;
  unsigned long long count = 0;
  auto pass = [&](uint64_t cap, uint32_t* os, uint32_t* ov, double* oq, double* oq2) {
    hipError_t e = hipMemsetAsync(cnt.p, 0, sizeof(unsigned long long), s);
    if (e == hipSuccess)
      e = launch_influence_compact(static_cast<const uint64_t*>(c->d_ikeys.p), static_cast<const double*>(c->d_iq.p),
                                   static_cast<const double*>(c->d_iq2.p), c->islots, os, ov, oq, oq2, cap,
                                   static_cast<unsigned long long*>(cnt.p), s);
    if (e == hipSuccess) e = hipMemcpyAsync(&count, cnt.p, sizeof(count), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e;
  };
  hipError_t e = pass(0, nullptr, nullptr, nullptr, nullptr);
  if (e != hipSuccess) {
    dfree(cnt);
    return hip_fail(c, e, "count influence entries");
  }
  *n = count;
  if (!source && !voxel && !sum_q && !sum_q2) {
    dfree(cnt);
    return MCX_OK;
  }
  if (!source || !voxel || !sum_q || !sum_q2) {
    dfree(cnt);
    return fail(c, MCX_E_INVALID, "pass all four output arrays, or none to count");
  }
  if (capacity < count) {
    dfree(cnt);
    return fail(c, MCX_E_RANGE, "influence output needs %llu entries", count);
  }
  DevBuf out;
  if ((rc = dalloc(c, out, size_t(count) * (2 * sizeof(uint32_t) + 2 * sizeof(double)) + 64, "influence staging"))) {
    dfree(cnt);
    return rc;
  }
  double* oq = static_cast<double*>(out.p);
  double* oq2 = oq + count;
  uint32_t* os = reinterpret_cast<uint32_t*>(oq2 + count);
  uint32_t* ov = os + count;
  const unsigned long long expect = count;
  e = pass(expect, os, ov, oq, oq2);
  if (e == hipSuccess && count != expect) e = hipErrorUnknown;
  if (e == hipSuccess && count) {
    e = hipMemcpy(source, os, size_t(count) * sizeof(uint32_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(voxel, ov, size_t(count) * sizeof(uint32_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(sum_q, oq, size_t(count) * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(sum_q2, oq2, size_t(count) * sizeof(double), hipMemcpyDeviceToHost);
  }
  dfree(out);
  dfree(cnt);
  if (e != hipSuccess) return hip_fail(c, e, "read influence entries");
  return MCX_OK;
}

int mcx_synchronize(mcx_ctx* c) {
  if (!c) return MCX_E_INVALID;
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, MCX_E_DEVICE, "hipSetDevice");
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(c, e, "synchronize");
  return MCX_OK;
}

int mcx_cancel(mcx_ctx* c) {
  if (!c) return MCX_E_INVALID;
  c->cancel.store(1);
  return MCX_OK;
}

int mcx_workspace_size(mcx_ctx* c, size_t* bytes) {
  if (!c || !bytes) return MCX_E_INVALID;
  *bytes = ws_fixed_bytes(c) + size_t(kTableSlots * kSlotBytes);
  return MCX_OK;
}

int mcx_set_workspace(mcx_ctx* c, void* dev, size_t bytes) {
  if (!c) return MCX_E_INVALID;
  if (dev && (reinterpret_cast<uintptr_t>(dev) & 255u)) return fail(c, MCX_E_INVALID, "workspace must be 256-byte aligned");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, MCX_E_DEVICE, "hipSetDevice");
  // the memory may have been written by other streams until now
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(c, e, "synchronize before the workspace change");
  // the loop and statistics counters are the context's own and stay
  for (DevBuf* b : {&c->d_queues, &c->d_htab}) dfree(*b);
  c->queue_cap_built = 0;
  c->ws = dev;
  c->ws_bytes = dev ? bytes : 0;
  c->ws_cap = 0;
  c->hslots = kTableSlots;
  int rc = dev ? carve_workspace(c) : MCX_OK;
  if (rc) {  // too small: back to library-owned memory
    for (DevBuf* b : {&c->d_queues, &c->d_htab}) dfree(*b);
    c->ws = nullptr;
    c->ws_bytes = 0;
  }
  return rc;
}

}  // extern "C"
