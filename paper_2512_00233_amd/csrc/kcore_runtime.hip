// Host runtime and C ABI of libkcore: workspace per device, the round driver
// (first round over every vertex, later rounds enqueued in chunks, convergence
// polled on a pinned copy of the device control block) and argument checking.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/kcore.h"
#include "kcore_kernels_impl.h"
#include "kcore_runtime.h"

namespace kcore {

static thread_local std::string g_last_error;

kcore_status fail(kcore_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

kcore_status hip_fail(hipError_t e, const char* what) {
  return fail(KCORE_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define KC_HIP(call)                                   \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return hip_fail(e_, #call);  \
  } while (0)

// ------------------------------------------------------------------ workspace
struct Workspace {
  int device = -1;
  int num_cus = 0;
  int64_t cap_n = 0;
  int64_t cap_nnz = 0;
  int32_t* stamp = nullptr;
  uint8_t* cls = nullptr;
  int32_t* lists[2] = {nullptr, nullptr};
  int32_t* slist = nullptr;
  int32_t* plen = nullptr;
  int32_t* plow = nullptr;
  int32_t* vbase = nullptr;
  int32_t* slack = nullptr;
  int32_t* defer = nullptr;  // deferred same-kernel checks, 3 ints each
  int64_t defer_cap = 0;
  uint8_t* dirty = nullptr;  // dirty-piece marks, two arrays (by round parity) of dirty_pieces bytes
  int64_t dirty_pieces = 0;
  int32_t* pruned = nullptr;
  Ctl* ctl = nullptr;
  Ctl* host_ctl = nullptr;      // pinned
  int32_t* verr = nullptr;      // validation result (device)
  int32_t* host_verr = nullptr;  // pinned
  int32_t* aux = nullptr;       // update runs: bounds over the inserted edges, search counters (device)
  int32_t* host_aux = nullptr;  // pinned
  int32_t* cert = nullptr;      // certificate: worst (code << 32 | vertex) as two words, then the largest core
  int32_t* host_cert = nullptr; // pinned
  int64_t* host_nnz = nullptr;   // pinned
  int32_t epoch = 1;
  // degree relabelling (single-graph calls on skewed graphs)
  struct Relabel {
    int64_t cap_n = 0, cap_nnz = 0;
    uint32_t* keys[2] = {nullptr, nullptr};
    int32_t* ids = nullptr;
    int32_t* order = nullptr;
    int32_t* new_of = nullptr;
    int64_t* new_deg = nullptr;
    int64_t* nrp = nullptr;
    int32_t* ncol = nullptr;
    int32_t* nout = nullptr;
    void* temp = nullptr;
    size_t temp_bytes = 0;
    unsigned long long* probe = nullptr;       // device [2]
    unsigned long long* host_probe = nullptr;  // pinned [2]
  } rl;
  std::vector<hipEvent_t> events;  // timing mode: one pair per round launch
  struct GraphEntry {
    std::string key;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;  // captured chunks of round launches, by launch shape
  std::mutex mu;

  void drop_graphs() {
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.exec);
    graphs.clear();
  }

  kcore_status need_events(size_t count) {
    while (events.size() < count) {
      hipEvent_t e;
      KC_HIP(hipEventCreate(&e));
      events.push_back(e);
    }
    return KCORE_OK;
  }

  void release_relabel() {
    for (void* p : {(void*)rl.keys[0], (void*)rl.keys[1], (void*)rl.ids, (void*)rl.order, (void*)rl.new_of,
                    (void*)rl.new_deg, (void*)rl.nrp, (void*)rl.ncol, (void*)rl.nout, rl.temp})
      if (p) (void)hipFree(p);
    unsigned long long* probe = rl.probe;
    unsigned long long* host_probe = rl.host_probe;
    rl = Relabel();
    rl.probe = probe;
    rl.host_probe = host_probe;
  }

  void release() {
    drop_graphs();
    release_relabel();
    for (void* p : {(void*)stamp, (void*)cls, (void*)lists[0], (void*)lists[1], (void*)slist, (void*)plen,
                    (void*)plow, (void*)vbase, (void*)slack, (void*)defer, (void*)pruned, (void*)dirty})
      (void)hipFree(p);
    stamp = nullptr;
    cls = nullptr;
    lists[0] = lists[1] = nullptr;
    slist = plen = plow = vbase = slack = defer = pruned = nullptr;
    dirty = nullptr;
    defer_cap = 0;
    dirty_pieces = 0;
    cap_n = 0;
    cap_nnz = 0;
  }
};

static std::mutex g_ws_mu;
static Workspace* g_ws[64];

static kcore_status get_workspace(Workspace** out) {
  int dev = 0;
  KC_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(KCORE_E_INVALID, "device index out of range");
  std::lock_guard<std::mutex> lk(g_ws_mu);
  if (!g_ws[dev]) {
    auto* ws = new Workspace();
    ws->device = dev;
    hipDeviceProp_t prop;
    KC_HIP(hipGetDeviceProperties(&prop, dev));
    ws->num_cus = prop.multiProcessorCount;
    KC_HIP(hipMalloc(&ws->ctl, sizeof(Ctl)));
    KC_HIP(hipHostMalloc(&ws->host_ctl, sizeof(Ctl), hipHostMallocDefault));
    KC_HIP(hipMalloc(&ws->verr, sizeof(int32_t)));
    KC_HIP(hipHostMalloc(&ws->host_verr, sizeof(int32_t), hipHostMallocDefault));
    KC_HIP(hipHostMalloc(&ws->host_nnz, sizeof(int64_t), hipHostMallocDefault));
    KC_HIP(hipMalloc(&ws->aux, 16 * sizeof(int32_t)));
    KC_HIP(hipHostMalloc(&ws->host_aux, 16 * sizeof(int32_t), hipHostMallocDefault));
    KC_HIP(hipMalloc(&ws->cert, 4 * sizeof(int32_t)));
    KC_HIP(hipHostMalloc(&ws->host_cert, 4 * sizeof(int32_t), hipHostMallocDefault));
    g_ws[dev] = ws;
  }
  *out = g_ws[dev];
  return KCORE_OK;
}

// Deferred same-kernel checks per round: a quarter of the vertices, at least 1M
// (beyond it, such neighbours are simply re-activated).
static int64_t defer_capacity(int64_t n) {
  return std::min<int64_t>(std::max<int64_t>(n / 4, 1 << 20), INT32_MAX / 3);
}

static kcore_status ensure_capacity(Workspace* ws, int64_t n, int64_t nnz, bool batched, hipStream_t st) {
  const bool need_vbase = batched && !ws->vbase;
  if (n <= ws->cap_n && nnz <= ws->cap_nnz && !need_vbase) return KCORE_OK;
  KC_HIP(hipStreamSynchronize(st));
  const int64_t cap = std::max<int64_t>({n, ws->cap_n, 1024});
  const int64_t cap_e = std::max<int64_t>({nnz, ws->cap_nnz, 1024});
  const bool keep_vbase = batched || ws->vbase;
  ws->release();
  bool ok = hipMalloc(&ws->stamp, sizeof(int32_t) * cap) == hipSuccess &&
            hipMalloc(&ws->cls, sizeof(uint8_t) * cap) == hipSuccess &&
            hipMalloc(&ws->lists[0], sizeof(int32_t) * cap) == hipSuccess &&
            hipMalloc(&ws->lists[1], sizeof(int32_t) * cap) == hipSuccess &&
            hipMalloc(&ws->slist, sizeof(int32_t) * cap) == hipSuccess &&
            hipMalloc(&ws->plen, sizeof(int32_t) * cap) == hipSuccess &&
            hipMalloc(&ws->plow, sizeof(int32_t) * cap) == hipSuccess &&
            hipMalloc(&ws->slack, sizeof(int32_t) * cap) == hipSuccess &&
            hipMalloc(&ws->defer, sizeof(int32_t) * 3 * defer_capacity(cap)) == hipSuccess &&
            (!keep_vbase || hipMalloc(&ws->vbase, sizeof(int32_t) * cap) == hipSuccess) &&
            hipMalloc(&ws->dirty, 2 * ((cap + kCompactPiece - 1) / kCompactPiece)) == hipSuccess &&

            hipMalloc(&ws->pruned, sizeof(int32_t) * cap_e) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    ws->release();
    return fail(KCORE_E_NOMEM, "workspace allocation failed for n=" + std::to_string(n) +
                                   " nnz=" + std::to_string(nnz));
  }
  KC_HIP(hipMemsetAsync(ws->stamp, 0, sizeof(int32_t) * cap, st));
  ws->dirty_pieces = (cap + kCompactPiece - 1) / kCompactPiece;
  KC_HIP(hipMemsetAsync(ws->dirty, 0, 2 * ws->dirty_pieces, st));
  ws->cap_n = cap;
  ws->cap_nnz = cap_e;
  ws->defer_cap = defer_capacity(cap);
  ws->epoch = 1;
  return KCORE_OK;
}

// ------------------------------------------------------------------ tuning
// Most rounds in one chunk of launches (the timing mode keeps events for this many).
constexpr int kMaxChunkRounds = 64;

Tuning resolve_tuning(const kcore_tuning* t, int num_cus) {
  Tuning r;
  r.t0 = kLaneMaxDeg;
  r.t1 = kGroupMaxDeg;
  r.t2 = kWaveMaxDeg;
  r.tail = 2048;
  r.tail_auto = 1;
  r.grid = 8 * num_cus;
  r.grid_auto = 1;
  // class 3: four workgroups fit a compute unit at a time; launching four
  // times more lets the hardware hand vertices to whichever unit frees up first
  r.big_grid = 16 * num_cus;
  r.big_grid_auto = 1;
  r.poll = 4;
  r.one_sided = -1;
  r.timing = 0;
  r.list_cap = 8192;
  r.list_cap_auto = 1;
  r.prune = 1;
  r.use_graph = 1;
  r.max_rounds = 0;
  r.relabel = 0;
  r.defer = -1;
  r.tail_cap = kTailRoundCap;
  r.tail_order = 0;
  r.tail_big = 0;
  r.renorm = kRoundRenorm;
  r.big_wave = 0;
  r.dirty = 1;
  if (const char* e = std::getenv("KCORE_TAIL")) {
    r.tail = std::atoi(e);
    r.tail_auto = 0;
  }
  if (t) {
    if (t->thread_max_deg > 0) r.t0 = std::min(t->thread_max_deg, kLaneMaxDeg);
    if (t->group_max_deg > 0) r.t1 = std::min(t->group_max_deg, kGroupMaxDeg);
    if (t->wave_max_deg > 0) r.t2 = std::min(t->wave_max_deg, kWaveMaxDeg);
    if (t->tail_threshold > 0) r.tail = t->tail_threshold;
    else if (t->tail_threshold < 0) r.tail = 0;  // tail disabled
    if (t->tail_threshold != 0) r.tail_auto = 0;
    if (t->grid_blocks > 0) {
      r.grid = t->grid_blocks;
      r.grid_auto = 0;
    }
    if (t->big_grid_blocks > 0) {
      r.big_grid = t->big_grid_blocks;
      r.big_grid_auto = 0;
    }
    if (t->rounds_per_poll > 0) r.poll = std::min(t->rounds_per_poll, kMaxChunkRounds);
    if (t->activation == 1 || t->activation == 2) r.one_sided = t->activation == 1;
    r.timing = t->timing == 1;
    if (t->list_cap > 0) {
      r.list_cap = t->list_cap;
      r.list_cap_auto = 0;
    }
    r.prune = t->no_prune != 1;
    r.use_graph = t->no_graph != 1;
    r.relabel = t->relabel == 2;
    if (t->deferred == 1 || t->deferred == 2) r.defer = t->deferred == 1;
    if (t->tail_round_cap > 0) r.tail_cap = t->tail_round_cap;
    r.tail_order = t->tail_order == 1;
    r.tail_big = t->tail_big == 1;
    if (t->big_wave == 1 || t->big_wave == 2) r.big_wave = t->big_wave == 1;
    if (t->dense_sweep == 1 || t->dense_sweep == 2) r.dirty = t->dense_sweep == 1;
    if (t->round_renorm > 0) r.renorm = std::max(t->round_renorm, 1024);
    if (t->max_rounds > 0) {
      r.max_rounds = t->max_rounds;
      r.tail = 0;
      r.tail_auto = 0;
    }
  }
  r.t0 = std::max(r.t0, 1);
  r.t1 = std::max(r.t1, r.t0);
  r.t2 = std::max(r.t2, r.t1);
  r.grid = std::max(8, (r.grid + 7) / 8 * 8);
  r.big_grid = std::max(1, r.big_grid);
  return r;
}

// On very sparse graphs (road networks: mean degree 2-3) a dropped estimate
// rarely leaves a neighbour's support intact, so the two-sided filter saves few
// recomputations and its slack atomics cost more than they save; there the
// one-sided rule is faster.  Denser graphs gain from the filter.
constexpr int64_t kOneSidedMeanDeg = 4;
// Deferred same-kernel checks remove most conservative re-activations, but cost
// one more launch per round: measured, they pay on large single graphs and not
// on small ones or on batches of many graphs.
constexpr int64_t kDeferMinVertices = 1 << 20;
// Small-class workgroups: 8 per compute unit, up to 32 per compute unit for very
// large inputs (about one per 32K vertices): the 2048-graph batch (304M
// vertices) runs 6% faster with 32 per unit, graphs of 16.8M vertices gain
// nothing from it.
constexpr int64_t kVerticesPerSmallBlock = 1 << 15;
// The defaults that depend on the input (n vertices, nnz adjacency entries; a
// batch is many graphs sharing the rounds): small-class grid, activation rule,
// deferred checks, list cap, class-3 grid and tail threshold.  Knobs the caller set are kept.
void settle_tuning(Tuning* tu, int64_t n, int64_t nnz, bool batch) {
  if (tu->grid_auto) {
    const int64_t want = (n + kVerticesPerSmallBlock - 1) / kVerticesPerSmallBlock;
    tu->grid = (int)std::min<int64_t>(std::max<int64_t>(want, tu->grid), 4 * (int64_t)tu->grid);
    tu->grid = std::max(8, (tu->grid + 7) / 8 * 8);
  }
  if (tu->one_sided < 0) tu->one_sided = nnz < kOneSidedMeanDeg * n;
  if (tu->defer < 0) tu->defer = !batch && !tu->one_sided && n >= kDeferMinVertices;
  // List cap (appends vs compaction from the stamps) of single graphs: sparse
  // graphs (one-sided rule) have thin frontiers, where appends beat a scan of
  // every stamp; large dense graphs see many repeated activations, which plain
  // stores and a compaction absorb best.  Measured: road 1.78 ms at 8192, 1.59
  // ms at 32768, 1.69 ms at 65536; rmat24 27.8 ms at 8192, 26.2 ms at 2048,
  // 26.0 ms at 1024, 26.2 ms at 512; ER small (10,000 vertices) best at 8192.
  if (tu->list_cap_auto && !batch) {
    if (tu->one_sided) tu->list_cap = 32768;
    else if (n >= kDeferMinVertices) tu->list_cap = 1024;
  }
  // Class-3 workgroups: twice as many for large single graphs under the
  // two-sided rule (rmat24 25.9 ms against 26.2 ms); road, ER small and the
  // 2048-graph batch measured the same or slower.
  if (tu->big_grid_auto && !batch && !tu->one_sided && n >= kDeferMinVertices) tu->big_grid *= 2;
  // Single graphs hand over to the one-workgroup tail later (road 1.59 ms at
  // 2048, 1.56 ms at 512; rmat24 never reaches it; ER small unchanged).  The
  // batched and served forms keep 2048 (the 2048-graph batch measured the same
  // at 512).
  if (tu->tail_auto && !batch) tu->tail = 512;
}

static bool env_flag(const char* name) {
  const char* e = std::getenv(name);
  return e && e[0] == '1';
}

// ------------------------------------------------------------------ driver
constexpr int kBlock = 256;

// Workgroups of the compaction kernel: at least 4 pieces of kCompactPerLane
// vertices per lane each, at most 16 per compute unit (measured on the 2048-graph
// batch's compaction: 61 ms with two per unit, 37 ms with eight, 33 ms with 16).
static int compact_grid(int64_t n, int num_cus) {
  const int64_t per_block = (int64_t)kCompactBlock * kCompactPerLane * 4;
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + per_block - 1) / per_block, 4 * (int64_t)num_cus));
}

// The two update kernels of a round (slot relative to the round base), in
// kBigFirst order, then the deferred checks.  With ev (4 events) the launches
// are bracketed: ev[0] before the first, ev[1] between, ev[2] after the second,
// ev[3] after the deferred checks.
template <bool FIRST, bool BATCH, typename Off>
static void launch_updates(const Args<Off>& a, const Tuning& tu, int32_t slot, int32_t collect, hipStream_t st,
                           hipEvent_t* ev) {
  if (ev) (void)hipEventRecord(ev[0], st);
  if (!FIRST && a.big_wave)
    hipLaunchKernelGGL((k_big_wave<BATCH, Off>), dim3(tu.big_grid), dim3(256), 0, st, a, slot, collect);
  if (kBigFirst)
    hipLaunchKernelGGL((k_big<FIRST, BATCH, Off>), dim3(tu.big_grid), dim3(kBigBlock), 0, st, a, slot, collect);
  else
    hipLaunchKernelGGL((k_round<kBlock, FIRST, BATCH, Off>), dim3(tu.grid), dim3(kBlock), 0, st, a, slot, collect);
  if (ev) (void)hipEventRecord(ev[1], st);
  if (kBigFirst)
    hipLaunchKernelGGL((k_round<kBlock, FIRST, BATCH, Off>), dim3(tu.grid), dim3(kBlock), 0, st, a, slot, collect);
  else
    hipLaunchKernelGGL((k_big<FIRST, BATCH, Off>), dim3(tu.big_grid), dim3(kBigBlock), 0, st, a, slot, collect);
  // the deferred same-kernel checks of the round (none in the first round, nor under the one-sided
  // rule, which re-activates every candidate)
  if (ev) (void)hipEventRecord(ev[2], st);
  if (!FIRST && a.defer && !a.one_sided)
    hipLaunchKernelGGL((k_defer<Off>), dim3(4 * kDeferRegions), dim3(kBlock), 0, st, a, slot, collect);
  if (ev) (void)hipEventRecord(ev[3], st);
}

// The compaction of a round (a no-op unless its lists overflowed).
template <typename Off>
static void launch_compact(const Args<Off>& a, int cgrid, int32_t slot, hipStream_t st) {
  hipLaunchKernelGGL((k_compact<false, Off>), dim3(cgrid), dim3(kCompactBlock), 0, st, a, slot);
}

// Launch one chunk of K rounds (slots 0..K-1 relative to ctl->rbase) and
// advance the round base.  With use_graph the chunk is captured once per
// launch shape and replayed.
template <bool BATCH, typename Off>
static kcore_status launch_chunk(Workspace* ws, const Args<Off>& a, const Tuning& tu, int cgrid, int K,
                                 int32_t collect, bool use_graph, hipStream_t st) {
  auto enqueue = [&]() {
    for (int i = 0; i < K; ++i) {
      launch_compact<Off>(a, cgrid, i, st);
      launch_updates<false, BATCH, Off>(a, tu, i, collect, st, nullptr);
    }
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, st, a.ctl, K);
  };
  if (!use_graph) {
    enqueue();
    KC_HIP(hipGetLastError());
    return KCORE_OK;
  }
  std::string key(reinterpret_cast<const char*>(&a), sizeof(a));
  const int32_t shape[6] = {K, cgrid, tu.grid, tu.big_grid, collect, (int32_t)(BATCH * 2 + (sizeof(Off) == 8))};
  key.append(reinterpret_cast<const char*>(shape), sizeof(shape));
  for (auto& g : ws->graphs)
    if (g.key == key) {
      KC_HIP(hipGraphLaunch(g.exec, st));
      return KCORE_OK;
    }
  hipGraph_t graph;
  KC_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  enqueue();
  const hipError_t launch_err = hipGetLastError();
  const hipError_t end_err = hipStreamEndCapture(st, &graph);
  if (launch_err != hipSuccess) return hip_fail(launch_err, "round launch during capture");
  if (end_err != hipSuccess) return hip_fail(end_err, "hipStreamEndCapture");
  hipGraphExec_t exec;
  const hipError_t inst_err = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (inst_err != hipSuccess) return hip_fail(inst_err, "hipGraphInstantiate");
  if (ws->graphs.size() >= 48) {
    (void)hipGraphExecDestroy(ws->graphs.front().exec);
    ws->graphs.erase(ws->graphs.begin());
  }
  ws->graphs.push_back({key, exec});
  KC_HIP(hipGraphLaunch(exec, st));
  return KCORE_OK;
}

// Timing mode: one round with an event before and after each of its kernels
// (compaction, class 3, classes 0..2, deferred checks), then the base advance.
constexpr int kRoundEvents = 5;
template <bool BATCH, typename Off>
static void launch_round_timed(const Args<Off>& a, const Tuning& tu, int cgrid, int32_t collect, hipEvent_t* ev,
                               hipStream_t st) {
  (void)hipEventRecord(ev[0], st);
  launch_compact<Off>(a, cgrid, 0, st);
  launch_updates<false, BATCH, Off>(a, tu, 0, collect, st, ev + 1);
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, st, a.ctl, 1);
}

// A kernel's counter, summed over its copies.
static unsigned long long kstat(const Ctl& h, int kid, int q) {
  unsigned long long t = 0;
  for (int c = 0; c < kStatCopies; ++c) t += h.kstats[c][kid][q];
  return t;
}

static float elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0;
  (void)hipEventElapsedTime(&ms, a, b);
  return ms;
}

// Start of an update run (kcore_update): the old coreness, the per-vertex
// flags of the edge changes and the number of inserted edges.
struct UpdateStart {
  const int32_t* prev;
  const int32_t* flag;
  int64_t rise, cap;  // on A: x = max(c_old, min(degree, c_old + rise, cap))
  bool heavy;         // the heavy-vertex rule: rise 1 outside Z
  int32_t all_from;   // A also holds every vertex of old coreness >= all_from (INT32_MAX: none)
  bool insert_only;
};

// Every vertex of every graph (one graph: vbase unused) to its fixpoint.
// row_ptr holds global edge offsets; with BATCH, col holds graph-local ids.
// With upd, the run starts from the bounds of an update instead of the degrees,
// and its first round is an ordinary later round over the update's frontier.
template <bool BATCH, typename Off>
static kcore_status run_rounds(Workspace* ws, int64_t n, int64_t nnz, const Off* row_ptr, const int32_t* col,
                               int32_t* out, const Tuning& tu, kcore_stats* stats, hipStream_t st,
                               std::vector<kcore_round_record>* rec = nullptr, const UpdateStart* upd = nullptr) {
  const int init_grid = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, (int64_t)ws->num_cus * 16);
  const int cgrid = compact_grid(n, ws->num_cus);
  if (ws->epoch > (1 << 29)) {
    const int fgrid = (int)std::min<int64_t>((ws->cap_n + kBlock - 1) / kBlock, (int64_t)ws->num_cus * 16);
    hipLaunchKernelGGL(k_fill, dim3(std::max(fgrid, 1)), dim3(kBlock), 0, st, ws->stamp, ws->cap_n, 0);
    ws->epoch = 1;
  }
  Args<Off> a;
  std::memset(&a, 0, sizeof(a));
  a.n = n;
  a.row_ptr = row_ptr;
  a.col = col;
  a.vbase = BATCH ? ws->vbase : nullptr;
  a.est = out;
  a.stamp = ws->stamp;
  a.cls = ws->cls;
  a.lists[0] = ws->lists[0];
  a.lists[1] = ws->lists[1];
  a.slist = ws->slist;
  a.pruned = ws->pruned;
  a.plen = ws->plen;
  a.plow = ws->plow;
  a.ctl = ws->ctl;
  a.slack = ws->slack;
  a.tail_threshold = tu.tail;
  a.list_cap = tu.list_cap;
  a.one_sided = tu.one_sided;
  a.defer = tu.defer > 0 ? ws->defer : nullptr;
  a.defer_cap = (int32_t)ws->defer_cap;
  a.prune = tu.prune;
  a.tail_cap = tu.tail_cap;
  a.tail_order = tu.tail_order;
  a.tail_big = tu.tail_big;
  a.big_wave = tu.big_wave && a.slist && a.prune;
  a.dirty = tu.dirty ? ws->dirty : nullptr;
  a.dirty_pieces = ws->dirty_pieces;
  const int32_t collect = (stats || rec) ? 1 : 0;
  const bool trace_env = env_flag("KCORE_TRACE");
  const bool trace = trace_env || rec != nullptr;  // one round per launch, counters read after each
  const bool timing = tu.timing || trace;
  const bool use_graph = tu.use_graph && !timing && st != nullptr;  // no capture on the null stream
  int32_t r0 = ws->epoch;
  double kms[KCORE_K_COUNT] = {0, 0, 0, 0, 0, 0};
  double init_ms = 0;
  if (timing) {
    kcore_status s = ws->need_events(kRoundEvents * kMaxChunkRounds);
    if (s != KCORE_OK) return s;
  }
  hipEvent_t* ev = timing ? ws->events.data() : nullptr;
  if (timing) KC_HIP(hipEventRecord(ev[0], st));
  hipLaunchKernelGGL(k_zero_ctl, dim3(1), dim3(256), 0, st, ws->ctl);
  if (upd) {
    hipLaunchKernelGGL(k_upd_init<Off>, dim3(init_grid), dim3(kBlock), 0, st, a, upd->prev, upd->flag, upd->rise,
                       (int32_t)upd->heavy, upd->cap, upd->all_from, (int32_t)upd->insert_only, r0 + 1, tu.t0, tu.t1, tu.t2);
    hipLaunchKernelGGL(k_pop_sum, dim3(1), dim3(64), 0, st, ws->ctl);
    if (timing)
      for (int i = 1; i <= 4; ++i) KC_HIP(hipEventRecord(ev[i], st));
  } else {
    hipLaunchKernelGGL(k_init<Off>, dim3(init_grid), dim3(kBlock), 0, st, a, r0, tu.t0, tu.t1, tu.t2);
    hipLaunchKernelGGL(k_pop_sum, dim3(1), dim3(64), 0, st, ws->ctl);
    hipLaunchKernelGGL((k_compact<true, Off>), dim3(cgrid), dim3(kCompactBlock), 0, st, a, 0);
    launch_updates<true, BATCH, Off>(a, tu, 0, collect, st, timing ? ev + 1 : nullptr);
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, st, ws->ctl, 1);
  }
  KC_HIP(hipGetLastError());
  unsigned long long prev[KI_COUNT][kLaneStats];
  std::memset(prev, 0, sizeof(prev));
  unsigned long long prev_tail = 0;
  auto trace_line = [&](const Ctl& h, int32_t r, const char* what, float ms, float big_ms) {
    unsigned long long d[2][kLaneStats];  // [0]: class-3 kernels and deferred checks, [1]: classes 0..2
    std::memset(d, 0, sizeof(d));
    for (int k = 0; k < KI_COUNT; ++k)
      for (int q = 0; q < kLaneStats; ++q) {
        const unsigned long long now = kstat(h, k, q);
        d[k == KI_BIG_FIRST || k == KI_BIG || k == KI_DEFER ? 0 : 1][q] += now - prev[k][q];
        prev[k][q] = now;
      }
    if (rec) {
      kcore_round_record x;
      std::memset(&x, 0, sizeof(x));
      x.round = (int32_t)rec->size() + 1;
      x.tail_rounds = (int32_t)(h.stats[ST_TAIL_ROUNDS] - prev_tail);
      x.vertex_updates = (int64_t)(d[0][ST_UPDATES] + d[1][ST_UPDATES]);
      x.edge_visits = (int64_t)(d[0][ST_VISITS] + d[1][ST_VISITS]);
      x.changes = (int64_t)(d[0][ST_CHANGES] + d[1][ST_CHANGES]);
      x.activations = (int64_t)(d[0][ST_ACTIVATIONS] + d[1][ST_ACTIVATIONS]);
      x.max_full_scan = (int64_t)h.maxscan_round;
      x.ms = ms;
      x.big_ms = big_ms;
      rec->push_back(x);
    }
    prev_tail = h.stats[ST_TAIL_ROUNDS];
    if (!trace_env) return;
    std::fprintf(stderr, "[kcore-trace] %s round=%d front=%d/%d/%d/%d dense=%d | big upd=%llu vis=%llu chg=%llu "
                 "act=%llu full=%llu maxscan=%u big_ms=%.3f | small upd=%llu vis=%llu chg=%llu act=%llu full=%llu | "
                 "tail=%llu ms=%.3f\n",
                 what, r - r0, h.cnt[r % 3][0], h.cnt[r % 3][kCtr], h.cnt[r % 3][2 * kCtr], h.cnt[r % 3][3 * kCtr],
                 h.overflow[r % 3][0], d[0][ST_UPDATES], d[0][ST_VISITS], d[0][ST_CHANGES], d[0][ST_ACTIVATIONS],
                 d[0][ST_FULL_SCANS], h.maxscan_round, big_ms, d[1][ST_UPDATES], d[1][ST_VISITS], d[1][ST_CHANGES],
                 d[1][ST_ACTIVATIONS], d[1][ST_FULL_SCANS], h.stats[ST_TAIL_ROUNDS], ms);
  };
  if (timing) {
    KC_HIP(hipMemcpyAsync(ws->host_ctl, ws->ctl, kCtlHostBytes, hipMemcpyDeviceToHost, st));
    KC_HIP(hipStreamSynchronize(st));
    init_ms = elapsed(ev[0], ev[1]);
    kms[KCORE_K_BIG_FIRST] = kBigFirst ? elapsed(ev[1], ev[2]) : elapsed(ev[2], ev[3]);
    kms[KCORE_K_ROUND_FIRST] = kBigFirst ? elapsed(ev[2], ev[3]) : elapsed(ev[1], ev[2]);
    if (trace_env)
      std::fprintf(stderr, "[kcore-trace] n=%lld nnz=%lld pop=%d/%d/%d/%d init_ms=%.3f\n", (long long)n,
                   (long long)nnz, ws->host_ctl->pop[0], ws->host_ctl->pop[1], ws->host_ctl->pop[2],
                   ws->host_ctl->pop[3], init_ms);
    if (trace && !upd) trace_line(*ws->host_ctl, r0 + 1, "first", (float)(kms[0] + kms[1]), (float)kms[0]);
  }
  const int64_t first_launches = upd ? 0 : 1;  // the first (all-vertex) round
  int64_t launches = first_launches;
  int K = trace ? 1 : tu.poll;
  int32_t r = r0 + 1;
  int64_t rounds_done = 1;  // round numbers, across renumberings
  for (;;) {
    if (tu.max_rounds > 0) {
      if (launches >= tu.max_rounds) {
        KC_HIP(hipMemcpyAsync(ws->host_ctl, ws->ctl, kCtlHostBytes, hipMemcpyDeviceToHost, st));
        KC_HIP(hipStreamSynchronize(st));
        r = ws->host_ctl->rbase;
        break;
      }
      K = (int)std::min<int64_t>(K, tu.max_rounds - launches);
    }
    if (timing) {
      for (int i = 0; i < K; ++i) launch_round_timed<BATCH, Off>(a, tu, cgrid, collect, ev + kRoundEvents * i, st);
      KC_HIP(hipGetLastError());
    } else {
      kcore_status s = launch_chunk<BATCH, Off>(ws, a, tu, cgrid, K, collect, use_graph, st);
      if (s != KCORE_OK) return s;
    }
    launches += K;
    KC_HIP(hipMemcpyAsync(ws->host_ctl, ws->ctl, kCtlHostBytes, hipMemcpyDeviceToHost, st));
    KC_HIP(hipStreamSynchronize(st));
    const Ctl& h = *ws->host_ctl;
    rounds_done += (int64_t)h.rbase - r;
    r = h.rbase;
    if (timing) {
      for (int i = 0; i < K; ++i) {
        hipEvent_t* e = ev + kRoundEvents * i;
        kms[KCORE_K_COMPACT] += elapsed(e[0], e[1]);
        kms[KCORE_K_BIG] += kBigFirst ? elapsed(e[1], e[2]) : elapsed(e[2], e[3]);
        kms[KCORE_K_ROUND] += kBigFirst ? elapsed(e[2], e[3]) : elapsed(e[1], e[2]);
        kms[KCORE_K_DEFER] += elapsed(e[3], e[4]);
        if (trace) trace_line(h, r - 1, "", elapsed(e[0], e[4]), kBigFirst ? elapsed(e[1], e[2]) : elapsed(e[2], e[3]));
      }
    }
    const int32_t* c = h.cnt[r % 3];
    if (h.overflow[r % 3][0] == 0 && c[0] == 0 && c[kCtr] == 0 && c[2 * kCtr] == 0 && c[3 * kCtr] == 0) break;
    // Every round but the last lowers an estimate (a round without a change
    // activates nobody), and the estimates fall by at most the sum of the
    // degrees: more rounds than that mean a fault, not a long run.
    if (rounds_done > nnz + 16) return fail(KCORE_E_HIP, "round count above its bound (internal error)");
    if (r > tu.renorm) {
      // round numbers stay far from the int32 range: renumber the stamps of every workspace vertex
      const int32_t d = (r - 64) / 6 * 6;
      const int rgrid = (int)std::min<int64_t>((ws->cap_n + kBlock - 1) / kBlock, (int64_t)ws->num_cus * 16);
      hipLaunchKernelGGL(k_rebase, dim3(rgrid), dim3(kBlock), 0, st, ws->stamp, (int32_t*)nullptr, ws->cap_n, d,
                         ws->ctl);
      KC_HIP(hipGetLastError());
      r -= d;
      r0 -= d;
    }
    // chunks double up to 16 rounds: past the fixpoint the rest of a chunk
    // replays empty rounds (about 9 us each against a poll of a few tens of
    // us); rmat24 (66 rounds) left 59 of them at 64 and takes 25.4 ms at 16,
    // 25.8 ms at 32, 25.9 ms at 64
    K = trace ? 1 : std::min(2 * K, 16);
  }
  // the estimates carry their class during the run
  hipLaunchKernelGGL(k_decode, dim3(init_grid), dim3(kBlock), 0, st, out, n);
  KC_HIP(hipGetLastError());
  const Ctl& hc = *ws->host_ctl;
  ws->epoch = r + 4;  // the round base already counts the tail's rounds
  if (stats) {
    stats->rounds = (int64_t)hc.stats[ST_ROUNDS];
    stats->tail_rounds = (int64_t)hc.stats[ST_TAIL_ROUNDS];
    stats->launches = launches;
    stats->dense_rounds = (int64_t)hc.stats[ST_DENSE_ROUNDS];
    stats->init_ms = init_ms;
    const bool defer_on = a.defer && !a.one_sided;
    const int64_t later = launches - first_launches;
    const int64_t kl[KCORE_K_COUNT] = {first_launches, first_launches, later, later, later, defer_on ? later : 0};
    // counters by public kernel index (the compaction kernel has none)
    const int kid[KCORE_K_COUNT] = {KI_BIG_FIRST, KI_ROUND_FIRST, KI_BIG, KI_ROUND, -1, KI_DEFER};
    for (int k = 0; k < KCORE_K_COUNT; ++k) {
      kcore_kernel_stats& o = stats->kernel[k];
      o.launches = kl[k];
      o.ms = kms[k];
      if (kid[k] >= 0) {
        o.vertex_updates = (int64_t)kstat(hc, kid[k], ST_UPDATES);
        o.edge_visits = (int64_t)kstat(hc, kid[k], ST_VISITS);
        o.changes = (int64_t)kstat(hc, kid[k], ST_CHANGES);
        o.activations = (int64_t)kstat(hc, kid[k], ST_ACTIVATIONS);
        o.prune_writes = (int64_t)kstat(hc, kid[k], ST_PRUNE_WRITES);
        o.full_scans = (int64_t)kstat(hc, kid[k], ST_FULL_SCANS);
        o.max_full_scan = (int64_t)hc.maxscan_run[kid[k]];
        stats->vertex_updates += o.vertex_updates;
        stats->edge_visits += o.edge_visits;
        stats->changes += o.changes;
        stats->activations += o.activations;
        stats->prune_writes += o.prune_writes;
        stats->full_scans += o.full_scans;
      }
      stats->total_ms += o.ms;
    }
    stats->total_ms += init_ms;
  }
  return KCORE_OK;
}

template <typename Off>
static kcore_status validate_csr(Workspace* ws, int64_t n, const Off* row_ptr, const int32_t* col,
                                 hipStream_t st) {
  const int grid = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, (int64_t)ws->num_cus * 16);
  hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, st, ws->verr, (int64_t)1, (int32_t)0x7f7f7f7f);
  hipLaunchKernelGGL(k_validate<Off>, dim3(grid), dim3(kBlock), 0, st, n, row_ptr, col, ws->verr);
  KC_HIP(hipGetLastError());
  KC_HIP(hipMemcpyAsync(ws->host_verr, ws->verr, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  KC_HIP(hipStreamSynchronize(st));
  const int32_t code = *ws->host_verr;
  if (code != 0x7f7f7f7f) {
    static const char* what[] = {"", "neighbour id out of range", "self-loop", "row not strictly increasing",
                                 "graph not symmetric"};
    return fail(KCORE_E_INVALID, std::string("KCORE_VALIDATE: ") + what[std::min(code, 4)]);
  }
  return KCORE_OK;
}

// Buffers of the relabelled copy (grown on demand).
static kcore_status ensure_relabel(Workspace* ws, int64_t n, int64_t nnz, hipStream_t st) {
  auto& rl = ws->rl;
  if (!rl.probe) {
    KC_HIP(hipMalloc(&rl.probe, 2 * sizeof(unsigned long long)));
    KC_HIP(hipHostMalloc(&rl.host_probe, 2 * sizeof(unsigned long long), hipHostMallocDefault));
  }
  if (n <= rl.cap_n && nnz <= rl.cap_nnz) return KCORE_OK;
  KC_HIP(hipStreamSynchronize(st));
  const int64_t cn = std::max(n, rl.cap_n), ce = std::max<int64_t>({nnz, rl.cap_nnz, 1});
  ws->release_relabel();
  size_t sort_bytes = 0, scan_bytes = 0;
  KC_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, (uint32_t*)nullptr, (uint32_t*)nullptr,
                                            (int32_t*)nullptr, (int32_t*)nullptr, (int)cn, 0, 10, st));
  KC_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, scan_bytes, (int64_t*)nullptr, (int64_t*)nullptr, (int)(cn + 1),
                                          st));
  rl.temp_bytes = std::max<size_t>({sort_bytes, scan_bytes, 256});
  const bool ok = hipMalloc(&rl.keys[0], sizeof(uint32_t) * cn) == hipSuccess &&
                  hipMalloc(&rl.keys[1], sizeof(uint32_t) * cn) == hipSuccess &&
                  hipMalloc(&rl.ids, sizeof(int32_t) * cn) == hipSuccess &&
                  hipMalloc(&rl.order, sizeof(int32_t) * cn) == hipSuccess &&
                  hipMalloc(&rl.new_of, sizeof(int32_t) * cn) == hipSuccess &&
                  hipMalloc(&rl.new_deg, sizeof(int64_t) * (cn + 1)) == hipSuccess &&
                  hipMalloc(&rl.nrp, sizeof(int64_t) * (cn + 1)) == hipSuccess &&
                  hipMalloc(&rl.ncol, sizeof(int32_t) * ce) == hipSuccess &&
                  hipMalloc(&rl.nout, sizeof(int32_t) * cn) == hipSuccess &&
                  hipMalloc(&rl.temp, rl.temp_bytes) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    ws->release_relabel();
    return fail(KCORE_E_NOMEM, "relabel buffers: allocation failed");
  }
  rl.cap_n = cn;
  rl.cap_nnz = ce;
  return KCORE_OK;
}

// Rows of degree > kRelabelLongDeg and the entries in them (synchronises the stream).
template <typename Off>
static kcore_status relabel_probe(Workspace* ws, int64_t n, const Off* row_ptr, int64_t* rows, int64_t* entries,
                                  hipStream_t st) {
  kcore_status s = ensure_relabel(ws, 0, 0, st);
  if (s != KCORE_OK) return s;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, (int64_t)ws->num_cus * 8));
  KC_HIP(hipMemsetAsync(ws->rl.probe, 0, 2 * sizeof(unsigned long long), st));
  hipLaunchKernelGGL(k_relabel_probe<Off>, dim3(grid), dim3(kBlock), 0, st, n, row_ptr, ws->rl.probe);
  KC_HIP(hipGetLastError());
  KC_HIP(hipMemcpyAsync(ws->rl.host_probe, ws->rl.probe, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
  KC_HIP(hipStreamSynchronize(st));
  *rows = (int64_t)ws->rl.host_probe[0];
  *entries = (int64_t)ws->rl.host_probe[1];
  return KCORE_OK;
}

// Decomposition of the graph renumbered by decreasing degree; results in the caller's numbering.
template <typename Off>
static kcore_status decompose_relabelled(Workspace* ws, int64_t n, int64_t nnz, const Off* row_ptr,
                                         const int32_t* col, int32_t* out, int64_t nlong, const Tuning& tu,
                                         kcore_stats* stats, hipStream_t st, std::vector<kcore_round_record>* rec) {
  kcore_status s = ensure_relabel(ws, n, nnz, st);
  if (s != KCORE_OK) return s;
  auto& rl = ws->rl;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, (int64_t)ws->num_cus * 16));
  hipLaunchKernelGGL(k_relabel_keys<Off>, dim3(grid), dim3(kBlock), 0, st, n, row_ptr, rl.keys[0], rl.ids);
  KC_HIP(hipGetLastError());
  size_t bytes = rl.temp_bytes;
  KC_HIP(hipcub::DeviceRadixSort::SortPairs(rl.temp, bytes, rl.keys[0], rl.keys[1], rl.ids, rl.order, (int)n, 0,
                                            10, st));
  hipLaunchKernelGGL(k_relabel_inverse<Off>, dim3(grid), dim3(kBlock), 0, st, n, row_ptr, rl.order, rl.new_of,
                     rl.new_deg);
  KC_HIP(hipGetLastError());
  bytes = rl.temp_bytes;
  KC_HIP(hipcub::DeviceScan::ExclusiveSum(rl.temp, bytes, rl.new_deg, rl.nrp, (int)(n + 1), st));
  hipLaunchKernelGGL(k_relabel_rows<Off>, dim3(grid), dim3(kBlock), 0, st, n, nlong, row_ptr, col, rl.order,
                     rl.new_of, rl.nrp, rl.ncol);
  KC_HIP(hipGetLastError());
  s = run_rounds<false, int64_t>(ws, n, nnz, rl.nrp, rl.ncol, rl.nout, tu, stats, st, rec);
  if (s != KCORE_OK) return s;
  hipLaunchKernelGGL(k_relabel_out, dim3(grid), dim3(kBlock), 0, st, n, rl.new_of, rl.nout, out);
  KC_HIP(hipGetLastError());
  return KCORE_OK;
}

template <typename Off>
static kcore_status decompose_impl(int64_t n, const Off* row_ptr, const int32_t* col, int32_t* out,
                                   const kcore_tuning* tuning, kcore_stats* stats, hipStream_t st,
                                   std::vector<kcore_round_record>* rec = nullptr) {
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (n < 0 || n > INT32_MAX) return fail(KCORE_E_INVALID, "n must be in [0, 2^31-1]");
  if (n == 0) return KCORE_OK;
  if (!row_ptr || !col || !out) return fail(KCORE_E_INVALID, "null pointer argument");
  Workspace* ws = nullptr;
  kcore_status s = get_workspace(&ws);
  if (s != KCORE_OK) return s;
  std::lock_guard<std::mutex> lk(ws->mu);
  *ws->host_nnz = 0;
  KC_HIP(hipMemcpyAsync(ws->host_nnz, row_ptr + n, sizeof(Off), hipMemcpyDeviceToHost, st));
  KC_HIP(hipStreamSynchronize(st));
  const int64_t nnz = sizeof(Off) == 8 ? *ws->host_nnz : (int64_t)*(const int32_t*)ws->host_nnz;
  if (nnz < 0) return fail(KCORE_E_INVALID, "row_ptr[n] is negative");
  s = ensure_capacity(ws, n, nnz, false, st);
  if (s != KCORE_OK) return s;
  if (env_flag("KCORE_VALIDATE")) {
    s = validate_csr<Off>(ws, n, row_ptr, col, st);
    if (s != KCORE_OK) return s;
  }
  Tuning tu = resolve_tuning(tuning, ws->num_cus);
  settle_tuning(&tu, n, nnz, false);
  if (tu.relabel && n > 1 && n < INT32_MAX - 1 && nnz > 0) {
    int64_t long_rows = 0, long_entries = 0;
    s = relabel_probe<Off>(ws, n, row_ptr, &long_rows, &long_entries, st);
    if (s != KCORE_OK) return s;
    return decompose_relabelled<Off>(ws, n, nnz, row_ptr, col, out, long_rows, tu, stats, st, rec);
  }
  return run_rounds<false, Off>(ws, n, nnz, row_ptr, col, out, tu, stats, st, rec);
}

// ------------------------------------------------------------------ no-allocation entry point
// kcore_decompose_noalloc keeps its whole workspace in one device array of
// fixed size, `scratch`, which the code object defines: every device the
// library runs on holds its own copy from the first kernel launch until the
// process ends, and the call itself allocates nothing (no hipMalloc, no
// pinned host buffer, no captured graph).  Host code never passes the array's
// name to a kernel: that name is a host-side stand-in, not a device address.
// The device address comes from hipGetSymbolAddress, once per device, at the
// first call on it, and is kept per device.
constexpr int64_t kNoAllocMaxN = KCORE_NOALLOC_MAX_VERTICES;
constexpr int64_t kNoAllocMaxNnz = KCORE_NOALLOC_MAX_ENTRIES;
constexpr size_t align256(size_t x) { return (x + 255) / 256 * 256; }
// Layout: control block, validation word, then the per-vertex arrays (stamp,
// class, two frontier lists, first-round list, pruned length, pruned threshold,
// slack) and the pruned adjacency.
constexpr size_t kScratchCtl = 0;
constexpr size_t kScratchVerr = kScratchCtl + align256(sizeof(Ctl));
constexpr size_t kScratchStamp = kScratchVerr + 256;
constexpr size_t kScratchCls = kScratchStamp + align256(4 * kNoAllocMaxN);
constexpr size_t kScratchList0 = kScratchCls + align256(kNoAllocMaxN);
constexpr size_t kScratchList1 = kScratchList0 + align256(4 * kNoAllocMaxN);
constexpr size_t kScratchSlist = kScratchList1 + align256(4 * kNoAllocMaxN);
constexpr size_t kScratchPlen = kScratchSlist + align256(4 * kNoAllocMaxN);
constexpr size_t kScratchPlow = kScratchPlen + align256(4 * kNoAllocMaxN);
constexpr size_t kScratchSlack = kScratchPlow + align256(4 * kNoAllocMaxN);
constexpr size_t kScratchPruned = kScratchSlack + align256(4 * kNoAllocMaxN);
constexpr size_t kScratchBytes = kScratchPruned + align256(4 * kNoAllocMaxNnz);
static_assert(kScratchBytes <= KCORE_NOALLOC_SCRATCH_BYTES, "scratch larger than the header states");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct NoAllocState {
  unsigned char* dev = nullptr;  // device address of this device's scratch
  int num_cus = 0;
  int32_t epoch = 1;             // next round base (stamps of earlier calls are all below it)
  Ctl host_ctl;                  // host copy of the control block (plain host memory)
  int64_t host_word = 0;         // host copy of row_ptr[n] or of the validation word
};
static std::mutex g_noalloc_mu;
static NoAllocState g_noalloc[64];

// Device address of the scratch array on the current device (kept per device); the stamps start at 0.
static kcore_status noalloc_setup(int dev, hipStream_t st) {
  NoAllocState& S = g_noalloc[dev];
  if (S.dev) return KCORE_OK;
  void* ptr = nullptr;
  KC_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) return fail(KCORE_E_HIP, "hipGetSymbolAddress(scratch) returned no address");
  int cus = 0;
  KC_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  unsigned char* base = static_cast<unsigned char*>(ptr);
  const int grid = (int)std::min<int64_t>((kNoAllocMaxN + kBlock - 1) / kBlock, (int64_t)cus * 16);
  hipLaunchKernelGGL(k_fill, dim3(grid), dim3(kBlock), 0, st, reinterpret_cast<int32_t*>(base + kScratchStamp),
                     kNoAllocMaxN, 0);
  KC_HIP(hipGetLastError());
  S.dev = base;
  S.num_cus = cus;
  S.epoch = 1;
  return KCORE_OK;
}

static kcore_status decompose_noalloc_impl(int64_t n, const int64_t* row_ptr, const int32_t* col, int32_t* out,
                                           hipStream_t st) {
  if (n < 0 || n > INT32_MAX) return fail(KCORE_E_INVALID, "n must be in [0, 2^31-1]");
  if (n > kNoAllocMaxN)
    return fail(KCORE_E_TOO_LARGE, "kcore_decompose_noalloc: n=" + std::to_string(n) + " exceeds " +
                                       std::to_string(kNoAllocMaxN) + " vertices");
  if (n == 0) return KCORE_OK;
  if (!row_ptr || !col || !out) return fail(KCORE_E_INVALID, "null pointer argument");
  int dev = 0;
  KC_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(KCORE_E_INVALID, "device index out of range");
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  kcore_status s = noalloc_setup(dev, st);
  if (s != KCORE_OK) return s;
  NoAllocState& S = g_noalloc[dev];
  S.host_word = -1;
  KC_HIP(hipMemcpyAsync(&S.host_word, row_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  KC_HIP(hipStreamSynchronize(st));
  const int64_t nnz = S.host_word;
  if (nnz < 0) return fail(KCORE_E_INVALID, "row_ptr[n] is negative");
  if (nnz > kNoAllocMaxNnz)
    return fail(KCORE_E_TOO_LARGE, "kcore_decompose_noalloc: " + std::to_string(nnz) + " adjacency entries exceed " +
                                       std::to_string(kNoAllocMaxNnz));
  // A workspace view of the scratch array (registered nowhere; it owns nothing).
  Workspace ws;
  ws.device = dev;
  ws.num_cus = S.num_cus;
  ws.cap_n = kNoAllocMaxN;
  ws.cap_nnz = kNoAllocMaxNnz;
  ws.ctl = reinterpret_cast<Ctl*>(S.dev + kScratchCtl);
  ws.verr = reinterpret_cast<int32_t*>(S.dev + kScratchVerr);
  ws.stamp = reinterpret_cast<int32_t*>(S.dev + kScratchStamp);
  ws.cls = S.dev + kScratchCls;
  ws.lists[0] = reinterpret_cast<int32_t*>(S.dev + kScratchList0);
  ws.lists[1] = reinterpret_cast<int32_t*>(S.dev + kScratchList1);
  ws.slist = reinterpret_cast<int32_t*>(S.dev + kScratchSlist);
  ws.plen = reinterpret_cast<int32_t*>(S.dev + kScratchPlen);
  ws.plow = reinterpret_cast<int32_t*>(S.dev + kScratchPlow);
  ws.slack = reinterpret_cast<int32_t*>(S.dev + kScratchSlack);
  ws.pruned = reinterpret_cast<int32_t*>(S.dev + kScratchPruned);
  ws.host_ctl = &S.host_ctl;
  ws.host_verr = reinterpret_cast<int32_t*>(&S.host_word);
  ws.epoch = S.epoch;
  if (env_flag("KCORE_VALIDATE")) {
    s = validate_csr<int64_t>(&ws, n, row_ptr, col, st);
    if (s != KCORE_OK) return s;
  }
  Tuning tu = resolve_tuning(nullptr, S.num_cus);
  tu.use_graph = 0;  // instantiating a graph allocates
  tu.defer = 0;      // no deferred-check buffer: such neighbours are re-activated
  settle_tuning(&tu, n, nnz, false);
  s = run_rounds<false, int64_t>(&ws, n, nnz, row_ptr, col, out, tu, nullptr, st);
  S.epoch = ws.epoch;
  return s;
}

// ------------------------------------------------------------------ core maintenance (kcore_update)
template <typename Off>
static kcore_status update_impl(int64_t n, const Off* row_ptr, const int32_t* col, const int32_t* prev, int64_t nd,
                                const int32_t* del, int64_t ni, const int32_t* ins, int32_t* out,
                                const kcore_tuning* tuning, kcore_stats* stats, hipStream_t st) {
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (n < 0 || n > INT32_MAX) return fail(KCORE_E_INVALID, "n must be in [0, 2^31-1]");
  if (nd < 0 || ni < 0) return fail(KCORE_E_INVALID, "edge counts must be >= 0");
  if (n == 0) return KCORE_OK;
  if (!row_ptr || !col || !prev || !out || (nd > 0 && !del) || (ni > 0 && !ins))
    return fail(KCORE_E_INVALID, "null pointer argument");
  Workspace* ws = nullptr;
  kcore_status s = get_workspace(&ws);
  if (s != KCORE_OK) return s;
  std::lock_guard<std::mutex> lk(ws->mu);
  *ws->host_nnz = 0;
  KC_HIP(hipMemcpyAsync(ws->host_nnz, row_ptr + n, sizeof(Off), hipMemcpyDeviceToHost, st));
  KC_HIP(hipStreamSynchronize(st));
  const int64_t nnz = sizeof(Off) == 8 ? *ws->host_nnz : (int64_t)*(const int32_t*)ws->host_nnz;
  if (nnz < 0) return fail(KCORE_E_INVALID, "row_ptr[n] is negative");
  s = ensure_capacity(ws, n, nnz, false, st);
  if (s != KCORE_OK) return s;
  if (env_flag("KCORE_VALIDATE")) {
    s = validate_csr<Off>(ws, n, row_ptr, col, st);
    if (s != KCORE_OK) return s;
  }
  Tuning tu = resolve_tuning(tuning, ws->num_cus);
  settle_tuning(&tu, n, nnz, false);
  tu.max_rounds = 0;
  // the flags live in the pruned-threshold array until the run starts (no pruned list exists then)
  int32_t* flag = ws->plow;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, (int64_t)ws->num_cus * 16));
  hipLaunchKernelGGL(k_fill, dim3(grid), dim3(kBlock), 0, st, flag, n, 0);
  // aux: [0] smallest and [1] largest min(c_old(u), c_old(v)) over I, [2] D, [3..5] the search's rotating
  // queue counters, [6] D' and [7] T' of the heavy-vertex rule, [8..11] the search's two 64-bit long-row
  // counters, [12..13] the 64-bit count of states reached, [14] the number of neighbours of Z
  hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, st, ws->aux, (int64_t)1, INT32_MAX);
  hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, st, ws->aux + 1, (int64_t)15, 0);
  // per-vertex counts of inserted edges live in the flag word above bit 1, which holds
  // counts below 2^29; larger batches take D = |I|
  const bool count = ni < (1 << 28);
  if (nd + ni > 0) {
    const int egrid = (int)std::max<int64_t>(1, std::min<int64_t>((nd + ni + kBlock - 1) / kBlock,
                                                                    (int64_t)ws->num_cus * 16));
    hipLaunchKernelGGL(k_upd_edges, dim3(egrid), dim3(kBlock), 0, st, del, nd, ins, ni, prev, flag, (int32_t)count,
                       ws->aux);
  }
  KC_HIP(hipGetLastError());
  int64_t rise = 0, cap = 0;
  int32_t all_from = INT32_MAX;
  bool heavy = false;
  if (ni > 0) {
    KC_HIP(hipMemcpyAsync(ws->host_aux, ws->aux, 3 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    KC_HIP(hipStreamSynchronize(st));
    int64_t T = ws->host_aux[0];
    rise = count ? ws->host_aux[2] : ni;
    cap = (int64_t)ws->host_aux[1] + rise;
    // the window rule while D is small (window offsets fit two bits of a queue entry, ids 30 bits),
    // otherwise the threshold rule; the slack array, not yet in use, holds the reached window offsets
    // (and, for the heavy-vertex rule, its counts)
    const bool window = rise <= kUpdWindowMax && n <= (int64_t)kStateMask + 1;
    int32_t* vis = ws->slack;
    if (window || rise >= 2) hipLaunchKernelGGL(k_fill, dim3(grid), dim3(kBlock), 0, st, vis, n, 0);
    // breadth-first search; the frontier lists serve as the search queues and the pruned-entry array,
    // not in use before the run, as the list of long rows (two ints per row, at most
    // kUpdWindowMax * nnz / kBfsLongRow rows; the rows of Z: at most |I| <= nnz / 2)
    int32_t* cnt = ws->aux + 3;
    unsigned long long* lcnt = reinterpret_cast<unsigned long long*>(ws->aux + 8);
    const int sgrid = (int)std::max<int64_t>(1, std::min<int64_t>((2 * ni + kBlock - 1) / kBlock,
                                                                   (int64_t)ws->num_cus * 16));
    const int lgrid = ws->num_cus * 8;
    constexpr int kLevelsPerPoll = 4;
    // (never above n, the queues' capacity: a level that overflows a queue also passes the budget)
    const int64_t budget = std::min<int64_t>(std::max<int64_t>(n / 16, 4096), n);
    bool give_up = false;
    UpdSearch q{(int32_t)T, window ? (int32_t)rise : 0, flag, vis, n};
    // The heavy-vertex rule, tried when some vertex has two or more inserted edges: Z's rows are
    // registered in the second long-row list (the first level clears it), D', T' and the number of
    // neighbours of Z are counted, and when D' <= 1 the search is the one of that rule.
    if (count && rise >= 2 && n <= (int64_t)kStateMask + 1 && 2 * ni <= nnz) {
      const UpdSearch zq{0, 1, flag, vis, n};
      hipLaunchKernelGGL(k_upd_zreg<Off>, dim3(sgrid), dim3(kBlock), 0, st, row_ptr, ins, ni, flag, vis, ws->pruned,
                         lcnt + 1, ws->aux);
      hipLaunchKernelGGL(k_upd_zcount<Off>, dim3(lgrid), dim3(kBlock), 0, st, row_ptr, col, prev, zq, ins, ni,
                         ws->pruned, lcnt + 1, ws->aux);
      KC_HIP(hipGetLastError());
      KC_HIP(hipMemcpyAsync(ws->host_aux + 6, ws->aux + 6, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
      KC_HIP(hipMemcpyAsync(ws->host_aux + 14, ws->aux + 14, sizeof(int32_t), hipMemcpyDeviceToHost, st));
      KC_HIP(hipStreamSynchronize(st));
      if (ws->host_aux[6] <= 1) {
        heavy = true;
        T = ws->host_aux[7];
        q = zq;
        // more sources than the budget allows gives the search up at once (Z still goes into A)
        give_up = ws->host_aux[14] > budget;
        hipLaunchKernelGGL(k_upd_zsrc<Off>, dim3(lgrid), dim3(kBlock), 0, st, row_ptr, col, prev, q, ws->pruned,
                           lcnt + 1, (int32_t)!give_up, ws->lists[0], cnt);
      }
    }
    if (give_up) {
      all_from = (int32_t)std::min<int64_t>(T, INT32_MAX);
    } else {
      hipLaunchKernelGGL(k_upd_bfs_start, dim3(sgrid), dim3(kBlock), 0, st, ins, ni, prev, q, ws->lists[0], cnt);
      KC_HIP(hipGetLastError());
      // A search that reaches more than a sixteenth of the vertices (in states; at least 4096, at most n)
      // is given up: A then also takes every vertex of old coreness >= T, a superset, since on a graph
      // whose cores hang together the search would have reached nearly all of them at the cost of a
      // traversal of the graph.  Levels are launched in bursts of kLevelsPerPoll on a fixed grid (each
      // level reads its queue's length on the device); the host then reads the current queue's length and
      // the states reached so far.  A level past the queues' capacity leaves an incomplete search behind
      // it, but its count alone exceeds the budget, so the search is given up at the next look.
      // Levels holding at most kBfsSmallBlock states (and kBfsSmallEntries entries) run inside one
      // workgroup (k_upd_bfs_small, which stops at a larger level); the first level is known to be small
      // when the sources are few.
      unsigned long long* reached = reinterpret_cast<unsigned long long*>(ws->aux + 12);
      const int64_t sources = 2 * ni * std::max<int32_t>(1, q.D) + (heavy ? ws->host_aux[14] : 0);
      bool small = sources <= kBfsSmallBlock;
      for (int level = 0;;) {
        if (small) {
          hipLaunchKernelGGL(k_upd_bfs_small<Off>, dim3(1), dim3(kBfsSmallBlock), 0, st, row_ptr, col, prev, q,
                             ws->lists[0], ws->lists[1], cnt, level, budget, reached, lcnt, ws->aux);
        } else {
          for (int b = 0; b < kLevelsPerPoll; ++b, ++level) {
            int32_t* cnt_in = cnt + level % 3;
            int32_t* cnt_out = cnt + (level + 1) % 3;
            int32_t* const qin = ws->lists[level & 1];
            int32_t* const qout = ws->lists[(level + 1) & 1];
            hipLaunchKernelGGL(k_upd_bfs_level<Off>, dim3(lgrid), dim3(kBlock), 0, st, row_ptr, col, prev, q, qin,
                               cnt_in, qout, cnt_out, cnt + (level + 2) % 3, ws->pruned, lcnt + (level & 1),
                               lcnt + ((level + 1) & 1), reached);
            hipLaunchKernelGGL(k_upd_bfs_long<Off>, dim3(ws->num_cus * 4), dim3(kBlock), 0, st, row_ptr, col,
                               prev, q, ws->pruned, lcnt + (level & 1), qout, cnt_out);
          }
        }
        KC_HIP(hipGetLastError());
        // aux[3..15]: the queue counters, the long-row counters, the states reached, the small kernel's level
        KC_HIP(hipMemcpyAsync(ws->host_aux + 3, ws->aux + 3, 13 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
        KC_HIP(hipStreamSynchronize(st));
        if (small) level = ws->host_aux[15];
        const int64_t nq = ws->host_aux[3 + level % 3];
        unsigned long long total = 0;
        std::memcpy(&total, ws->host_aux + 12, sizeof(total));
        if ((int64_t)total + nq > budget) {
          all_from = (int32_t)std::min<int64_t>(T, INT32_MAX);
          break;
        }
        if (nq == 0) break;
        // a small launch that returns with a live level stopped at a large one: a burst follows
        small = !small && nq <= kBfsSmallBlock;
      }
    }
  }
  const UpdateStart upd{prev, flag, rise, cap, heavy, all_from, nd == 0};
  return run_rounds<false, Off>(ws, n, nnz, row_ptr, col, out, tu, stats, st, nullptr, &upd);
}

// ------------------------------------------------------------------ certificate (kcore_certify)
template <typename Off>
static kcore_status certify_impl(int64_t n, const Off* row_ptr, const int32_t* col, const int32_t* core,
                                 int32_t* out_code, int64_t* out_vertex, hipStream_t st) {
  if (!out_code || !out_vertex) return fail(KCORE_E_INVALID, "null result pointer");
  *out_code = 0;
  *out_vertex = -1;
  if (n < 0 || n > INT32_MAX) return fail(KCORE_E_INVALID, "n must be in [0, 2^31-1]");
  if (n == 0) return KCORE_OK;
  if (!row_ptr || !col || !core) return fail(KCORE_E_INVALID, "null pointer argument");
  Workspace* ws = nullptr;
  kcore_status s = get_workspace(&ws);
  if (s != KCORE_OK) return s;
  std::lock_guard<std::mutex> lk(ws->mu);
  *ws->host_nnz = 0;
  KC_HIP(hipMemcpyAsync(ws->host_nnz, row_ptr + n, sizeof(Off), hipMemcpyDeviceToHost, st));
  hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, st, ws->cert, (int64_t)2, (int32_t)-1);
  hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, st, ws->cert + 2, (int64_t)2, 0);
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((n * kWave + kBlock - 1) / kBlock,
                                                                (int64_t)ws->num_cus * 32));
  hipLaunchKernelGGL(k_certify<Off>, dim3(grid), dim3(kBlock), 0, st, n, row_ptr, col, core,
                     reinterpret_cast<unsigned long long*>(ws->cert), ws->cert + 2);
  KC_HIP(hipGetLastError());
  KC_HIP(hipMemcpyAsync(ws->host_cert, ws->cert, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  KC_HIP(hipStreamSynchronize(st));
  const int64_t nnz = sizeof(Off) == 8 ? *ws->host_nnz : (int64_t)*(const int32_t*)ws->host_nnz;
  unsigned long long w;
  std::memcpy(&w, ws->host_cert, sizeof(w));
  if (w != ~0ull) {
    *out_vertex = (int64_t)(w >> 32);
    *out_code = (int32_t)(w & 0xffffffffull);
    return KCORE_OK;
  }
  const int64_t km = ws->host_cert[2];
  if (km * (km + 1) / 2 > nnz / 2) *out_code = 4;
  return KCORE_OK;
}

template <typename Off>
static kcore_status validate_batch(Workspace* ws, int64_t n, const Off* row_ptr, const int32_t* col,
                                   hipStream_t st) {
  const int grid = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, (int64_t)ws->num_cus * 16);
  KC_HIP(hipMemsetAsync(ws->verr, 0x7f, sizeof(int32_t), st));
  hipLaunchKernelGGL(k_validate_batch<Off>, dim3(grid), dim3(kBlock), 0, st, n, row_ptr, col, ws->vbase, ws->verr);
  KC_HIP(hipGetLastError());
  KC_HIP(hipMemcpyAsync(ws->host_verr, ws->verr, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  KC_HIP(hipStreamSynchronize(st));
  const int32_t code = *ws->host_verr;
  if (code != 0x7f7f7f7f) {
    static const char* what[] = {"", "neighbour id outside its graph", "self-loop", "row not strictly increasing",
                                 "graph not symmetric"};
    return fail(KCORE_E_INVALID, std::string("KCORE_VALIDATE: ") + what[std::min(code, 4)]);
  }
  return KCORE_OK;
}

// ------------------------------------------------------------------ tuning cache (autotuner results)
struct TuneEntry {
  int32_t G;
  int32_t logn, lognnz;  // log2 buckets of the vertex and entry counts
  kcore_tuning t;
};
static std::mutex g_tune_mu;
static std::vector<TuneEntry> g_tune;

static int ilog2(int64_t x) {
  int l = 0;
  while (x > 1) {
    x >>= 1;
    ++l;
  }
  return l;
}

static bool tune_lookup(int32_t G, int64_t n, int64_t nnz, kcore_tuning* out) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const auto& e : g_tune)
    if (e.G == G && e.logn == ilog2(n) && e.lognnz == ilog2(nnz)) {
      *out = e.t;
      return true;
    }
  return false;
}

static void tune_store(int32_t G, int64_t n, int64_t nnz, const kcore_tuning& t) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (auto& e : g_tune)
    if (e.G == G && e.logn == ilog2(n) && e.lognnz == ilog2(nnz)) {
      e.t = t;
      return;
    }
  g_tune.push_back({G, ilog2(n), ilog2(nnz), t});
}

// Batched decomposition: read the sizes, build the per-vertex graph base, run.
static kcore_status batch_prepare(Workspace* ws, int32_t G, const int64_t* gvo, const int64_t* row_ptr,
                                  int64_t* n_out, int64_t* nnz_out, hipStream_t st) {
  KC_HIP(hipMemcpyAsync(ws->host_nnz, gvo + G, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  KC_HIP(hipStreamSynchronize(st));
  const int64_t n = *ws->host_nnz;
  if (n < 0 || n > INT32_MAX) return fail(KCORE_E_INVALID, "total vertex count must be in [0, 2^31-1]");
  int64_t nnz = 0;
  if (n > 0) {
    KC_HIP(hipMemcpyAsync(ws->host_nnz, row_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    KC_HIP(hipStreamSynchronize(st));
    nnz = *ws->host_nnz;
    if (nnz < 0) return fail(KCORE_E_INVALID, "row_ptr[N] is negative");
  }
  *n_out = n;
  *nnz_out = nnz;
  if (n == 0) return KCORE_OK;
  kcore_status s = ensure_capacity(ws, n, nnz, true, st);
  if (s != KCORE_OK) return s;
  hipLaunchKernelGGL(k_vbase, dim3(G), dim3(256), 0, st, gvo, ws->vbase);
  KC_HIP(hipGetLastError());
  return KCORE_OK;
}

static kcore_status batch_impl(int32_t G, const int64_t* gvo, const int64_t* row_ptr, const int32_t* col,
                               int32_t* out, const kcore_tuning* tuning, kcore_stats* stats, hipStream_t st) {
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (G < 0) return fail(KCORE_E_INVALID, "num_graphs must be >= 0");
  if (G == 0) return KCORE_OK;
  if (!gvo || !row_ptr || !col || !out) return fail(KCORE_E_INVALID, "null pointer argument");
  Workspace* ws = nullptr;
  kcore_status s = get_workspace(&ws);
  if (s != KCORE_OK) return s;
  std::lock_guard<std::mutex> lk(ws->mu);
  int64_t n = 0, nnz = 0;
  s = batch_prepare(ws, G, gvo, row_ptr, &n, &nnz, st);
  if (s != KCORE_OK || n == 0) return s;
  if (env_flag("KCORE_VALIDATE")) {
    s = validate_batch<int64_t>(ws, n, row_ptr, col, st);
    if (s != KCORE_OK) return s;
  }
  kcore_tuning cached;
  const kcore_tuning* use = tuning;
  if (!use && tune_lookup(G, n, nnz, &cached)) use = &cached;
  Tuning tu = resolve_tuning(use, ws->num_cus);
  settle_tuning(&tu, n, nnz, true);
  return run_rounds<true, int64_t>(ws, n, nnz, row_ptr, col, out, tu, stats, st);
}

// Coordinate descent over the launch knobs; each candidate is timed (median
// of `reps` runs, HIP events on the stream) on the caller's batch.
static kcore_status autotune_impl(int32_t G, const int64_t* gvo, const int64_t* row_ptr, const int32_t* col,
                                  int32_t* out, int32_t reps, kcore_tuning* best, float* best_ms, hipStream_t st) {
  if (G <= 0 || !gvo || !row_ptr || !col || !out || !best) return fail(KCORE_E_INVALID, "bad autotune arguments");
  reps = std::max(1, std::min(reps, 15));
  Workspace* ws = nullptr;
  kcore_status s = get_workspace(&ws);
  if (s != KCORE_OK) return s;
  int cus = ws->num_cus;
  hipEvent_t e0, e1;
  KC_HIP(hipEventCreate(&e0));
  KC_HIP(hipEventCreate(&e1));
  auto measure = [&](const kcore_tuning& t, float* ms) -> kcore_status {
    std::vector<float> v;
    for (int i = 0; i < reps + 1; ++i) {
      KC_HIP(hipEventRecord(e0, st));
      kcore_status r = batch_impl(G, gvo, row_ptr, col, out, &t, nullptr, st);
      if (r != KCORE_OK) return r;
      KC_HIP(hipEventRecord(e1, st));
      KC_HIP(hipEventSynchronize(e1));
      float x = 0;
      KC_HIP(hipEventElapsedTime(&x, e0, e1));
      if (i > 0) v.push_back(x);  // first run warms the workspace and the graph cache
    }
    std::sort(v.begin(), v.end());
    *ms = v[v.size() / 2];
    return KCORE_OK;
  };
  kcore_tuning cur;
  std::memset(&cur, 0, sizeof(cur));
  float cur_ms = 0;
  s = measure(cur, &cur_ms);
  if (s != KCORE_OK) return s;
  struct Knob {
    int32_t kcore_tuning::*field;
    std::vector<int32_t> values;
  };
  const std::vector<Knob> knobs = {
      {&kcore_tuning::grid_blocks, {4 * cus, 8 * cus, 16 * cus}},
      {&kcore_tuning::big_grid_blocks, {4 * cus, 16 * cus, 32 * cus}},
      {&kcore_tuning::list_cap, {2048, 8192, 32768}},
      {&kcore_tuning::tail_threshold, {512, 2048, 8192}},
      {&kcore_tuning::group_max_deg, {32, 64}},
      {&kcore_tuning::wave_max_deg, {256, 512}},
      {&kcore_tuning::rounds_per_poll, {2, 4, 8}},
      {&kcore_tuning::activation, {1, 2}},
  };
  for (const auto& k : knobs) {
    for (int32_t val : k.values) {
      kcore_tuning cand = cur;
      cand.*(k.field) = val;
      float ms = 0;
      s = measure(cand, &ms);
      if (s != KCORE_OK) return s;
      if (ms < cur_ms * 0.99f) {
        cur = cand;
        cur_ms = ms;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *best = cur;
  if (best_ms) *best_ms = cur_ms;
  int64_t n = 0, nnz = 0;
  {
    std::lock_guard<std::mutex> lk(ws->mu);
    s = batch_prepare(ws, G, gvo, row_ptr, &n, &nnz, st);
    if (s != KCORE_OK) return s;
  }
  tune_store(G, n, nnz, cur);
  return KCORE_OK;
}

// ------------------------------------------------------------------ served graphs (device side)
static Args<int64_t> serve_args(const ServeArena* A) {
  Args<int64_t> a;
  std::memset(&a, 0, sizeof(a));
  a.n = A->nv;
  a.row_ptr = A->row_ptr;
  a.col = A->col;
  a.vbase = A->vbase;
  a.est = A->est;
  a.stamp = A->stamp;
  a.cls = A->cls;
  a.lists[0] = A->lists[0];
  a.lists[1] = A->lists[1];
  a.slist = nullptr;  // no first (all-vertex) round: graphs join through compaction rounds
  a.pruned = A->pruned;
  a.plen = A->plen;
  a.plow = A->plow;
  a.ctl = static_cast<Ctl*>(A->ctl);
  a.slack = A->slack;
  a.served = 1;
  a.tail_threshold = A->tu.tail;
  a.list_cap = A->tu.list_cap;
  a.one_sided = A->tu.one_sided;
  a.prune = A->tu.prune;
  a.gact = A->gact;
  a.tail_cap = A->tu.tail_cap;
  a.tail_order = A->tu.tail_order;
  a.tail_big = A->tu.tail_big;
  return a;
}

void serve_arena_destroy(ServeArena* A) {
  if (A->step_exec) (void)hipGraphExecDestroy(static_cast<hipGraphExec_t>(A->step_exec));
  A->step_exec = nullptr;
  for (void* p : {(void*)A->row_ptr, (void*)A->est, (void*)A->stamp, (void*)A->cls, (void*)A->lists[0],
                  (void*)A->lists[1], (void*)A->plen, (void*)A->plow, (void*)A->vbase, (void*)A->slack, (void*)A->gact,

                  (void*)A->col, (void*)A->pruned, A->ctl, A->slots, (void*)A->slot_vb, (void*)A->status})
    if (p) (void)hipFree(p);
  *A = ServeArena();
}

kcore_status serve_arena_create(ServeArena* A, int device, int64_t nv, int64_t ne, int32_t max_slots,
                                const kcore_tuning* tuning, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  *A = ServeArena();
  A->device = device;
  hipDeviceProp_t prop;
  KC_HIP(hipGetDeviceProperties(&prop, device));
  A->num_cus = prop.multiProcessorCount;
  A->nv = nv;
  A->ne = std::max<int64_t>(ne, 1);
  A->max_slots = max_slots;
  A->tu = resolve_tuning(tuning, A->num_cus);
  if (A->tu.one_sided < 0) A->tu.one_sided = 0;  // graphs of any density share the rounds
  A->tu.defer = 0;                               // the arenas keep no deferred-check buffer
  size_t bytes = 0;
  auto alloc = [&](auto** p, size_t count) {
    const size_t b = sizeof(**p) * std::max<size_t>(count, 1);
    bytes += b;
    return hipMalloc(reinterpret_cast<void**>(p), b) == hipSuccess;
  };
  const bool ok = alloc(&A->row_ptr, nv) && alloc(&A->est, nv) && alloc(&A->stamp, nv) && alloc(&A->cls, nv) &&
                  alloc(&A->lists[0], nv) && alloc(&A->lists[1], nv) && alloc(&A->plen, nv) &&
                  alloc(&A->plow, nv) && alloc(&A->vbase, nv) && alloc(&A->slack, nv) && alloc(&A->gact, nv) &&
 alloc(&A->col, A->ne) &&
                  alloc(&A->pruned, A->ne) && alloc(reinterpret_cast<Ctl**>(&A->ctl), 1) &&
                  alloc(reinterpret_cast<SlotDesc**>(&A->slots), max_slots) && alloc(&A->slot_vb, max_slots) &&
                  alloc(&A->status, max_slots);
  if (!ok) {
    (void)hipGetLastError();
    serve_arena_destroy(A);
    return fail(KCORE_E_NOMEM, "server arena allocation failed (" + std::to_string(bytes) + " bytes requested)");
  }
  A->bytes = bytes;
  KC_HIP(hipMemsetAsync(A->stamp, 0, sizeof(int32_t) * nv, st));
  KC_HIP(hipMemsetAsync(A->slot_vb, 0xff, sizeof(int32_t) * max_slots, st));
  hipLaunchKernelGGL(k_serve_reset, dim3(1), dim3(256), 0, st, static_cast<Ctl*>(A->ctl), 2);
  KC_HIP(hipGetLastError());
  KC_HIP(hipStreamSynchronize(st));
  return KCORE_OK;
}

kcore_status serve_join(ServeArena* A, int32_t nslots, int64_t max_n, const int32_t pop[4], int32_t nhi,
                        void* stream) {
  hipStream_t st = (hipStream_t)stream;
  const Args<int64_t> a = serve_args(A);
  const SlotDesc* slots = static_cast<const SlotDesc*>(A->slots);
  if (nslots > 0) {
    const int gx = (int)std::max<int64_t>(1, std::min<int64_t>((max_n + kBlock) / kBlock, 64));
    hipLaunchKernelGGL(k_slot_init<int64_t>, dim3(gx, nslots), dim3(kBlock), 0, st, a, slots, A->tu.t0, A->tu.t1,
                       A->tu.t2);
    hipLaunchKernelGGL(k_slot_shift, dim3(gx, nslots), dim3(kBlock), 0, st, A->row_ptr, slots);
  }
  hipLaunchKernelGGL(k_serve_join, dim3(1), dim3(64), 0, st, static_cast<Ctl*>(A->ctl), pop[0], pop[1], pop[2],
                     pop[3], nhi);
  KC_HIP(hipGetLastError());
  return KCORE_OK;
}

kcore_status serve_decode(ServeArena* A, int64_t vb, int64_t n, hipStream_t st) {
  if (n <= 0) return KCORE_OK;
  const int grid = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, (int64_t)A->num_cus * 4);
  hipLaunchKernelGGL(k_decode, dim3(grid), dim3(kBlock), 0, st, A->est + vb, n);
  KC_HIP(hipGetLastError());
  return KCORE_OK;
}

kcore_status serve_step(ServeArena* A, int32_t rounds, int32_t nslots, int32_t* host_status, void* host_ctl,
                        void* stream) {
  hipStream_t st = (hipStream_t)stream;
  const Args<int64_t> a = serve_args(A);
  const Tuning& tu = A->tu;
  const int cgrid = compact_grid(A->nv, A->num_cus);
  auto enqueue = [&]() {
    for (int i = 0; i < rounds; ++i) {
      hipLaunchKernelGGL((k_compact<false, int64_t>), dim3(cgrid), dim3(kCompactBlock), 0, st, a, i);
      launch_updates<false, true, int64_t>(a, tu, i, 0, st, nullptr);
    }
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, st, a.ctl, rounds);
  };
  if (!tu.use_graph) {
    enqueue();
    KC_HIP(hipGetLastError());
  } else {
    if (A->step_exec && A->step_rounds != rounds) {
      (void)hipGraphExecDestroy(static_cast<hipGraphExec_t>(A->step_exec));
      A->step_exec = nullptr;
    }
    if (!A->step_exec) {
      hipGraph_t graph;
      KC_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      enqueue();
      const hipError_t launch_err = hipGetLastError();
      const hipError_t end_err = hipStreamEndCapture(st, &graph);
      if (launch_err != hipSuccess) return hip_fail(launch_err, "step launch during capture");
      if (end_err != hipSuccess) return hip_fail(end_err, "hipStreamEndCapture");
      hipGraphExec_t exec;
      const hipError_t inst_err = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (inst_err != hipSuccess) return hip_fail(inst_err, "hipGraphInstantiate");
      A->step_exec = exec;
      A->step_rounds = rounds;
    }
    KC_HIP(hipGraphLaunch(static_cast<hipGraphExec_t>(A->step_exec), st));
  }
  if (nslots > 0) {
    hipLaunchKernelGGL(k_slot_status, dim3((nslots + 255) / 256), dim3(256), 0, st, A->gact, A->slot_vb, nslots,
                       A->status);
    KC_HIP(hipGetLastError());
    KC_HIP(hipMemcpyAsync(host_status, A->status, sizeof(int32_t) * nslots, hipMemcpyDeviceToHost, st));
  }
  KC_HIP(hipMemcpyAsync(host_ctl, A->ctl, kCtlHostBytes, hipMemcpyDeviceToHost, st));
  return KCORE_OK;
}

int32_t serve_ctl_rbase(const void* host_ctl) { return static_cast<const Ctl*>(host_ctl)->rbase; }
size_t serve_ctl_size() { return sizeof(Ctl); }

kcore_status serve_rebase(ServeArena* A, int64_t nhi, int32_t d, void* stream) {
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((nhi + kBlock - 1) / kBlock, (int64_t)A->num_cus * 16));
  hipLaunchKernelGGL(k_rebase, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream, A->stamp, A->gact, nhi, d,
                     static_cast<Ctl*>(A->ctl));
  KC_HIP(hipGetLastError());
  return KCORE_OK;
}

}  // namespace kcore

using namespace kcore;

extern "C" {

kcore_status kcore_decompose(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, int32_t* out_core,
                             void* stream) {
  return decompose_impl<int64_t>(n, row_ptr, col_idx, out_core, nullptr, nullptr, (hipStream_t)stream);
}

kcore_status kcore_decompose32(int64_t n, const int32_t* row_ptr, const int32_t* col_idx, int32_t* out_core,
                               void* stream) {
  return decompose_impl<int32_t>(n, row_ptr, col_idx, out_core, nullptr, nullptr, (hipStream_t)stream);
}

kcore_status kcore_decompose_ex(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, int32_t* out_core,
                                const kcore_tuning* tuning, kcore_stats* stats, void* stream) {
  return decompose_impl<int64_t>(n, row_ptr, col_idx, out_core, tuning, stats, (hipStream_t)stream);
}

kcore_status kcore_decompose32_ex(int64_t n, const int32_t* row_ptr, const int32_t* col_idx, int32_t* out_core,
                                  const kcore_tuning* tuning, kcore_stats* stats, void* stream) {
  return decompose_impl<int32_t>(n, row_ptr, col_idx, out_core, tuning, stats, (hipStream_t)stream);
}

kcore_status kcore_decompose_noalloc(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, int32_t* out_core,
                                     void* stream) {
  return decompose_noalloc_impl(n, row_ptr, col_idx, out_core, (hipStream_t)stream);
}

kcore_status kcore_update(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, const int32_t* prev_core,
                          int64_t n_removed, const int32_t* removed, int64_t n_inserted, const int32_t* inserted,
                          int32_t* out_core, const kcore_tuning* tuning, kcore_stats* stats, void* stream) {
  return update_impl<int64_t>(n, row_ptr, col_idx, prev_core, n_removed, removed, n_inserted, inserted, out_core,
                              tuning, stats, (hipStream_t)stream);
}

kcore_status kcore_update32(int64_t n, const int32_t* row_ptr, const int32_t* col_idx, const int32_t* prev_core,
                            int64_t n_removed, const int32_t* removed, int64_t n_inserted, const int32_t* inserted,
                            int32_t* out_core, const kcore_tuning* tuning, kcore_stats* stats, void* stream) {
  return update_impl<int32_t>(n, row_ptr, col_idx, prev_core, n_removed, removed, n_inserted, inserted, out_core,
                              tuning, stats, (hipStream_t)stream);
}

kcore_status kcore_certify(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, const int32_t* core,
                           int32_t* out_code, int64_t* out_vertex, void* stream) {
  return certify_impl<int64_t>(n, row_ptr, col_idx, core, out_code, out_vertex, (hipStream_t)stream);
}

kcore_status kcore_certify32(int64_t n, const int32_t* row_ptr, const int32_t* col_idx, const int32_t* core,
                             int32_t* out_code, int64_t* out_vertex, void* stream) {
  return certify_impl<int32_t>(n, row_ptr, col_idx, core, out_code, out_vertex, (hipStream_t)stream);
}

kcore_status kcore_decompose_rounds(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, int32_t* out_core,
                                    const kcore_tuning* tuning, kcore_round_record* records, int32_t max_records,
                                    int32_t* n_records, void* stream) {
  if (!n_records || max_records < 0 || (max_records > 0 && !records))
    return fail(KCORE_E_INVALID, "bad record buffer arguments");
  *n_records = 0;
  std::vector<kcore_round_record> rec;
  const kcore_status s =
      decompose_impl<int64_t>(n, row_ptr, col_idx, out_core, tuning, nullptr, (hipStream_t)stream, &rec);
  const int32_t k = (int32_t)std::min<size_t>(rec.size(), (size_t)max_records);
  if (k > 0) std::memcpy(records, rec.data(), sizeof(kcore_round_record) * k);
  *n_records = k;
  return s;
}

kcore_status kcore_decompose_batch(int32_t num_graphs, const int64_t* graph_vtx_off, const int64_t* row_ptr,
                                   const int32_t* col_idx, int32_t* out_core, const kcore_tuning* tuning,
                                   kcore_stats* stats, void* stream) {
  return batch_impl(num_graphs, graph_vtx_off, row_ptr, col_idx, out_core, tuning, stats, (hipStream_t)stream);
}

kcore_status kcore_autotune_batch(int32_t num_graphs, const int64_t* graph_vtx_off, const int64_t* row_ptr,
                                  const int32_t* col_idx, int32_t* out_core, int32_t reps, kcore_tuning* best,
                                  float* best_ms, void* stream) {
  return autotune_impl(num_graphs, graph_vtx_off, row_ptr, col_idx, out_core, reps, best, best_ms,
                       (hipStream_t)stream);
}

kcore_status kcore_tuning_cache_set(int32_t num_graphs, int64_t total_vertices, int64_t total_entries,
                                    const kcore_tuning* tuning) {
  if (!tuning || num_graphs <= 0) return fail(KCORE_E_INVALID, "bad tuning cache key or value");
  tune_store(num_graphs, total_vertices, total_entries, *tuning);
  return KCORE_OK;
}

kcore_status kcore_tuning_cache_get(int32_t num_graphs, int64_t total_vertices, int64_t total_entries,
                                    kcore_tuning* tuning) {
  if (!tuning) return fail(KCORE_E_INVALID, "null tuning");
  if (!tune_lookup(num_graphs, total_vertices, total_entries, tuning)) return fail(KCORE_E_AGAIN, "no entry");
  return KCORE_OK;
}

const char* kcore_last_error(void) { return g_last_error.c_str(); }

const char* kcore_version(void) { return "kcore-mi355x 0.2.0 (gfx950)"; }

kcore_status kcore_release_workspace(void) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return fail(KCORE_E_HIP, "no device");
  std::lock_guard<std::mutex> lk(g_ws_mu);
  Workspace* ws = g_ws[dev];
  if (ws) {
    std::lock_guard<std::mutex> lk2(ws->mu);
    (void)hipDeviceSynchronize();
    ws->release();
  }
  return KCORE_OK;
}

}  // extern "C"
