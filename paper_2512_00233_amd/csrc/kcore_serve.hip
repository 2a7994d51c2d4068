// Serving loop of libkcore (continuous batching of independent graphs).
//
// Requests arrive as host CSR buffers.  The server thread admits them into a
// vertex arena and an entry arena by device footprint, copies them in on an
// upload stream while the resident graphs compute on the compute stream, lets
// them join the running rounds at the next step boundary (a step is a
// captured chunk of rounds), and retires every graph whose activity word shows
// no pending round: its estimates are copied to the caller's buffer on a
// download stream, then its arena space is freed.  Host code only: the kernels
// and their launches live in the runtime translation unit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/kcore.h"
#include "kcore_kernels.h"
#include "kcore_runtime.h"

#define KC_HIP_RET(call)                                 \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return kcore::hip_fail(e_, #call); \
  } while (0)

static_assert(kcore::kServeVertexBytes == KCORE_SERVE_VERTEX_BYTES, "vertex footprint out of date");
constexpr int kUploadStreams = 2;
static_assert(kcore::kServeEntryBytes == KCORE_SERVE_ENTRY_BYTES, "entry footprint out of date");

namespace kcore {
namespace {

double now_us() {
  return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over [0, cap).  Zero-length requests get offset 0 and
// hold nothing.
class RangeAlloc {
 public:
  void reset(int64_t cap) {
    cap_ = cap;
    free_.clear();
    if (cap > 0) free_[0] = cap;
  }
  bool alloc(int64_t len, int64_t* off) {
    if (len == 0) {
      *off = 0;
      return true;
    }
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < len) continue;
      *off = it->first;
      const int64_t rest = it->second - len, start = it->first + len;
      free_.erase(it);
      if (rest > 0) free_[start] = rest;
      return true;
    }
    return false;
  }
  void release(int64_t off, int64_t len) {
    if (len == 0) return;
    auto it = free_.emplace(off, len).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  // One past the highest allocated position.
  int64_t high_water() const {
    if (free_.empty()) return cap_;
    auto last = std::prev(free_.end());
    return last->first + last->second == cap_ ? last->first : cap_;
  }

 private:
  int64_t cap_ = 0;
  std::map<int64_t, int64_t> free_;
};

enum class St { Queued, Staging, Resident, Retiring };

struct Request {
  uint64_t id = 0;
  int64_t n = 0, nnz = 0;
  const int64_t* row_ptr = nullptr;
  const int32_t* col = nullptr;
  int32_t* out = nullptr;
  int32_t cls[kClasses] = {0, 0, 0, 0};
  double t_submit = 0, t_admit = 0;
  int64_t vb = 0, eb = 0;
  int32_t slot = -1;
  int32_t r_join = 0, r_last = 0;
  hipEvent_t ev = nullptr;
  St st = St::Queued;
};

// Host-side CSR checks done at submission.  The degree classes are needed for
// the list regions; the full precondition check runs only with KCORE_VALIDATE=1.
kcore_status check_request(int64_t n, const int64_t* row_ptr, const int32_t* col, const Tuning& tu, bool full,
                           int32_t cls[kClasses], int64_t* nnz_out) {
  const int64_t nnz = row_ptr[n];
  if (row_ptr[0] != 0) return fail(KCORE_E_INVALID, "row_ptr[0] must be 0");
  if (nnz < 0) return fail(KCORE_E_INVALID, "row_ptr[n] is negative");
  if (nnz > 0 && !col) return fail(KCORE_E_INVALID, "null col_idx");
  for (int k = 0; k < kClasses; ++k) cls[k] = 0;
  for (int64_t v = 0; v < n; ++v) {
    const int64_t d = row_ptr[v + 1] - row_ptr[v];
    if (d < 0) return fail(KCORE_E_INVALID, "row_ptr is not non-decreasing");
    cls[d <= tu.t0 ? 0 : (d <= tu.t1 ? 1 : (d <= tu.t2 ? 2 : 3))] += 1;
  }
  if (full) {
    for (int64_t v = 0; v < n; ++v) {
      for (int64_t j = row_ptr[v]; j < row_ptr[v + 1]; ++j) {
        const int32_t u = col[j];
        if (u < 0 || u >= n) return fail(KCORE_E_INVALID, "KCORE_VALIDATE: neighbour id out of range");
        if (u == v) return fail(KCORE_E_INVALID, "KCORE_VALIDATE: self-loop");
        if (j > row_ptr[v] && col[j - 1] >= u)
          return fail(KCORE_E_INVALID, "KCORE_VALIDATE: row not strictly increasing");
        const int32_t* b = col + row_ptr[u];
        const int32_t* e = col + row_ptr[u + 1];
        if (!std::binary_search(b, e, (int32_t)v)) return fail(KCORE_E_INVALID, "KCORE_VALIDATE: graph not symmetric");
      }
    }
  }
  *nnz_out = nnz;
  return KCORE_OK;
}

}  // namespace
}  // namespace kcore

using namespace kcore;

struct kcore_server {
  // configuration
  int device = 0;
  int32_t max_slots = 0, max_queue = 0, rounds_per_step = 0;
  int64_t nv = 0, ne = 0;
  ServeArena arena;
  hipStream_t cs = nullptr, down = nullptr;
  hipStream_t up[kUploadStreams] = {};  // uploads alternate between these (several copy engines)
  int next_up = 0;
  hipEvent_t step_ev = nullptr;
  std::vector<hipEvent_t> spare_events;
  // pinned host buffers
  void* host_ctl = nullptr;
  int32_t* host_status = nullptr;
  int32_t* host_slot_vb = nullptr;
  SlotDesc* host_slots = nullptr;
  bool validate = false;

  // shared with client threads (mu)
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> queue;
  std::list<kcore_completion> done;
  std::unordered_map<uint64_t, std::list<kcore_completion>::iterator> done_by_id;
  std::unordered_map<uint64_t, bool> pending;  // submitted, completion not yet delivered
  uint64_t next_id = 1;
  bool stop = false;
  kcore_status fatal = KCORE_OK;
  std::string fatal_msg;
  int64_t n_submitted = 0, n_completed = 0, n_cancelled = 0, n_rejected = 0, n_inflight = 0;
  int64_t n_steps = 0, n_rounds = 0, bytes_used = 0, bytes_peak = 0, n_rebases = 0;
  double t_first_submit = -1, t_last_done = 0;
  std::vector<double> latencies;

  // server thread only
  RangeAlloc vspace, espace;
  std::vector<Request*> staging, resident, retiring;
  std::vector<Request*> slot_of;  // slot index -> resident or retiring request
  std::vector<int32_t> free_slots;
  int64_t pop[kClasses] = {0, 0, 0, 0};  // class populations of every slot holding arena space
  int32_t rbase = 2;
  int64_t head_skips = 0;
  std::thread thread;

  hipEvent_t take_event() {
    if (!spare_events.empty()) {
      hipEvent_t e = spare_events.back();
      spare_events.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
  }

  int64_t footprint(const Request* r) const {
    return KCORE_SERVE_VERTEX_BYTES * (r->n + 1) + KCORE_SERVE_ENTRY_BYTES * r->nnz;
  }

  // Deliver a completion (caller holds mu).
  void complete_locked(Request* r, int32_t status, double t) {
    kcore_completion c;
    std::memset(&c, 0, sizeof(c));
    c.req_id = r->id;
    c.status = status;
    c.rounds = r->r_last > r->r_join ? r->r_last - r->r_join : 0;
    c.latency_us = t - r->t_submit;
    c.queue_us = r->t_admit > 0 ? r->t_admit - r->t_submit : 0;
    done.push_back(c);
    done_by_id[r->id] = std::prev(done.end());
    if (status == KCORE_OK) {
      ++n_completed;
      latencies.push_back(c.latency_us);
      t_last_done = t;
    } else {
      ++n_cancelled;
    }
    --n_inflight;
    if (r->ev) spare_events.push_back(r->ev);
    delete r;
    cv_done.notify_all();
  }

  void release_space(Request* r) {
    vspace.release(r->vb, r->n + 1);
    espace.release(r->eb, r->nnz);
    std::lock_guard<std::mutex> lk(mu);
    bytes_used -= footprint(r);
  }

  kcore_status set_fatal(kcore_status s) {
    std::lock_guard<std::mutex> lk(mu);
    if (fatal == KCORE_OK) {
      fatal = s;
      fatal_msg = kcore_last_error();
    }
    return s;
  }

  // Retired graphs whose result has reached the host: complete them.
  kcore_status finish_retired() {
    for (size_t i = 0; i < retiring.size();) {
      Request* r = retiring[i];
      const hipError_t q = hipEventQuery(r->ev);
      if (q == hipErrorNotReady) {
        ++i;
        continue;
      }
      if (q != hipSuccess) return hip_fail(q, "download event");
      const double t = now_us();
      retiring[i] = retiring.back();
      retiring.pop_back();
      slot_of[r->slot] = nullptr;
      free_slots.push_back(r->slot);
      for (int k = 0; k < kClasses; ++k) pop[k] -= r->cls[k];
      release_space(r);
      std::lock_guard<std::mutex> lk(mu);
      complete_locked(r, KCORE_OK, t);
    }
    return KCORE_OK;
  }

  // Move queued requests into the arenas (first fit, with bounded bypass of a
  // head that does not fit) and start their uploads.
  kcore_status admit() {
    std::vector<Request*> taken;
    {
      std::lock_guard<std::mutex> lk(mu);
      const int64_t room = (int64_t)max_slots - (int64_t)(staging.size() + resident.size() + retiring.size());
      size_t i = 0;
      while (i < queue.size() && (int64_t)taken.size() < room && i < 64) {
        Request* r = queue[i];
        const bool head = i == 0;
        if (!head && head_skips > 256) break;  // let the head through before anyone else
        int64_t vb = 0, eb = 0;
        if (vspace.alloc(r->n + 1, &vb)) {
          if (espace.alloc(r->nnz, &eb)) {
            r->vb = vb;
            r->eb = eb;
            queue.erase(queue.begin() + i);
            taken.push_back(r);
            bytes_used += footprint(r);
            bytes_peak = std::max(bytes_peak, bytes_used);
            head_skips = head ? 0 : head_skips + 1;
            continue;
          }
          vspace.release(vb, r->n + 1);
        }
        ++i;
      }
    }
    const double t = now_us();
    for (Request* r : taken) {
      hipStream_t us = up[next_up];
      next_up = (next_up + 1) % kUploadStreams;
      r->t_admit = t;
      r->st = St::Staging;
      r->ev = take_event();
      if (!r->ev) return fail(KCORE_E_HIP, "hipEventCreate failed");
      KC_HIP_RET(hipMemcpyAsync(arena.row_ptr + r->vb, r->row_ptr, sizeof(int64_t) * (r->n + 1),
                                hipMemcpyHostToDevice, us));
      if (r->nnz > 0)
        KC_HIP_RET(hipMemcpyAsync(arena.col + r->eb, r->col, sizeof(int32_t) * r->nnz, hipMemcpyHostToDevice, us));
      KC_HIP_RET(hipEventRecord(r->ev, us));
      staging.push_back(r);
    }
    return KCORE_OK;
  }

  // Staged graphs whose upload has finished join at the current round base.
  kcore_status join() {
    std::vector<Request*> ready;
    for (size_t i = 0; i < staging.size();) {
      const hipError_t q = hipEventQuery(staging[i]->ev);
      if (q == hipErrorNotReady) {
        ++i;
        continue;
      }
      if (q != hipSuccess) return hip_fail(q, "upload event");
      ready.push_back(staging[i]);
      staging[i] = staging.back();
      staging.pop_back();
    }
    if (ready.empty()) return KCORE_OK;
    int64_t max_n = 0;
    for (size_t j = 0; j < ready.size(); ++j) {
      Request* r = ready[j];
      r->slot = free_slots.back();
      free_slots.pop_back();
      slot_of[r->slot] = r;
      r->st = St::Resident;
      r->r_join = rbase;
      for (int k = 0; k < kClasses; ++k) pop[k] += r->cls[k];
      host_slots[j] = SlotDesc{r->eb, (int32_t)r->vb, (int32_t)r->n};
      max_n = std::max(max_n, r->n);
      resident.push_back(r);
    }
    for (int32_t s = 0; s < max_slots; ++s) host_slot_vb[s] = slot_of[s] ? (int32_t)slot_of[s]->vb : -1;
    KC_HIP_RET(hipMemcpyAsync(arena.slots, host_slots, sizeof(SlotDesc) * ready.size(), hipMemcpyHostToDevice, cs));
    KC_HIP_RET(hipMemcpyAsync(arena.slot_vb, host_slot_vb, sizeof(int32_t) * max_slots, hipMemcpyHostToDevice, cs));
    const int32_t p[kClasses] = {(int32_t)pop[0], (int32_t)pop[1], (int32_t)pop[2], (int32_t)pop[3]};
    return serve_join(&arena, (int32_t)ready.size(), max_n, p, (int32_t)vspace.high_water(), cs);
  }

  // Highest slot index in use + 1.
  int32_t slot_count() const {
    int32_t hi = 0;
    for (int32_t s = 0; s < max_slots; ++s)
      if (slot_of[s]) hi = s + 1;
    return hi;
  }

  // One step over the resident graphs; meanwhile keep retiring and admitting.
  kcore_status step() {
    const int32_t ns = slot_count();
    kcore_status s = serve_step(&arena, rounds_per_step, ns, host_status, host_ctl, cs);
    if (s != KCORE_OK) return s;
    KC_HIP_RET(hipEventRecord(step_ev, cs));
    for (;;) {
      const hipError_t q = hipEventQuery(step_ev);
      if (q == hipSuccess) break;
      if (q != hipErrorNotReady) return hip_fail(q, "step event");
      if ((s = finish_retired()) != KCORE_OK) return s;
      if ((s = admit()) != KCORE_OK) return s;
      std::this_thread::yield();
    }
    const int32_t r_new = serve_ctl_rbase(host_ctl);
    {
      std::lock_guard<std::mutex> lk(mu);
      ++n_steps;
      n_rounds += r_new - rbase;
    }
    rbase = r_new;
    for (size_t i = 0; i < resident.size();) {
      Request* r = resident[i];
      const int32_t act = host_status[r->slot];
      if (act >= rbase) {
        ++i;
        continue;
      }
      // no pending round: the estimates are final; copy them out behind this step
      r->r_last = act;
      r->st = St::Retiring;
      KC_HIP_RET(hipStreamWaitEvent(down, step_ev, 0));
      if ((s = serve_decode(&arena, r->vb, r->n, down)) != KCORE_OK) return s;
      if (r->n > 0)
        KC_HIP_RET(hipMemcpyAsync(r->out, arena.est + r->vb, sizeof(int32_t) * r->n, hipMemcpyDeviceToHost, down));
      KC_HIP_RET(hipEventRecord(r->ev, down));
      retiring.push_back(r);
      resident[i] = resident.back();
      resident.pop_back();
    }
    if (rbase > arena.tu.renorm) {
      // round numbers stay far from the int32 range: renumber the live stamps and activity words
      // (a multiple of 6 keeps every round's counter slot and list parity) before the next step or join
      const int32_t d = (rbase - 64) / 6 * 6;
      if ((s = serve_rebase(&arena, vspace.high_water(), d, cs)) != KCORE_OK) return s;
      rbase -= d;
      for (Request* r : resident) r->r_join -= d;
      std::lock_guard<std::mutex> lk(mu);
      ++n_rebases;
    }
    return KCORE_OK;
  }

  kcore_status loop_once(bool* idle) {
    kcore_status s;
    if ((s = finish_retired()) != KCORE_OK) return s;
    if ((s = admit()) != KCORE_OK) return s;
    if ((s = join()) != KCORE_OK) return s;
    *idle = false;
    if (!resident.empty()) return step();
    *idle = staging.empty() && retiring.empty();
    return KCORE_OK;
  }

  void run() {
    (void)hipSetDevice(device);
    for (;;) {
      {
        std::unique_lock<std::mutex> lk(mu);
        if (stop) break;
      }
      bool idle = false;
      const kcore_status s = loop_once(&idle);
      if (s != KCORE_OK) {
        set_fatal(s);
        break;
      }
      if (idle) {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait_for(lk, std::chrono::milliseconds(50), [&] { return stop || !queue.empty(); });
      } else if (resident.empty()) {
        std::this_thread::yield();  // uploads or downloads in flight
      }
    }
    // drain the device, then cancel whatever is left
    (void)hipStreamSynchronize(cs);
    for (hipStream_t st : up) (void)hipStreamSynchronize(st);
    (void)hipStreamSynchronize(down);
    std::lock_guard<std::mutex> lk(mu);
    const int32_t status = fatal == KCORE_OK ? KCORE_E_CANCELLED : fatal;
    const double t = now_us();
    for (auto* list : {&staging, &resident, &retiring}) {
      for (Request* r : *list) complete_locked(r, status, t);
      list->clear();
    }
    for (Request* r : queue) complete_locked(r, status, t);
    queue.clear();
    stop = true;
  }
};

namespace {

kcore_status create_impl(const kcore_serve_config* cfg_in, kcore_server** out) {
  if (!out) return fail(KCORE_E_INVALID, "null output pointer");
  *out = nullptr;
  kcore_serve_config cfg;
  std::memset(&cfg, 0, sizeof(cfg));
  if (cfg_in) cfg = *cfg_in;
  int ndev = 0;
  KC_HIP_RET(hipGetDeviceCount(&ndev));
  if (cfg.device < 0 || cfg.device >= ndev) return fail(KCORE_E_INVALID, "device ordinal out of range");
  if (cfg.max_slots < 0 || cfg.max_queue < 0 || cfg.rounds_per_step < 0 || cfg.entries_per_vertex < 0 ||
      cfg.hbm_budget_bytes < 0)
    return fail(KCORE_E_INVALID, "negative configuration value");
  int prev = 0;
  KC_HIP_RET(hipGetDevice(&prev));
  KC_HIP_RET(hipSetDevice(cfg.device));
  auto* S = new kcore_server();
  auto cleanup = [&](kcore_status s) {
    serve_arena_destroy(&S->arena);
    for (hipStream_t st : {S->cs, S->down})
      if (st) (void)hipStreamDestroy(st);
    for (hipStream_t st : S->up)
      if (st) (void)hipStreamDestroy(st);
    if (S->step_ev) (void)hipEventDestroy(S->step_ev);
    for (void* p : {S->host_ctl, (void*)S->host_status, (void*)S->host_slot_vb, (void*)S->host_slots})
      if (p) (void)hipHostFree(p);
    delete S;
    (void)hipSetDevice(prev);
    return s;
  };
  S->device = cfg.device;
  S->max_slots = cfg.max_slots > 0 ? std::min(cfg.max_slots, 1 << 16) : 1024;
  S->max_queue = cfg.max_queue > 0 ? cfg.max_queue : 65536;
  S->rounds_per_step = cfg.rounds_per_step > 0 ? std::min(cfg.rounds_per_step, 256) : 8;
  const int64_t epv = cfg.entries_per_vertex > 0 ? cfg.entries_per_vertex : 16;
  int64_t budget = cfg.hbm_budget_bytes;
  if (budget == 0) {
    size_t fr = 0, tot = 0;
    KC_HIP_RET(hipMemGetInfo(&fr, &tot));
    budget = std::min<int64_t>((int64_t)64 << 30, (int64_t)(fr / 2));
  }
  int64_t nv = budget / (KCORE_SERVE_VERTEX_BYTES + KCORE_SERVE_ENTRY_BYTES * epv);
  nv = std::min<int64_t>(nv, (int64_t)INT32_MAX - 1);
  if (nv < 64) return cleanup(fail(KCORE_E_INVALID, "hbm_budget_bytes too small"));
  S->nv = nv;
  S->ne = nv * epv;
  kcore_status s = serve_arena_create(&S->arena, cfg.device, S->nv, S->ne, S->max_slots, &cfg.tuning, nullptr);
  if (s != KCORE_OK) return cleanup(s);
  bool streams_ok = true;
  for (hipStream_t& st : S->up) streams_ok = streams_ok && hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
  if (!streams_ok || hipStreamCreateWithFlags(&S->cs, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&S->down, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&S->step_ev, hipEventDisableTiming) != hipSuccess ||
      hipHostMalloc(&S->host_ctl, serve_ctl_size(), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&S->host_status, sizeof(int32_t) * S->max_slots, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&S->host_slot_vb, sizeof(int32_t) * S->max_slots, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&S->host_slots, sizeof(SlotDesc) * S->max_slots, hipHostMallocDefault) != hipSuccess)
    return cleanup(fail(KCORE_E_HIP, "server stream, event or pinned buffer creation failed"));
  S->vspace.reset(S->nv);
  S->espace.reset(S->ne);
  S->slot_of.assign(S->max_slots, nullptr);
  for (int32_t i = S->max_slots - 1; i >= 0; --i) S->free_slots.push_back(i);
  S->validate = [] {
    const char* e = std::getenv("KCORE_VALIDATE");
    return e && e[0] == '1';
  }();
  S->thread = std::thread([S] { S->run(); });
  (void)hipSetDevice(prev);
  *out = S;
  return KCORE_OK;
}

}  // namespace

extern "C" {

kcore_status kcore_serve_create(const kcore_serve_config* cfg, kcore_server** out) { return create_impl(cfg, out); }

kcore_status kcore_serve_submit(kcore_server* S, int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                                int32_t* out_core, uint64_t* out_req_id) {
  if (!S || !out_req_id) return fail(KCORE_E_INVALID, "null server or request-id pointer");
  auto reject = [&](kcore_status s) {
    std::lock_guard<std::mutex> lk(S->mu);
    ++S->n_rejected;
    return s;
  };
  if (n < 0 || n >= INT32_MAX) return reject(fail(KCORE_E_INVALID, "n must be in [0, 2^31-2]"));
  if (n > 0 && (!row_ptr || !out_core)) return reject(fail(KCORE_E_INVALID, "null pointer argument"));
  auto* r = new Request();
  r->n = n;
  r->row_ptr = row_ptr;
  r->col = col_idx;
  r->out = out_core;
  if (n > 0) {
    const kcore_status s = check_request(n, row_ptr, col_idx, S->arena.tu, S->validate, r->cls, &r->nnz);
    if (s != KCORE_OK) {
      delete r;
      return reject(s);
    }
    if (n + 1 > S->nv || r->nnz > S->ne) {
      delete r;
      return reject(fail(KCORE_E_TOO_LARGE, "graph larger than the server's arenas (" + std::to_string(n) +
                                                " vertices, " + std::to_string(r->nnz) + " entries)"));
    }
  }
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->fatal != KCORE_OK) {
    delete r;
    ++S->n_rejected;
    return fail(S->fatal, "server failed: " + S->fatal_msg);
  }
  if (S->stop) {
    delete r;
    ++S->n_rejected;
    return fail(KCORE_E_CANCELLED, "server is stopping");
  }
  if ((int64_t)S->queue.size() >= S->max_queue) {
    delete r;
    ++S->n_rejected;
    return fail(KCORE_E_AGAIN, "queue full");
  }
  r->id = S->next_id++;
  r->t_submit = now_us();
  if (S->t_first_submit < 0) S->t_first_submit = r->t_submit;
  ++S->n_submitted;
  ++S->n_inflight;
  S->pending[r->id] = true;
  *out_req_id = r->id;
  if (n == 0) {
    S->complete_locked(r, KCORE_OK, now_us());
    return KCORE_OK;
  }
  S->queue.push_back(r);
  S->cv_work.notify_one();
  return KCORE_OK;
}

kcore_status kcore_serve_poll(kcore_server* S, kcore_completion* out, int32_t max, int32_t* n_out) {
  if (!S || !n_out || max < 0 || (max > 0 && !out)) return fail(KCORE_E_INVALID, "bad poll arguments");
  std::lock_guard<std::mutex> lk(S->mu);
  int32_t k = 0;
  while (k < max && !S->done.empty()) {
    out[k] = S->done.front();
    S->done_by_id.erase(out[k].req_id);
    S->pending.erase(out[k].req_id);
    S->done.pop_front();
    ++k;
  }
  *n_out = k;
  return KCORE_OK;
}

kcore_status kcore_serve_wait(kcore_server* S, uint64_t req_id, int64_t timeout_us, kcore_completion* out) {
  if (!S || !out) return fail(KCORE_E_INVALID, "bad wait arguments");
  std::unique_lock<std::mutex> lk(S->mu);
  if (!S->pending.count(req_id)) return fail(KCORE_E_INVALID, "unknown or already delivered request id");
  auto ready = [&] { return S->done_by_id.count(req_id) > 0; };
  if (timeout_us < 0) {
    S->cv_done.wait(lk, ready);
  } else if (!S->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
    return fail(KCORE_E_TIMEOUT, "request not complete");
  }
  auto it = S->done_by_id[req_id];
  *out = *it;
  S->done.erase(it);
  S->done_by_id.erase(req_id);
  S->pending.erase(req_id);
  return KCORE_OK;
}

kcore_status kcore_serve_stats(kcore_server* S, kcore_serve_report* out) {
  if (!S || !out) return fail(KCORE_E_INVALID, "bad stats arguments");
  std::lock_guard<std::mutex> lk(S->mu);
  std::memset(out, 0, sizeof(*out));
  out->submitted = S->n_submitted;
  out->completed = S->n_completed;
  out->cancelled = S->n_cancelled;
  out->rejected = S->n_rejected;
  out->queued = (int64_t)S->queue.size();
  out->resident = S->n_inflight - out->queued;
  out->steps = S->n_steps;
  out->rounds = S->n_rounds;
  out->rebases = S->n_rebases;
  out->bytes_budget = (int64_t)S->arena.bytes;
  out->bytes_peak = S->bytes_peak;
  if (!S->latencies.empty()) {
    std::vector<double> v = S->latencies;
    std::sort(v.begin(), v.end());
    auto pct = [&](double p) {
      const size_t i = (size_t)std::min<double>((double)v.size() - 1, std::ceil(p * (double)v.size()) - 1);
      return v[i];
    };
    out->p50_us = pct(0.50);
    out->p99_us = pct(0.99);
    out->max_us = v.back();
    double sum = 0;
    for (double x : v) sum += x;
    out->mean_us = sum / (double)v.size();
    const double span = S->t_last_done - S->t_first_submit;
    out->graphs_per_s = span > 0 ? (double)S->n_completed / (span * 1e-6) : 0;
  }
  return KCORE_OK;
}

kcore_status kcore_serve_destroy(kcore_server* S) {
  if (!S) return fail(KCORE_E_INVALID, "null server");
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    S->cv_work.notify_all();
  }
  if (S->thread.joinable()) S->thread.join();
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(S->device);
  serve_arena_destroy(&S->arena);
  for (hipStream_t st : {S->cs, S->down}) (void)hipStreamDestroy(st);
  for (hipStream_t st : S->up) (void)hipStreamDestroy(st);
  (void)hipEventDestroy(S->step_ev);
  for (hipEvent_t e : S->spare_events) (void)hipEventDestroy(e);
  for (void* p : {S->host_ctl, (void*)S->host_status, (void*)S->host_slot_vb, (void*)S->host_slots})
    (void)hipHostFree(p);
  (void)hipSetDevice(prev);
  delete S;
  return KCORE_OK;
}

}  // extern "C"
