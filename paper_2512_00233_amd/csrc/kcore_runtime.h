// Internal host-side declarations shared by the runtime translation units.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <string>

#include <hip/hip_runtime_api.h>

#include "../../include/kcore.h"

namespace kcore {

// Resolved launch parameters (library defaults overridden by kcore_tuning).
struct Tuning {
  int t0;         // class 0 (one lane): degree <= t0
  int t1;         // class 1 (16-lane group): degree <= t1
  int t2;         // class 2 (wavefront): degree <= t2; above: class 3 (workgroup)
  int tail;       // frontier work that hands the run to one workgroup
  int grid;       // workgroups per small-class round launch
  int grid_auto;  // 1: grid is the default, raised for very large inputs (settle_tuning)
  int big_grid;   // workgroups per class-3 round launch
  int poll;       // rounds in the first chunk between host checks
  int one_sided;  // activation rule: 1 one-sided, 0 two-sided, -1 chosen from the graph (settle_tuning)
  int timing;     // HIP events around every round launch
  int list_cap;   // sparse list capacity per class
  int list_cap_auto;  // 1: list_cap is the default, chosen per graph (settle_tuning)
  int big_grid_auto;  // 1: big_grid is the default, chosen per graph (settle_tuning)
  int tail_auto;      // 1: tail is the default, chosen per graph (settle_tuning)
  int prune;      // pruned adjacency on/off
  int use_graph;  // capture chunks of round launches as hipGraphs
  int max_rounds; // > 0: stop after this many rounds (tail off)
  int relabel;    // 1: renumber by degree first (single-graph calls)
  int defer;      // deferred same-kernel checks: 1 on, 0 off, -1 chosen from the graph (settle_tuning)
  int tail_cap;   // rounds per tail launch before it hands its frontier back
  int tail_order; // 1: lowest estimate first inside the tail
  int tail_big;   // 1: class-3 vertices may enter the tail
  int renorm;     // round number above which stamps are renumbered down
  int big_wave;   // 1: later rounds run the wavefront pass over class 3 before the workgroup kernel
  int dirty;      // 1: later-round activations mark their piece; compaction rounds skip unmarked pieces
};

Tuning resolve_tuning(const kcore_tuning* t, int num_cus);
// Fixes the defaults that depend on the input (small-class grid, activation rule, deferred
// same-kernel checks, list cap, class-3 grid, tail threshold) for a graph (or batch) of n vertices and nnz entries.
void settle_tuning(Tuning* tu, int64_t n, int64_t nnz, bool batch);
kcore_status fail(kcore_status s, const std::string& msg);
kcore_status hip_fail(hipError_t e, const char* what);

// ------------------------------------------------------------------ served graphs
// Device side of a server: a vertex arena and an entry arena holding every
// resident graph, the round kernels' state over them, and the captured step.
struct ServeArena {
  int device = 0;
  int num_cus = 0;
  int64_t nv = 0;       // vertex arena capacity (ids), < 2^31
  int64_t ne = 0;       // entry arena capacity
  int32_t max_slots = 0;
  Tuning tu{};
  size_t bytes = 0;     // device bytes held
  // vertex arena
  int64_t* row_ptr = nullptr;
  int32_t* est = nullptr;
  int32_t* stamp = nullptr;
  uint8_t* cls = nullptr;
  int32_t* lists[2] = {nullptr, nullptr};
  int32_t* plen = nullptr;
  int32_t* plow = nullptr;
  int32_t* vbase = nullptr;
  int32_t* slack = nullptr;
  int32_t* gact = nullptr;
  // entry arena
  int32_t* col = nullptr;
  int32_t* pruned = nullptr;
  // control and slot tables
  void* ctl = nullptr;          // Ctl
  void* slots = nullptr;        // SlotDesc[max_slots] of the slots joining at a boundary
  int32_t* slot_vb = nullptr;   // [max_slots] base vertex per slot index (-1: none)
  int32_t* status = nullptr;    // [max_slots] activity words
  void* step_exec = nullptr;    // hipGraphExec_t of one step
  int32_t step_rounds = 0;
};

// Bytes of device memory per vertex and per adjacency entry of a resident graph.
constexpr int64_t kServeVertexBytes = 8 + 4 + 4 + 1 + 8 + 4 + 4 + 4 + 4 + 4;
constexpr int64_t kServeEntryBytes = 4 + 4;

kcore_status serve_arena_create(ServeArena* A, int device, int64_t nv, int64_t ne, int32_t max_slots,
                                const kcore_tuning* tuning, void* stream);
void serve_arena_destroy(ServeArena* A);
// Slots already copied in (row offsets graph-local) join the next round.
kcore_status serve_join(ServeArena* A, int32_t nslots, int64_t max_n, const int32_t pop[4], int32_t nhi,
                        void* stream);
// One step: `rounds` rounds over every resident graph, then the slots' activity words and the
// control block are copied to the pinned host buffers.
kcore_status serve_step(ServeArena* A, int32_t rounds, int32_t nslots, int32_t* host_status, void* host_ctl,
                        void* stream);
// Strip the class bits from the estimates of a finished graph (vertices vb .. vb+n-1) before they are
// copied out.
kcore_status serve_decode(ServeArena* A, int64_t vb, int64_t n, hipStream_t st);
// Round base of a control block copied to the host.
int32_t serve_ctl_rbase(const void* host_ctl);
size_t serve_ctl_size();
// Renumber the round stamps and activity words of the live vertex range [0, nhi) down by d (a multiple of
// 6), between two steps; the device round base follows.
kcore_status serve_rebase(ServeArena* A, int64_t nhi, int32_t d, void* stream);

}  // namespace kcore
