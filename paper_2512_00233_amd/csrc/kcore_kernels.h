// Device kernels of the iterative coreness computation (gfx950, wave64).
//
// The method (paper: Sec. II-B, Alg. 1; FastK, Sec. IV, Alg. 4): each vertex u
// holds an estimate est[u], initially deg(u); a vertex of the frontier
// recomputes h = max{k <= est[u] : |{v in N(u) : est[v] >= k}| >= k} (the
// h-index of its neighbours' estimates, capped by its own) and lowers est[u]
// to h.  A change activates neighbours for the next round (FastK's activation,
// Sec. IV "Further Optimizations").  The run ends when the frontier is empty.
//
// GPU-specific choices (not from the paper):
//  * Updates are written in place and read by other lanes without
//    synchronisation inside a round.  Every value a lane can read lies between
//    the value at the start of the round and the final one; estimates only
//    decrease and never drop below the coreness, so any mixture of old and new
//    reads still yields a valid upper bound and the same fixed point.
//  * Activation: when u drops from a to b, neighbour v (estimate x read in
//    this round) is activated iff x > b and (x <= a, or v belongs to the
//    current frontier).  The first clause is the paper's two-sided filter;
//    the second covers the neighbours whose own value is still moving in this
//    round, for which x may be stale.  One-sided mode (x > b only) is kept as
//    an option.
//  * Frontier membership is a per-vertex round stamp (atomicMax dedup).  A
//    large frontier is swept densely from the stamps (no shared counters); a
//    small one is kept as three lists by degree class (lane / wavefront /
//    workgroup), appended with one atomic per wavefront and capped: overflow
//    switches the next round to the dense sweep.
//  * Pruned adjacency: after a full scan that yields h, a vertex of degree
//    > 8 keeps the neighbours whose estimate is >= L = 3h/4.  Estimates only
//    decrease, so the pruned-away neighbours stay below L forever, and a
//    search over the pruned list that finds h' >= L is exact; otherwise the
//    vertex rescans its full adjacency and rebuilds the list.
//  * When the frontier is small, one workgroup runs all remaining rounds
//    (the GPU analogue of FastK's switch to sequential processing, Sec. IV).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kcore {

constexpr int kWave = 64;
constexpr int kThreadMaxDeg = 8;    // compile-time register budget of the lane path
constexpr int kWaveRegs = 8;        // values per lane in the wavefront path (<= 512 neighbours)
constexpr int kBlockRegs = 8;       // values per thread in the workgroup path
constexpr int kHugeThresholds = 8;  // thresholds per pass of the multi-pass search

// Control block in device memory.  Counter slot s = round % 3.
struct Ctl {
  int32_t cnt[3][4];       // [slot][class] sparse list sizes (may exceed the cap: then overflow is set)
  int32_t overflow[3][4];  // [slot][0]: 1 when the round of this slot runs as a dense sweep
  int32_t tail_cnt[2][4];  // counters of the single-workgroup tail
  int32_t pop[4];          // vertices per degree class (static list sizes)
  unsigned long long stats[16];
  int32_t error;           // 1: the tail hit its round cap
  int32_t seed_fill[4];    // static-list fill counters of k_seed
  int32_t pad[3];
};
enum Stat {
  ST_UPDATES = 0, ST_VISITS, ST_CHANGES, ST_ACTIVATIONS, ST_PRUNE_WRITES, ST_FULL_SCANS, ST_ROUNDS,
  ST_TAIL_ROUNDS, ST_DENSE_ROUNDS
};
constexpr int kLaneStats = 6;  // stats accumulated per lane (ST_UPDATES .. ST_FULL_SCANS)

// Hard cap on rounds inside one tail invocation (a correct run needs far fewer;
// the cap only guarantees that the kernel terminates).
constexpr int32_t kTailRoundCap = 1 << 22;

template <typename Off>
struct Args {
  int64_t n;
  const Off* row_ptr;
  const int32_t* col;
  int32_t* est;
  int32_t* stamp;
  uint8_t* cls;
  int32_t* lists[2];  // sparse frontier lists by parity of the round (class regions at prefix offsets of pop)
  int32_t* slist;     // static lists: all class-1 vertices, then all class-2 vertices
  int32_t* pruned;    // pruned adjacency, same row offsets as col
  int32_t* plen;      // pruned list length (0: none yet)
  int32_t* plow;      // pruned list threshold L
  Ctl* ctl;
  int32_t t1, t2, t3;  // thread / wave / block degree limits
  int32_t tail_threshold;
  int32_t list_cap;    // sparse list capacity per class before overflow
  int32_t one_sided;
  int32_t prune;       // 0 disables the pruned adjacency
};

}  // namespace kcore
