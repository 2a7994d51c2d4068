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
//  * Frontier membership is a per-vertex round stamp (atomicMax dedup); the
//    next frontier is built as three lists by degree class (lane / wavefront /
//    workgroup), appended with one atomic per wavefront.
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
  int32_t cnt[3][4];      // [slot][class] frontier list sizes (class 3 unused padding)
  int32_t tail_cnt[2][4]; // counters of the single-workgroup tail
  int32_t pop[4];         // vertices per degree class (list region sizes)
  int32_t base[4];        // list region offsets (exclusive prefix of pop)
  unsigned long long stats[8];
  int32_t error;          // 1: the tail hit its round cap
  int32_t pad2[3];
};

// Hard cap on rounds inside one tail invocation (a correct run needs far fewer;
// the cap only guarantees that the kernel terminates).
constexpr int32_t kTailRoundCap = 1 << 22;
enum Stat { ST_UPDATES = 0, ST_VISITS, ST_CHANGES, ST_ACTIVATIONS, ST_ROUNDS, ST_TAIL_ROUNDS };

template <typename Off>
struct Args {
  int64_t n;
  const Off* row_ptr;
  const int32_t* col;
  int32_t* est;
  int32_t* stamp;
  const uint8_t* cls;
  int32_t* lists[2];  // frontier lists by parity of the round
  Ctl* ctl;
  int32_t t1, t2, t3;  // thread / wave / block degree limits
  int32_t tail_threshold;
  int32_t one_sided;
};

}  // namespace kcore
