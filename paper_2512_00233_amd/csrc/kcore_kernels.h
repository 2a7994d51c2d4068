// Device kernels of the iterative coreness computation (gfx950, wave64).
//
// The method (paper: Sec. II-B, Alg. 1; FastK, Sec. IV, Alg. 4): each vertex u
// holds an estimate est[u], initially deg(u); a vertex of the frontier
// recomputes h = max{k <= est[u] : |{v in N(u) : est[v] >= k}| >= k} (the
// h-index of its neighbours' estimates, capped by its own) and lowers est[u]
// to h.  A change activates neighbours for the next round (the activation of
// FastK, Sec. IV).  The run ends when the frontier is empty.
//
// GPU-specific choices (not from the paper):
//  * Updates are written in place and read by other lanes without
//    synchronisation inside a round.  Every value a lane can read lies between
//    the value at the start of the round and the final one; estimates only
//    decrease and never drop below the coreness, so any mixture of old and new
//    reads still yields a valid upper bound and the same fixed point.
//  * Activation: when u drops from a to b, neighbour v (estimate x read in
//    this round) matters only if x > b.  In the first round every such v is
//    activated (one-sided; every vertex is active).  Later, the two-sided
//    filter of the paper (x <= a: u was counted in v's support at v's level)
//    is applied exactly, through v's support slack (support at its level minus
//    the level, kept since v's last recomputation): v is activated only when
//    the slack goes negative.  A neighbour updated in the same kernel of this
//    round may have read u's old value and is re-activated; class 3 and the
//    small classes are separate kernels in a fixed order, so a neighbour of
//    the other group either reads u's new value later or has a final value
//    already (activate_changed); read above u's old level it needs nothing at
//    all.  The neighbour's class comes with its estimate (two low bits of the
//    estimate word during a run).  One-sided mode is kept as an option.
//  * Frontier membership is a per-vertex round stamp (atomicMax dedup).  The
//    frontier is processed as four lists by degree class (lane <= 8,
//    16-lane group <= 64, wavefront <= 512, workgroup above).  Activations
//    append to the next round's lists with one atomic per wavefront, up to a
//    cap; past the cap the next round rebuilds its lists from the stamps in
//    one compaction pass (one atomic per workgroup and class).
//  * The h-index search over values held in registers is k-ary: the first
//    pass tests e, e-1, e-3, ... and the lower bound at once (kKary thresholds;
//    most recomputations stop there), later passes split the remaining interval
//    evenly.  Long adjacency lists use a one-pass LDS histogram instead.
//  * Pruned adjacency: after a full scan that yields h, a vertex of degree
//    > 64 keeps the neighbours whose estimate is >= L = h - h/4.  Estimates only
//    decrease, so the pruned-away neighbours stay below L forever, and a
//    search over the pruned list that finds h' >= L is exact; otherwise the
//    vertex rescans its full adjacency and rebuilds the list.
//  * When the frontier is small, one workgroup runs all remaining rounds
//    (the GPU analogue of FastK's switch to sequential processing, Sec. IV).
//  * Batched graphs: neighbour ids are graph-local; a per-vertex base offset
//    turns them into global ids (pruned lists store global ids).
//  * Served graphs: graphs join a running sequence of rounds between two
//    launches.  Their vertices are stamped with the next round number, and that
//    round rebuilds its lists by compaction, so a new graph's first round is a
//    compaction round over all of its vertices.  Every activation also records
//    the round in a per-graph word, so the host can tell which graphs have no
//    work left and retire them while the others keep running.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace kcore {

constexpr int kWave = 64;
constexpr int kClasses = 4;
constexpr int kLaneMaxDeg = 8;      // class 0: one lane, registers
constexpr int kGroupLanes = 16;     // class 1: 16 lanes x 4 values
constexpr int kGroupRegs = 4;
constexpr int kGroupMaxDeg = kGroupLanes * kGroupRegs;  // 64
constexpr int kWaveRegs = 8;        // class 2: 64 lanes x 8 values
constexpr int kWaveMaxDeg = kWave * kWaveRegs;           // 512
// Search levels of an update run: one wavefront takes a row in slices of kBfsSlice entries; rows longer
// than kBfsLongRow are cut into slices shared out over the whole grid.
constexpr int kBfsSlice = 512;
// Threads of the single-workgroup search kernel, and the largest level it takes (in states and entries).
constexpr int kBfsSmallBlock = 1024;
constexpr int kBfsSmallEntries = 8 * kBfsSmallBlock;
// Widest window (largest number of inserted edges at one vertex) searched by window in an update run.
constexpr int kUpdWindowMax = 4;
// Starting slack of a vertex that no loss of support can move (an update with insertions only).
constexpr int32_t kSlackFinal = 1 << 30;
constexpr int kBfsLongRow = 1024;
constexpr int kBigBlock = 256;      // class 3: one workgroup per vertex
constexpr int kBigRegs = 8;         // values per thread held in registers (2048 per workgroup)
// Later rounds, optional (kcore_tuning.big_wave = 1): a first class-3 pass takes each vertex on one
// wavefront when its pruned list has at most kWave * kBigWaveRegs entries (most pruned lists hold a few
// hundred) and hands the others to the workgroup-per-vertex kernel.  Measured slower on rmat24 (26.3 ms
// against 25.3 ms: the pass and the hand-over cost more than the concurrency gains), so it is off by default.
constexpr int kBigWaveRegs = 16;
// Thresholds per pass of the k-ary search.  Each costs R ballots per pass and
// the number of passes falls like log_k of the interval, so few thresholds are
// cheapest (measured on rmat24: 3 best, 2 and 4 within 0.3%, 8 3% slower, 16 15%).
constexpr int kKary = 3;
constexpr int kHistBins = 4096;     // LDS histogram bins of the one-pass search (16 KB)
constexpr int kStash = 8192;        // LDS copies (16-bit) of the values read by the one-pass search (16 KB)
constexpr int kCompactPerLane = 16; // vertices per lane read at once by the compaction kernel
// Threads of a compaction workgroup: each workgroup reserves its list space with
// one atomic per class, and atomics on one line are served one at a time, so
// fewer, larger workgroups (the same wavefronts in all) wait less.
constexpr int kCompactBlock = 1024;
constexpr int kCompactPiece = 64 * kCompactPerLane;  // vertices a wavefront reads at once (a dirty-mark piece)
constexpr int kCompactPieceShift = 10;
static_assert(kCompactPiece == 1 << kCompactPieceShift, "piece size");
constexpr int kRelabelBuckets = 1024;  // degree buckets of the relabelling (larger degrees share the top one)
constexpr int kRelabelLongDeg = 64;    // rows above this degree are copied by a wavefront when renumbering
// Order of the two update kernels in a round: class 3 first (true) or classes 0..2 first.
constexpr bool kBigFirst = true;
constexpr int kPruneMarginNum = 1;  // pruned lists keep estimates >= h - h * num / den
constexpr int kPruneMarginDen = 4;
// Class-3 lists built in the first round, where estimates fall furthest, keep a
// wider margin (fewer full rescans in the second round).
constexpr int kPruneFirstMarginDen = 3;
constexpr int kDeferRegions = 128;  // regions of the deferred-check buffer (spreads the append counters)
constexpr int kPruneCompactDen = 16;  // a class-3 pruned list is compacted once >= 1/16 of it is below L
// Lists longer than this (hubs) are rebuilt with the wider threshold L = h / 2: a full rescan of a hub by one
// workgroup takes longer than a whole round elsewhere, so hubs trade a longer pruned list for fewer
// rescans (rmat24: 24.9 ms against 25.3 ms with the h - h/4 of other lists)
constexpr int kHubPruneDeg = 16384;
// Class-3 vertices above this degree sit out the first round (their first scan waits for lowered estimates).
constexpr int kHubDelayDeg = 16384;

// During a run the estimate array holds value << 2 | degree class (classes
// 0..3; a vertex of degree <= 1 is stored as class 0, it is never activated),
// so that the gather of a neighbour's estimate also tells which round kernel
// updates it.  Values fit 29 bits: the initial estimate is min(degree, kEstMax),
// still an upper bound of the coreness (a coreness above 2^29 would need more
// than 2^58 adjacency entries).  The last kernel of a run strips the class.
constexpr int kEstShift = 2;
constexpr int32_t kEstMax = (1 << 29) - 1;
__host__ __device__ inline int32_t est_enc(int32_t value, int32_t cls) { return (value << kEstShift) | (cls & 3); }
__host__ __device__ inline int32_t est_val(int32_t raw) { return raw >> kEstShift; }
__host__ __device__ inline int32_t est_cls(int32_t raw) { return raw & 3; }

constexpr int kPopCopies = 32;

// Control block in device memory.  Counter slot s = round % 3.
// List counters: the counter of class k sits at index k * kCtr of its array, one
// 128-byte line per class, since the atomics of all wavefronts on one line are
// served one at a time (about 11 ns each on MI355X, same address or not) and
// appends to different classes then proceed side by side.
constexpr int kCtr = 32;

struct Ctl {
  int32_t cnt[3][kClasses * kCtr];       // sparse list sizes per class (may exceed the cap: then overflow is set)
  int32_t overflow[3][4];                // [slot][0]: 1 when the round of this slot rebuilds its lists by compaction
  int32_t ccnt[2][kClasses * kCtr];      // list sizes produced by the compaction pass, by round parity
  int32_t tail_cnt[2][kClasses * kCtr];  // counters of the single-workgroup tail
  int32_t pop[kClasses];                 // vertices per degree class (list region sizes)
  int32_t seed_fill[kClasses * kCtr];    // first-round (static) list sizes: vertices of degree >= 2 per class
  unsigned long long stats[16];   // run counters (ST_ROUNDS ...)
  // per round kernel (KernelId) and counter (ST_UPDATES .. ST_FULL_SCANS), in kStatCopies
  // copies by workgroup, copy-major: one counter's copies lie 240 bytes apart, on different
  // lines, so that the flushes of a launch do not all meet on one line
  unsigned long long kstats[32][5][6];
  int32_t rbase;                  // round number of slot 0 of the next chunk of round launches
  int32_t tail_pending;           // rounds run by a tail since the last base advance (stamps up to rbase + this)
  int32_t nhi;                    // served graphs: vertex-id bound of the live slots (compaction range)
  // A tail that reached its round cap hands its frontier back to the round
  // launches: the round number of that frontier and its list sizes by class
  // (the lists of that round hold it, uncapped); the chunk's base advance then
  // moves the round base there instead of past the chunk.
  int32_t resume;
  int32_t resume_round;
  int32_t resume_cnt[kClasses];
  // longest full adjacency scan of the class-3 kernel: over the run by kernel, and in the current round
  uint32_t maxscan_run[5];
  uint32_t maxscan_round;
  int32_t resid_cnt;              // class-3 vertices the wavefront pass handed to the workgroup kernel this round
  int32_t dirty_from;             // first round whose compaction may skip pieces without a dirty mark
  // class counts of the initialisation kernels, summed into pop by k_pop_sum: a
  // workgroup adds to copy blockIdx.x % kPopCopies, one 128-byte line each, since
  // the atomics of thousands of workgroups on one line are served one at a time
  int32_t pop_part[kPopCopies][32];
  // deferred same-kernel checks appended in the current round, one counter per
  // buffer region (a workgroup appends to region blockIdx.x % kDeferRegions), at
  // index region * kCtr
  int32_t dcnt[kDeferRegions * kCtr];
};
// What the host reads of the control block (everything before the copies of the class counts and the
// deferred-check counters).
constexpr size_t kCtlHostBytes = offsetof(Ctl, pop_part);
enum Stat {
  ST_UPDATES = 0, ST_VISITS, ST_CHANGES, ST_ACTIVATIONS, ST_PRUNE_WRITES, ST_FULL_SCANS, ST_ROUNDS,
  ST_TAIL_ROUNDS, ST_DENSE_ROUNDS
};
constexpr int kLaneStats = 6;  // stats accumulated per lane (ST_UPDATES .. ST_FULL_SCANS)
constexpr int kStatCopies = 32;
static_assert(sizeof(Ctl::kstats) / sizeof(Ctl::kstats[0]) == kStatCopies, "statistics copies");
// Round kernels whose work is counted separately (the first round's two, the later rounds' two).
// (and the deferred checks, whose activations are counted too)
enum KernelId { KI_BIG_FIRST = 0, KI_ROUND_FIRST, KI_BIG, KI_ROUND, KI_DEFER, KI_COUNT };

// Rounds one tail launch runs before it hands its frontier back to the round
// launches (default of kcore_tuning.tail_round_cap).  A long chain of
// dependent drops (a path of n vertices needs about n/2 rounds) thus never
// keeps one kernel running for long, and no run has a round limit.
constexpr int32_t kTailRoundCap = 1 << 16;
// Round number above which the stamps are renumbered down by a multiple of 6
// (which keeps every round's counter slot, round % 3, and list parity), so that
// round numbers never approach the int32 range (default of
// kcore_tuning.round_renorm).
constexpr int32_t kRoundRenorm = 1 << 30;

template <typename Off>
struct Args {
  int64_t n;
  const Off* row_ptr;
  const int32_t* col;
  const int32_t* vbase;  // batched graphs: global id of the first vertex of each vertex's graph (nullptr: 0)
  int32_t* est;
  int32_t* stamp;
  uint8_t* cls;
  int32_t* lists[2];  // frontier lists by parity of the round (class regions at prefix offsets of pop)
  int32_t* slist;     // first-round lists: vertices of degree >= 2, same class regions
  int32_t* pruned;    // pruned adjacency (global ids), same row offsets as col
  int32_t* plen;      // pruned list length (0: none yet)
  int32_t* plow;      // pruned list threshold L
  Ctl* ctl;
  int32_t tail_threshold;
  int32_t list_cap;    // sparse list capacity per class before overflow
  int32_t one_sided;
  int32_t prune;       // 0 disables the pruned adjacency
  int32_t* slack;      // support at the own level minus the level, from the last recomputation
  int32_t* gact;       // served graphs: per graph (indexed by its base vertex) the last round it has work for
  int32_t served;      // 1: the served arenas (compaction range from the control block)
  // Deferred same-kernel checks: (v, e, h) triples of frontier neighbours that
  // may have read a vertex's old value e before it dropped to h (nullptr: such
  // neighbours are re-activated instead).
  int32_t* defer;
  int32_t defer_cap;   // triples
  int32_t tail_cap;    // rounds per tail launch before the frontier is handed back (kTailRoundCap)
  int32_t tail_order;  // 1: the tail takes its frontier lowest estimate first, a bounded amount of work per step
  int32_t tail_big;    // 1: class-3 vertices may enter the tail (64 work units each)
  int32_t big_wave;    // 1: later rounds run the wavefront pass over class 3 first (needs slist for the hand-over)
  // Dirty pieces (kCompactPiece vertices each), two arrays by the parity of the stamped round: every later-round
  // activation marks its piece, so that a round that rebuilds its lists from the stamps skips unmarked pieces
  // (nullptr: every piece is read)
  uint8_t* dirty;
  int64_t dirty_pieces;  // pieces per parity
};

// A served graph's place in the arenas.
struct SlotDesc {
  int64_t eb;  // first entry of its adjacency in the entry arena
  int32_t vb;  // first vertex id in the vertex arena (its rows are vb .. vb+n-1; row_ptr[vb+n] ends the last row)
  int32_t n;   // vertices
};

}  // namespace kcore
