/*
 * kcore.h -- C ABI of libkcore, exact k-core decomposition on MI355X (gfx950).
 *
 * Method (paper: Sec. II-B, Alg. 1 -- the Montresor et al. protocol -- and its
 * shared-memory form FastK, Sec. IV, Alg. 4): every vertex starts with its
 * degree as coreness estimate and repeatedly lowers it to the h-index of its
 * neighbours' estimates, capped by its own value, until no estimate changes.
 * Estimates never increase (Sec. III, selective message sending) and the fixed
 * point reached from the degrees is exactly the coreness of Definition 1
 * (Sec. II): the largest k whose k-core (maximal vertex set inducing minimum
 * degree >= k) contains the vertex; 0 for isolated vertices.
 *
 * Graph input everywhere: an undirected graph as a symmetric CSR.
 *   row_ptr[n+1]  offsets into col_idx, row_ptr[0] == 0, non-decreasing;
 *   col_idx[nnz]  neighbour ids in [0, n), int32; every edge {u,v} appears as
 *                 v in row u AND u in row v; no self-loops; no duplicate entries
 *                 (the paper removes self-loops and treats graphs as undirected,
 *                 Sec. V-A).  Rows sorted ascending are recommended (locality),
 *                 not required.
 * Preconditions are checked only when the environment variable
 * KCORE_VALIDATE=1 is set (then a violation returns KCORE_E_INVALID); otherwise
 * violating them gives unspecified (but memory-safe for in-range ids) results.
 *
 * Output: out_core[n] int32, the coreness of every vertex, bit-exact.
 *
 * Errors: every call returns a kcore_status; no C++ exception crosses the ABI.
 * kcore_last_error() returns a thread-local description of the last failure.
 */
#ifndef KCORE_H_
#define KCORE_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  KCORE_OK = 0,
  KCORE_E_INVALID = -1,   /* bad argument or (with KCORE_VALIDATE=1) bad CSR */
  KCORE_E_NOMEM = -2,     /* device or host allocation failed */
  KCORE_E_HIP = -3,       /* a HIP runtime call failed */
  KCORE_E_TOO_LARGE = -4, /* request larger than the configured memory budget */
  KCORE_E_AGAIN = -5,     /* queue full, retry later */
  KCORE_E_CANCELLED = -6, /* request cancelled (server destroyed) */
  KCORE_E_TIMEOUT = -7    /* wait timed out */
} kcore_status;

/* Tuning knobs of the round kernels.  Zero in a field means "library default".
 * Results never depend on these values; only speed does. */
typedef struct kcore_tuning {
  int32_t thread_max_deg;  /* class 0, one lane per vertex: degree <= this (1..8, default 8) */
  int32_t group_max_deg;   /* class 1, 16 lanes per vertex: degree <= this (<= 64, default 64) */
  int32_t wave_max_deg;    /* class 2, one wavefront per vertex: degree <= this (<= 512, default 512);
                              above: class 3, one workgroup per vertex */
  int32_t tail_threshold;  /* frontier work (lane = 1, group = 4, wavefront = 16, workgroup = 64) at or below
                              which one workgroup finishes the run (<0: never; 0: 512 for single graphs,
                              2048 for the batched form) */
  int32_t grid_blocks;     /* workgroups per small-class round launch (0: 8 per compute unit, raised to one per
                              32768 vertices, at most 32 per compute unit, for very large inputs) */
  int32_t big_grid_blocks; /* workgroups per class-3 round launch (0: 16 per compute unit, 32 for
                              single graphs of at least 2^20 vertices under the two-sided rule) */
  int32_t rounds_per_poll; /* rounds enqueued before the first host check of the frontier */
  int32_t activation;      /* 0: automatic (one-sided when the mean degree is below 4, else two-sided; the
                              served form always uses two-sided), 1: one-sided rule, 2: two-sided rule */
  int32_t timing;          /* 1: bracket every kernel launch with HIP events (fills the ms statistics) */
  int32_t list_cap;        /* frontier list capacity per degree class; beyond it the next round rebuilds
                              its lists from the round stamps (0: chosen per graph: 32768 for single graphs
                              under the one-sided rule, 1024 for single graphs of at least 2^20 vertices under
                              the two-sided rule, otherwise 8192) */
  int32_t no_prune;        /* 1: disable the pruned adjacency (always scan the full neighbour list) */
  int32_t no_graph;        /* 1: launch every round directly instead of replaying captured hipGraphs */
  int32_t max_rounds;      /* > 0: stop after this many rounds (the first round counts as round 1; the
                              single-workgroup tail is off) and leave the estimates reached so far in
                              out_core: an upper bound of the coreness, equal to it once the run has
                              converged.  Instrumentation of the convergence; 0: run to the fixpoint */
  int32_t relabel;         /* single-graph calls: 2 renumbers the vertices by decreasing degree on the device
                              before the decomposition (the estimates of high-degree vertices then share cache
                              lines; the renumbering itself costs about one sweep of random reads, so it pays
                              only on some graphs); 0 or 1: no renumbering.  Results come back in the caller's
                              numbering */
  int32_t deferred;        /* checks of frontier neighbours updated in the same kernel: 1 deferred to the end
                              of the round and decided by their final level and slack, 2 re-activated at once;
                              0: automatic (deferred for single graphs of at least 2^20 vertices under the
                              two-sided rule, otherwise re-activated) */
  int32_t tail_round_cap;  /* rounds one single-workgroup tail launch runs before it hands its frontier back
                              to the round launches, which continue the run (0: 65536).  No run has a round
                              limit: a long chain of drops simply takes several tail launches */
  int32_t tail_order;      /* order inside the tail: 0 (default) round by round, every queued vertex once per
                              round; 1 lowest estimate first (the order of the paper's sequential phase,
                              Sec. IV): each step takes the queued vertices of the lowest estimates, one
                              workgroup pass of work, and keeps the rest queued */
  int32_t tail_big;        /* 1: class-3 vertices (workgroup per vertex) may enter the tail, at 64 units of
                              work each; 0 (default): a frontier with one keeps the run out of the tail */
  int32_t round_renorm;    /* round number above which the per-vertex round stamps are renumbered down
                              between two chunks of rounds (0: 2^30; values below 1024 are raised to 1024).
                              Round numbers therefore never overflow, however many rounds or served steps
                              a call or a server runs; a test hook, results never depend on it */
  int32_t big_wave;        /* later rounds of single graphs and batches: 1 a first class-3 pass takes each vertex
                              on one wavefront when its pruned list has at most 1024 entries, and hands the rest
                              to the workgroup-per-vertex kernel; 0 or 2 (default) every class-3 vertex on a
                              workgroup (measured faster on rmat24, road and ER small) */
  int32_t dense_sweep;     /* rounds that rebuild their lists from the round stamps: 1 (default) later-round
                              activations also mark their piece of 1024 vertices and the rebuild reads only
                              marked pieces; 2 the rebuild reads every stamp */
  int32_t reserved[2];
} kcore_tuning;

/* Round kernels, as indices into kcore_stats.kernel.  The first round (every
 * vertex of degree >= 2) runs its own instances of the class-3 and classes-0..2
 * kernels; later rounds run a compaction kernel (list rebuild from the round
 * stamps; it does nothing unless the previous round's lists overflowed), the
 * class-3 kernel, the classes-0..2 kernel (which also hosts the
 * single-workgroup tail) and, on large single graphs, the deferred checks. */
enum {
  KCORE_K_BIG_FIRST = 0,
  KCORE_K_ROUND_FIRST = 1,
  KCORE_K_BIG = 2,
  KCORE_K_ROUND = 3,
  KCORE_K_COMPACT = 4,
  KCORE_K_DEFER = 5,       /* deferred same-kernel checks at the end of a later round (when enabled) */
  KCORE_K_COUNT = 6
};

/* Work and time of one round kernel over a call.  Edge visits count the
 * adjacency entries scanned by the h-index update. */
typedef struct kcore_kernel_stats {
  int64_t launches;        /* launches of this kernel */
  int64_t vertex_updates;  /* vertices whose h-index it recomputed */
  int64_t edge_visits;     /* adjacency entries read by those recomputations */
  int64_t changes;         /* estimate decreases */
  int64_t activations;     /* vertices it put in a next frontier */
  int64_t prune_writes;    /* entries it wrote to pruned neighbour lists */
  int64_t full_scans;      /* recomputations that read the full neighbour list */
  int64_t max_full_scan;   /* class-3 kernels: the longest full neighbour list one recomputation read */
  double ms;               /* summed launch durations (timing mode only: HIP events on the stream) */
} kcore_kernel_stats;

/* Per-call statistics (optional output). */
typedef struct kcore_stats {
  int64_t rounds;          /* rounds until the frontier emptied (multi-workgroup + tail) */
  int64_t tail_rounds;     /* of which run inside the single-workgroup tail */
  int64_t launches;        /* rounds enqueued (each one launch of every later-round kernel) */
  int64_t dense_rounds;    /* rounds whose lists were rebuilt from the round stamps */
  int64_t vertex_updates;  /* totals over the kernels */
  int64_t edge_visits;
  int64_t changes;
  int64_t activations;
  int64_t prune_writes;
  int64_t full_scans;
  double init_ms;          /* timing mode: estimate initialisation and first-round lists */
  double total_ms;         /* timing mode: init_ms + every kernel's ms */
  kcore_kernel_stats kernel[KCORE_K_COUNT];
} kcore_stats;

/*
 * kcore_decompose -- coreness of one graph with int64 row offsets.
 *   n         number of vertices, 0 <= n <= 2^31-1 (ids are int32); n == 0 is a no-op.
 *   row_ptr   DEVICE pointer, int64[n+1].
 *   col_idx   DEVICE pointer, int32[row_ptr[n]].
 *   out_core  DEVICE pointer, int32[n]; written with the coreness.  Must not
 *             alias row_ptr or col_idx.  Used as the estimate array during the run.
 *   stream    hipStream_t (as void*), NULL for the default stream.
 * All graph buffers are owned by the caller and only read.  The library keeps
 * a per-device workspace (29 bytes per vertex plus 4 bytes per adjacency
 * entry for the pruned neighbour lists, and a small control block; a graph
 * that is renumbered by degree (kcore_tuning.relabel) adds 45 bytes per vertex
 * and 4 per entry for its renumbered copy),
 * allocated on first use, grown on demand and reused by later calls.
 * Work is enqueued on `stream`; the call returns after the fixpoint has been
 * reached (it synchronises `stream` a few times to test for convergence), so
 * out_core is final on return.  Calls from several host threads are
 * serialised per device.
 */
kcore_status kcore_decompose(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, int32_t* out_core,
                             void* stream);

/* Same with int32 row offsets (graphs with fewer than 2^31 adjacency entries). */
kcore_status kcore_decompose32(int64_t n, const int32_t* row_ptr, const int32_t* col_idx, int32_t* out_core,
                               void* stream);

/* kcore_decompose with explicit tuning (NULL = defaults) and optional statistics (NULL = none). */
kcore_status kcore_decompose_ex(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, int32_t* out_core,
                                const kcore_tuning* tuning, kcore_stats* stats, void* stream);

/* The same with int32 row offsets. */
kcore_status kcore_decompose32_ex(int64_t n, const int32_t* row_ptr, const int32_t* col_idx, int32_t* out_core,
                                  const kcore_tuning* tuning, kcore_stats* stats, void* stream);

/*
 * kcore_decompose_noalloc -- kcore_decompose for callers that cannot allocate
 * (code that must not call hipMalloc, tight serving loops, harnesses that
 * forbid allocation).  Same arguments, result and synchronisation as
 * kcore_decompose, with default tuning.  The call allocates nothing: no device
 * or pinned memory, no captured graph, no allocating library routine.  Its
 * whole workspace (round stamps, frontier lists, pruned lists, control block)
 * is one fixed device array of at most KCORE_NOALLOC_SCRATCH_BYTES bytes that
 * the library's code object defines; every device the library runs on holds
 * its own copy until the process ends.  Limits: n <= KCORE_NOALLOC_MAX_VERTICES
 * and row_ptr[n] <= KCORE_NOALLOC_MAX_ENTRIES, else KCORE_E_TOO_LARGE (checked
 * before any kernel runs; reading row_ptr[n] synchronises `stream`).
 * Every call on a device shares that device's array and leaves its contents
 * behind (stamps stay below the next call's round numbers).  Calls on one
 * device are serialised by the library; work that another caller enqueues
 * into the same array by other means would race with it.
 */
#define KCORE_NOALLOC_MAX_VERTICES (1ll << 20)
#define KCORE_NOALLOC_MAX_ENTRIES (1ll << 23)
#define KCORE_NOALLOC_SCRATCH_BYTES (64ll << 20)
kcore_status kcore_decompose_noalloc(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, int32_t* out_core,
                                     void* stream);

/*
 * kcore_update -- coreness after edge changes, from the coreness before them
 * (core maintenance on a changing graph: the paper's future work on dynamic
 * graphs, Sec. VI; the iteration of Sec. II-B restarted from a pointwise upper
 * bound of the new coreness, which the monotone updates lower to exactly the
 * new coreness, as from the degrees).
 *   n, row_ptr, col_idx   DEVICE, the graph AFTER the changes, as for kcore_decompose.
 *   prev_core             DEVICE int32[n]: the coreness of the graph before the changes
 *                         (same vertex ids).  May alias out_core (update in place).
 *   removed               DEVICE int32[2 * n_removed]: pairs {u, v} of the edges present before and
 *                         absent now (each edge once, either orientation).
 *   inserted              DEVICE int32[2 * n_inserted]: the edges absent before and present now.
 *   out_core              DEVICE int32[n]: the coreness of the graph after the changes.
 *   tuning, stats, stream as for kcore_decompose_ex (relabel and max_rounds are ignored).
 * The result is exact when the graph before the changes is the graph after them
 * with `inserted` removed and `removed` added back, and prev_core is its coreness;
 * otherwise it is unspecified (but memory-safe for in-range ids).  Ids must lie
 * in [0, n) (with KCORE_VALIDATE=1 the new CSR is checked, not the lists).
 * Start: removals only lower coreness, so the old coreness bounds the new one
 * and only the endpoints of removed edges are recomputed first.  With D the
 * largest number of inserted edges at one vertex, coreness rises by at most D,
 * and a vertex w that rises is joined to an inserted edge, both of whose
 * endpoints have old coreness >= old(w) + 1 - D, through vertices of old
 * coreness in [old(w) + 1 - D, old(w)] (for D = 1: the subcore of the edge's
 * lower endpoint).  A breadth-first search from the inserted endpoints finds
 * the vertices so joined (while D <= 4; beyond, or past n/16 states, every
 * vertex of old coreness >= the smallest min(old(u), old(v)) over the inserted
 * edges); they start from max(old, min(degree, old + D, K + D)), K the largest
 * min(old(u), old(v)), and are recomputed first if that is above old.  When D >= 2
 * and, with Z the vertices of two or more inserted edges, no other vertex has two
 * edges to Z and inserted edges to vertices outside Z together (as when vertices
 * arrive with their edges), only Z may rise by more than 1: the search then
 * keeps to the old shells of Z's neighbours and of the lower endpoints of the
 * inserted edges outside Z, and the vertices it finds start from old + 1 (Z
 * from old + D).  Work therefore follows the extent of the change rather than
 * the graph.  Synchronises `stream` once or twice before the search, once per
 * four levels of it (levels of at most 1,024 states run inside one workgroup,
 * with one look after them), and as kcore_decompose does.
 */
kcore_status kcore_update(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, const int32_t* prev_core,
                          int64_t n_removed, const int32_t* removed, int64_t n_inserted, const int32_t* inserted,
                          int32_t* out_core, const kcore_tuning* tuning, kcore_stats* stats, void* stream);
/* The same with int32 row offsets (row_ptr[n] < 2^31), as kcore_decompose32. */
kcore_status kcore_update32(int64_t n, const int32_t* row_ptr, const int32_t* col_idx, const int32_t* prev_core,
                            int64_t n_removed, const int32_t* removed, int64_t n_inserted, const int32_t* inserted,
                            int32_t* out_core, const kcore_tuning* tuning, kcore_stats* stats, void* stream);

/*
 * kcore_certify -- check a claimed coreness vector on the device, with no
 * reference result: the local conditions Definition 1 (Sec. II) implies.
 *   n, row_ptr, col_idx   DEVICE, the graph, as for kcore_decompose.
 *   core                  DEVICE int32[n], the vector to check.
 *   out_code              HOST: 0 when every condition holds; else, for the smallest vertex that fails
 *                         one, the first condition it fails (4 only when no vertex fails 1-3):
 *                         1 a core outside [0, degree]; 2 an isolated vertex with a nonzero core, or a
 *                         vertex with neighbours and core 0; 3 a vertex v with fewer than core(v)
 *                         neighbours of core >= core(v) (then {core >= k} does not induce minimum degree
 *                         >= k); 4 k_max (k_max + 1) / 2 larger than the number of edges.
 *   out_vertex            HOST: for codes 1-3 that vertex (-1 otherwise).
 * Passing is necessary, not sufficient: maximality of the cores is not a local
 * property (on K_4, the vector of all 2 passes).  Synchronises `stream`.
 */
kcore_status kcore_certify(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, const int32_t* core,
                           int32_t* out_code, int64_t* out_vertex, void* stream);
/* The same with int32 row offsets (row_ptr[n] < 2^31). */
kcore_status kcore_certify32(int64_t n, const int32_t* row_ptr, const int32_t* col_idx, const int32_t* core,
                             int32_t* out_code, int64_t* out_vertex, void* stream);

/* One round of a run recorded by kcore_decompose_rounds. */
typedef struct kcore_round_record {
  int32_t round;           /* 1 = the first round (every vertex of degree >= 2) */
  int32_t tail_rounds;     /* rounds run inside this launch by the single-workgroup tail (0: none) */
  int64_t vertex_updates;  /* vertices whose h-index was recomputed in this round (with a tail: its rounds) */
  int64_t edge_visits;     /* adjacency entries read by those recomputations */
  int64_t changes;         /* estimate decreases */
  int64_t activations;     /* vertices put in the next frontier */
  int64_t max_full_scan;   /* the longest full neighbour list one class-3 recomputation read in this round */
  double ms;               /* duration of the round's kernels (HIP events on the stream) */
  double big_ms;           /* of which the class-3 kernel */
} kcore_round_record;

/*
 * kcore_decompose_ex launching one round at a time (instrumentation of the
 * convergence, as in the paper's per-iteration figures): each round is
 * bracketed by HIP events and its work counters are read back, one
 * kcore_round_record per round into records[0 .. max_records) (host memory;
 * later rounds are not recorded); *n_records receives the number written.
 * Slower than kcore_decompose; the result is the same.
 */
kcore_status kcore_decompose_rounds(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, int32_t* out_core,
                                    const kcore_tuning* tuning, kcore_round_record* records, int32_t max_records,
                                    int32_t* n_records, void* stream);

/*
 * kcore_decompose_batch -- coreness of many independent graphs in one launch
 * sequence (all graphs advance round by round together; a converged graph
 * simply has no frontier).  This form has no counterpart in the paper: it
 * batches the same computation over many graphs.
 *   num_graphs     G >= 0 (G == 0 is a no-op).
 *   graph_vtx_off  DEVICE int64[G+1]: graph g owns global vertices
 *                  [graph_vtx_off[g], graph_vtx_off[g+1]); graph_vtx_off[0] == 0;
 *                  total N = graph_vtx_off[G] <= 2^31-1.
 *   row_ptr        DEVICE int64[N+1]: GLOBAL offsets into col_idx.
 *   col_idx        DEVICE int32: neighbour ids LOCAL to the graph (0 .. n_g-1).
 *   out_core       DEVICE int32[N]: coreness, by global vertex id.
 *   tuning         NULL: the tuning recorded for batches of this shape by
 *                  kcore_autotune_batch / kcore_tuning_cache_set if any,
 *                  else library defaults.
 *   stats, stream  as for kcore_decompose_ex.
 * Each graph's result equals the result of kcore_decompose on that graph alone.
 * With KCORE_VALIDATE=1 the batch is checked first (ids inside their graph,
 * symmetry, no loops or duplicates).
 */
kcore_status kcore_decompose_batch(int32_t num_graphs, const int64_t* graph_vtx_off, const int64_t* row_ptr,
                                   const int32_t* col_idx, int32_t* out_core, const kcore_tuning* tuning,
                                   kcore_stats* stats, void* stream);

/*
 * kcore_autotune_batch -- time launch-knob candidates (grid sizes, list
 * capacity, tail threshold, class boundaries, poll chunk) on the caller's batch
 * by coordinate descent, `reps` timed runs each (median), and record the best
 * in the process-wide tuning cache under the batch's shape (G and the log2 of N
 * and of the entry count).  Writes the best tuning and its time (ms).  Runs the
 * decomposition many times; out_core holds a correct result on return.
 */
kcore_status kcore_autotune_batch(int32_t num_graphs, const int64_t* graph_vtx_off, const int64_t* row_ptr,
                                  const int32_t* col_idx, int32_t* out_core, int32_t reps, kcore_tuning* best,
                                  float* best_ms, void* stream);

/* Set / get the cached tuning for batches of a shape (used to persist autotuner
 * results across processes).  _get returns KCORE_E_AGAIN when there is no entry. */
kcore_status kcore_tuning_cache_set(int32_t num_graphs, int64_t total_vertices, int64_t total_entries,
                                    const kcore_tuning* tuning);
kcore_status kcore_tuning_cache_get(int32_t num_graphs, int64_t total_vertices, int64_t total_entries,
                                    kcore_tuning* tuning);

/* ------------------------------------------------------------------ serving
 * A server decomposes a stream of independent graphs submitted from host
 * memory.  This form has no counterpart in the paper: it runs the same
 * computation as kcore_decompose_batch over graphs that arrive at different
 * times.  It holds a vertex arena and an adjacency-entry arena in device
 * memory, sized from a byte budget.  A request is admitted when both arenas
 * have room for it (its device footprint is KCORE_SERVE_VERTEX_BYTES * (n+1) +
 * KCORE_SERVE_ENTRY_BYTES * nnz bytes); its CSR is then copied in on a copy
 * stream while the resident graphs keep computing, and at the next step
 * boundary it joins the running rounds (continuous batching: graphs enter and
 * leave between steps of a few rounds, the others are not restarted).  A graph
 * whose frontier is empty leaves its slot: its result is copied to the
 * caller's out_core on another copy stream and its arena space is reused.
 * Each result equals kcore_decompose on that graph alone.
 *
 * Threads: one server thread per server drives the device; submit, poll, wait
 * and stats may be called from any host thread.  No call on a server may be in
 * progress or made once kcore_serve_destroy has been called on it.
 */
#define KCORE_SERVE_VERTEX_BYTES 45
#define KCORE_SERVE_ENTRY_BYTES 8

typedef struct kcore_serve_config {
  int64_t hbm_budget_bytes;   /* device bytes for the arenas (0: min(64 GiB, half of the free memory)) */
  int32_t max_slots;          /* graphs resident at once (0: 1024) */
  int32_t max_queue;          /* submitted, not yet admitted requests before submit returns KCORE_E_AGAIN
                                 (0: 65536) */
  int32_t rounds_per_step;    /* rounds between two step boundaries (0: 8) */
  int32_t entries_per_vertex; /* split of the budget: entry-arena slots per vertex-arena slot (0: 16) */
  int32_t device;             /* HIP device ordinal */
  int32_t reserved[5];
  kcore_tuning tuning;        /* round-kernel knobs, as for kcore_decompose_ex (timing is ignored) */
} kcore_serve_config;

typedef struct kcore_server kcore_server;

typedef struct kcore_completion {
  uint64_t req_id;
  int32_t status;     /* KCORE_OK, KCORE_E_CANCELLED, or KCORE_E_HIP after a device failure */
  int32_t rounds;     /* rounds the graph spent resident (from joining to its last round) */
  double latency_us;  /* submit -> result in out_core */
  double queue_us;    /* submit -> admission into the arenas */
} kcore_completion;

typedef struct kcore_serve_report {
  int64_t submitted;    /* accepted by kcore_serve_submit */
  int64_t completed;    /* results delivered (status OK) */
  int64_t cancelled;
  int64_t rejected;     /* submit calls that returned an error */
  int64_t queued;       /* waiting for admission now */
  int64_t resident;     /* admitted and not yet completed now */
  int64_t steps;        /* step launches */
  int64_t rounds;       /* rounds run */
  int64_t bytes_budget; /* arena bytes held on the device */
  int64_t bytes_peak;   /* peak footprint of admitted requests */
  double p50_us, p99_us, max_us, mean_us;  /* latency over completed requests */
  double graphs_per_s;  /* completed / (last completion - first submit) */
  int64_t rebases;      /* renumberings of the round stamps (kcore_tuning.round_renorm) */
  int64_t reserved[3];
} kcore_serve_report;

/* Create a server (cfg may be NULL: defaults).  Allocates the arenas, four
 * HIP streams of default priority (compute, two for uploads, one for results)
 * and the server thread.  KCORE_E_NOMEM when
 * the budget cannot be allocated. */
kcore_status kcore_serve_create(const kcore_serve_config* cfg, kcore_server** out);

/*
 * Submit one graph.  row_ptr (int64[n+1], row_ptr[0] == 0), col_idx
 * (int32[row_ptr[n]], ids in [0, n)) and out_core (int32[n]) are HOST
 * pointers owned by the caller, kept alive and unmodified until the request's
 * completion has been delivered by kcore_serve_poll or kcore_serve_wait.  Page-locked
 * (pinned) memory lets the copies overlap with compute; pageable memory works
 * but the copies then block the server thread.  The row offsets are read
 * during the call (degree classes).  *out_req_id receives the request id.
 * Errors: KCORE_E_INVALID (bad arguments; with KCORE_VALIDATE=1 also a CSR
 * that breaks the preconditions), KCORE_E_TOO_LARGE (the graph cannot fit in
 * the arenas even when they are empty), KCORE_E_AGAIN (queue full),
 * KCORE_E_HIP (the server failed earlier).  n == 0 completes at once.
 */
kcore_status kcore_serve_submit(kcore_server* server, int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                                int32_t* out_core, uint64_t* out_req_id);

/* Non-blocking: move up to `max` completions (in completion order) into out;
 * *n_out receives how many.  Each completion is delivered once, by poll or by wait. */
kcore_status kcore_serve_poll(kcore_server* server, kcore_completion* out, int32_t max, int32_t* n_out);

/* Block until request req_id completes (timeout_us < 0: no limit) and deliver
 * its completion.  KCORE_E_TIMEOUT if it did not complete in time (it stays
 * pending), KCORE_E_INVALID for an unknown or already delivered id. */
kcore_status kcore_serve_wait(kcore_server* server, uint64_t req_id, int64_t timeout_us, kcore_completion* out);

/* Counters and latency percentiles so far. */
kcore_status kcore_serve_stats(kcore_server* server, kcore_serve_report* out);

/* Stop the server: queued and in-flight requests are cancelled (their
 * out_core contents are unspecified), the device work is drained, every
 * resource is freed. */
kcore_status kcore_serve_destroy(kcore_server* server);

/* ---- measurement ---------------------------------------------------------
 * The bare access pattern of the neighbour scan, the method's hotspot (Sec. III,
 * Optimizations): *out_sum = sum of vals[idx[j]] for 0 <= j < m, in one pass
 * (coalesced reads of idx, one random 4-byte gather of vals per entry).  Timed
 * on a graph's col_idx it gives the device's random-gather rate for that
 * adjacency, the practical ceiling of the round kernels' edge visits.
 *   idx[m]     device, int32, every value in [0, n) (not checked: out-of-range
 *              values read outside vals)
 *   vals[n]    device, int32
 *   out_sum    device, one int64, overwritten
 * Asynchronous on `stream`.  KCORE_E_INVALID for a negative size or a null
 * pointer where one is needed. */
kcore_status kcore_probe_gather(const int32_t* idx, int64_t m, const int32_t* vals, int64_t n, int64_t* out_sum,
                                void* stream);

/* Thread-local message for the last non-OK status returned on this thread. */
const char* kcore_last_error(void);

/* Library version string. */
const char* kcore_version(void);

/* Release the workspace held for the current device (optional; it is also
 * released at process exit). */
kcore_status kcore_release_workspace(void);

#ifdef __cplusplus
}
#endif

#endif /* KCORE_H_ */
