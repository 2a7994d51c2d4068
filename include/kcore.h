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
  int32_t tail_threshold;  /* frontier work (lane = 1, group = 4, wavefront = 16) at or below which one
                              workgroup finishes the run (<0: never; default 2048) */
  int32_t grid_blocks;     /* workgroups per small-class round launch (0: 8 per compute unit) */
  int32_t big_grid_blocks; /* workgroups per class-3 round launch (0: 4 per compute unit) */
  int32_t rounds_per_poll; /* rounds enqueued before the first host check of the frontier */
  int32_t activation;      /* 0: guarded two-sided rule (default), 1: one-sided rule */
  int32_t timing;          /* 1: bracket every round launch with HIP events (fills the *_ms statistics) */
  int32_t list_cap;        /* frontier list capacity per degree class; beyond it the next round rebuilds
                              its lists from the round stamps (0: library default 8192) */
  int32_t no_prune;        /* 1: disable the pruned adjacency (always scan the full neighbour list) */
  int32_t no_graph;        /* 1: launch every round directly instead of replaying captured hipGraphs */
  int32_t reserved[4];
} kcore_tuning;

/* Per-call statistics (optional output).  Edge visits count the adjacency
 * entries scanned by the h-index update. */
typedef struct kcore_stats {
  int64_t rounds;          /* rounds until the frontier emptied (multi-workgroup + tail) */
  int64_t tail_rounds;     /* of which run inside the single-workgroup tail */
  int64_t launches;        /* round-kernel launches */
  int64_t vertex_updates;  /* vertices whose h-index was recomputed */
  int64_t edge_visits;     /* adjacency entries read by those recomputations */
  int64_t changes;         /* estimate decreases */
  int64_t activations;     /* vertices appended to a next frontier */
  /* first round (every vertex of degree >= 2) alone; filled only when tuning.timing == 1 */
  int64_t dense_vertex_updates;
  int64_t dense_edge_visits;
  int64_t dense_changes;
  int64_t dense_activations;
  double dense_ms;         /* duration of the dense round kernel (timing mode) */
  double sparse_ms;        /* summed durations of all later round kernels (timing mode) */
  int64_t full_scans;      /* recomputations that read the full neighbour list */
  int64_t prune_writes;    /* entries written to pruned neighbour lists */
  int64_t dense_rounds;    /* rounds whose lists were rebuilt from the round stamps */
  int64_t reserved2;
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
 * a per-device workspace (about 21 bytes per vertex plus 4 bytes per adjacency
 * entry for the pruned neighbour lists, and a small control block),
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
