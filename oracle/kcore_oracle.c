/*
 * CPU oracle for k-core decomposition -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * call this code.  It shares nothing with the GPU library: no headers, helpers,
 * tables or pre/post-processing.  Plain, sequential, integer-only C.
 *
 * What is computed (paper, Sec. II, Definition 1 and the paragraph after it):
 * for a positive integer k the k-core of an undirected graph is the
 * inclusion-maximal vertex set whose induced subgraph has minimum degree >= k;
 * the coreness of v is the largest k whose k-core contains v (0 when v lies in
 * no 1-core, i.e. v is isolated).  The method under test (Sec. II-B, Alg. 1,
 * and FastK, Sec. IV) converges to exactly this value, so the oracle is the
 * definition itself, with no approximation.
 *
 * Three routines:
 *   oracle_core_levels  the definition written out: for k = 1, 2, ... delete,
 *                       until none is left, every remaining vertex with fewer
 *                       than k remaining neighbours; what survives is the
 *                       k-core (nested in the (k-1)-core, so each level starts
 *                       from the survivors of the previous one); a vertex
 *                       deleted at level k has coreness k-1.
 *   oracle_core_bz      Batagelj-Zaversnik bucket peeling (the linear-time
 *                       sequential algorithm the paper cites in Sec. II and its
 *                       Related Work): an independent second implementation.
 *   oracle_check        the local certificate: 0 <= core <= deg, isolated <=> 0,
 *                       every v has >= core(v) neighbours u with
 *                       core(u) >= core(v), and kmax(kmax+1)/2 <= m.
 *
 * Input: CSR with int64 row offsets [n+1] and int32 neighbour ids, undirected
 * (both directions present), no self-loops, no duplicate entries.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- levels */
/* Returns 0 on success, -1 on allocation failure. */
int oracle_core_levels(int64_t n, const int64_t* row_ptr, const int32_t* col, int32_t* core) {
  if (n <= 0) return 0;
  int64_t* deg = (int64_t*)malloc(sizeof(int64_t) * n);     /* remaining-neighbour count */
  char* alive = (char*)malloc(n);
  char* queued = (char*)malloc(n);
  int32_t* remaining = (int32_t*)malloc(sizeof(int32_t) * n); /* vertices not yet deleted */
  int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * n);
  if (!deg || !alive || !queued || !remaining || !queue) {
    free(deg); free(alive); free(queued); free(remaining); free(queue);
    return -1;
  }
  int64_t nrem = n;
  for (int64_t v = 0; v < n; ++v) {
    deg[v] = row_ptr[v + 1] - row_ptr[v];
    alive[v] = 1;
    queued[v] = 0;
    remaining[v] = (int32_t)v;
  }
  for (int64_t k = 1; nrem > 0; ++k) {
    /* seed the deletion queue with every remaining vertex of degree < k */
    int64_t qh = 0, qt = 0;
    for (int64_t i = 0; i < nrem; ++i) {
      int32_t v = remaining[i];
      if (deg[v] < k) { queue[qt++] = v; queued[v] = 1; }
    }
    /* delete until every remaining vertex has >= k remaining neighbours */
    while (qh < qt) {
      int32_t v = queue[qh++];
      alive[v] = 0;
      core[v] = (int32_t)(k - 1);
      for (int64_t j = row_ptr[v]; j < row_ptr[v + 1]; ++j) {
        int32_t u = col[j];
        if (!alive[u]) continue;
        deg[u] -= 1;
        if (deg[u] < k && !queued[u]) { queue[qt++] = u; queued[u] = 1; }
      }
    }
    /* the survivors are the k-core */
    int64_t w = 0;
    for (int64_t i = 0; i < nrem; ++i)
      if (alive[remaining[i]]) remaining[w++] = remaining[i];
    nrem = w;
  }
  free(deg); free(alive); free(queued); free(remaining); free(queue);
  return 0;
}

/* ---------------------------------------------------------------- BZ */
/* Batagelj & Zaversnik, "An O(m) Algorithm for Cores Decomposition of
 * Networks" (2003).  Vertices are kept in an array ordered by current degree,
 * with the start of each degree block recorded; processing vertices in that
 * order, each neighbour of higher current degree is moved to the front of its
 * block, the block boundary is advanced past it and its degree drops by one.
 * When a vertex is reached its current degree is its coreness. */
int oracle_core_bz(int64_t n, const int64_t* row_ptr, const int32_t* col, int32_t* core) {
  if (n <= 0) return 0;
  int32_t maxd = 0;
  int32_t* d = core; /* current degree, becomes the coreness in place */
  for (int64_t v = 0; v < n; ++v) {
    d[v] = (int32_t)(row_ptr[v + 1] - row_ptr[v]);
    if (d[v] > maxd) maxd = d[v];
  }
  int64_t* start = (int64_t*)calloc((size_t)maxd + 2, sizeof(int64_t)); /* first index of each degree block */
  int32_t* order = (int32_t*)malloc(sizeof(int32_t) * n);             /* vertices by current degree */
  int64_t* where = (int64_t*)malloc(sizeof(int64_t) * n);             /* index of v in order */
  if (!start || !order || !where) {
    free(start); free(order); free(where);
    return -1;
  }
  /* counting sort by degree */
  for (int64_t v = 0; v < n; ++v) start[d[v] + 1] += 1;
  for (int32_t k = 0; k <= maxd; ++k) start[k + 1] += start[k];
  {
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * ((size_t)maxd + 1));
    if (!fill) { free(start); free(order); free(where); return -1; }
    memcpy(fill, start, sizeof(int64_t) * ((size_t)maxd + 1));
    for (int64_t v = 0; v < n; ++v) {
      where[v] = fill[d[v]]++;
      order[where[v]] = (int32_t)v;
    }
    free(fill);
  }
  for (int64_t i = 0; i < n; ++i) {
    int32_t v = order[i];
    for (int64_t j = row_ptr[v]; j < row_ptr[v + 1]; ++j) {
      int32_t u = col[j];
      if (d[u] > d[v]) {
        int32_t du = d[u];
        int64_t pu = where[u];
        int64_t pw = start[du]; /* first slot of u's degree block */
        int32_t w = order[pw];
        if (u != w) { /* swap u to the front of its block */
          order[pu] = w; where[w] = pu;
          order[pw] = u; where[u] = pw;
        }
        start[du] += 1; /* u now belongs to the block of degree du-1 */
        d[u] = du - 1;
      }
    }
  }
  free(start); free(order); free(where);
  return 0;
}

/* ---------------------------------------------------------------- certificate */
/* Returns 0 when the local certificate holds, otherwise a positive code:
 * 1 core < 0 or core > deg, 2 isolated vertex with core != 0 or
 * non-isolated vertex with core == 0, 3 local support violated,
 * 4 kmax(kmax+1)/2 > m.  *bad receives the first offending vertex (or -1). */
int oracle_check(int64_t n, const int64_t* row_ptr, const int32_t* col, const int32_t* core, int64_t* bad) {
  *bad = -1;
  int64_t kmax = 0;
  for (int64_t v = 0; v < n; ++v) {
    int64_t dv = row_ptr[v + 1] - row_ptr[v];
    int64_t c = core[v];
    if (c < 0 || c > dv) { *bad = v; return 1; }
    if ((dv == 0) != (c == 0)) { *bad = v; return 2; }
    int64_t support = 0;
    for (int64_t j = row_ptr[v]; j < row_ptr[v + 1]; ++j)
      if (core[col[j]] >= c) support += 1;
    if (support < c) { *bad = v; return 3; }
    if (c > kmax) kmax = c;
  }
  int64_t m = row_ptr[n] / 2;
  if (kmax * (kmax + 1) / 2 > m) return 4;
  return 0;
}

/* ---------------------------------------------------------------- batched */
/* Concatenated graphs: graph g owns vertices [vo[g], vo[g+1]); row_ptr holds
 * global edge offsets and col holds graph-local ids.  Each graph is decomposed
 * independently with oracle_core_levels (method 0) or oracle_core_bz
 * (method 1); graphs are shared among `threads` POSIX threads. */
struct batch_job {
  int32_t G;
  const int64_t* vo;
  const int64_t* row_ptr;
  const int32_t* col;
  int32_t* core;
  int method;
  int64_t next; /* guarded by mu */
  pthread_mutex_t mu;
  int err;
};

static void* batch_worker(void* arg) {
  struct batch_job* jb = (struct batch_job*)arg;
  for (;;) {
    pthread_mutex_lock(&jb->mu);
    int64_t g = jb->next++;
    pthread_mutex_unlock(&jb->mu);
    if (g >= jb->G) break;
    int64_t v0 = jb->vo[g], n = jb->vo[g + 1] - v0;
    int64_t e0 = jb->row_ptr[v0];
    int64_t* rp = (int64_t*)malloc(sizeof(int64_t) * (n + 1));
    if (!rp) { jb->err = -1; continue; }
    for (int64_t v = 0; v <= n; ++v) rp[v] = jb->row_ptr[v0 + v] - e0;
    int r = jb->method == 0 ? oracle_core_levels(n, rp, jb->col + e0, jb->core + v0)
                            : oracle_core_bz(n, rp, jb->col + e0, jb->core + v0);
    if (r) jb->err = r;
    free(rp);
  }
  return NULL;
}

int oracle_core_batch(int32_t G, const int64_t* vo, const int64_t* row_ptr, const int32_t* col, int32_t* core,
                      int32_t method, int32_t threads) {
  struct batch_job jb;
  jb.G = G; jb.vo = vo; jb.row_ptr = row_ptr; jb.col = col; jb.core = core;
  jb.method = method; jb.next = 0; jb.err = 0;
  pthread_mutex_init(&jb.mu, NULL);
  if (threads < 1) threads = 1;
  if (threads > 256) threads = 256;
  pthread_t th[256];
  for (int t = 0; t < threads; ++t) pthread_create(&th[t], NULL, batch_worker, &jb);
  for (int t = 0; t < threads; ++t) pthread_join(th[t], NULL);
  pthread_mutex_destroy(&jb.mu);
  return jb.err;
}
