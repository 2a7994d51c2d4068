// Seeded synthetic graph generators and the edge-list -> CSR builder.
//
// This module produces INPUTS only. It holds none of the coreness arithmetic:
// it draws edges, symmetrises, removes self-loops and duplicates, and lays the
// result out as a CSR (row offsets int64, neighbour ids int32, each row sorted
// ascending). Both the CPU oracle and the GPU path consume its output.
//
// Randomness is counter-based: every draw is splitmix64 applied to a key made
// from (seed, stream, index), so a graph depends only on its parameters and
// seed, never on the number of threads used to build it.
//
// Graph families:
//   * G(n, m): m distinct undirected edges, endpoints uniform, u != v; the
//     first m distinct pairs in counter order are kept (equivalent to
//     sequential rejection of duplicates).
//   * Road-like lattice: rows x cols grid, each lattice edge kept with
//     probability p; each vertex, with probability chord_prob, gets one chord
//     to a vertex at Manhattan distance 1..maxdist inside the grid.
//   * R-MAT (Chakrabarti, Zhan, Faloutsos 2004) with per-level multiplicative
//     noise shared by all samples (in the spirit of the noisy stochastic
//     Kronecker model of Seshadhri, Pinar, Kolda), optional seeded relabel.
//   * Chung-Lu: weights w_i proportional to (i+1)^(-1/(gamma-1)), endpoints
//     drawn in proportion to w through a Vose alias table.
//   * Batch: many graphs of log-uniform size drawn from the three families,
//     concatenated with per-graph vertex offsets and graph-local ids.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <thread>
#include <vector>

namespace {

// ---------------------------------------------------------------- RNG
inline uint64_t mix64(uint64_t z) {
  // splitmix64 finaliser (Steele, Lea, Flood 2014; constants as published by Vigna)
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
inline uint64_t rand_key(uint64_t seed, uint64_t stream) {
  return mix64(mix64(seed) ^ (stream * 0xD1B54A32D192ED03ull + 0x632BE59BD9B4E019ull));
}
inline uint64_t rand_at(uint64_t key, uint64_t i) {
  return mix64(key + (i + 1) * 0x9E3779B97F4A7C15ull);
}
inline double u01(uint64_t x) { return (double)(x >> 11) * (1.0 / 9007199254740992.0); }
// Uniform integer in [0, r) by multiply-high (bias < r / 2^64).
inline uint64_t below(uint64_t x, uint64_t r) {
  return (uint64_t)(((unsigned __int128)x * (unsigned __int128)r) >> 64);
}

enum : uint64_t {
  S_ER = 1, S_KEEP = 2, S_CHORD = 3, S_CHORD_OFF = 4, S_RMAT = 5, S_NOISE = 6,
  S_PERM = 7, S_CL = 8, S_BATCH = 9, S_PARAM = 10
};

int default_threads() {
  const char* e = std::getenv("GG_THREADS");
  if (!e) e = std::getenv("OMP_NUM_THREADS");
  int t = e ? std::atoi(e) : 0;
  if (t <= 0) t = (int)std::thread::hardware_concurrency();
  if (t <= 0) t = 1;
  return std::min(t, 64);
}

template <class F>
void parallel_for(int64_t n, int nthreads, F&& f) {
  // f(begin, end, thread_index) over contiguous chunks
  if (nthreads <= 1 || n < 4096) {
    f((int64_t)0, n, 0);
    return;
  }
  std::vector<std::thread> th;
  int64_t chunk = (n + nthreads - 1) / nthreads;
  for (int t = 0; t < nthreads; ++t) {
    int64_t b = t * chunk, e = std::min(n, b + chunk);
    if (b >= e) break;
    th.emplace_back([&f, b, e, t] { f(b, e, t); });
  }
  for (auto& x : th) x.join();
}

// ---------------------------------------------------------------- CSR
struct Csr {
  int64_t n = 0;
  int64_t nnz = 0;
  int64_t* row_ptr = nullptr;  // malloc'd, n+1
  int32_t* col = nullptr;      // malloc'd, nnz
  ~Csr() {
    std::free(row_ptr);
    std::free(col);
  }
};

// Build a symmetric, loop-free, duplicate-free CSR with sorted rows from an
// undirected edge list given as parallel src/dst arrays of length m.
Csr* build_csr(int64_t n, int64_t m, const uint32_t* src, const uint32_t* dst, int nthreads) {
  auto* g = new Csr();
  g->n = n;
  g->row_ptr = (int64_t*)std::malloc(sizeof(int64_t) * (n + 1));
  std::vector<int64_t> off(n + 1, 0);
  std::vector<uint32_t> tmp;
  if (nthreads <= 1) {
    for (int64_t i = 0; i < m; ++i)
      if (src[i] != dst[i]) { off[src[i] + 1]++; off[dst[i] + 1]++; }
    for (int64_t v = 0; v < n; ++v) off[v + 1] += off[v];
    tmp.resize(off[n]);
    std::vector<int64_t> cur(off.begin(), off.end() - 1);
    for (int64_t i = 0; i < m; ++i)
      if (src[i] != dst[i]) { tmp[cur[src[i]]++] = dst[i]; tmp[cur[dst[i]]++] = src[i]; }
  } else {
    std::unique_ptr<std::atomic<uint32_t>[]> cnt(new std::atomic<uint32_t>[n]);
    parallel_for(n, nthreads, [&](int64_t b, int64_t e, int) {
      for (int64_t v = b; v < e; ++v) cnt[v].store(0, std::memory_order_relaxed);
    });
    parallel_for(m, nthreads, [&](int64_t b, int64_t e, int) {
      for (int64_t i = b; i < e; ++i)
        if (src[i] != dst[i]) {
          cnt[src[i]].fetch_add(1, std::memory_order_relaxed);
          cnt[dst[i]].fetch_add(1, std::memory_order_relaxed);
        }
    });
    for (int64_t v = 0; v < n; ++v) off[v + 1] = off[v] + cnt[v].load(std::memory_order_relaxed);
    tmp.resize(off[n]);
    parallel_for(n, nthreads, [&](int64_t b, int64_t e, int) {
      for (int64_t v = b; v < e; ++v) cnt[v].store(0, std::memory_order_relaxed);
    });
    parallel_for(m, nthreads, [&](int64_t b, int64_t e, int) {
      for (int64_t i = b; i < e; ++i)
        if (src[i] != dst[i]) {
          uint32_t u = src[i], v = dst[i];
          tmp[off[u] + cnt[u].fetch_add(1, std::memory_order_relaxed)] = v;
          tmp[off[v] + cnt[v].fetch_add(1, std::memory_order_relaxed)] = u;
        }
    });
  }
  // sort + dedup each row in place, record the new degree
  std::vector<int64_t> deg(n);
  parallel_for(n, nthreads, [&](int64_t b, int64_t e, int) {
    for (int64_t v = b; v < e; ++v) {
      uint32_t* s = tmp.data() + off[v];
      uint32_t* t = tmp.data() + off[v + 1];
      std::sort(s, t);
      deg[v] = std::unique(s, t) - s;
    }
  });
  g->row_ptr[0] = 0;
  for (int64_t v = 0; v < n; ++v) g->row_ptr[v + 1] = g->row_ptr[v] + deg[v];
  g->nnz = g->row_ptr[n];
  g->col = (int32_t*)std::malloc(sizeof(int32_t) * std::max<int64_t>(g->nnz, 1));
  parallel_for(n, nthreads, [&](int64_t b, int64_t e, int) {
    for (int64_t v = b; v < e; ++v)
      std::memcpy(g->col + g->row_ptr[v], tmp.data() + off[v], sizeof(uint32_t) * deg[v]);
  });
  return g;
}

// ---------------------------------------------------------------- generators
Csr* gen_er(int64_t n, int64_t m, uint64_t seed, int nthreads) {
  // keep the first m distinct unordered pairs (u != v) in counter order
  int64_t maxm = n * (n - 1) / 2;
  if (m > maxm) m = maxm;
  uint64_t key = rand_key(seed, S_ER);
  uint64_t next = 0;
  int64_t have = 0;
  std::vector<uint64_t> chosen;  // pair keys kept so far, sorted
  while (have < m) {
    int64_t want = (m - have) + (m - have) / 8 + 64;
    // draw `want` candidates with counters next..next+want-1
    std::vector<std::pair<uint64_t, uint64_t>> cand(want);  // (pairkey, counter)
    parallel_for(want, nthreads, [&](int64_t b, int64_t e, int) {
      for (int64_t i = b; i < e; ++i) {
        uint64_t c = next + i;
        uint64_t r = rand_at(key, c);
        uint64_t r2 = rand_at(key, c ^ 0x8000000000000000ull);
        uint64_t u = below(r, n), v = below(r2, n);
        if (u == v) { cand[i] = {~0ull, c}; continue; }
        if (u > v) std::swap(u, v);
        cand[i] = {(u << 32) | v, c};
      }
    });
    next += want;
    std::sort(cand.begin(), cand.end());
    std::vector<std::pair<uint64_t, uint64_t>> fresh;  // (counter, pairkey) first occurrence, not already chosen
    for (size_t i = 0; i < cand.size(); ++i) {
      if (cand[i].first == ~0ull) continue;
      if (i > 0 && cand[i].first == cand[i - 1].first) continue;
      if (std::binary_search(chosen.begin(), chosen.end(), cand[i].first)) continue;
      fresh.push_back({cand[i].second, cand[i].first});
    }
    std::sort(fresh.begin(), fresh.end());
    int64_t take = std::min<int64_t>((int64_t)fresh.size(), m - have);
    for (int64_t i = 0; i < take; ++i) chosen.push_back(fresh[i].second);
    std::sort(chosen.begin(), chosen.end());
    have += take;
  }
  std::vector<uint32_t> s(m), d(m);
  for (int64_t i = 0; i < m; ++i) { s[i] = (uint32_t)(chosen[i] >> 32); d[i] = (uint32_t)(chosen[i] & 0xffffffffu); }
  return build_csr(n, m, s.data(), d.data(), nthreads);
}

Csr* gen_lattice(int64_t rows, int64_t cols, double p, double chord_prob, int maxdist, uint64_t seed,
                 int nthreads) {
  int64_t n = rows * cols;
  int64_t nh = rows * (cols - 1), nv = (rows - 1) * cols;
  uint64_t kkey = rand_key(seed, S_KEEP), ckey = rand_key(seed, S_CHORD), okey = rand_key(seed, S_CHORD_OFF);
  // offsets (dr, dc) with 1 <= |dr|+|dc| <= maxdist, in a fixed enumeration order
  std::vector<std::pair<int, int>> offs;
  for (int dr = -maxdist; dr <= maxdist; ++dr)
    for (int dc = -maxdist; dc <= maxdist; ++dc) {
      int l1 = std::abs(dr) + std::abs(dc);
      if (l1 >= 1 && l1 <= maxdist) offs.push_back({dr, dc});
    }
  // pass 1: per chunk count kept edges, pass 2: write them in index order
  int T = std::max(1, nthreads);
  int64_t total = nh + nv + n;  // lattice edges, then one chord slot per vertex
  int64_t chunk = (total + T - 1) / T;
  std::vector<int64_t> cnt(T + 1, 0);
  auto edge_of = [&](int64_t i, uint32_t& a, uint32_t& b) -> bool {
    if (i < nh) {
      if (u01(rand_at(kkey, i)) >= p) return false;
      int64_t r = i / (cols - 1), c = i % (cols - 1);
      a = (uint32_t)(r * cols + c); b = a + 1;
      return true;
    }
    if (i < nh + nv) {
      int64_t j = i - nh;
      if (u01(rand_at(kkey, i)) >= p) return false;
      int64_t r = j / cols, c = j % cols;
      a = (uint32_t)(r * cols + c); b = (uint32_t)((r + 1) * cols + c);
      return true;
    }
    int64_t x = i - nh - nv;
    if (u01(rand_at(ckey, x)) >= chord_prob) return false;
    int64_t r = x / cols, c = x % cols;
    for (int attempt = 0; attempt < 256; ++attempt) {
      uint64_t k = below(rand_at(okey, (uint64_t)x * 256 + attempt), offs.size());
      int64_t r2 = r + offs[k].first, c2 = c + offs[k].second;
      if (r2 < 0 || r2 >= rows || c2 < 0 || c2 >= cols) continue;
      a = (uint32_t)x; b = (uint32_t)(r2 * cols + c2);
      return true;
    }
    return false;
  };
  std::vector<std::thread> th;
  for (int t = 0; t < T; ++t)
    th.emplace_back([&, t] {
      int64_t b = t * chunk, e = std::min(total, b + chunk);
      uint32_t x, y;
      int64_t c = 0;
      for (int64_t i = b; i < e; ++i) c += edge_of(i, x, y);
      cnt[t + 1] = c;
    });
  for (auto& x : th) x.join();
  th.clear();
  for (int t = 0; t < T; ++t) cnt[t + 1] += cnt[t];
  std::vector<uint32_t> s(cnt[T]), d(cnt[T]);
  for (int t = 0; t < T; ++t)
    th.emplace_back([&, t] {
      int64_t b = t * chunk, e = std::min(total, b + chunk);
      int64_t o = cnt[t];
      uint32_t x, y;
      for (int64_t i = b; i < e; ++i)
        if (edge_of(i, x, y)) { s[o] = x; d[o] = y; ++o; }
    });
  for (auto& x : th) x.join();
  return build_csr(n, cnt[T], s.data(), d.data(), nthreads);
}

void fisher_yates(std::vector<uint32_t>& perm, uint64_t seed) {
  uint64_t key = rand_key(seed, S_PERM);
  for (size_t i = 0; i < perm.size(); ++i) perm[i] = (uint32_t)i;
  for (size_t i = perm.size(); i > 1; --i) {
    size_t j = below(rand_at(key, i), i);
    std::swap(perm[i - 1], perm[j]);
  }
}

Csr* gen_rmat(int scale, int64_t samples, double a, double b, double c, double d, double noise, int relabel,
              uint64_t seed, int nthreads) {
  int64_t n = (int64_t)1 << scale;
  uint64_t nkey = rand_key(seed, S_NOISE), rkey = rand_key(seed, S_RMAT);
  // per-level thresholds in 32-bit fixed point
  std::vector<uint64_t> ta(scale), tab(scale), tabc(scale);
  for (int l = 0; l < scale; ++l) {
    double f[4], base[4] = {a, b, c, d}, s = 0;
    for (int j = 0; j < 4; ++j) {
      f[j] = base[j] * (1.0 + noise * (2.0 * u01(rand_at(nkey, (uint64_t)l * 4 + j)) - 1.0));
      s += f[j];
    }
    double pa = f[0] / s, pb = f[1] / s, pc = f[2] / s;
    ta[l] = (uint64_t)(pa * 4294967296.0);
    tab[l] = (uint64_t)((pa + pb) * 4294967296.0);
    tabc[l] = (uint64_t)((pa + pb + pc) * 4294967296.0);
  }
  std::vector<uint32_t> perm;
  if (relabel) {
    perm.resize(n);
    fisher_yates(perm, seed);
  }
  std::vector<uint32_t> s(samples), t(samples);
  int W = (scale + 1) / 2;
  parallel_for(samples, nthreads, [&](int64_t bb, int64_t ee, int) {
    for (int64_t i = bb; i < ee; ++i) {
      uint32_t u = 0, v = 0;
      for (int l = 0; l < scale; ++l) {
        uint64_t w = rand_at(rkey, (uint64_t)i * W + (l >> 1));
        uint64_t r = (l & 1) ? (w >> 32) : (w & 0xffffffffull);
        uint32_t bit = 1u << (scale - 1 - l);
        if (r < ta[l]) {
        } else if (r < tab[l]) {
          v |= bit;
        } else if (r < tabc[l]) {
          u |= bit;
        } else {
          u |= bit; v |= bit;
        }
      }
      if (relabel) { u = perm[u]; v = perm[v]; }
      s[i] = u; t[i] = v;
    }
  });
  return build_csr(n, samples, s.data(), t.data(), nthreads);
}

Csr* gen_chung_lu(int64_t n, double gamma, double avg_deg, uint64_t seed, int nthreads) {
  // Vose alias table over w_i = (i+1)^(-1/(gamma-1))
  std::vector<double> w(n);
  double ex = -1.0 / (gamma - 1.0), sw = 0;
  for (int64_t i = 0; i < n; ++i) { w[i] = std::pow((double)(i + 1), ex); sw += w[i]; }
  std::vector<double> prob(n);
  std::vector<uint32_t> alias(n);
  {
    std::vector<double> q(n);
    std::vector<uint32_t> small, large;
    for (int64_t i = 0; i < n; ++i) {
      q[i] = w[i] * n / sw;
      (q[i] < 1.0 ? small : large).push_back((uint32_t)i);
    }
    while (!small.empty() && !large.empty()) {
      uint32_t l = small.back(); small.pop_back();
      uint32_t g = large.back(); large.pop_back();
      prob[l] = q[l]; alias[l] = g;
      q[g] = (q[g] + q[l]) - 1.0;
      (q[g] < 1.0 ? small : large).push_back(g);
    }
    for (uint32_t g : large) { prob[g] = 1.0; alias[g] = g; }
    for (uint32_t l : small) { prob[l] = 1.0; alias[l] = l; }
  }
  int64_t m = (int64_t)std::llround(n * avg_deg / 2.0);
  uint64_t key = rand_key(seed, S_CL);
  std::vector<uint32_t> s(m), t(m);
  auto draw = [&](uint64_t x) -> uint32_t {
    uint64_t i = below(x, n);
    double coin = u01(mix64(x));
    return coin < prob[i] ? (uint32_t)i : alias[i];
  };
  parallel_for(m, nthreads, [&](int64_t b, int64_t e, int) {
    for (int64_t i = b; i < e; ++i) {
      s[i] = draw(rand_at(key, 2 * (uint64_t)i));
      t[i] = draw(rand_at(key, 2 * (uint64_t)i + 1));
    }
  });
  return build_csr(n, m, s.data(), t.data(), nthreads);
}

// ---------------------------------------------------------------- batch
struct Batch {
  int32_t G = 0;
  int64_t total_n = 0, total_nnz = 0;
  int64_t* graph_vtx_off = nullptr;  // G+1
  int64_t* row_ptr = nullptr;        // total_n + 1, global edge offsets
  int32_t* col = nullptr;            // graph-local ids
  int32_t* kind = nullptr;           // 0 = ER, 1 = Chung-Lu, 2 = lattice
  ~Batch() {
    std::free(graph_vtx_off); std::free(row_ptr); std::free(col); std::free(kind);
  }
};

struct GraphSpec {
  int kind;
  int64_t n;
  double p1, p2;
  uint64_t seed;
};

GraphSpec batch_spec(uint64_t seed, int64_t g, int64_t nmin, int64_t nmax, int kinds_mask) {
  uint64_t key = rand_key(seed, S_BATCH + (uint64_t)g * 16);
  GraphSpec s;
  double lo = std::log((double)nmin), hi = std::log((double)nmax);
  s.n = (int64_t)std::llround(std::exp(lo + (hi - lo) * u01(rand_at(key, 0))));
  int allowed[3], na = 0;
  for (int k = 0; k < 3; ++k)
    if (kinds_mask & (1 << k)) allowed[na++] = k;
  if (na == 0) allowed[na++] = 0;
  s.kind = allowed[below(rand_at(key, 1), na)];
  s.p1 = u01(rand_at(key, 2));
  s.p2 = u01(rand_at(key, 3));
  s.seed = rand_at(key, 4);
  if (s.kind == 2) {
    int64_t side = (int64_t)std::ceil(std::sqrt((double)s.n));
    s.n = side * side;
  }
  return s;
}

Csr* gen_spec(const GraphSpec& s, int nthreads) {
  if (s.kind == 0) {
    double deg = 8.0 + 24.0 * s.p1;
    int64_t m = (int64_t)std::llround(s.n * deg / 2.0);
    return gen_er(s.n, m, s.seed, nthreads);
  }
  if (s.kind == 1) {
    double gamma = 2.1 + 0.6 * s.p1, deg = 8.0 + 24.0 * s.p2;
    return gen_chung_lu(s.n, gamma, deg, s.seed, nthreads);
  }
  int64_t side = (int64_t)std::llround(std::sqrt((double)s.n));
  return gen_lattice(side, side, 0.6, 0.01, 8, s.seed, nthreads);
}

}  // namespace

extern "C" {

uint64_t gg_rand(uint64_t seed, uint64_t stream, uint64_t i) { return rand_at(rand_key(seed, stream), i); }

void* gg_er(int64_t n, int64_t m, uint64_t seed) { return gen_er(n, m, seed, default_threads()); }
void* gg_lattice(int64_t rows, int64_t cols, double p, double chord_prob, int32_t maxdist, uint64_t seed) {
  return gen_lattice(rows, cols, p, chord_prob, maxdist, seed, default_threads());
}
void* gg_rmat(int32_t scale, int64_t samples, double a, double b, double c, double d, double noise,
              int32_t relabel, uint64_t seed) {
  return gen_rmat(scale, samples, a, b, c, d, noise, relabel, seed, default_threads());
}
void* gg_chung_lu(int64_t n, double gamma, double avg_deg, uint64_t seed) {
  return gen_chung_lu(n, gamma, avg_deg, seed, default_threads());
}
// Undirected edge list (any order, loops and duplicates allowed) -> CSR.
void* gg_from_edges(int64_t n, int64_t m, const int32_t* src, const int32_t* dst) {
  return build_csr(n, m, (const uint32_t*)src, (const uint32_t*)dst, default_threads());
}
int64_t gg_n(void* h) { return ((Csr*)h)->n; }
int64_t gg_nnz(void* h) { return ((Csr*)h)->nnz; }
int64_t* gg_row_ptr(void* h) { return ((Csr*)h)->row_ptr; }
int32_t* gg_col(void* h) { return ((Csr*)h)->col; }
void gg_free(void* h) { delete (Csr*)h; }

// Per-graph specification of the batch (size, family, parameters), cheap to query.
void gg_batch_spec(uint64_t seed, int64_t g, int64_t nmin, int64_t nmax, int32_t kinds_mask, int32_t* kind,
                   int64_t* n) {
  GraphSpec s = batch_spec(seed, g, nmin, nmax, kinds_mask);
  *kind = s.kind;
  *n = s.n;
}

// Generate graphs [g0, g0 + count) of the batch, concatenated.
void* gg_batch(uint64_t seed, int64_t g0, int32_t count, int64_t nmin, int64_t nmax, int32_t kinds_mask) {
  int T = default_threads();
  std::vector<std::unique_ptr<Csr>> parts(count);
  std::vector<int32_t> kinds(count);
  std::atomic<int32_t> next(0);
  // largest graphs first for load balance
  std::vector<GraphSpec> specs(count);
  std::vector<int32_t> order(count);
  for (int32_t i = 0; i < count; ++i) {
    specs[i] = batch_spec(seed, g0 + i, nmin, nmax, kinds_mask);
    kinds[i] = specs[i].kind;
    order[i] = i;
  }
  std::sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return specs[x].n > specs[y].n; });
  std::vector<std::thread> th;
  for (int t = 0; t < T; ++t)
    th.emplace_back([&] {
      for (;;) {
        int32_t k = next.fetch_add(1);
        if (k >= count) break;
        int32_t i = order[k];
        parts[i].reset(gen_spec(specs[i], 1));
      }
    });
  for (auto& x : th) x.join();
  auto* b = new Batch();
  b->G = count;
  b->graph_vtx_off = (int64_t*)std::malloc(sizeof(int64_t) * (count + 1));
  b->kind = (int32_t*)std::malloc(sizeof(int32_t) * std::max(count, 1));
  b->graph_vtx_off[0] = 0;
  std::vector<int64_t> eoff(count + 1, 0);
  for (int32_t i = 0; i < count; ++i) {
    b->graph_vtx_off[i + 1] = b->graph_vtx_off[i] + parts[i]->n;
    eoff[i + 1] = eoff[i] + parts[i]->nnz;
    b->kind[i] = kinds[i];
  }
  b->total_n = b->graph_vtx_off[count];
  b->total_nnz = eoff[count];
  b->row_ptr = (int64_t*)std::malloc(sizeof(int64_t) * (b->total_n + 1));
  b->col = (int32_t*)std::malloc(sizeof(int32_t) * std::max<int64_t>(b->total_nnz, 1));
  next.store(0);
  th.clear();
  for (int t = 0; t < T; ++t)
    th.emplace_back([&] {
      for (;;) {
        int32_t i = next.fetch_add(1);
        if (i >= count) break;
        const Csr* p = parts[i].get();
        int64_t vo = b->graph_vtx_off[i], eo = eoff[i];
        for (int64_t v = 0; v < p->n; ++v) b->row_ptr[vo + v] = eo + p->row_ptr[v];
        std::memcpy(b->col + eo, p->col, sizeof(int32_t) * p->nnz);
        parts[i].reset();
      }
    });
  for (auto& x : th) x.join();
  b->row_ptr[b->total_n] = b->total_nnz;
  return b;
}
int32_t gg_batch_count(void* h) { return ((Batch*)h)->G; }
int64_t gg_batch_total_n(void* h) { return ((Batch*)h)->total_n; }
int64_t gg_batch_total_nnz(void* h) { return ((Batch*)h)->total_nnz; }
int64_t* gg_batch_graph_vtx_off(void* h) { return ((Batch*)h)->graph_vtx_off; }
int64_t* gg_batch_row_ptr(void* h) { return ((Batch*)h)->row_ptr; }
int32_t* gg_batch_col(void* h) { return ((Batch*)h)->col; }
int32_t* gg_batch_kind(void* h) { return ((Batch*)h)->kind; }
void gg_batch_free(void* h) { delete (Batch*)h; }

// Check the CSR preconditions. Returns 0 if valid, otherwise a positive code:
// 1 row_ptr[0] != 0, 2 row_ptr not monotone, 3 id out of range, 4 self-loop,
// 5 row not strictly increasing (unsorted or duplicate), 6 not symmetric.
int32_t gg_validate(int64_t n, const int64_t* row_ptr, const int32_t* col) {
  if (n == 0) return 0;
  if (row_ptr[0] != 0) return 1;
  for (int64_t v = 0; v < n; ++v)
    if (row_ptr[v + 1] < row_ptr[v]) return 2;
  std::atomic<int32_t> err(0);
  parallel_for(n, default_threads(), [&](int64_t b, int64_t e, int) {
    for (int64_t v = b; v < e && err.load(std::memory_order_relaxed) == 0; ++v) {
      for (int64_t j = row_ptr[v]; j < row_ptr[v + 1]; ++j) {
        int32_t u = col[j];
        int32_t code = 0;
        if (u < 0 || u >= n) code = 3;
        else if (u == v) code = 4;
        else if (j > row_ptr[v] && col[j - 1] >= u) code = 5;
        else if (!std::binary_search(col + row_ptr[u], col + row_ptr[u + 1], (int32_t)v)) code = 6;
        if (code) { int32_t z = 0; err.compare_exchange_strong(z, code); break; }
      }
    }
  });
  return err.load();
}

}  // extern "C"
