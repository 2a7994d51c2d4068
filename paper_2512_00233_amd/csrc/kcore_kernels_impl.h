// Kernels of the iterative coreness computation (included by the runtime TU).
// See kcore_kernels.h for the method, the citations and the GPU-specific design.
#pragma once
#include "kcore_kernels.h"

namespace kcore {

// ------------------------------------------------------------------ wave helpers
__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }
__device__ __forceinline__ int popc(uint64_t m) { return __popcll(m); }
__device__ __forceinline__ int lanes_below(uint64_t m) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
__device__ __forceinline__ int32_t ld_counter(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t uni(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ int32_t wave_incl_scan(int32_t x) {
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    int32_t t = __shfl_up(x, o);
    if (lane >= o) x += t;
  }
  return x;
}

template <typename Off>
__device__ __forceinline__ int32_t* list_of(const Args<Off>& a, int32_t round) {
  return (round & 1) ? a.lists[1] : a.lists[0];  // select, not an indexed load from the argument struct
}

struct LaneStats {
  uint64_t v[kLaneStats] = {0, 0, 0, 0, 0, 0};
};

// Where activated vertices go.
struct Sink {
  int32_t* list;      // next sparse frontier list
  int32_t* cnt;       // its three class counters
  int32_t* overflow;  // flag of the next round (nullptr: never overflows)
  int32_t stamp;      // round number of the next frontier
  int32_t b[3];       // class region offsets in the list
  int32_t cap[3];     // class capacities
};

template <typename Off>
__device__ __forceinline__ Sink make_sink(const Args<Off>& a, int32_t next_round, int32_t* cnt, int32_t* overflow,
                                          bool capped) {
  const Ctl* ctl = a.ctl;
  Sink s;
  s.list = list_of(a, next_round);
  s.cnt = cnt;
  s.overflow = overflow;
  s.stamp = next_round;
  const int32_t p0 = ctl->pop[0], p1 = ctl->pop[1], p2 = ctl->pop[2];
  s.b[0] = 0;
  s.b[1] = p0;
  s.b[2] = p0 + p1;
  s.cap[0] = capped ? min(p0, a.list_cap) : p0;
  s.cap[1] = capped ? min(p1, a.list_cap) : p1;
  s.cap[2] = capped ? min(p2, a.list_cap) : p2;
  return s;
}

// Activate up to N candidates per lane for the next round: deduplicate on the
// round stamp (all atomics of a lane in flight together), then, unless the next
// round already overflowed to a dense sweep, append the winners to the list of
// their degree class with one atomic per class per wavefront.  Every active lane
// of the wavefront must call this.
template <int N, typename Off>
__device__ __forceinline__ void activate_batch(const Args<Off>& a, const Sink& s, const int32_t (&v)[N],
                                               const bool (&want)[N], LaneStats& st) {
  bool anyw = false;
#pragma unroll
  for (int i = 0; i < N; ++i) anyw |= want[i];
  if (!ballot(anyw)) return;
  int32_t p[N];
#pragma unroll
  for (int i = 0; i < N; ++i) p[i] = want[i] ? a.stamp[v[i]] : INT32_MAX;
#pragma unroll
  for (int i = 0; i < N; ++i) p[i] = (p[i] < s.stamp) ? atomicMax(&a.stamp[v[i]], s.stamp) : INT32_MAX;
  uint32_t first = 0;
#pragma unroll
  for (int i = 0; i < N; ++i) first |= (p[i] < s.stamp ? 1u : 0u) << i;
  st.v[ST_ACTIVATIONS] += __popc(first);
  const bool dense_next = s.overflow && *(volatile int32_t*)s.overflow;
  if (dense_next || !ballot(first != 0)) return;
#pragma unroll
  for (int i = 0; i < N; ++i) p[i] = (first >> i & 1u) ? (int32_t)a.cls[v[i]] : 3;  // degree class of winners
  const int lane = lane_id();
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    int32_t mine = 0;
#pragma unroll
    for (int i = 0; i < N; ++i) mine += p[i] == k;
    const int32_t incl = wave_incl_scan(mine);
    const int32_t tot = __shfl(incl, kWave - 1);
    if (tot == 0) continue;
    int32_t base = 0;
    if (lane == kWave - 1) base = atomicAdd(&s.cnt[k], tot);
    base = __shfl(base, kWave - 1);
    int32_t pos = base + incl - mine;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      if (p[i] == k) {
        if (pos < s.cap[k]) s.list[s.b[k] + pos] = v[i];
        ++pos;
      }
    }
    if (lane == kWave - 1 && base + tot > s.cap[k] && s.overflow) *(volatile int32_t*)s.overflow = 1;
  }
}

// Should neighbour v, whose estimate read in this round is x, be activated
// after the current vertex dropped from e to h?
template <typename Off>
__device__ __forceinline__ bool wants(const Args<Off>& a, int32_t v, int32_t x, int32_t e, int32_t h, bool dense,
                                      int32_t round) {
  if (x <= h) return false;
  if (a.one_sided || x <= e || dense) return true;
  return a.stamp[v] >= round;  // v is in the current frontier: its value may still be moving
}

// ------------------------------------------------------------------ lane path
// One lane per vertex, degree <= kThreadMaxDeg, values held in registers.
template <typename Off>
__device__ __forceinline__ void upd_lane(const Args<Off>& a, const Sink& s, int32_t u, bool valid, bool dense,
                                         int32_t round, LaneStats& st) {
  int32_t e = 0, d = 0;
  Off beg = 0;
  if (valid) {
    beg = a.row_ptr[u];
    d = (int32_t)(a.row_ptr[u + 1] - beg);
    e = a.est[u];
  }
  valid = valid && e >= 2;  // an estimate of 1 is final: every non-isolated vertex has coreness >= 1
  int32_t c[kThreadMaxDeg], x[kThreadMaxDeg];
#pragma unroll
  for (int i = 0; i < kThreadMaxDeg; ++i) c[i] = (valid && i < d) ? a.col[beg + i] : 0;
#pragma unroll
  for (int i = 0; i < kThreadMaxDeg; ++i) x[i] = (valid && i < d) ? a.est[c[i]] : 0;
  int32_t h = e;
  if (valid) {
    st.v[ST_UPDATES] += 1;
    st.v[ST_VISITS] += (uint64_t)d;
    int cnt = 0;
#pragma unroll
    for (int i = 0; i < kThreadMaxDeg; ++i) cnt += x[i] >= e;
    if (cnt < e) {
      h = 1;
      for (int k = e - 1; k >= 2; --k) {
        int sk = 0;
#pragma unroll
        for (int i = 0; i < kThreadMaxDeg; ++i) sk += x[i] >= k;
        if (sk >= k) {
          h = k;
          break;
        }
      }
      a.est[u] = h;
      st.v[ST_CHANGES] += 1;
    }
  }
  const bool changed = valid && h < e;
  if (!ballot(changed)) return;
  bool w[kThreadMaxDeg];
#pragma unroll
  for (int i = 0; i < kThreadMaxDeg; ++i) w[i] = changed && i < d && wants(a, c[i], x[i], e, h, dense, round);
  activate_batch<kThreadMaxDeg>(a, s, c, w, st);
}

// ------------------------------------------------------------------ wavefront path
// One 64-lane wavefront per vertex, degree <= 64 * kWaveRegs; searches its
// pruned list first when it has one.
template <typename Off>
__device__ __forceinline__ void upd_wave(const Args<Off>& a, const Sink& s, int32_t u, bool dense, int32_t round,
                                         LaneStats& st) {
  constexpr int R = kWaveRegs;
  const int lane = lane_id();
  const Off beg = a.row_ptr[u];
  const int32_t d = uni((int32_t)(a.row_ptr[u + 1] - beg));
  const int32_t e = uni(a.est[u]);
  if (e < 2) return;
  const int32_t pl = a.prune ? uni(a.plen[u]) : 0;
  const int32_t L = pl > 0 ? uni(a.plow[u]) : 1;
  int32_t c[R], x[R];
  int32_t len = 0;
  auto load = [&](const int32_t* src, int32_t n_) {
    len = n_;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int j = lane + kWave * i;
      c[i] = (kWave * i < n_ && j < n_) ? src[beg + j] : 0;
    }
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int j = lane + kWave * i;
      x[i] = (kWave * i < n_ && j < n_) ? a.est[c[i]] : 0;
    }
  };
  auto count = [&](int32_t k) {
    int tot = 0;
#pragma unroll
    for (int i = 0; i < R; ++i)
      if (kWave * i < len) tot += popc(ballot(x[i] >= k));
    return tot;
  };
  auto search = [&](int32_t lo, int32_t hi) {  // max k in [lo, hi] with count(k) >= k, given count(lo) >= lo
    while (lo < hi) {
      const int32_t mid = (lo + hi + 1) >> 1;
      if (count(mid) >= mid) lo = mid;
      else hi = mid - 1;
    }
    return lo;
  };
  if (lane == 0) st.v[ST_UPDATES] += 1;
  int32_t h = -1;
  if (pl > 0) {
    load(a.pruned, pl);
    if (lane == 0) st.v[ST_VISITS] += pl;
    if (count(e) >= e) h = e;
    else if (count(L) >= L) h = search(L, e - 1);
  }
  if (h < 0) {
    load(a.col, d);
    if (lane == 0) {
      st.v[ST_VISITS] += d;
      st.v[ST_FULL_SCANS] += 1;
    }
    h = count(e) >= e ? e : search(1, e - 1);
    if (a.prune) {
      const int32_t L2 = max(2, (3 * h) / 4);
      int32_t off = 0;
#pragma unroll
      for (int i = 0; i < R; ++i) {
        if (kWave * i < len) {
          const bool keep = (lane + kWave * i < len) && x[i] >= L2;
          const uint64_t m = ballot(keep);
          if (keep) a.pruned[beg + off + lanes_below(m)] = c[i];
          off += popc(m);
        }
      }
      if (lane == 0) {
        a.plen[u] = off;
        a.plow[u] = L2;
        st.v[ST_PRUNE_WRITES] += off;
      }
    }
  }
  if (h == e) return;
  if (lane == 0) {
    a.est[u] = h;
    st.v[ST_CHANGES] += 1;
  }
  bool w[R];
#pragma unroll
  for (int i = 0; i < R; ++i) w[i] = (lane + kWave * i < len) && wants(a, c[i], x[i], e, h, dense, round);
  activate_batch<R>(a, s, c, w, st);
}

// ------------------------------------------------------------------ workgroup paths
// Sum over the workgroup of one value per wavefront (lane 0 holds it).
template <int BLOCK>
__device__ __forceinline__ int32_t block_sum_waves(int32_t wave_val, int32_t* red) {
  const int wave = threadIdx.x / kWave;
  if (lane_id() == 0) red[wave] = wave_val;
  __syncthreads();
  int32_t t = 0;
#pragma unroll
  for (int w = 0; w < BLOCK / kWave; ++w) t += red[w];
  __syncthreads();
  return t;
}

// Exclusive prefix over the workgroup of one value per thread; also returns the total.
template <int BLOCK>
__device__ __forceinline__ int32_t block_excl_scan(int32_t x, int32_t& total, int32_t* red) {
  const int wave = threadIdx.x / kWave;
  const int32_t incl = wave_incl_scan(x);
  if (lane_id() == kWave - 1) red[wave] = incl;
  __syncthreads();
  int32_t before = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < BLOCK / kWave; ++w) {
    const int32_t r = red[w];
    before += w < wave ? r : 0;
    tot += r;
  }
  __syncthreads();
  total = tot;
  return before + incl - x;
}

// Workgroup-wide search over a list in global memory, re-read on each pass:
// the largest k in [lo, hi] with |{j < len : est[src[j]] >= k}| >= k, or lo - 1
// when count(lo) < lo.  Each pass tests kHugeThresholds thresholds.
template <int BLOCK, typename Off>
__device__ __forceinline__ int32_t mp_search(const Args<Off>& a, const int32_t* src, int32_t len, int32_t lo,
                                             int32_t hi, int32_t* red) {
  constexpr int S = kHugeThresholds;
  constexpr int NW = BLOCK / kWave;
  const int tid = threadIdx.x;
  bool lo_known = false;
  while (!(lo_known && lo >= hi)) {
    // unknown lo: thr(0) = lo and the rest spread over (lo, hi]; known lo: spread over (lo, hi]
    const int first = lo_known ? 0 : 1;
    const int slots = S - first;
    const int64_t span = (int64_t)hi - lo;
    auto thr = [&](int q) -> int32_t {
      if (q < first) return lo;
      const int r = q - first;
      if (span >= slots) return (int32_t)(lo + ((int64_t)(r + 1) * span + slots - 1) / slots);
      return (r < span) ? lo + 1 + r : INT32_MAX;
    };
    int32_t t[S], cnt[S];
#pragma unroll
    for (int q = 0; q < S; ++q) {
      t[q] = uni(thr(q));
      cnt[q] = 0;
    }
    for (int32_t j = tid; j < len; j += BLOCK) {
      const int32_t xv = a.est[src[j]];
#pragma unroll
      for (int q = 0; q < S; ++q) cnt[q] += xv >= t[q];
    }
    const int wave = tid / kWave;
#pragma unroll
    for (int q = 0; q < S; ++q) {
      const int32_t w = wave_sum(cnt[q]);
      if (lane_id() == 0) red[q * NW + wave] = w;
    }
    __syncthreads();
    int32_t best = -1;
#pragma unroll
    for (int q = 0; q < S; ++q) {
      int32_t tot = 0;
#pragma unroll
      for (int w = 0; w < NW; ++w) tot += red[q * NW + w];
      if (t[q] != INT32_MAX && tot >= t[q]) best = q;  // count(k) - k is decreasing: the hits form a prefix
    }
    __syncthreads();
    best = uni(best);
    if (!lo_known) {
      if (best < 0) return lo - 1;
      lo_known = true;
    }
    if (best < 0) {
      hi = thr(0) - 1;
    } else {
      const int32_t nlo = thr(best);
      if (best + 1 < S && thr(best + 1) != INT32_MAX) hi = thr(best + 1) - 1;
      lo = nlo;
    }
  }
  return lo;
}

// One workgroup per vertex (degree class 2).  Lists of up to BLOCK * kBlockRegs
// entries are held in registers (binary search with wavefront ballots);
// longer ones use the multi-pass search.  The pruned list is tried first.
template <int BLOCK, typename Off>
__device__ __forceinline__ void upd_big(const Args<Off>& a, const Sink& s, int32_t u, bool dense, int32_t round,
                                        LaneStats& st, int32_t* red) {
  constexpr int R = kBlockRegs;
  constexpr int CAPR = BLOCK * R;
  const int tid = threadIdx.x;
  const Off beg = a.row_ptr[u];
  const int32_t d = uni((int32_t)(a.row_ptr[u + 1] - beg));
  const int32_t e = uni(a.est[u]);
  if (e < 2) return;
  const int32_t pl = a.prune ? uni(a.plen[u]) : 0;
  const int32_t L = pl > 0 ? uni(a.plow[u]) : 1;
  int32_t c[R], x[R];
  int32_t len = 0;
  bool inreg = false;
  const int32_t* src = a.col;
  auto load = [&](const int32_t* from, int32_t n_) {
    len = n_;
    src = from;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int j = tid + BLOCK * i;
      c[i] = (BLOCK * i < n_ && j < n_) ? from[beg + j] : 0;
    }
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int j = tid + BLOCK * i;
      x[i] = (BLOCK * i < n_ && j < n_) ? a.est[c[i]] : 0;
    }
  };
  auto count = [&](int32_t k) {
    int tot = 0;
#pragma unroll
    for (int i = 0; i < R; ++i)
      if (BLOCK * i < len) tot += popc(ballot(x[i] >= k));
    return block_sum_waves<BLOCK>(tot, red);
  };
  auto search = [&](int32_t lo, int32_t hi) {
    while (lo < hi) {
      const int32_t mid = (lo + hi + 1) >> 1;
      if (count(mid) >= mid) lo = mid;
      else hi = mid - 1;
    }
    return lo;
  };
  if (tid == 0) st.v[ST_UPDATES] += 1;
  int32_t h = -1;
  if (pl > 0) {
    if (tid == 0) st.v[ST_VISITS] += pl;
    if (pl <= CAPR) {
      load(a.pruned, pl);
      inreg = true;
      if (count(e) >= e) h = e;
      else if (count(L) >= L) h = search(L, e - 1);
    } else {
      inreg = false;
      len = pl;
      src = a.pruned;
      const int32_t hp = mp_search<BLOCK>(a, a.pruned + beg, pl, L, e, red);
      if (hp >= L) h = hp;
    }
  }
  bool rebuild_pass = false;
  if (h < 0) {
    if (tid == 0) {
      st.v[ST_VISITS] += d;
      st.v[ST_FULL_SCANS] += 1;
    }
    if (d <= CAPR) {
      load(a.col, d);
      inreg = true;
      h = count(e) >= e ? e : search(1, e - 1);
      if (a.prune) {
        const int32_t L2 = max(2, (3 * h) / 4);
        int32_t mine = 0;
#pragma unroll
        for (int i = 0; i < R; ++i) mine += (tid + BLOCK * i < len) && x[i] >= L2;
        int32_t total = 0;
        int32_t off = block_excl_scan<BLOCK>(mine, total, red);
#pragma unroll
        for (int i = 0; i < R; ++i)
          if ((tid + BLOCK * i < len) && x[i] >= L2) a.pruned[beg + off++] = c[i];
        if (tid == 0) {
          a.plen[u] = total;
          a.plow[u] = L2;
          st.v[ST_PRUNE_WRITES] += total;
        }
      }
    } else {
      inreg = false;
      len = d;
      src = a.col;
      h = mp_search<BLOCK>(a, a.col + beg, d, 1, e, red);
      rebuild_pass = a.prune != 0;
    }
  }
  const bool changed = h < e;
  if (!changed && !rebuild_pass) return;
  if (changed && tid == 0) {
    a.est[u] = h;
    st.v[ST_CHANGES] += 1;
  }
  if (inreg) {
    bool w[R];
#pragma unroll
    for (int i = 0; i < R; ++i) w[i] = (tid + BLOCK * i < len) && wants(a, c[i], x[i], e, h, dense, round);
    activate_batch<R>(a, s, c, w, st);
    return;
  }
  // streaming pass over the list: activation and/or rebuilding the pruned list
  const int32_t L2 = max(2, (3 * h) / 4);
  int32_t written = 0;
  for (int32_t j0 = 0; j0 < len; j0 += BLOCK) {
    const int32_t j = j0 + tid;
    int32_t v[1] = {0};
    int32_t xv = 0;
    if (j < len) {
      v[0] = src[beg + j];
      xv = a.est[v[0]];
    }
    if (rebuild_pass) {
      const int32_t keep = (j < len) && xv >= L2;
      int32_t total = 0;
      const int32_t off = block_excl_scan<BLOCK>(keep, total, red);
      if (keep) a.pruned[beg + written + off] = v[0];
      written += total;
    }
    if (changed) {
      bool w[1] = {(j < len) && wants(a, v[0], xv, e, h, dense, round)};
      activate_batch<1>(a, s, v, w, st);
    }
  }
  if (rebuild_pass && tid == 0) {
    a.plen[u] = written;
    a.plow[u] = L2;
    st.v[ST_PRUNE_WRITES] += written;
  }
}

// ------------------------------------------------------------------ statistics
template <int BLOCK>
__device__ __forceinline__ void flush_stats(Ctl* ctl, const LaneStats& st, unsigned long long* red64) {
  constexpr int NW = BLOCK / kWave;
  const int wave = threadIdx.x / kWave;
#pragma unroll
  for (int q = 0; q < kLaneStats; ++q) {
    const unsigned long long w = wave_sum((unsigned long long)st.v[q]);
    if (lane_id() == 0) red64[q * NW + wave] = w;
  }
  __syncthreads();
  if (threadIdx.x < kLaneStats) {
    unsigned long long t = 0;
    for (int w = 0; w < NW; ++w) t += red64[threadIdx.x * NW + w];
    if (t) atomicAdd(&ctl->stats[threadIdx.x], t);
  }
}

// ------------------------------------------------------------------ frontier sweeps
// Sparse round: the three class lists of the current round.
template <int BLOCK, typename Off>
__device__ __forceinline__ void sweep_lists(const Args<Off>& a, const Sink& s, const int32_t* cur, int32_t n0,
                                            int32_t n1, int32_t n2, int32_t round, int32_t b1, int32_t b2,
                                            int32_t worker, int32_t workers, LaneStats& st, int32_t* red) {
  constexpr int NW = BLOCK / kWave;
  for (int32_t i = worker; i < n2; i += workers) upd_big<BLOCK>(a, s, cur[b2 + i], false, round, st, red);
  const int32_t gw = worker * NW + threadIdx.x / kWave;
  for (int32_t i = gw; i < n1; i += workers * NW) upd_wave(a, s, cur[b1 + i], false, round, st);
  for (int32_t i = worker * BLOCK + threadIdx.x; i - lane_id() < n0; i += workers * BLOCK) {
    const bool valid = i < n0;
    upd_lane(a, s, valid ? cur[i] : 0, valid, false, round, st);
  }
}

// Workgroup id -> logical id such that consecutive logical ids (consecutive
// vertex ranges in the dense sweep) land on the same XCD (workgroups are
// dispatched round-robin over the 8 XCDs).
__device__ __forceinline__ int32_t xcd_logical_block(int32_t b, int32_t G) {
  constexpr int X = 8;
  if (G % X != 0) return b;
  return (b % X) * (G / X) + b / X;
}

// Dense round: active vertices found from the stamps (FIRST: every vertex of degree >= 2).
template <int BLOCK, bool FIRST, typename Off>
__device__ __forceinline__ void sweep_dense(const Args<Off>& a, const Sink& s, int32_t round, LaneStats& st,
                                            int32_t* red, int32_t* sh_u, unsigned long long* sh_mask) {
  const Ctl* ctl = a.ctl;
  const int32_t pop1 = ctl->pop[1], pop2 = ctl->pop[2];
  const int32_t G = gridDim.x;
  const int lane = lane_id();
  // workgroup class: static list, 64 entries per group examined by wavefront 0
  {
    const int32_t* S2 = a.slist + pop1;
    const int32_t groups = (pop2 + (int32_t)G * kWave - 1) / ((int32_t)G * kWave);
    for (int32_t g = 0; g < groups; ++g) {
      if (threadIdx.x < kWave) {
        const int32_t i = (int32_t)blockIdx.x + G * (g * kWave + lane);
        bool act = false;
        int32_t u = 0;
        if (i < pop2) {
          u = S2[i];
          act = FIRST || a.stamp[u] == round;
        }
        const uint64_t m = ballot(act);
        sh_u[lane] = u;
        if (lane == 0) *sh_mask = m;
      }
      __syncthreads();
      uint64_t m = *sh_mask;
      __syncthreads();
      while (m) {
        const int b = __ffsll((unsigned long long)m) - 1;
        m &= m - 1;
        upd_big<BLOCK>(a, s, sh_u[b], FIRST, round, st, red);
      }
      __syncthreads();
    }
  }
  // wavefront class: static list, 64 consecutive entries per wavefront
  {
    constexpr int NW = BLOCK / kWave;
    const int32_t* S1 = a.slist;
    const int32_t gw = blockIdx.x * NW + threadIdx.x / kWave;
    for (int32_t i0 = gw * kWave; i0 < pop1; i0 += G * NW * kWave) {
      const int32_t i = i0 + lane;
      int32_t u = 0;
      bool act = false;
      if (i < pop1) {
        u = S1[i];
        act = FIRST || a.stamp[u] == round;
      }
      uint64_t m = ballot(act);
      while (m) {
        const int b = __ffsll((unsigned long long)m) - 1;
        m &= m - 1;
        upd_wave(a, s, __shfl(u, b), FIRST, round, st);
      }
    }
  }
  // lane class: sweep of the vertex range of this workgroup
  {
    const int32_t lb = xcd_logical_block(blockIdx.x, G);
    const int64_t chunk = ((a.n + G - 1) / G + BLOCK - 1) / BLOCK * BLOCK;
    const int64_t v_end = min(a.n, (lb + 1) * chunk);
    for (int64_t v0 = lb * chunk; v0 < v_end; v0 += BLOCK) {
      const int64_t v = v0 + threadIdx.x;
      bool valid = false;
      if (v < v_end) {
        if (FIRST) {
          valid = a.cls[v] == 0;
        } else if (a.stamp[v] == round) {
          valid = a.cls[v] == 0;
        }
      }
      upd_lane(a, s, (int32_t)v, valid, FIRST, round, st);
    }
  }
}

// ------------------------------------------------------------------ tail
// One workgroup runs the remaining rounds on uncapped lists.  Within the
// workgroup, stores become visible to all its wavefronts at each barrier, so no
// launch is needed per round.
template <int BLOCK, typename Off>
__device__ __forceinline__ void run_tail(const Args<Off>& a, int32_t round, LaneStats& st, int32_t* red) {
  Ctl* ctl = a.ctl;
  const int tid = threadIdx.x;
  const int32_t p0 = ctl->pop[0], p1 = ctl->pop[1];
  if (tid < 4) {
    ctl->tail_cnt[0][tid] = 0;
    ctl->tail_cnt[1][tid] = 0;
  }
  __syncthreads();
  int32_t t = 0;
  for (;; ++t) {
    const int32_t r = round + t;
    const int32_t* cc = (t == 0) ? ctl->cnt[round % 3] : ctl->tail_cnt[t & 1];
    const int32_t n0 = ld_counter(cc + 0), n1 = ld_counter(cc + 1), n2 = ld_counter(cc + 2);
    if (n0 + n1 + n2 == 0) break;
    if (t >= kTailRoundCap) {
      if (tid == 0) ctl->error = 1;
      break;
    }
    const Sink s = make_sink(a, r + 1, ctl->tail_cnt[(t + 1) & 1], nullptr, false);
    sweep_lists<BLOCK>(a, s, list_of(a, r), n0, n1, n2, r, p0, p0 + p1, 0, 1, st, red);
    __syncthreads();
    if (t > 0 && tid < 4) ctl->tail_cnt[t & 1][tid] = 0;  // reused by round t+2
    __syncthreads();
  }
  if (tid < 4) {
    ctl->cnt[(round + 1) % 3][tid] = 0;
    ctl->cnt[(round + 2) % 3][tid] = 0;
    ctl->overflow[(round + 1) % 3][tid] = 0;
    ctl->overflow[(round + 2) % 3][tid] = 0;
  }
  if (tid == 0) {
    atomicAdd(&ctl->stats[ST_TAIL_ROUNDS], (unsigned long long)t);
    atomicAdd(&ctl->stats[ST_ROUNDS], (unsigned long long)t);
  }
}

// ------------------------------------------------------------------ kernels
// est = degree, degree class, class populations (one atomic per workgroup and class).
template <typename Off>
__global__ __launch_bounds__(256) void k_init(Args<Off> a) {
  __shared__ uint32_t part[3][256 / kWave];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  uint32_t p[3] = {0, 0, 0};
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += stride) {
    const int32_t d = (int32_t)(a.row_ptr[v + 1] - a.row_ptr[v]);
    a.est[v] = d;
    a.plen[v] = 0;
    const uint8_t c = d <= a.t1 ? 0 : (d <= a.t2 ? 1 : 2);
    a.cls[v] = c;
    p[c] += 1;
  }
  const int wave = threadIdx.x / kWave;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const uint32_t w = wave_sum(p[k]);
    if (lane_id() == 0) part[k][wave] = w;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    uint32_t t = 0;
    for (int w = 0; w < 256 / kWave; ++w) t += part[threadIdx.x][w];
    if (t) atomicAdd(&a.ctl->pop[threadIdx.x], (int32_t)t);
  }
}

// Static lists of the wavefront and workgroup classes.  Each workgroup owns a
// contiguous vertex range: a counting pass, one atomic per class, a writing pass.
template <typename Off>
__global__ __launch_bounds__(256) void k_seed(Args<Off> a) {
  int32_t* fill = a.ctl->seed_fill;
  constexpr int BLOCK = 256;
  __shared__ int32_t red[BLOCK / kWave];
  __shared__ int32_t base_sh[3];
  const int64_t chunk = (a.n + gridDim.x - 1) / gridDim.x;
  const int64_t v0 = (int64_t)blockIdx.x * chunk, v1 = min(a.n, v0 + chunk);
  int32_t mine[3] = {0, 0, 0};
  for (int64_t v = v0 + threadIdx.x; v < v1; v += BLOCK) {
    const int c = a.cls[v];
    mine[1] += c == 1;
    mine[2] += c == 2;
  }
  const int32_t pop1 = a.ctl->pop[1];
  for (int k = 1; k < 3; ++k) {
    int32_t total = 0;
    (void)block_excl_scan<BLOCK>(mine[k], total, red);
    if (threadIdx.x == 0) base_sh[k] = total ? atomicAdd(&fill[k], total) : 0;
  }
  __syncthreads();
  int32_t run[3] = {0, base_sh[1], base_sh[2]};
  for (int64_t vb = v0; vb < v1; vb += BLOCK) {
    const int64_t v = vb + threadIdx.x;
    const int c = v < v1 ? a.cls[v] : 0;
    for (int k = 1; k < 3; ++k) {
      int32_t total = 0;
      const int32_t off = block_excl_scan<BLOCK>(c == k ? 1 : 0, total, red);
      if (c == k) a.slist[(k == 2 ? pop1 : 0) + run[k] + off] = (int32_t)v;
      run[k] += total;
    }
  }
}

// One round (round number `round`).  FIRST: the dense first round over every
// vertex of degree >= 2.  Otherwise the round runs densely from the stamps when
// its sparse lists overflowed, else from the lists; a small list frontier is
// handed to the single-workgroup tail.
template <int BLOCK, bool FIRST, typename Off>
__global__ __launch_bounds__(BLOCK) void k_round(Args<Off> a, int32_t round, int32_t collect_stats) {
  __shared__ int32_t red[kHugeThresholds * (BLOCK / kWave)];
  __shared__ unsigned long long red64[kLaneStats * (BLOCK / kWave)];
  __shared__ int32_t sh_u[kWave];
  __shared__ unsigned long long sh_mask;
  Ctl* ctl = a.ctl;
  const int slot = round % 3;
  const bool dense = FIRST || ctl->overflow[slot][0] != 0;
  const int32_t n0 = ctl->cnt[slot][0], n1 = ctl->cnt[slot][1], n2 = ctl->cnt[slot][2];
  if (blockIdx.x == 0 && threadIdx.x < 4) {
    ctl->cnt[(round + 2) % 3][threadIdx.x] = 0;
    ctl->overflow[(round + 2) % 3][threadIdx.x] = 0;
  }
  LaneStats st;
  if (!dense) {
    const int32_t tot = n0 + n1 + n2;
    if (tot == 0) return;
    if (tot <= a.tail_threshold) {
      if (blockIdx.x == 0) {
        run_tail<BLOCK>(a, round, st, red);
        if (collect_stats) flush_stats<BLOCK>(ctl, st, red64);
      }
      return;
    }
  }
  const int nslot = (round + 1) % 3;
  const Sink s = make_sink(a, round + 1, ctl->cnt[nslot], &ctl->overflow[nslot][0], true);
  if (dense) {
    sweep_dense<BLOCK, FIRST>(a, s, round, st, red, sh_u, &sh_mask);
  } else {
    const int32_t p0 = ctl->pop[0], p1 = ctl->pop[1];
    sweep_lists<BLOCK>(a, s, list_of(a, round), n0, n1, n2, round, p0, p0 + p1, blockIdx.x, gridDim.x, st, red);
  }
  if (collect_stats) flush_stats<BLOCK>(ctl, st, red64);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    atomicAdd(&ctl->stats[ST_ROUNDS], 1ull);
    if (dense) atomicAdd(&ctl->stats[ST_DENSE_ROUNDS], 1ull);
  }
}

// Precondition check (only when requested): ids in range, no self-loops,
// strictly increasing rows (no duplicates), and symmetry by binary search.
// err[0] receives the smallest violated code (1 range, 2 loop, 3 order, 4 asymmetry).
template <typename Off>
__global__ void k_validate(int64_t n, const Off* row_ptr, const int32_t* col, int32_t* err) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const Off b = row_ptr[v], e = row_ptr[v + 1];
    if (e < b) {
      atomicMin(err, 3);
      continue;
    }
    for (Off j = b; j < e; ++j) {
      const int32_t u = col[j];
      if (u < 0 || u >= n) {
        atomicMin(err, 1);
        break;
      }
      if (u == v) {
        atomicMin(err, 2);
        break;
      }
      if (j > b && col[j - 1] >= u) {
        atomicMin(err, 3);
        break;
      }
      Off lo = row_ptr[u], hi = row_ptr[u + 1];
      bool found = false;
      while (lo < hi) {
        const Off mid = lo + (hi - lo) / 2;
        const int32_t w = col[mid];
        if (w == (int32_t)v) {
          found = true;
          break;
        }
        if (w < (int32_t)v) lo = mid + 1;
        else hi = mid;
      }
      if (!found) {
        atomicMin(err, 4);
        break;
      }
    }
  }
}

}  // namespace kcore
