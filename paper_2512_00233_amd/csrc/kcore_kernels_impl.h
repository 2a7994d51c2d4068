// Kernels of the iterative coreness computation (included by the runtime TU).  See kcore_kernels.h for the
// method, the citations and the GPU-specific design.
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

template <typename Off>
__device__ __forceinline__ int32_t* list_of(const Args<Off>& a, int32_t round) {
  return (round & 1) ? a.lists[1] : a.lists[0];  // select, not an indexed load from the argument struct
}

struct LaneStats {
  uint32_t updates = 0, changes = 0, acts = 0;
  uint64_t visits = 0;
};

// Region offsets of the three degree classes inside a frontier list.
struct Bases {
  int32_t b[3];
};
__device__ __forceinline__ Bases load_bases(const Ctl* ctl) {
  Bases B;
  int32_t p0 = ctl->pop[0], p1 = ctl->pop[1];
  B.b[0] = 0;
  B.b[1] = p0;
  B.b[2] = p0 + p1;
  return B;
}

// Where activated vertices go.
struct Sink {
  int32_t* list;  // next frontier list
  int32_t* cnt;   // its three class counters
  int32_t stamp;  // round number of the next frontier
  Bases B;
};

// Activate v (lanes with want=true) for the next round: deduplicate on the
// round stamp, then append to the list of v's degree class with one atomic per
// class per wavefront.  Every active lane of the wavefront must call this.
template <typename Off>
__device__ __forceinline__ void activate(const Args<Off>& a, const Sink& s, int32_t v, bool want, LaneStats& st) {
  bool first = false;
  int c = 0;
  if (want && a.stamp[v] < s.stamp) {
    first = atomicMax(&a.stamp[v], s.stamp) < s.stamp;
    if (first) c = a.cls[v];
  }
  uint64_t any = ballot(first);
  if (!any) return;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    bool p = first && c == k;
    uint64_t m = ballot(p);
    if (m) {
      int leader = __ffsll((unsigned long long)m) - 1;
      int b = 0;
      if (lane_id() == leader) b = atomicAdd(&s.cnt[k], popc(m));
      b = __shfl(b, leader);
      if (p) s.list[s.B.b[k] + b + lanes_below(m)] = v;
    }
  }
  st.acts += first;
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
__device__ __forceinline__ void upd_lane(const Args<Off>& a, const Sink& s, int32_t u, bool valid, bool dense, int32_t round,
                         LaneStats& st) {
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
    st.updates += 1;
    st.visits += (uint64_t)d;
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
      st.changes += 1;
    }
  }
  bool changed = valid && h < e;
  if (!ballot(changed)) return;
#pragma unroll
  for (int i = 0; i < kThreadMaxDeg; ++i) {
    bool w = changed && i < d && wants(a, c[i], x[i], e, h, dense, round);
    activate(a, s, c[i], w, st);
  }
}

// ------------------------------------------------------------------ wavefront path
// One 64-lane wavefront per vertex, degree <= 64 * kWaveRegs.
template <typename Off>
__device__ __forceinline__ void upd_wave(const Args<Off>& a, const Sink& s, int32_t u, bool dense, int32_t round, LaneStats& st) {
  const int lane = lane_id();
  const Off beg = a.row_ptr[u];
  const int32_t d = uni((int32_t)(a.row_ptr[u + 1] - beg));
  const int32_t e = uni(a.est[u]);
  if (e < 2) return;
  const int nr = (d + kWave - 1) / kWave;
  int32_t c[kWaveRegs], x[kWaveRegs];
#pragma unroll
  for (int i = 0; i < kWaveRegs; ++i) {
    int j = lane + kWave * i;
    c[i] = 0;
    if (i < nr && j < d) c[i] = a.col[beg + j];
  }
#pragma unroll
  for (int i = 0; i < kWaveRegs; ++i) {
    int j = lane + kWave * i;
    x[i] = 0;
    if (i < nr && j < d) x[i] = a.est[c[i]];
  }
  auto count = [&](int32_t k) {
    int tot = 0;
#pragma unroll
    for (int i = 0; i < kWaveRegs; ++i)
      if (i < nr) tot += popc(ballot(x[i] >= k));
    return tot;
  };
  if (lane == 0) {
    st.updates += 1;
    st.visits += (uint64_t)d;
  }
  int32_t h = e;
  if (count(e) < e) {
    int32_t lo = 1, hi = e - 1;  // count(1) = d >= 1 always holds
    while (lo < hi) {
      int32_t mid = (lo + hi + 1) >> 1;
      if (count(mid) >= mid) lo = mid;
      else hi = mid - 1;
    }
    h = lo;
    if (lane == 0) {
      a.est[u] = h;
      st.changes += 1;
    }
  }
  if (h == e) return;
#pragma unroll
  for (int i = 0; i < kWaveRegs; ++i) {
    if (i < nr) {
      bool w = (lane + kWave * i < d) && wants(a, c[i], x[i], e, h, dense, round);
      activate(a, s, c[i], w, st);
    }
  }
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

// One workgroup per vertex, degree <= BLOCK * kBlockRegs: values in registers,
// binary search on k with wavefront ballots.
template <int BLOCK, typename Off>
__device__ __forceinline__ void upd_block(const Args<Off>& a, const Sink& s, int32_t u, bool dense, int32_t round, LaneStats& st,
                          int32_t* red) {
  const int tid = threadIdx.x;
  const Off beg = a.row_ptr[u];
  const int32_t d = uni((int32_t)(a.row_ptr[u + 1] - beg));
  const int32_t e = uni(a.est[u]);
  if (e < 2) return;
  const int nr = (d + BLOCK - 1) / BLOCK;
  int32_t c[kBlockRegs], x[kBlockRegs];
#pragma unroll
  for (int i = 0; i < kBlockRegs; ++i) {
    int j = tid + BLOCK * i;
    c[i] = 0;
    if (i < nr && j < d) c[i] = a.col[beg + j];
  }
#pragma unroll
  for (int i = 0; i < kBlockRegs; ++i) {
    int j = tid + BLOCK * i;
    x[i] = 0;
    if (i < nr && j < d) x[i] = a.est[c[i]];
  }
  auto count = [&](int32_t k) {
    int tot = 0;
#pragma unroll
    for (int i = 0; i < kBlockRegs; ++i)
      if (i < nr) tot += popc(ballot(x[i] >= k));
    return block_sum_waves<BLOCK>(tot, red);
  };
  if (tid == 0) {
    st.updates += 1;
    st.visits += (uint64_t)d;
  }
  int32_t h = e;
  if (count(e) < e) {
    int32_t lo = 1, hi = e - 1;
    while (lo < hi) {
      int32_t mid = (lo + hi + 1) >> 1;
      if (count(mid) >= mid) lo = mid;
      else hi = mid - 1;
    }
    h = lo;
    if (tid == 0) {
      a.est[u] = h;
      st.changes += 1;
    }
  }
  if (h == e) return;
#pragma unroll
  for (int i = 0; i < kBlockRegs; ++i) {
    if (i < nr) {
      bool w = (tid + BLOCK * i < d) && wants(a, c[i], x[i], e, h, dense, round);
      activate(a, s, c[i], w, st);
    }
  }
}

// One workgroup per vertex of any degree: the answer interval [lo, hi] is cut
// into kHugeThresholds pieces per pass over the adjacency (re-read each pass),
// counting neighbours at or above each threshold.
template <int BLOCK, typename Off>
__device__ __forceinline__ void upd_huge(const Args<Off>& a, const Sink& s, int32_t u, bool dense, int32_t round, LaneStats& st,
                         int32_t* red) {
  constexpr int S = kHugeThresholds;
  constexpr int NW = BLOCK / kWave;
  const int tid = threadIdx.x;
  const Off beg = a.row_ptr[u];
  const int32_t d = uni((int32_t)(a.row_ptr[u + 1] - beg));
  const int32_t e = uni(a.est[u]);
  if (e < 2) return;
  if (tid == 0) {
    st.updates += 1;
    st.visits += (uint64_t)d;
  }
  // invariant: h in [lo, hi] and count(lo) >= lo
  int32_t lo = 1, hi = e;
  while (lo < hi) {
    // thresholds thr(0) < ... < thr(S-1) == hi split (lo, hi]; INT32_MAX marks unused slots
    const int64_t span = (int64_t)hi - lo;
    auto thr = [&](int q) -> int32_t {
      if (span >= S) return (int32_t)(lo + ((int64_t)(q + 1) * span + S - 1) / S);
      return (q < span) ? lo + 1 + q : INT32_MAX;
    };
    int32_t cnt[S];
#pragma unroll
    for (int q = 0; q < S; ++q) cnt[q] = 0;
    for (int32_t j = tid; j < d; j += BLOCK) {
      int32_t xv = a.est[a.col[beg + j]];
#pragma unroll
      for (int q = 0; q < S; ++q) cnt[q] += xv >= thr(q);
    }
    const int wave = tid / kWave;
#pragma unroll
    for (int q = 0; q < S; ++q) {
      int32_t w = wave_sum(cnt[q]);
      if (lane_id() == 0) red[q * NW + wave] = w;
    }
    __syncthreads();
    int32_t best = -1;
#pragma unroll
    for (int q = 0; q < S; ++q) {
      int32_t tot = 0;
#pragma unroll
      for (int w = 0; w < NW; ++w) tot += red[q * NW + w];
      const int32_t tq = thr(q);
      if (tq != INT32_MAX && tot >= tq) best = q;  // count(k) - k is decreasing: the last hit is the largest
    }
    __syncthreads();
    best = uni(best);
    if (best < 0) {
      hi = thr(0) - 1;
    } else {
      const int32_t nlo = thr(best);
      if (best + 1 < S && thr(best + 1) != INT32_MAX) hi = thr(best + 1) - 1;
      lo = nlo;
    }
  }
  const int32_t h = lo;
  if (h == e) return;
  if (tid == 0) {
    a.est[u] = h;
    st.changes += 1;
  }
  for (int32_t j0 = 0; j0 < d; j0 += BLOCK) {
    int32_t j = j0 + tid;
    bool w = false;
    int32_t v = 0;
    if (j < d) {
      v = a.col[beg + j];
      w = wants(a, v, a.est[v], e, h, dense, round);
    }
    activate(a, s, v, w, st);
  }
}

template <int BLOCK, typename Off>
__device__ __forceinline__ void upd_big(const Args<Off>& a, const Sink& s, int32_t u, bool dense, int32_t round,
                                        LaneStats& st, int32_t* red) {
  const int32_t d = uni((int32_t)(a.row_ptr[u + 1] - a.row_ptr[u]));
  if (d <= a.t3) upd_block<BLOCK>(a, s, u, dense, round, st, red);
  else upd_huge<BLOCK>(a, s, u, dense, round, st, red);
}

// ------------------------------------------------------------------ statistics
template <int BLOCK>
__device__ __forceinline__ void flush_stats(Ctl* ctl, const LaneStats& st, unsigned long long* red64) {
  constexpr int NW = BLOCK / kWave;
  const int wave = threadIdx.x / kWave;
  unsigned long long v[4] = {st.updates, st.visits, st.changes, st.acts};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    unsigned long long w = wave_sum(v[q]);
    if (lane_id() == 0) red64[q * NW + wave] = w;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    unsigned long long t = 0;
    for (int w = 0; w < NW; ++w) t += red64[threadIdx.x * NW + w];
    if (t) atomicAdd(&ctl->stats[ST_UPDATES + threadIdx.x], t);
  }
}

// ------------------------------------------------------------------ tail
// One workgroup runs the remaining rounds.  Within the workgroup, stores become
// visible to all its wavefronts at each barrier, so no launch is needed per round.
template <int BLOCK, typename Off>
__device__ __forceinline__ void run_tail(const Args<Off>& a, int32_t round, LaneStats& st, int32_t* red) {
  Ctl* ctl = a.ctl;
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  constexpr int NW = BLOCK / kWave;
  const Bases B = load_bases(ctl);
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
    const int32_t* cur = list_of(a, r);
    Sink s{list_of(a, r + 1), ctl->tail_cnt[(t + 1) & 1], r + 1, B};
    for (int32_t i = 0; i < n2; ++i) upd_big<BLOCK>(a, s, cur[B.b[2] + i], false, r, st, red);
    for (int32_t i = wave; i < n1; i += NW) upd_wave(a, s, cur[B.b[1] + i], false, r, st);
    for (int32_t i = tid; i - lane_id() < n0; i += BLOCK) {
      bool valid = i < n0;
      upd_lane(a, s, valid ? cur[i] : 0, valid, false, r, st);
    }
    __syncthreads();
    if (t > 0 && tid < 4) ctl->tail_cnt[t & 1][tid] = 0;  // reused by round t+2
    __syncthreads();
  }
  if (tid < 4) {
    ctl->cnt[(round + 1) % 3][tid] = 0;
    ctl->cnt[(round + 2) % 3][tid] = 0;
  }
  if (tid == 0) {
    atomicAdd(&ctl->stats[ST_TAIL_ROUNDS], (unsigned long long)t);
    atomicAdd(&ctl->stats[ST_ROUNDS], (unsigned long long)t);
  }
}

// ------------------------------------------------------------------ kernels
// Workgroup id -> logical id such that consecutive logical ids (consecutive
// vertex ranges in the dense sweep) land on the same XCD (workgroups are
// dispatched round-robin over the 8 XCDs).
__device__ __forceinline__ int32_t xcd_logical_block(int32_t b, int32_t G) {
  constexpr int X = 8;
  if (G % X != 0) return b;
  return (b % X) * (G / X) + b / X;
}

// est = degree, degree class, class populations.
template <typename Off>
__global__ void k_init(Args<Off> a) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  uint32_t p[3] = {0, 0, 0};
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += stride) {
    int32_t d = (int32_t)(a.row_ptr[v + 1] - a.row_ptr[v]);
    a.est[v] = d;
    uint8_t c = d <= a.t1 ? 0 : (d <= a.t2 ? 1 : 2);
    const_cast<uint8_t*>(a.cls)[v] = c;
    p[c] += 1;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    uint32_t w = wave_sum(p[k]);
    if (lane_id() == 0 && w) atomicAdd(&a.ctl->pop[k], (int32_t)w);
  }
}

// Seed the first (dense) round: vertices of the wavefront and workgroup classes
// with degree >= 2 go to the round's lists; the lane class is swept implicitly.
template <typename Off>
__global__ void k_seed(Args<Off> a, int32_t round) {
  const Bases B = load_bases(a.ctl);
  int32_t* list = list_of(a, round);
  int32_t* cnt = a.ctl->cnt[round % 3];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v0 = (int64_t)blockIdx.x * blockDim.x; v0 < a.n; v0 += stride) {
    int64_t v = v0 + threadIdx.x;
    int c = v < a.n ? a.cls[v] : 0;
#pragma unroll
    for (int k = 1; k < 3; ++k) {
      bool p = c == k;
      uint64_t m = ballot(p);
      if (m) {
        int leader = __ffsll((unsigned long long)m) - 1;
        int b = 0;
        if (lane_id() == leader) b = atomicAdd(&cnt[k], popc(m));
        b = __shfl(b, leader);
        if (p) list[B.b[k] + b + lanes_below(m)] = (int32_t)v;
      }
    }
  }
}

// One round over the current frontier (round number `round`).  DENSE: the
// first round, where the lane class is every vertex of degree >= 2.
template <int BLOCK, bool DENSE, typename Off>
__global__ __launch_bounds__(BLOCK) void k_round(Args<Off> a, int32_t round) {
  __shared__ int32_t red[kHugeThresholds * (BLOCK / kWave)];
  __shared__ unsigned long long red64[4 * (BLOCK / kWave)];
  Ctl* ctl = a.ctl;
  const int32_t* cc = ctl->cnt[round % 3];
  const int32_t n0 = DENSE ? 0 : cc[0];
  const int32_t n1 = cc[1], n2 = cc[2];
  if (blockIdx.x == 0 && threadIdx.x < 4) ctl->cnt[(round + 2) % 3][threadIdx.x] = 0;
  LaneStats st;
  if (!DENSE) {
    const int32_t tot = n0 + n1 + n2;
    if (tot == 0) return;
    if (tot <= a.tail_threshold) {
      if (blockIdx.x == 0) {
        run_tail<BLOCK>(a, round, st, red);
        flush_stats<BLOCK>(ctl, st, red64);
      }
      return;
    }
  }
  const Bases B = load_bases(ctl);
  const int32_t* cur = list_of(a, round);
  Sink s{list_of(a, round + 1), ctl->cnt[(round + 1) % 3], round + 1, B};
  const int32_t G = gridDim.x;
  // workgroup class
  for (int32_t i = blockIdx.x; i < n2; i += G) upd_big<BLOCK>(a, s, cur[B.b[2] + i], DENSE, round, st, red);
  // wavefront class
  {
    constexpr int NW = BLOCK / kWave;
    const int32_t gw = blockIdx.x * NW + threadIdx.x / kWave;
    for (int32_t i = gw; i < n1; i += G * NW) upd_wave(a, s, cur[B.b[1] + i], DENSE, round, st);
  }
  // lane class
  if (DENSE) {
    const int32_t lb = xcd_logical_block(blockIdx.x, G);
    const int64_t chunk = ((a.n + G - 1) / G + BLOCK - 1) / BLOCK * BLOCK;
    const int64_t v_end = min(a.n, (lb + 1) * chunk);
    for (int64_t v0 = lb * chunk; v0 < v_end; v0 += BLOCK) {
      int64_t v = v0 + threadIdx.x;
      bool valid = v < v_end && a.cls[v] == 0;
      upd_lane(a, s, (int32_t)v, valid, true, round, st);
    }
  } else {
    const int32_t T = G * BLOCK;
    for (int32_t i = blockIdx.x * BLOCK + threadIdx.x; i - lane_id() < n0; i += T) {
      bool valid = i < n0;
      upd_lane(a, s, valid ? cur[i] : 0, valid, false, round, st);
    }
  }
  flush_stats<BLOCK>(ctl, st, red64);
  if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&ctl->stats[ST_ROUNDS], 1ull);
}

// Precondition check (only when requested): ids in range, no self-loops,
// strictly increasing rows (no duplicates), and symmetry by binary search.
// err[0] receives the smallest violated code (1 range, 2 loop, 3 order, 4 asymmetry).
template <typename Off>
__global__ void k_validate(int64_t n, const Off* row_ptr, const int32_t* col, int32_t* err) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    Off b = row_ptr[v], e = row_ptr[v + 1];
    if (e < b) { atomicMin(err, 3); continue; }
    for (Off j = b; j < e; ++j) {
      int32_t u = col[j];
      if (u < 0 || u >= n) { atomicMin(err, 1); break; }
      if (u == v) { atomicMin(err, 2); break; }
      if (j > b && col[j - 1] >= u) { atomicMin(err, 3); break; }
      Off lo = row_ptr[u], hi = row_ptr[u + 1];
      bool found = false;
      while (lo < hi) {
        Off mid = lo + (hi - lo) / 2;
        int32_t w = col[mid];
        if (w == (int32_t)v) { found = true; break; }
        if (w < (int32_t)v) lo = mid + 1;
        else hi = mid;
      }
      if (!found) { atomicMin(err, 4); break; }
    }
  }
}

}  // namespace kcore
