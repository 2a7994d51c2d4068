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
__device__ __forceinline__ int32_t wave_max(int32_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ int32_t wave_min(int32_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ int32_t wave_incl_scan(int32_t x) {
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int32_t t = __shfl_up(x, o);
    if (lane >= o) x += t;
  }
  return x;
}

template <typename Off>
__device__ __forceinline__ int32_t* list_of(const Args<Off>& a, int32_t round) {
  return (round & 1) ? a.lists[1] : a.lists[0];  // select, not an indexed load from the argument struct
}

__device__ __forceinline__ void region_bases(const Ctl* ctl, int32_t (&b)[kClasses]) {
  int32_t acc = 0;
#pragma unroll
  for (int k = 0; k < kClasses; ++k) {
    b[k] = acc;
    acc += ctl->pop[k];
  }
}

struct LaneStats {
  uint64_t v[kLaneStats] = {0, 0, 0, 0, 0, 0};
};

// Where activated vertices go.
struct Sink {
  int32_t* list;      // next frontier list
  int32_t* cnt;       // its class counters
  int32_t* overflow;  // flag of the next round (nullptr: uncapped, never overflows)
  int32_t stamp;      // round number of the next frontier
  int32_t b[kClasses];
  int32_t cap[kClasses];
  int32_t* dcnt;      // this workgroup's deferred-check counter (nullptr: re-activate instead)
  int32_t dbase;      // first triple of its buffer region
  int32_t dcap;       // triples in the region
  uint8_t* dirty;     // dirty-piece marks of the next round (nullptr: none kept)
};

template <typename Off>
__device__ __forceinline__ Sink make_sink(const Args<Off>& a, int32_t next_round, int32_t* cnt, int32_t* overflow,
                                          bool capped) {
  Sink s;
  s.list = list_of(a, next_round);
  s.cnt = cnt;
  s.overflow = overflow;
  s.stamp = next_round;
  s.dcnt = nullptr;
  s.dbase = 0;
  s.dcap = 0;
  s.dirty = a.dirty ? a.dirty + (next_round & 1) * a.dirty_pieces : nullptr;
  region_bases(a.ctl, s.b);
#pragma unroll
  for (int k = 0; k < kClasses; ++k) s.cap[k] = capped ? min(a.ctl->pop[k], a.list_cap) : a.ctl->pop[k];
  return s;
}

// The current vertex dropped from e to h; up to N neighbours per lane (ids v,
// estimates x read in this round, valid where `in`) are candidates for the
// next round.  Neighbour v needs a recomputation only if the current vertex
// was counted in v's support at v's level x (x <= e) and no longer is (x > h).
// v keeps its support slack (support at its level minus the level, set when v
// was last recomputed): the loss is subtracted, and v is activated only when
// the slack goes negative.
// A vertex of the current frontier is updated in this round too.  Class-3
// vertices are updated by the class-3 kernel, the others by the classes-0..2
// kernel; one of the two completes before the other starts (kBigFirst; in the
// tail the same order holds behind a barrier).  So, with BIG telling which
// kernel the current vertex belongs to:
//  * v updated by the same kernel may have read the old value of the current
//    vertex, and x may be stale: v is re-activated;
//  * v updated by the later kernel (the current one runs first): v reads the
//    new value, nothing to do;
//  * v updated by the earlier kernel: v's update is done, x is its new value
//    and its slack counts the current vertex's old value: the exact rule applies.
// A vertex already activated for the next round needs nothing.  In the first
// round (dense) and in one-sided mode every candidate with x > h is activated.
// Winners of the round-stamp dedup (atomicMax) are appended to the list of
// their degree class with one atomic per class per wavefront, unless the next
// round already rebuilds its lists by compaction (then the stamps are plain
// stores and the activation count includes repeats).
// Loads and atomics of a lane are issued together at each step.  Every active
// lane of the wavefront must call this.
template <int N, bool BIG, typename Off>
__device__ __forceinline__ void activate_changed(const Args<Off>& a, const Sink& s, int32_t (&v)[N],
                                                 const int32_t (&x)[N], const bool (&in)[N], int32_t e, int32_t h,
                                                 bool dense, int32_t round, LaneStats& st, int32_t gb, uint32_t cb) {
  const bool always = a.one_sided || dense;
  // cb holds each neighbour's class (2 bits each, from its estimate word).  A
  // neighbour updated by the other kernel, read above e, needs nothing, under
  // either rule and in any round: if that kernel runs later it reads the new
  // value, otherwise x is already its value for the round (nothing updates it
  // concurrently), and the current vertex was never counted at that level.  Its
  // stamp is not even read.  In the first round every class-3 vertex is in the
  // next frontier already (k_big), so the classes-0..2 kernel skips them all.
  bool cand[N];
  bool any = false;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const bool other = (((cb >> (2 * i)) & 3u) == 3u) != BIG;
    const bool skip = other && (x[i] > e || (!BIG && dense && kBigFirst));
    cand[i] = in[i] && x[i] > h && !skip;
    any |= cand[i];
  }
  if (!ballot(any)) return;
  const bool compact_next = s.overflow && *(volatile int32_t*)s.overflow;
  if (always && compact_next) {
    // every candidate is activated and the next round's lists come from the
    // stamps: plain stores (all writers of this round store the same value)
#pragma unroll
    for (int i = 0; i < N; ++i)
      if (cand[i]) {
        a.stamp[v[i]] = s.stamp;
        if (s.dirty) s.dirty[v[i] >> kCompactPieceShift] = 1;
      }
    uint32_t nc = 0;
#pragma unroll
    for (int i = 0; i < N; ++i) nc += cand[i];
    st.v[ST_ACTIVATIONS] += nc;
    if (a.gact && nc) a.gact[gb] = s.stamp;
    return;
  }
  int32_t sv[N], cv[N];
#pragma unroll
  for (int i = 0; i < N; ++i) sv[i] = cand[i] ? a.stamp[v[i]] : INT32_MAX;
  // the class tells frontier members' kernel and winners' list
#pragma unroll
  for (int i = 0; i < N; ++i) cv[i] = (int32_t)((cb >> (2 * i)) & 3u);
  uint32_t want = 0, sub = 0, dfr = 0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    if (!cand[i] || sv[i] >= s.stamp) continue;  // not a candidate, or already in the next frontier
    bool w = false, d = false, q = false;
    if (always) w = true;
    else if (sv[i] == round && (cv[i] == 3) == BIG) (s.dcnt ? q : w) = true;  // same kernel
    else if (sv[i] == round && BIG == kBigFirst) w = false;  // v's kernel runs after this one
    else if (x[i] <= e) d = true;
    want |= (w ? 1u : 0u) << i;
    sub |= (d ? 1u : 0u) << i;
    dfr |= (q ? 1u : 0u) << i;
  }
  const int lane = lane_id();
  // A neighbour updated in this same kernel may have read the old value e.  Its
  // check is deferred until the kernel is over (k_defer): then its level is
  // final, and the drop matters only if it crossed that level, which the
  // neighbour's slack decides.  Past the buffer's capacity it is re-activated.
  if (s.dcnt && ballot(dfr != 0)) {
    const int32_t mine = __popc(dfr);
    const int32_t incl = wave_incl_scan(mine);
    const int32_t tot = __shfl(incl, kWave - 1);
    int32_t base = 0;
    if (lane == kWave - 1) base = atomicAdd(s.dcnt, tot);
    base = __shfl(base, kWave - 1);
    int32_t pos = base + incl - mine;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      if (dfr >> i & 1u) {
        if (pos < s.dcap) {
          int32_t* t = a.defer + 3 * ((int64_t)s.dbase + pos);
          t[0] = v[i];
          t[1] = e;
          t[2] = h;
        } else {
          want |= 1u << i;
        }
        ++pos;
      }
    }
  }
  int32_t p[N];
#pragma unroll
  for (int i = 0; i < N; ++i) p[i] = (sub >> i & 1u) ? atomicSub(&a.slack[v[i]], 1) : 1;
#pragma unroll
  for (int i = 0; i < N; ++i) want |= ((sub >> i & 1u) && p[i] <= 0 ? 1u : 0u) << i;
  if (compact_next) {
    // the next round's lists come from the stamps: no dedup needed, plain stores
#pragma unroll
    for (int i = 0; i < N; ++i)
      if (want >> i & 1u) {
        a.stamp[v[i]] = s.stamp;
        if (s.dirty) s.dirty[v[i] >> kCompactPieceShift] = 1;
      }
    st.v[ST_ACTIVATIONS] += __popc(want);
    if (a.gact && want) a.gact[gb] = s.stamp;
    return;
  }
#pragma unroll
  for (int i = 0; i < N; ++i) p[i] = (want >> i & 1u) ? atomicMax(&a.stamp[v[i]], s.stamp) : INT32_MAX;
  uint32_t first = 0;
#pragma unroll
  for (int i = 0; i < N; ++i) first |= (p[i] < s.stamp ? 1u : 0u) << i;
  st.v[ST_ACTIVATIONS] += __popc(first);
  // the next round may still overflow its lists and rebuild them from the stamps
  if (s.dirty) {
#pragma unroll
    for (int i = 0; i < N; ++i)
      if (first >> i & 1u) s.dirty[v[i] >> kCompactPieceShift] = 1;
  }
  // served graphs: the graph has work in the next round (all candidates share the current vertex's graph)
  if (a.gact && first) a.gact[gb] = s.stamp;
  if (!ballot(first != 0)) return;
#pragma unroll
  for (int i = 0; i < N; ++i) p[i] = (first >> i & 1u) ? cv[i] : kClasses;  // class of winners
#pragma unroll
  for (int k = 0; k < kClasses; ++k) {
    int32_t mine = 0;
#pragma unroll
    for (int i = 0; i < N; ++i) mine += p[i] == k;
    if (!ballot(mine != 0)) continue;  // no winner of this class in the wavefront
    const int32_t incl = wave_incl_scan(mine);
    const int32_t tot = __shfl(incl, kWave - 1);
    if (tot == 0) continue;
    int32_t base = 0;
    if (lane == kWave - 1) base = atomicAdd(&s.cnt[k * kCtr], tot);
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

// ------------------------------------------------------------------ k-ary search over register values
// Each group of G lanes holds R values per lane.  Returns, per group, the
// largest k in [lo, e] with |{values >= k}| >= k (and that count in `count`),
// or lo - 1 when the count at lo is below lo (possible only when the caller
// does not know count(lo) >= lo).
// Pass 1 tests e, e-1, e-3, ... (kKary - 1 of them) and lo; later passes cut the
// remaining interval into kKary pieces.  Every lane of the wavefront must call this.
template <int G, int R>
__device__ __forceinline__ int32_t kary_regs(const int32_t (&x)[R], int32_t e, int32_t lo, bool active,
                                             int32_t& count) {
  constexpr int S = kKary;
  const int lane = lane_id();
  const uint64_t gm = (G == kWave) ? ~0ull : (((1ull << G) - 1) << (lane & ~(G - 1)));
  int32_t hi = e, res = lo - 1, clo = 0;
  bool done = !active, first = true;
  while (ballot(!done)) {
    int32_t t[S];
    if (first) {
#pragma unroll
      for (int q = 0; q < S - 1; ++q) t[q] = max(lo, e - ((1 << q) - 1));
      t[S - 1] = lo;
    } else {
      const int32_t span = hi - lo;
      const int32_t step = (span + S - 1) / S;
#pragma unroll
      for (int q = 0; q < S; ++q) t[q] = lo + (int32_t)min((int64_t)span, (int64_t)(q + 1) * step);
    }
    int32_t c[S];
#pragma unroll
    for (int q = 0; q < S; ++q) c[q] = 0;
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int q = 0; q < S; ++q) c[q] += popc(ballot(x[r] >= t[q]) & gm);
    if (!done) {
      if (first) {
        int qs = -1;  // thresholds descend: the first hit is the largest satisfied value
#pragma unroll
        for (int q = S - 1; q >= 0; --q)
          if (c[q] >= t[q]) qs = q;
        if (qs < 0) {
          done = true;
        } else {
          int32_t nhi = e, nlo = t[0], nc = c[0];
#pragma unroll
          for (int q = 1; q < S; ++q)
            if (q == qs) {
              nhi = t[q - 1] - 1;
              nlo = t[q];
              nc = c[q];
            }
          lo = nlo;
          hi = nhi;
          clo = nc;
        }
        first = false;
      } else {
        int qs = -1;  // thresholds ascend: the last hit is the largest satisfied value
#pragma unroll
        for (int q = 0; q < S; ++q)
          if (c[q] >= t[q]) qs = q;
        if (qs < 0) {
          hi = t[0] - 1;
        } else {
          int32_t nlo = t[0], nhi = hi, nc = c[0];
#pragma unroll
          for (int q = 0; q < S; ++q) {
            if (q == qs) {
              nlo = t[q];
              nc = c[q];
            }
            if (q == qs + 1) nhi = t[q] - 1;
          }
          lo = nlo;
          hi = nhi;
          clo = nc;
        }
      }
      if (!done && lo >= hi) {
        res = lo;
        done = true;
      }
    }
  }
  count = clo;
  return res;
}

// ------------------------------------------------------------------ class 0: lane per vertex
template <bool BATCH, typename Off>
__device__ __forceinline__ void upd_lane(const Args<Off>& a, const Sink& s, int32_t u, bool valid, bool dense,
                                         int32_t round, LaneStats& st) {
  int32_t e = 0, d = 0, gb = 0;
  Off beg = 0;
  if (valid) {
    beg = a.row_ptr[u];
    d = (int32_t)(a.row_ptr[u + 1] - beg);
    e = est_val(a.est[u]);
    if (BATCH) gb = a.vbase[u];
  }
  valid = valid && e >= 2;  // an estimate of 1 is final: every non-isolated vertex has coreness >= 1
  int32_t c[kLaneMaxDeg], x[kLaneMaxDeg];
#pragma unroll
  for (int i = 0; i < kLaneMaxDeg; ++i) c[i] = (valid && i < d) ? gb + a.col[beg + i] : 0;
#pragma unroll
  for (int i = 0; i < kLaneMaxDeg; ++i) x[i] = (valid && i < d) ? a.est[c[i]] : 0;
  uint32_t cb = 0;
#pragma unroll
  for (int i = 0; i < kLaneMaxDeg; ++i) {
    cb |= (uint32_t)est_cls(x[i]) << (2 * i);
    x[i] = est_val(x[i]);
  }
  int32_t h = e;
  if (valid) {
    st.v[ST_UPDATES] += 1;
    st.v[ST_VISITS] += (uint64_t)d;
    int cnt = 0;
#pragma unroll
    for (int i = 0; i < kLaneMaxDeg; ++i) cnt += x[i] >= e;
    if (cnt < e) {
      h = 1;
      cnt = d;  // every neighbour of a vertex of degree >= 1 has an estimate >= 1
      for (int k = e - 1; k >= 2; --k) {
        int sk = 0;
#pragma unroll
        for (int i = 0; i < kLaneMaxDeg; ++i) sk += x[i] >= k;
        if (sk >= k) {
          h = k;
          cnt = sk;
          break;
        }
      }
      a.est[u] = est_enc(h, 0);
      st.v[ST_CHANGES] += 1;
    }
    a.slack[u] = cnt - h;
  }
  const bool changed = valid && h < e;
  bool in[kLaneMaxDeg];
#pragma unroll
  for (int i = 0; i < kLaneMaxDeg; ++i) in[i] = changed && i < d;
  activate_changed<kLaneMaxDeg, false>(a, s, c, x, in, e, h, dense, round, st, gb, cb);
}

// Threshold of a pruned list built after a full scan that gave h: neighbours
// whose estimate is at least this are kept.
__device__ __forceinline__ int32_t prune_low(int32_t h) { return max(2, h - (h * kPruneMarginNum) / kPruneMarginDen); }
// The same for class-3 lists built in the first round.
__device__ __forceinline__ int32_t prune_low_first(int32_t h) { return max(2, h - h / kPruneFirstMarginDen); }

// ------------------------------------------------------------------ class 1: 16-lane group per vertex
template <bool BATCH, typename Off>
__device__ __forceinline__ void upd_group(const Args<Off>& a, const Sink& s, int32_t u, bool valid, bool dense,
                                          int32_t round, LaneStats& st) {
  constexpr int G = kGroupLanes, R = kGroupRegs;
  const int gl = lane_id() & (G - 1);
  int32_t e = 0, d = 0, gb = 0;
  Off beg = 0;
  if (valid) {
    beg = a.row_ptr[u];
    d = (int32_t)(a.row_ptr[u + 1] - beg);
    e = est_val(a.est[u]);
    if (BATCH) gb = a.vbase[u];
  }
  valid = valid && e >= 2;
  int32_t c[R], x[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = gl + G * r;
    c[r] = (valid && j < d) ? gb + a.col[beg + j] : 0;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) x[r] = (valid && gl + G * r < d) ? a.est[c[r]] : 0;
  uint32_t cb = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    cb |= (uint32_t)est_cls(x[r]) << (2 * r);
    x[r] = est_val(x[r]);
  }
  if (valid && gl == 0) {
    st.v[ST_UPDATES] += 1;
    st.v[ST_VISITS] += (uint64_t)d;
  }
  int32_t cnt = 0;
  const int32_t h = kary_regs<G, R>(x, e, 1, valid, cnt);
  const bool changed = valid && h < e;
  if (changed && gl == 0) {
    a.est[u] = est_enc(h, 1);
    st.v[ST_CHANGES] += 1;
  }
  if (valid && gl == 0) a.slack[u] = cnt - h;
  bool in[R];
#pragma unroll
  for (int r = 0; r < R; ++r) in[r] = changed && (gl + G * r < d);
  activate_changed<R, false>(a, s, c, x, in, e, h, dense, round, st, gb, cb);
}

// ------------------------------------------------------------------ class 2: wavefront per vertex
// Searches its pruned list first when it has one.
template <bool BATCH, typename Off>
__device__ __forceinline__ void upd_wave(const Args<Off>& a, const Sink& s, int32_t u, bool dense, int32_t round,
                                         LaneStats& st) {
  constexpr int R = kWaveRegs;
  const int lane = lane_id();
  const Off beg = a.row_ptr[u];
  const int32_t d = uni((int32_t)(a.row_ptr[u + 1] - beg));
  const int32_t e = uni(est_val(a.est[u]));
  if (e < 2) return;
  const int32_t gb = BATCH ? uni(a.vbase[u]) : 0;
  const int32_t pl = a.prune ? uni(a.plen[u]) : 0;
  const int32_t L = pl > 0 ? uni(a.plow[u]) : 1;
  int32_t c[R], x[R];
  uint32_t cb = 0;  // neighbour classes, 2 bits each
  int32_t len = 0;
  auto load = [&](const int32_t* src, int32_t n_, int32_t off) {
    len = n_;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int j = lane + kWave * i;
      c[i] = (kWave * i < n_ && j < n_) ? off + src[beg + j] : 0;
    }
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int j = lane + kWave * i;
      x[i] = (kWave * i < n_ && j < n_) ? a.est[c[i]] : 0;
    }
    cb = 0;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      cb |= (uint32_t)est_cls(x[i]) << (2 * i);
      x[i] = est_val(x[i]);
    }
  };
  if (lane == 0) st.v[ST_UPDATES] += 1;
  int32_t h = -1, cnt = 0;
  if (pl > 0) {
    load(a.pruned, pl, 0);
    if (lane == 0) st.v[ST_VISITS] += pl;
    const int32_t hp = kary_regs<kWave, R>(x, e, L, true, cnt);
    if (hp >= L) h = hp;
  }
  if (h < 0) {
    load(a.col, d, gb);
    if (lane == 0) {
      st.v[ST_VISITS] += d;
      st.v[ST_FULL_SCANS] += 1;
    }
    h = kary_regs<kWave, R>(x, e, 1, true, cnt);
    if (a.prune) {
      const int32_t L2 = prune_low(h);
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
  if (lane == 0) a.slack[u] = cnt - h;
  if (h == e) return;
  if (lane == 0) {
    a.est[u] = est_enc(h, 2);
    st.v[ST_CHANGES] += 1;
  }
  bool in[R];
#pragma unroll
  for (int i = 0; i < R; ++i) in[i] = lane + kWave * i < len;
  activate_changed<R, false>(a, s, c, x, in, e, h, dense, round, st, gb, cb);
}

// ------------------------------------------------------------------ class 3: workgroup per vertex
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

// Workgroup version of kary_regs (the whole workgroup is one group); red holds
// kKary * (BLOCK / 64) ints.
template <int BLOCK, int R>
__device__ __forceinline__ int32_t kary_block(const int32_t (&x)[R], int32_t e, int32_t lo, int32_t* red,
                                              int32_t& count, int32_t* count_lo = nullptr) {
  constexpr int S = kKary;
  constexpr int NW = BLOCK / kWave;
  const int wave = threadIdx.x / kWave;
  int32_t hi = e, clo = 0;
  bool first = true;
  for (;;) {
    int32_t t[S];
    if (first) {
#pragma unroll
      for (int q = 0; q < S - 1; ++q) t[q] = max(lo, e - ((1 << q) - 1));
      t[S - 1] = lo;
    } else {
      const int32_t span = hi - lo;
      const int32_t step = (span + S - 1) / S;
#pragma unroll
      for (int q = 0; q < S; ++q) t[q] = lo + (int32_t)min((int64_t)span, (int64_t)(q + 1) * step);
    }
#pragma unroll
    for (int q = 0; q < S; ++q) {
      int32_t cq = 0;
#pragma unroll
      for (int r = 0; r < R; ++r) cq += popc(ballot(x[r] >= t[q]));
      if (lane_id() == 0) red[q * NW + wave] = cq;
    }
    __syncthreads();
    int32_t c[S];
#pragma unroll
    for (int q = 0; q < S; ++q) {
      int32_t tot = 0;
#pragma unroll
      for (int w = 0; w < NW; ++w) tot += red[q * NW + w];
      c[q] = tot;
    }
    __syncthreads();
    if (first) {
      if (count_lo) *count_lo = c[S - 1];  // the first pass tests lo itself
      int qs = -1;
#pragma unroll
      for (int q = S - 1; q >= 0; --q)
        if (c[q] >= t[q]) qs = q;
      if (qs < 0) return lo - 1;
      int32_t nhi = e, nlo = t[0], nc = c[0];
#pragma unroll
      for (int q = 1; q < S; ++q)
        if (q == qs) {
          nhi = t[q - 1] - 1;
          nlo = t[q];
          nc = c[q];
        }
      lo = nlo;
      hi = nhi;
      clo = nc;
      first = false;
    } else {
      int qs = -1;
#pragma unroll
      for (int q = 0; q < S; ++q)
        if (c[q] >= t[q]) qs = q;
      if (qs < 0) {
        hi = t[0] - 1;
      } else {
        int32_t nlo = t[0], nhi = hi, nc = c[0];
#pragma unroll
        for (int q = 0; q < S; ++q) {
          if (q == qs) {
            nlo = t[q];
            nc = c[q];
          }
          if (q == qs + 1) nhi = t[q] - 1;
        }
        lo = nlo;
        hi = nhi;
        clo = nc;
      }
    }
    if (lo >= hi) {
      count = clo;
      return lo;
    }
  }
}

// Workgroup-wide search over a list in global memory, re-read on each pass:
// the largest k in [lo, hi] with count(k) >= k (and that count), or lo - 1
// when count(lo) < lo.
// Each pass tests kKary thresholds (used only for cores above kHistBins).
template <int BLOCK, typename Off>
__device__ __forceinline__ int32_t mp_search(const Args<Off>& a, const int32_t* src, int32_t off, int32_t len,
                                             int32_t lo, int32_t hi, int32_t* red, int32_t& count) {
  constexpr int S = kKary;
  constexpr int NW = BLOCK / kWave;
  const int tid = threadIdx.x;
  bool lo_known = false;
  int32_t clo = 0;
  while (!(lo_known && lo >= hi)) {
    const int first = lo_known ? 0 : 1;
    const int slots = S - first;
    const int64_t span = (int64_t)hi - lo;
    int32_t t[S], cnt[S];
#pragma unroll
    for (int q = 0; q < S; ++q) {
      int32_t tq;
      if (q < first) tq = lo;
      else if (span >= slots) tq = (int32_t)(lo + ((int64_t)(q - first + 1) * span + slots - 1) / slots);
      else tq = (q - first < span) ? lo + 1 + (q - first) : INT32_MAX;
      t[q] = uni(tq);
      cnt[q] = 0;
    }
    for (int32_t j = tid; j < len; j += BLOCK) {
      const int32_t xv = est_val(a.est[off + src[j]]);
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
    int32_t best = -1, cbest = 0;
#pragma unroll
    for (int q = 0; q < S; ++q) {
      int32_t tot = 0;
#pragma unroll
      for (int w = 0; w < NW; ++w) tot += red[q * NW + w];
      if (t[q] != INT32_MAX && tot >= t[q]) {  // count(k) - k is decreasing: the hits form a prefix
        best = q;
        cbest = tot;
      }
    }
    __syncthreads();
    best = uni(best);
    cbest = uni(cbest);
    if (!lo_known) {
      if (best < 0) return lo - 1;
      lo_known = true;
    }
    if (best < 0) {
      hi = t[0] - 1;
    } else {
      int32_t nlo = t[0], nhi = hi;
#pragma unroll
      for (int q = 0; q < S; ++q) {
        if (q == best) nlo = t[q];
        if (q == best + 1 && t[q] != INT32_MAX) nhi = t[q] - 1;
      }
      lo = nlo;
      hi = nhi;
      clo = cbest;
    }
  }
  count = clo;
  return lo;
}

// One-pass search over a long list in global memory: the largest k in [lo, e]
// with count(k) >= k, or lo - 1.  Values in [lo, top] (top = min(e, lo +
// kHistBins - 1)) go to an LDS histogram, larger ones to one counter; if the
// answer lies above top, the multi-pass search finishes over (top, e].
// With `stash`, value j is also kept in LDS as min(x, e + 1) with its class
// (the estimate word's layout, 16 bits), which keeps every comparison the later
// passes make (x > h, x <= e, x >= L for L <= h <= e), so that they need not
// gather the estimates again (the caller checks len <= kStash and e + 1 < 2^14).
// `kept` receives the number of values >= lo.
template <int BLOCK, typename Off>
__device__ __forceinline__ int32_t hist_search(const Args<Off>& a, const int32_t* src, int32_t off, int32_t len,
                                               int32_t lo, int32_t e, int32_t* red, int32_t* hist, int32_t& count,
                                               uint16_t* stash, int32_t& kept) {
  constexpr int U = 8;  // loads in flight per thread
  const int tid = threadIdx.x;
  const int32_t top = (int32_t)min((int64_t)e, (int64_t)lo + kHistBins - 1);
  const int32_t nb = top - lo + 1;
  for (int32_t i = tid; i < nb; i += BLOCK) hist[i] = 0;
  __syncthreads();
  int32_t above = 0;
  for (int32_t j0 = 0; j0 < len; j0 += BLOCK * U) {
    int32_t c[U], x[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int32_t j = j0 + q * BLOCK + tid;
      c[q] = j < len ? off + src[j] : -1;
    }
#pragma unroll
    for (int q = 0; q < U; ++q) x[q] = c[q] >= 0 ? a.est[c[q]] : -1;
    if (stash) {
#pragma unroll
      for (int q = 0; q < U; ++q)
        if (c[q] >= 0) stash[j0 + q * BLOCK + tid] = (uint16_t)est_enc(min(est_val(x[q]), e + 1), est_cls(x[q]));
    }
#pragma unroll
    for (int q = 0; q < U; ++q) x[q] = c[q] >= 0 ? est_val(x[q]) : -1;
#pragma unroll
    for (int q = 0; q < U; ++q) {
      if (x[q] > top) above += 1;
      else if (x[q] >= lo) atomicAdd(&hist[x[q] - lo], 1);
    }
  }
  const int32_t tot_above = block_sum_waves<BLOCK>(wave_sum(above), red);
  // thread t owns bins [t*pb, t*pb + pb): suffix sums, then the highest k with count(k) >= k
  const int32_t pb = (nb + BLOCK - 1) / BLOCK;
  const int32_t b0 = tid * pb, b1 = min(nb, b0 + pb);
  int32_t local = 0;
  for (int32_t b = b0; b < b1; ++b) local += hist[b];
  int32_t total = 0;
  const int32_t before = block_excl_scan<BLOCK>(local, total, red);
  kept = total + tot_above;
  int32_t run = tot_above + (total - before - local);  // values above my bins
  // candidate and its count, packed so that the maximum picks the largest candidate
  long long cand = -1;
  for (int32_t b = b1 - 1; b >= b0; --b) {
    run += hist[b];
    if (run >= lo + b) {
      cand = ((long long)b << 32) | (unsigned)run;
      break;
    }
  }
  long long wm = cand;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const long long other = __shfl_xor(wm, o);
    wm = other > wm ? other : wm;
  }
  const int wave = tid / kWave;
  long long* red64 = reinterpret_cast<long long*>(hist);  // bins are no longer needed
  __syncthreads();
  if (lane_id() == 0) red64[wave] = wm;
  __syncthreads();
  long long best = -1;
#pragma unroll
  for (int w = 0; w < BLOCK / kWave; ++w) best = red64[w] > best ? red64[w] : best;
  __syncthreads();
  if (top < e && tot_above >= top + 1) return mp_search<BLOCK>(a, src, off, len, top + 1, e, red, count);
  if (best < 0) return lo - 1;
  count = (int32_t)(best & 0xffffffffll);
  return lo + (int32_t)(best >> 32);
}

// A class-3 vertex whose pruned list holds at most kWave * kBigWaveRegs
// entries, on one wavefront: the search over that list with the values in
// registers (ballots only, no barrier).  Returns true when the vertex is done:
// its value was found there (h >= L) and the update, the compaction of the list
// and the activation are written, or its estimate is already final.  Returns
// false, having written nothing but statistics, when the vertex needs the
// workgroup: no pruned list, a longer one, or a result below L.
template <bool BATCH, typename Off>
__device__ __forceinline__ bool upd_big_wave(const Args<Off>& a, const Sink& s, int32_t u, int32_t round,
                                             LaneStats& st) {
  constexpr int R = kBigWaveRegs;
  const int lane = lane_id();
  const int32_t e = uni(est_val(a.est[u]));
  if (e < 2) return true;
  const int32_t pl = a.prune ? uni(a.plen[u]) : 0;
  if (pl <= 0 || pl > kWave * R) return false;
  const Off beg = a.row_ptr[u];
  const int32_t L = uni(a.plow[u]);
  const int32_t gb = BATCH ? uni(a.vbase[u]) : 0;
  int32_t c[R], x[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int j = lane + kWave * i;
    c[i] = (kWave * i < pl && j < pl) ? a.pruned[beg + j] : 0;
  }
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int j = lane + kWave * i;
    x[i] = (kWave * i < pl && j < pl) ? a.est[c[i]] : 0;
  }
  uint32_t cb = 0;
#pragma unroll
  for (int i = 0; i < R; ++i) {
    cb |= (uint32_t)est_cls(x[i]) << (2 * i);
    x[i] = est_val(x[i]);
  }
  if (lane == 0) st.v[ST_VISITS] += pl;
  int32_t cnt = 0;
  const int32_t h = kary_regs<kWave, R>(x, e, L, true, cnt);
  if (h < L) return false;
  if (lane == 0) st.v[ST_UPDATES] += 1;
  // entries fallen below L never rise again: compact the list once 1/kPruneCompactDen of it has
  int32_t kept = 0;
#pragma unroll
  for (int i = 0; i < R; ++i)
    if (kWave * i < pl) kept += popc(ballot(lane + kWave * i < pl && x[i] >= L));
  if ((pl - kept) * kPruneCompactDen >= pl) {
    int32_t off = 0;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      if (kWave * i < pl) {
        const bool keep = lane + kWave * i < pl && x[i] >= L;
        const uint64_t m = ballot(keep);
        if (keep) a.pruned[beg + off + lanes_below(m)] = c[i];
        off += popc(m);
      }
    }
    if (lane == 0) {
      a.plen[u] = kept;
      st.v[ST_PRUNE_WRITES] += kept;
    }
  }
  if (lane == 0) a.slack[u] = cnt - h;
  if (h == e) return true;
  if (lane == 0) {
    a.est[u] = est_enc(h, 3);
    st.v[ST_CHANGES] += 1;
  }
  bool in[R];
#pragma unroll
  for (int i = 0; i < R; ++i) in[i] = lane + kWave * i < pl;
  activate_changed<R, true>(a, s, c, x, in, e, h, false, round, st, gb, cb);
  return true;
}

// One workgroup per vertex of class 3.  Lists of up to BLOCK * kBigRegs entries
// are held in registers (k-ary search); longer ones use the one-pass LDS
// histogram.  The pruned list is tried first.  When a search over it succeeds
// and at least 1/kPruneCompactDen of its entries have fallen below its
// threshold L (they can never rise again), the list is compacted in place.
template <int BLOCK, bool BATCH, typename Off>
__device__ __forceinline__ void upd_big(const Args<Off>& a, const Sink& s, int32_t u, bool dense, int32_t round,
                                        LaneStats& st, int32_t* red, int32_t* hist, uint16_t* stash, bool track,
                                        bool wave_tried) {
  constexpr int R = kBigRegs;
  constexpr int CAPR = BLOCK * R;
  const int tid = threadIdx.x;
  const Off beg = a.row_ptr[u];
  const int32_t d = uni((int32_t)(a.row_ptr[u + 1] - beg));
  const int32_t e = uni(est_val(a.est[u]));
  if (e < 2) return;
  const int32_t gb = BATCH ? uni(a.vbase[u]) : 0;
  const int32_t pl = a.prune ? uni(a.plen[u]) : 0;
  const int32_t L = pl > 0 ? uni(a.plow[u]) : 1;
  int32_t c[R], x[R];
  uint32_t cb = 0;  // register path: neighbour classes, 2 bits each
  int32_t len = 0, soff = 0;
  bool inreg = false;
  // the last one-pass search kept its values in LDS
  bool stashed = false;
  const bool stash_ok = e < (1 << 14) - 1;
  const int32_t* src = a.col;
  auto load = [&](const int32_t* from, int32_t n_, int32_t off) {
    len = n_;
    src = from;
    soff = off;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int j = tid + BLOCK * i;
      c[i] = (BLOCK * i < n_ && j < n_) ? off + from[beg + j] : 0;
    }
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int j = tid + BLOCK * i;
      x[i] = (BLOCK * i < n_ && j < n_) ? a.est[c[i]] : 0;
    }
    cb = 0;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      cb |= (uint32_t)est_cls(x[i]) << (2 * i);
      x[i] = est_val(x[i]);
    }
  };
  if (tid == 0) st.v[ST_UPDATES] += 1;
  int32_t h = -1, cnt = 0;
  bool compact_pass = false;  // the streaming pass compacts the pruned list
  // a pruned list short enough for the wavefront pass was searched there already, without success
  if (pl > 0 && !(wave_tried && pl <= kWave * kBigWaveRegs)) {
    if (tid == 0) st.v[ST_VISITS] += pl;
    if (pl <= CAPR) {
      load(a.pruned, pl, 0);
      inreg = true;
      int32_t kept = 0;  // entries still >= L
      const int32_t hp = kary_block<BLOCK, R>(x, e, L, red, cnt, &kept);
      if (hp >= L) {
        h = hp;
        if ((pl - kept) * kPruneCompactDen >= pl) {
          int32_t mine = 0;
#pragma unroll
          for (int i = 0; i < R; ++i) mine += (tid + BLOCK * i < pl) && x[i] >= L;
          int32_t off = block_excl_scan<BLOCK>(mine, kept, red);
#pragma unroll
          for (int i = 0; i < R; ++i)
            if ((tid + BLOCK * i < pl) && x[i] >= L) a.pruned[beg + off++] = c[i];
          if (tid == 0) {
            a.plen[u] = kept;
            st.v[ST_PRUNE_WRITES] += kept;
          }
        }
      }
    } else {
      inreg = false;
      len = pl;
      src = a.pruned;
      soff = 0;
      stashed = stash_ok && pl <= kStash;
      int32_t kept = 0;
      const int32_t hp =
          hist_search<BLOCK>(a, a.pruned + beg, 0, pl, L, e, red, hist, cnt, stashed ? stash : nullptr, kept);
      if (hp >= L) {
        h = hp;
        compact_pass = (pl - kept) * kPruneCompactDen >= pl;
      }
    }
  }
  bool rebuild_pass = false;
  if (h < 0) {
    if (tid == 0) {
      st.v[ST_VISITS] += d;
      st.v[ST_FULL_SCANS] += 1;
      if (track) {  // counted runs: the longest full scan, over the run and in this round
        atomicMax(&a.ctl->maxscan_run[dense ? KI_BIG_FIRST : KI_BIG], (uint32_t)d);
        atomicMax(&a.ctl->maxscan_round, (uint32_t)d);
      }
    }
    if (d <= CAPR) {
      load(a.col, d, gb);
      inreg = true;
      h = kary_block<BLOCK, R>(x, e, 1, red, cnt);
      if (a.prune) {
        const int32_t L2 = dense ? prune_low_first(h) : prune_low(h);
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
      soff = gb;
      stashed = stash_ok && d <= kStash;
      int32_t kept = 0;
      h = hist_search<BLOCK>(a, a.col + beg, gb, d, 1, e, red, hist, cnt, stashed ? stash : nullptr, kept);
      rebuild_pass = a.prune != 0;
    }
  }
  if (tid == 0) a.slack[u] = cnt - h;
  const bool changed = h < e;
  if (changed && tid == 0) {
    a.est[u] = est_enc(h, 3);
    st.v[ST_CHANGES] += 1;
  }
  // In the first round the neighbours need no notice: the classes-0..2 ones are
  // updated after this kernel and read the new value, and every class-3 vertex
  // puts itself in the next frontier (k_big).
  const bool notify = changed && !(dense && kBigFirst);
  if (!notify && !rebuild_pass && !compact_pass) return;
  if (inreg) {
    bool in[R];
#pragma unroll
    for (int i = 0; i < R; ++i) in[i] = tid + BLOCK * i < len;
    activate_changed<R, true>(a, s, c, x, in, e, h, dense, round, st, gb, cb);
    return;
  }
  // streaming pass over the list, U entries per thread at a time: activation
  // and/or writing the pruned list (one workgroup scan per U * BLOCK entries):
  // a rebuild from the full list keeps values >= prune_low(h); the compaction of
  // the pruned list in place keeps values >= L (a position is written only after
  // the barrier that follows its read, and never ahead of the positions read)
  constexpr int U = 8;
  const bool write_pass = rebuild_pass || compact_pass;
  const int32_t L2 = compact_pass ? L : (d > kHubPruneDeg ? max(2, h / 2) : (dense ? prune_low_first(h) : prune_low(h)));
  int32_t written = 0;
  for (int32_t j0 = 0; j0 < len; j0 += BLOCK * U) {
    int32_t v[U], xv[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int32_t j = j0 + q * BLOCK + tid;
      v[q] = j < len ? soff + src[beg + j] : -1;
    }
#pragma unroll
    for (int q = 0; q < U; ++q)
      xv[q] = v[q] < 0 ? 0 : (stashed ? (int32_t)stash[j0 + q * BLOCK + tid] : a.est[v[q]]);
    uint32_t qb = 0;  // classes, 2 bits each
#pragma unroll
    for (int q = 0; q < U; ++q) {
      qb |= (uint32_t)est_cls(xv[q]) << (2 * q);
      xv[q] = est_val(xv[q]);
    }
    if (write_pass) {
      int32_t mine = 0;
#pragma unroll
      for (int q = 0; q < U; ++q) mine += v[q] >= 0 && xv[q] >= L2;
      int32_t total = 0;
      int32_t off = block_excl_scan<BLOCK>(mine, total, red);
#pragma unroll
      for (int q = 0; q < U; ++q)
        if (v[q] >= 0 && xv[q] >= L2) a.pruned[beg + written + off++] = v[q];
      written += total;
    }
    if (notify) {
      bool in[U];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        in[q] = v[q] >= 0;
        v[q] = max(v[q], 0);
      }
      activate_changed<U, true>(a, s, v, xv, in, e, h, dense, round, st, gb, qb);
    }
  }
  if (write_pass && tid == 0) {
    a.plen[u] = written;
    a.plow[u] = L2;
    st.v[ST_PRUNE_WRITES] += written;
  }
}

// Class-3 vertex inside the single-workgroup tail (rare: the tail starts only
// without class-3 vertices): multi-pass search over the pruned list (or the
// full list when it fails), then one streaming activation pass.  Uses few
// registers; a full-list result below the pruned threshold drops the pruned list.
template <int BLOCK, bool BATCH, typename Off>
__device__ __forceinline__ void upd_big_lite(const Args<Off>& a, const Sink& s, int32_t u, int32_t round,
                                             LaneStats& st, int32_t* red) {
  const int tid = threadIdx.x;
  const Off beg = a.row_ptr[u];
  const int32_t d = uni((int32_t)(a.row_ptr[u + 1] - beg));
  const int32_t e = uni(est_val(a.est[u]));
  if (e < 2) return;
  const int32_t gb = BATCH ? uni(a.vbase[u]) : 0;
  const int32_t pl = a.prune ? uni(a.plen[u]) : 0;
  const int32_t L = pl > 0 ? uni(a.plow[u]) : 1;
  if (tid == 0) st.v[ST_UPDATES] += 1;
  int32_t h = -1, cnt = 0;
  const int32_t* src = a.col + beg;
  int32_t len = d, off = gb;
  if (pl > 0) {
    if (tid == 0) st.v[ST_VISITS] += pl;
    h = mp_search<BLOCK>(a, a.pruned + beg, 0, pl, L, e, red, cnt);
    if (h >= L) {
      src = a.pruned + beg;
      len = pl;
      off = 0;
    } else {
      h = -1;
    }
  }
  if (h < 0) {
    if (tid == 0) {
      st.v[ST_VISITS] += d;
      st.v[ST_FULL_SCANS] += 1;
      if (pl > 0) a.plen[u] = 0;
    }
    h = mp_search<BLOCK>(a, a.col + beg, gb, d, 1, e, red, cnt);
  }
  if (tid == 0) a.slack[u] = cnt - h;
  if (h == e) return;
  if (tid == 0) {
    a.est[u] = est_enc(h, 3);
    st.v[ST_CHANGES] += 1;
  }
  for (int32_t j0 = 0; j0 < len; j0 += BLOCK) {
    const int32_t j = j0 + tid;
    int32_t v[1] = {0}, xv[1] = {0};
    uint32_t cb = 0;
    bool in[1] = {j < len};
    if (in[0]) {
      v[0] = off + src[j];
      xv[0] = a.est[v[0]];
      cb = (uint32_t)est_cls(xv[0]);
      xv[0] = est_val(xv[0]);
    }
    activate_changed<1, true>(a, s, v, xv, in, e, h, false, round, st, gb, cb);
  }
}

// ------------------------------------------------------------------ statistics
template <int BLOCK>
__device__ __forceinline__ void flush_stats(Ctl* ctl, int kid, const LaneStats& st, unsigned long long* red64) {
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
    if (t) atomicAdd(&ctl->kstats[blockIdx.x % kStatCopies][kid][threadIdx.x], t);
  }
}

// ------------------------------------------------------------------ frontier lists
struct Frontier {
  const int32_t* list;
  int32_t n[kClasses];
  int32_t b[kClasses];
};

// The lists of round `round`: first round = the static lists; a round whose
// appends overflowed = the compaction output; otherwise the appended lists.
template <bool FIRST, typename Off>
__device__ __forceinline__ Frontier frontier_of(const Args<Off>& a, int32_t round, bool& dense) {
  const Ctl* ctl = a.ctl;
  Frontier f;
  region_bases(ctl, f.b);
  dense = FIRST || ctl->overflow[round % 3][0] != 0;
  const int32_t* cn = FIRST ? ctl->seed_fill : (dense ? ctl->ccnt[round & 1] : ctl->cnt[round % 3]);
#pragma unroll
  for (int k = 0; k < kClasses; ++k) f.n[k] = cn[k * kCtr];
  f.list = FIRST ? a.slist : list_of(a, round);
  return f;
}

// Classes 0..2 of a frontier, shared among `workers` workgroups.
template <int BLOCK, bool BATCH, typename Off>
__device__ __forceinline__ void sweep_small(const Args<Off>& a, const Sink& s, const Frontier& f, bool dense,
                                            int32_t round, int32_t worker, int32_t workers, LaneStats& st) {
  constexpr int NW = BLOCK / kWave;
  const int lane = lane_id();
  const int32_t gw = worker * NW + threadIdx.x / kWave;
  // class 2: one wavefront per vertex
  for (int32_t i = gw; i < f.n[2]; i += workers * NW) upd_wave<BATCH>(a, s, f.list[f.b[2] + i], dense, round, st);
  // class 1: four 16-lane groups per wavefront
  constexpr int GPW = kWave / kGroupLanes;
  for (int32_t i0 = gw * GPW; i0 < f.n[1]; i0 += workers * NW * GPW) {
    const int32_t i = i0 + lane / kGroupLanes;
    const bool valid = i < f.n[1];
    upd_group<BATCH>(a, s, valid ? f.list[f.b[1] + i] : 0, valid, dense, round, st);
  }
  // class 0: one lane per vertex
  for (int32_t i = worker * BLOCK + threadIdx.x; i - lane < f.n[0]; i += workers * BLOCK) {
    const bool valid = i < f.n[0];
    upd_lane<BATCH>(a, s, valid ? f.list[f.b[0] + i] : 0, valid, dense, round, st);
  }
}

// ------------------------------------------------------------------ tail
// Whether the frontier f of a round goes to the single-workgroup tail: a round
// that is not dense, whose work (lane = 1, 16-lane group = 4, wavefront = 16,
// workgroup = 64) is at most the threshold, with no class-3 vertex unless
// tail_big admits them.  The class-3 kernel, which runs before the
// classes-0..2 kernel of the same round, makes the same decision and then
// leaves the round to the tail.
template <typename Off>
__device__ __forceinline__ bool tail_eligible(const Args<Off>& a, const Frontier& f, bool dense) {
  if (dense || (f.n[3] > 0 && !a.tail_big)) return false;
  const int64_t work = (int64_t)f.n[0] + 4ll * f.n[1] + 16ll * f.n[2] + 64ll * f.n[3];
  return work > 0 && work <= a.tail_threshold;
}

// Lowest estimate first inside the tail (the order of FastK's sequential
// phase, Sec. IV: the vertex with the lowest estimate is taken next, so that
// vertices of high coreness are not recomputed for every change below them).
// Of the frontier f of round r, the tail keeps the vertices whose estimate is
// at most tau, the lowest level at which their work (lanes: 1, 16, 64 and a
// workgroup by class) fills one pass of the workgroup; every vertex is kept
// when the whole frontier fits one pass.  The others move to the next round's
// lists with the next round's stamp, before anything of this round is
// processed, so activations see them as already queued.  Estimates at or above
// kTailBins - 1 share the top bin.  bins holds kTailBins ints of LDS.
constexpr int kTailBins = 256;
template <int BLOCK, typename Off>
__device__ __forceinline__ void tail_select(const Args<Off>& a, Frontier& f, int32_t r, int32_t* ncnt,
                                            int32_t* bins, int32_t* red) {
  static_assert(BLOCK == kTailBins, "one bin per thread");
  const int tid = threadIdx.x;
  constexpr int32_t w[kClasses] = {1, kGroupLanes, kWave, BLOCK};
  int64_t total = 0;
#pragma unroll
  for (int k = 0; k < kClasses; ++k) total += (int64_t)f.n[k] * w[k];
  if (total <= BLOCK) return;
  bins[tid] = 0;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kClasses; ++k)
    for (int32_t i = tid; i < f.n[k]; i += BLOCK)
      atomicAdd(&bins[min(est_val(a.est[f.list[f.b[k] + i]]), kTailBins - 1)], w[k]);
  __syncthreads();
  int32_t tot = 0;
  const int32_t before = block_excl_scan<BLOCK>(bins[tid], tot, red);
  // the lowest bin whose cumulative work reaches one pass
  const bool reach = before + bins[tid] >= BLOCK;
  int32_t first = reach ? tid : kTailBins;
  first = min(first, __shfl_xor(first, 32));
  first = min(first, __shfl_xor(first, 16));
  first = min(first, __shfl_xor(first, 8));
  first = min(first, __shfl_xor(first, 4));
  first = min(first, __shfl_xor(first, 2));
  first = min(first, __shfl_xor(first, 1));
  if (lane_id() == 0) red[tid / kWave] = first;
  __syncthreads();
  int32_t bin = kTailBins;
#pragma unroll
  for (int q = 0; q < BLOCK / kWave; ++q) bin = min(bin, red[q]);
  __syncthreads();
  const int32_t tau = bin >= kTailBins - 1 ? INT32_MAX : bin;
  int32_t* next = list_of(a, r + 1);
  const int lane = lane_id();
#pragma unroll
  for (int k = 0; k < kClasses; ++k) {
    int32_t kept = 0;
    for (int32_t j0 = 0; j0 < f.n[k]; j0 += BLOCK) {
      const int32_t j = j0 + tid;
      const int32_t v = j < f.n[k] ? f.list[f.b[k] + j] : -1;
      const bool sel = v >= 0 && est_val(a.est[v]) <= tau;
      const bool carry = v >= 0 && !sel;
      int32_t chunk = 0;
      // every entry of the chunk is read before any is written (the scan's barriers);
      // writes stay below the positions still to be read
      const int32_t off = block_excl_scan<BLOCK>(sel ? 1 : 0, chunk, red);
      if (sel) const_cast<int32_t*>(f.list)[f.b[k] + kept + off] = v;
      kept += chunk;
      const uint64_t m = ballot(carry);
      if (m) {
        int32_t base = 0;
        if (lane == 0) base = atomicAdd(&ncnt[k * kCtr], popc(m));
        base = __shfl(base, 0);
        if (carry) {
          next[f.b[k] + base + lanes_below(m)] = v;
          a.stamp[v] = r + 1;
          if (a.gact) a.gact[a.vbase[v]] = r + 1;  // served graphs: the graph still has work
        }
      }
    }
    f.n[k] = kept;
  }
  __syncthreads();
}

// One workgroup runs the remaining rounds on uncapped lists.  Within the
// workgroup, stores become visible to all its wavefronts at each barrier, so no
// launch is needed per round.  After a_.tail_cap rounds a tail that still has
// a frontier hands it back to the round launches (Ctl::resume): the kernel
// always ends after a bounded number of rounds, and long runs continue in the
// next chunk of launches.
template <int BLOCK, bool BATCH, typename Off>
__device__ __forceinline__ void run_tail(const Args<Off>& a, int32_t round, const Frontier& f0, LaneStats& st,
                                         int32_t* red, int32_t* bins) {
  Ctl* ctl = a.ctl;
  const int tid = threadIdx.x;
  if (tid < kClasses) {
    ctl->tail_cnt[0][tid * kCtr] = 0;
    ctl->tail_cnt[1][tid * kCtr] = 0;
  }
  __syncthreads();
  int32_t t = 0;
  for (;; ++t) {
    const int32_t r = round + t;
    Frontier f = f0;
    if (t > 0) {
      f.list = list_of(a, r);
#pragma unroll
      for (int k = 0; k < kClasses; ++k) f.n[k] = ld_counter(&ctl->tail_cnt[t & 1][k * kCtr]);
    }
    if (f.n[0] + f.n[1] + f.n[2] + f.n[3] == 0) break;
    if (t >= a.tail_cap) {
      // the frontier of round r (stamps r, in the lists of round r) goes back to the round launches
      if (tid == 0) {
#pragma unroll
        for (int k = 0; k < kClasses; ++k) ctl->resume_cnt[k] = f.n[k];
        ctl->resume_round = r;
        ctl->resume = 1;
      }
      break;
    }
    int32_t* ncnt = ctl->tail_cnt[(t + 1) & 1];
    if (a.tail_order) tail_select<BLOCK>(a, f, r, ncnt, bins, red);
    Sink s = make_sink(a, r + 1, ncnt, nullptr, false);
    s.dirty = nullptr;  // tail lists are never rebuilt from the stamps
    // the two groups of classes in the order of the round kernels; the barrier
    // makes the first group's updates visible to the second
    if (kBigFirst)
      for (int32_t i = 0; i < f.n[3]; ++i) upd_big_lite<BLOCK, BATCH>(a, s, f.list[f.b[3] + i], r, st, red);
    else
      sweep_small<BLOCK, BATCH>(a, s, f, false, r, 0, 1, st);
    __syncthreads();
    if (kBigFirst)
      sweep_small<BLOCK, BATCH>(a, s, f, false, r, 0, 1, st);
    else
      for (int32_t i = 0; i < f.n[3]; ++i) upd_big_lite<BLOCK, BATCH>(a, s, f.list[f.b[3] + i], r, st, red);
    __syncthreads();
    if (t > 0 && tid < kClasses) ctl->tail_cnt[t & 1][tid * kCtr] = 0;  // reused by round t+2
    __syncthreads();
  }
  // Nothing is left in the round slots: clear them (the round base then skips
  // past the stamps the tail used, so none of them is read again; a handed-back
  // frontier is restored by the base advance).
  if (tid < 12) {
    ctl->cnt[tid / 4][(tid % 4) * kCtr] = 0;
    ctl->overflow[tid / 4][tid % 4] = 0;
  }
  if (tid == 0) {
    ctl->tail_pending += t;
    atomicAdd(&ctl->stats[ST_TAIL_ROUNDS], (unsigned long long)t);
    atomicAdd(&ctl->stats[ST_ROUNDS], (unsigned long long)t);
  }
}

// ------------------------------------------------------------------ kernels
// Deferred same-kernel checks of a round, after both update kernels: for each
// (v, e, h) whose drop from e to h may have been read stale by v, v's level is
// now final; the drop matters only if h < level <= e, and then it is charged
// to v's slack like any other loss (v is activated when the slack goes
// negative).  A charge for a drop that v had in fact seen only makes the rule
// more conservative.
template <typename Off>
__global__ __launch_bounds__(256) void k_defer(Args<Off> a, int32_t slot, int32_t collect_stats) {
  __shared__ unsigned long long red64[kLaneStats * (256 / kWave)];
  if (!a.defer) return;
  Ctl* ctl = a.ctl;
  const int32_t round = ctl->rbase + slot;
  // workgroups share out the regions: region blockIdx.x % kDeferRegions, slice blockIdx.x / kDeferRegions
  const int reg = blockIdx.x % kDeferRegions;
  const int slices = max(1u, gridDim.x / kDeferRegions);
  const int slice = blockIdx.x / kDeferRegions;
  if (slice >= slices) return;
  const int32_t rcap = a.defer_cap / kDeferRegions;
  const int32_t n = min(ctl->dcnt[reg * kCtr], rcap);
  if (n == 0) return;
  const int nslot = (round + 1) % 3;
  const Sink s = make_sink(a, round + 1, ctl->cnt[nslot], &ctl->overflow[nslot][0], true);
  LaneStats st;
  const int32_t* base = a.defer + 3 * (int64_t)reg * rcap;
  for (int32_t i0 = slice * blockDim.x; i0 < n; i0 += slices * blockDim.x) {
    const int32_t i = i0 + threadIdx.x;
    int32_t v[1] = {0};
    const int32_t one[1] = {1};
    bool act[1] = {false};
    uint32_t c = 0;
    if (i < n) {
      v[0] = base[3 * i];
      const int32_t e = base[3 * i + 1], h = base[3 * i + 2];
      const int32_t raw = a.est[v[0]];
      const int32_t lv = est_val(raw);
      c = (uint32_t)est_cls(raw);
      if (h < lv && lv <= e && a.stamp[v[0]] < s.stamp) act[0] = atomicSub(&a.slack[v[0]], 1) <= 0;
    }
    // activation as in the first round (unconditional for the lanes that set act)
    activate_changed<1, true>(a, s, v, one, act, INT32_MAX, 0, true, round, st, 0, c);
  }
  if (collect_stats) flush_stats<256>(ctl, KI_DEFER, st, red64);
}

// The estimates of a finished run (or of a stopped one) without their class bits.
__global__ void k_decode(int32_t* est, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) est[v] = est_val(est[v]);
}

// p[0 .. n) = value (a kernel rather than a memset, so that the sequence can be captured in a graph).
__global__ __launch_bounds__(256) void k_fill(int32_t* p, int64_t n, int32_t value) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = value;
}

// Zero the control block (a kernel rather than a memset, so that the sequence
// can be captured in a graph).
__global__ void k_zero_ctl(Ctl* ctl) {
  int32_t* p = reinterpret_cast<int32_t*>(ctl);
  for (int i = threadIdx.x; i < (int)(sizeof(Ctl) / sizeof(int32_t)); i += blockDim.x) p[i] = 0;
}

// Move the round base past a chunk of `k` round launches and past the rounds
// a tail ran inside it; after a tail that handed its frontier back, to the
// round of that frontier, whose list sizes become the round's counters (the
// rounds of the chunk after the tail found nothing to do).
__global__ void k_advance(Ctl* ctl, int32_t k) {
  if (threadIdx.x == 0) {
    if (ctl->resume) {
      const int32_t r = ctl->resume_round;
      ctl->rbase = r;
#pragma unroll
      for (int c = 0; c < kClasses; ++c) {
        ctl->cnt[r % 3][c * kCtr] = ctl->resume_cnt[c];
        ctl->overflow[r % 3][c] = 0;
      }
      ctl->resume = 0;
    } else {
      ctl->rbase += k + ctl->tail_pending;
    }
    ctl->tail_pending = 0;
  }
}

// Renumber the round stamps down by d (a multiple of 6, so that every round
// keeps its counter slot, round % 3, and its list parity), stamps older than d
// becoming 0, and the activity words of served graphs with them; the round base
// follows.  Run between two chunks, when no round is in flight.
__global__ __launch_bounds__(256) void k_rebase(int32_t* stamp, int32_t* gact, int64_t n, int32_t d, Ctl* ctl) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    stamp[v] = max(stamp[v] - d, 0);
    if (gact) gact[v] = max(gact[v] - d, 0);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->rbase -= d;
    ctl->dirty_from = max(ctl->dirty_from - d, 0);
  }
}

// Batched graphs: vbase[v] = first global vertex id of v's graph (one workgroup per graph).
__global__ void k_vbase(const int64_t* graph_vtx_off, int32_t* vbase) {
  const int64_t v0 = graph_vtx_off[blockIdx.x], v1 = graph_vtx_off[blockIdx.x + 1];
  for (int64_t v = v0 + threadIdx.x; v < v1; v += blockDim.x) vbase[v] = (int32_t)v0;
}

// A workgroup's class counts (per wavefront) added to its copy of the class populations.
__device__ __forceinline__ void add_pops(Ctl* ctl, const uint32_t (&part)[kClasses][256 / kWave]) {
  int32_t* slot = ctl->pop_part[blockIdx.x % kPopCopies];
#pragma unroll
  for (int k = 0; k < kClasses; ++k) {
    uint32_t t = 0;
    for (int w = 0; w < 256 / kWave; ++w) t += part[k][w];
    if (t) atomicAdd(&slot[k], (int32_t)t);
  }
}

// The class populations: the sum of the copies (one workgroup, after the initialisation kernel).
__global__ void k_pop_sum(Ctl* ctl) {
  if (threadIdx.x < kClasses) {
    int32_t t = 0;
    for (int c = 0; c < kPopCopies; ++c) t += ctl->pop_part[c][threadIdx.x];
    ctl->pop[threadIdx.x] = t;
  }
}

// est = degree, degree class, class populations (by copies, see add_pops).  A vertex of degree <= 1 already holds its coreness and can never be
// activated: it gets no class (kClasses) and no list space.  Only classes 2
// and 3 keep pruned lists.
template <typename Off>
__global__ __launch_bounds__(256) void k_init(Args<Off> a, int32_t r0, int32_t t0, int32_t t1, int32_t t2) {
  __shared__ uint32_t part[kClasses][256 / kWave];
  // the round after the first (all-vertices) round rebuilds its lists by compaction: no appends in the first round
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.ctl->overflow[(r0 + 1) % 3][0] = 1;
    a.ctl->rbase = r0;
    a.ctl->dirty_from = r0 + 2;  // the first round's activations are not marked
  }
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  uint32_t p[kClasses] = {0, 0, 0, 0};
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += stride) {
    const int32_t d = (int32_t)(a.row_ptr[v + 1] - a.row_ptr[v]);
    const uint8_t c = d <= 1 ? kClasses : (d <= t0 ? 0 : (d <= t1 ? 1 : (d <= t2 ? 2 : 3)));
    a.est[v] = est_enc(min(d, kEstMax), c);
    if (c == 2 || c == 3) a.plen[v] = 0;
    a.cls[v] = c;
#pragma unroll
    for (int k = 0; k < kClasses; ++k) p[k] += c == k;
  }
  const int wave = threadIdx.x / kWave;
#pragma unroll
  for (int k = 0; k < kClasses; ++k) {
    const uint32_t w = wave_sum(p[k]);
    if (lane_id() == 0) part[k][wave] = w;
  }
  __syncthreads();
  if (threadIdx.x == 0) add_pops(a.ctl, part);
}

// Build class lists from a per-vertex predicate: SEED = the first-round lists
// (every vertex of degree >= 2, into slist / seed_fill), otherwise the lists of
// a round whose appends overflowed (stamp == round, into ccnt).  Each workgroup
// owns a contiguous vertex range split among its wavefronts, read in pieces of
// kCompactPerLane vertices per lane with every load of a piece in flight at
// once: a counting pass, one atomic per workgroup and class, then a writing
// pass over the same range.
template <bool SEED, typename Off>
__global__ __launch_bounds__(kCompactBlock) void k_compact(Args<Off> a, int32_t slot) {
  constexpr int BLOCK = kCompactBlock, NW = BLOCK / kWave, P = kCompactPerLane, PIECE = kWave * P;
  __shared__ int32_t wcnt[NW][kClasses];
  __shared__ int32_t bbase[kClasses];
  Ctl* ctl = a.ctl;
  const int32_t round = ctl->rbase + slot;
  // this round's deferred checks start empty (the previous round's were consumed by its k_defer)
  if (!SEED && blockIdx.x == 0 && threadIdx.x < kDeferRegions) ctl->dcnt[threadIdx.x * kCtr] = 0;
  if (!SEED && blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->maxscan_round = 0;
    ctl->resid_cnt = 0;
  }
  const int wave = threadIdx.x / kWave, lane = lane_id();
  const int64_t n = a.served ? (int64_t)ctl->nhi : a.n;  // served graphs: the range of the live slots
  const int64_t chunk = ((n + gridDim.x - 1) / gridDim.x + PIECE * NW - 1) / (PIECE * NW) * (PIECE * NW);
  const int64_t wchunk = chunk / NW;
  const int64_t w0 = (int64_t)blockIdx.x * chunk + wave * wchunk, w1 = min(n, w0 + wchunk);
  static_assert(PIECE == kCompactPiece, "a wavefront piece is a dirty-mark piece");
  // this round's activations mark the next round's pieces: clear them first (every piece of [0, n) is in
  // exactly one wavefront's range)
  if (!SEED && a.dirty && lane == 0)
    for (int64_t pb = w0; pb < w1; pb += PIECE) a.dirty[((round + 1) & 1) * a.dirty_pieces + (pb >> kCompactPieceShift)] = 0;
  if (!SEED && ctl->overflow[round % 3][0] == 0) return;
  // pieces without a mark hold no vertex of this round (every later-round activation marks its piece)
  const uint8_t* marks = (!SEED && a.dirty && round >= ctl->dirty_from) ? a.dirty + (round & 1) * a.dirty_pieces : nullptr;
  // class of each vertex of a piece (kClasses: not in the list)
  auto piece = [&](int64_t pb, int32_t (&c)[P]) {
    if (SEED) {  // every vertex with a class (degree >= 2)
#pragma unroll
      for (int i = 0; i < P; ++i) {
        const int64_t v = pb + i * kWave + lane;
        c[i] = v < w1 ? (int32_t)a.cls[v] : kClasses;
      }
      return;
    }
    if (marks && marks[pb >> kCompactPieceShift] == 0) {
#pragma unroll
      for (int i = 0; i < P; ++i) c[i] = kClasses;
      return;
    }
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const int64_t v = pb + i * kWave + lane;
      c[i] = v < w1 ? a.stamp[v] : -1;
    }
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const int64_t v = pb + i * kWave + lane;
      c[i] = c[i] == round ? (int32_t)a.cls[v] : kClasses;
    }
  };
  int32_t mine[kClasses] = {0, 0, 0, 0};
  for (int64_t pb = w0; pb < w1; pb += PIECE) {
    int32_t c[P];
    piece(pb, c);
#pragma unroll
    for (int i = 0; i < P; ++i)
#pragma unroll
      for (int k = 0; k < kClasses; ++k) mine[k] += c[i] == k;
  }
#pragma unroll
  for (int k = 0; k < kClasses; ++k) {
    const int32_t w = wave_sum(mine[k]);
    if (lane == 0) wcnt[wave][k] = w;
  }
  __syncthreads();
  if (threadIdx.x < kClasses) {
    int32_t t = 0;
    for (int w = 0; w < NW; ++w) t += wcnt[w][threadIdx.x];
    int32_t* fill = SEED ? ctl->seed_fill : ctl->ccnt[round & 1];
    bbase[threadIdx.x] = t ? atomicAdd(&fill[threadIdx.x * kCtr], t) : 0;
  }
  __syncthreads();
  int32_t rb[kClasses];
  region_bases(ctl, rb);
  int32_t pos[kClasses];
#pragma unroll
  for (int k = 0; k < kClasses; ++k) {
    int32_t before = 0;
    for (int w = 0; w < wave; ++w) before += wcnt[w][k];
    pos[k] = rb[k] + bbase[k] + before;
  }
  int32_t* out = SEED ? a.slist : list_of(a, round);
  for (int64_t pb = w0; pb < w1; pb += PIECE) {
    int32_t c[P];
    piece(pb, c);
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const int64_t v = pb + i * kWave + lane;
#pragma unroll
      for (int k = 0; k < kClasses; ++k) {
        const uint64_t m = ballot(c[i] == k);
        if (c[i] == k) out[pos[k] + lanes_below(m)] = (int32_t)v;
        pos[k] += popc(m);
      }
    }
  }
}

// One round, classes 0..2 (round number `round`).  A small frontier without
// class-3 vertices is handed to the single-workgroup tail.
template <int BLOCK, bool FIRST, bool BATCH, typename Off>
__global__ __launch_bounds__(BLOCK) void k_round(Args<Off> a, int32_t slot, int32_t collect_stats) {
  __shared__ unsigned long long red64[kLaneStats * (BLOCK / kWave)];
  __shared__ int32_t red[kKary * (BLOCK / kWave)];
  __shared__ int32_t tbins[kTailBins];
  Ctl* ctl = a.ctl;
  const int32_t round = ctl->rbase + slot;
  bool dense = false;
  const Frontier f = frontier_of<FIRST>(a, round, dense);
  if (blockIdx.x == 0 && threadIdx.x < 4) {
    ctl->cnt[(round + 2) % 3][threadIdx.x * kCtr] = 0;
    ctl->overflow[(round + 2) % 3][threadIdx.x] = 0;
    ctl->ccnt[(round + 1) & 1][threadIdx.x * kCtr] = 0;  // compaction output of the next round
  }
  LaneStats st;
  const int32_t tot = f.n[0] + f.n[1] + f.n[2] + f.n[3];
  if (!FIRST && tot == 0) return;
  if (!FIRST && tail_eligible(a, f, dense)) {
    if (blockIdx.x == 0) {
      run_tail<BLOCK, BATCH>(a, round, f, st, red, tbins);
      if (collect_stats) flush_stats<BLOCK>(ctl, KI_ROUND, st, red64);
    }
    return;
  }
  const int nslot = (round + 1) % 3;
  Sink s = make_sink(a, round + 1, ctl->cnt[nslot], &ctl->overflow[nslot][0], true);
  if (FIRST) s.dirty = nullptr;  // the round after the first reads every piece
  if (!FIRST && a.defer) {
    const int reg = blockIdx.x % kDeferRegions;
    s.dcnt = &ctl->dcnt[reg * kCtr];
    s.dcap = a.defer_cap / kDeferRegions;
    s.dbase = reg * s.dcap;
  }
  sweep_small<BLOCK, BATCH>(a, s, f, FIRST, round, blockIdx.x, gridDim.x, st);
  if (collect_stats) flush_stats<BLOCK>(ctl, FIRST ? KI_ROUND_FIRST : KI_ROUND, st, red64);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    atomicAdd(&ctl->stats[ST_ROUNDS], 1ull);
    if (dense) atomicAdd(&ctl->stats[ST_DENSE_ROUNDS], 1ull);
  }
}

// Later rounds, class 3, first pass (before k_big): one wavefront per vertex.
// A vertex whose pruned list is short and holds the answer is finished here;
// the others go to the hand-over list (the class-3 region of the first-round
// list, unused after the first round), which k_big then takes one workgroup per
// vertex.  Both kernels run before the classes-0..2 kernel, so the activation
// rules see them as one class-3 kernel (a class-3 neighbour is always a
// same-kernel neighbour).
template <bool BATCH, typename Off>
__global__ __launch_bounds__(256) void k_big_wave(Args<Off> a, int32_t slot, int32_t collect_stats) {
  __shared__ unsigned long long red64[kLaneStats * (256 / kWave)];
  Ctl* ctl = a.ctl;
  const int32_t round = ctl->rbase + slot;
  bool dense = false;
  const Frontier f = frontier_of<false>(a, round, dense);
  if (f.n[3] == 0 || tail_eligible(a, f, dense)) return;
  LaneStats st;
  const int nslot = (round + 1) % 3;
  Sink s = make_sink(a, round + 1, ctl->cnt[nslot], &ctl->overflow[nslot][0], true);
  if (a.defer) {
    const int reg = blockIdx.x % kDeferRegions;
    s.dcnt = &ctl->dcnt[reg * kCtr];
    s.dcap = a.defer_cap / kDeferRegions;
    s.dbase = reg * s.dcap;
  }
  int32_t* hand = a.slist + f.b[3];
  const int32_t nw = (int32_t)(gridDim.x * (256 / kWave));
  for (int32_t i = (int32_t)(blockIdx.x * (256 / kWave) + threadIdx.x / kWave); i < f.n[3]; i += nw) {
    const int32_t u = uni(f.list[f.b[3] + i]);
    if (!upd_big_wave<BATCH>(a, s, u, round, st) && lane_id() == 0) hand[atomicAdd(&ctl->resid_cnt, 1)] = u;
  }
  if (collect_stats) flush_stats<256>(ctl, KI_BIG, st, red64);
}

// One round, class 3 (degree above the wavefront class): one workgroup per
// vertex.  Runs before k_round of the same round; a round handed to the tail
// has no class-3 vertex, so this kernel then finds nothing to do.
template <bool FIRST, bool BATCH, typename Off>
__global__ __launch_bounds__(kBigBlock, 4) void k_big(Args<Off> a, int32_t slot, int32_t collect_stats) {
  constexpr int BLOCK = kBigBlock, NW = BLOCK / kWave;
  __shared__ int32_t hist[kHistBins];
  __shared__ uint16_t stash[kStash];
  __shared__ int32_t red[kKary * NW];
  __shared__ unsigned long long red64[kLaneStats * NW];
  Ctl* ctl = a.ctl;
  const int32_t round = ctl->rbase + slot;
  bool dense = false;
  const Frontier f = frontier_of<FIRST>(a, round, dense);
  if (f.n[3] == 0) return;
  if (!FIRST && tail_eligible(a, f, dense)) return;  // the classes-0..2 kernel runs the round as a tail
  LaneStats st;
  const int nslot = (round + 1) % 3;
  Sink s = make_sink(a, round + 1, ctl->cnt[nslot], &ctl->overflow[nslot][0], true);
  if (FIRST) s.dirty = nullptr;
  if (!FIRST && a.defer) {
    const int reg = blockIdx.x % kDeferRegions;
    s.dcnt = &ctl->dcnt[reg * kCtr];
    s.dcap = a.defer_cap / kDeferRegions;
    s.dbase = reg * s.dcap;
  }
  // later rounds with the wavefront pass: only the vertices it handed over, from the hand-over list
  const bool resid = !FIRST && a.big_wave;
  const int32_t n3 = resid ? ld_counter(&ctl->resid_cnt) : f.n[3];
  const int32_t* l3 = resid ? a.slist + f.b[3] : f.list + f.b[3];
  for (int32_t i = blockIdx.x; i < n3; i += gridDim.x) {
    const int32_t u = l3[i];
    // In the first round a vertex of degree above kHubDelayDeg is not recomputed: it keeps its degree as
    // its bound and, like every class-3 vertex, enters the second round's frontier, where its first scan
    // meets estimates the first round has lowered (a lower h, so a pruned list closer to its final level).
    if (!(FIRST && kBigFirst) || uni((int32_t)(a.row_ptr[u + 1] - a.row_ptr[u])) <= kHubDelayDeg)
      upd_big<BLOCK, BATCH>(a, s, u, FIRST, round, st, red, hist, stash, collect_stats != 0, resid);
    if (FIRST && kBigFirst) {
      // every class-3 vertex is in the second round's frontier
      int32_t self[1] = {u};
      const int32_t one[1] = {1};
      const bool lead[1] = {threadIdx.x == 0};
      activate_changed<1, true>(a, s, self, one, lead, INT32_MAX, 0, true, round, st, BATCH ? uni(a.vbase[u]) : 0,
                                3u);
    }
  }
  if (collect_stats) flush_stats<BLOCK>(ctl, FIRST ? KI_BIG_FIRST : KI_BIG, st, red64);
}

// Certificate of a claimed coreness vector, a check that needs no reference
// result (the local conditions that Definition 1 implies): code 1 when a core
// lies outside [0, degree], 2 when an isolated vertex has a nonzero core or a
// vertex with neighbours has core 0, 3 when a vertex has fewer than core(v)
// neighbours of core >= core(v) (then {core >= k} would not induce minimum
// degree >= k).  The smallest failing vertex, with the first condition it
// fails, is kept as one 64-bit word (vertex << 32 | code) by atomicMin; the largest core goes to
// kmax for the host's check k_max (k_max + 1) / 2 <= m.  One wavefront per
// vertex counts its supporting neighbours.  Maximality (no larger vector
// passes) cannot be checked locally.
template <typename Off>
__global__ __launch_bounds__(256) void k_certify(int64_t n, const Off* row_ptr, const int32_t* col,
                                                 const int32_t* core, unsigned long long* worst, int32_t* kmax) {
  const int lane = lane_id();
  const int64_t nw = (int64_t)gridDim.x * blockDim.x / kWave;
  int32_t km = 0;
  for (int64_t v = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; v < n; v += nw) {
    const Off b = row_ptr[v], e = row_ptr[v + 1];
    const int64_t d = (int64_t)(e - b);
    const int32_t c = core[v];
    km = max(km, c);
    int code = 0;
    if (c < 0 || c > d) code = 1;
    else if ((d == 0) != (c == 0)) code = 2;
    else if (c > 0) {
      int64_t sup = 0;
      for (Off j = b + lane; j < e; j += kWave) sup += core[col[j]] >= c;
      sup = wave_sum(sup);
      if (sup < c) code = 3;
    }
    if (code && lane == 0) atomicMin(worst, ((unsigned long long)v << 32) | (unsigned long long)code);
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) km = max(km, __shfl_xor(km, o));
  if (lane == 0 && km > 0) atomicMax(kmax, km);
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

// Batched-graph precondition check: local ids inside their graph, no
// self-loops, strictly increasing rows, symmetry (codes as k_validate).
template <typename Off>
__global__ void k_validate_batch(int64_t n, const Off* row_ptr, const int32_t* col, const int32_t* vbase,
                                 int32_t* err) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const Off b = row_ptr[v], e = row_ptr[v + 1];
    if (e < b) {
      atomicMin(err, 3);
      continue;
    }
    const int32_t gb = vbase[v];
    const int32_t vl = (int32_t)(v - gb);
    for (Off j = b; j < e; ++j) {
      const int32_t ul = col[j];
      const int64_t u = (int64_t)gb + ul;
      if (ul < 0 || u >= n || vbase[u] != gb) {
        atomicMin(err, 1);
        break;
      }
      if (u == v) {
        atomicMin(err, 2);
        break;
      }
      if (j > b && col[j - 1] >= ul) {
        atomicMin(err, 3);
        break;
      }
      Off lo = row_ptr[u], hi = row_ptr[u + 1];
      bool found = false;
      while (lo < hi) {
        const Off mid = lo + (hi - lo) / 2;
        const int32_t w = col[mid];
        if (w == vl) {
          found = true;
          break;
        }
        if (w < vl) lo = mid + 1;
        else hi = mid;
      }
      if (!found) {
        atomicMin(err, 4);
        break;
      }
    }
  }
}

// ------------------------------------------------------------------ served graphs
// Graphs join the running rounds between two launches, each into a slot of the
// vertex arena (vb .. vb+n, the last entry holding the row end) and of the
// entry arena (eb ..).  The slot's graph-local row offsets have just been
// copied to row_ptr[vb .. vb+n].

// New slots (blockIdx.y = slot): est = degree, class, no pruned list, graph
// base, and for every vertex of degree >= 2 a stamp of the next round, which
// is then the graph's first round; the graph's activity word gets it too.
template <typename Off>
__global__ __launch_bounds__(256) void k_slot_init(Args<Off> a, const SlotDesc* slots, int32_t t0, int32_t t1,
                                                   int32_t t2) {
  const SlotDesc sd = slots[blockIdx.y];
  const int32_t r = a.ctl->rbase;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < sd.n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t v = sd.vb + i;
    const int32_t d = (int32_t)(a.row_ptr[v + 1] - a.row_ptr[v]);
    const uint8_t c = d <= t0 ? 0 : (d <= t1 ? 1 : (d <= t2 ? 2 : 3));
    a.est[v] = est_enc(min(d, kEstMax), c);
    a.plen[v] = 0;
    a.cls[v] = c;
    const_cast<int32_t*>(a.vbase)[v] = sd.vb;
    // a stamp left by an earlier graph in this range is overwritten (0 never equals a round)
    a.stamp[v] = d >= 2 ? r : 0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) a.gact[sd.vb] = r;
}

// Graph-local row offsets of the new slots -> entry-arena offsets (after k_slot_init has read them).
__global__ __launch_bounds__(256) void k_slot_shift(int64_t* row_ptr, const SlotDesc* slots) {
  const SlotDesc sd = slots[blockIdx.y];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= sd.n; i += (int64_t)gridDim.x * blockDim.x)
    row_ptr[sd.vb + i] += sd.eb;
}

// After slots joined (or left): new class populations, so the next round
// rebuilds its lists by compaction over the live vertex range; its append
// counters start from zero.
__global__ void k_serve_join(Ctl* ctl, int32_t p0, int32_t p1, int32_t p2, int32_t p3, int32_t nhi) {
  const int k = threadIdx.x;
  const int32_t r = ctl->rbase;
  if (k < kClasses) {
    ctl->pop[k] = k == 0 ? p0 : (k == 1 ? p1 : (k == 2 ? p2 : p3));
    ctl->ccnt[r & 1][k * kCtr] = 0;
    ctl->cnt[(r + 1) % 3][k * kCtr] = 0;
    ctl->overflow[(r + 1) % 3][k] = 0;
  }
  if (k == 0) {
    ctl->overflow[r % 3][0] = 1;
    ctl->nhi = nhi;
  }
}

// Activity word of every slot's graph (the host compares it with the round base).
__global__ void k_slot_status(const int32_t* gact, const int32_t* slot_vb, int32_t nslots, int32_t* out) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nslots; i += gridDim.x * blockDim.x)
    out[i] = slot_vb[i] >= 0 ? gact[slot_vb[i]] : 0;
}

// Control block of a server: zero, round base r0.
__global__ void k_serve_reset(Ctl* ctl, int32_t r0) {
  int32_t* p = reinterpret_cast<int32_t*>(ctl);
  for (int i = threadIdx.x; i < (int)(sizeof(Ctl) / sizeof(int32_t)); i += blockDim.x) p[i] = 0;
  __syncthreads();
  if (threadIdx.x == 0) ctl->rbase = r0;
}

// ------------------------------------------------------------------ core maintenance after edge changes
// The coreness c_old of a graph is known; edges R are removed and edges I
// inserted (the paper's future work on dynamic graphs, Sec. VI).  The run
// restarts the same iteration from a pointwise upper bound x of the new
// coreness c_new, with a frontier that holds every vertex whose bound may
// exceed the h-index of its neighbours' bounds.  Two facts about the new
// k-core H of a vertex w (k = c_new(w)) give the bounds.  (a) In the old graph
// H keeps every edge but the inserted ones, so with D the largest number of
// inserted edges at one vertex every vertex of H has at least k - D neighbours
// in H there: c_old >= c_new - D everywhere.  (b) For any level c, let S be
// the vertices of old coreness <= c in the new (c+1)-core N.  Every component C
// of S holds an endpoint of an inserted edge whose endpoints both lie in N:
// otherwise every vertex of C has its c+1 neighbours in N through old edges, so
// C together with the old (c+1)-core has minimum degree c+1 in the old graph.
//  * removals only lower coreness, so x = c_old bounds every vertex; only the
//    endpoints of R have a new neighbourhood;
//  * by (b) with c = c_old(w), a vertex w that rises is joined to an endpoint u
//    of such an edge (u, v) by vertices that all rise past c_old(w) (its
//    component of S), each of old coreness at most c_old(w) and, by (a), at
//    least c_old(w) + 1 - D.  A vertex of old coreness below T, the smallest
//    min(c_old(u), c_old(v)) over I, never rises (its component would hold an
//    endpoint of old coreness below T), so w lies in the set A of vertices
//    reached from the endpoints through vertices of old coreness >= T.  When
//    D = 1 the component keeps to old coreness exactly c_old(w), u included,
//    and c_old(v) >= c_old(w): u is the lower endpoint of its edge and w lies in
//    u's subcore (reached from u through vertices of the same old coreness), the
//    set a single insertion can raise, which the search then follows instead.
//    A search that grows too large is given up for the superset of all
//    vertices of old coreness >= T.  On A, x = max(c_old, min(degree, c_old + D, K_max + D)), K_max the largest
//    min(c_old(u), c_old(v)) over I (by (a) on w and, with c = c_new(w) - 1, on
//    the endpoints u, v); elsewhere x = c_old;
//  * x never falls below c_old at the start (so no neighbour loses support
//    unannounced), except on vertices left with degree <= 1, whose coreness is
//    then known (0 or 1): they take it, and their neighbour joins the frontier.
// A vertex whose bound stays c_old and that lost no edge sees at least c_old
// neighbours with bounds >= c_old (insertions only add neighbours), so its bound
// is at most their h-index: the frontier is the endpoints of R, the vertices
// whose bound rose, and the neighbours of vertices left with degree 1.  The
// slack of every vertex starts at 0, so the first loss of support at its level
// activates it; with insertions only, a vertex out of the frontier is final
// (c_old <= c_new <= x = c_old) and its slack starts out of reach.

// Flags (bit 0: endpoint of a removed edge, bit 1: in A, bits 2 and up: the
// number of inserted edges at the vertex when `count` is set) and, over the
// inserted edges, the smallest and the largest min(c_old(u), c_old(v)) and the
// largest count: out[0], out[1] and out[2].
__global__ __launch_bounds__(256) void k_upd_edges(const int32_t* del, int64_t nd, const int32_t* ins, int64_t ni,
                                                   const int32_t* prev, int32_t* flag, int32_t count, int32_t* out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int32_t lo = INT32_MAX, hi = -1, hits = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nd + ni; i += stride) {
    if (i < nd) {
      atomicOr(&flag[del[2 * i]], 1);
      atomicOr(&flag[del[2 * i + 1]], 1);
    } else {
      const int64_t j = i - nd;
      const int32_t u = ins[2 * j], v = ins[2 * j + 1];
      const int32_t k = min(prev[u], prev[v]);
      lo = min(lo, k);
      hi = max(hi, k);
      if (count) hits = max(hits, 1 + max(atomicAdd(&flag[u], 4) >> 2, atomicAdd(&flag[v], 4) >> 2));
    }
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    lo = min(lo, __shfl_xor(lo, o));
    hi = max(hi, __shfl_xor(hi, o));
    hits = max(hits, __shfl_xor(hits, o));
  }
  if (lane_id() == 0 && hi >= 0) {
    atomicMin(&out[0], lo);
    atomicMax(&out[1], hi);
    atomicMax(&out[2], hits);
  }
}

// The search for A.  With the window rule (D <= kUpdWindowMax) a search state
// is a vertex x with a window top c in [c_old(x), c_old(x) + D - 1], encoded as
// x | (c - c_old(x)) << 30; it moves to the neighbours y with c_old(y) in
// [c + 1 - D, c] (state y, c), and a vertex joins A when its state of window
// top c_old(y) is reached.  vis[y] holds one bit per window offset.  Without it
// (the threshold rule) a state is a vertex, and it moves to the neighbours of
// old coreness >= T.  Queues hold at most `cap` states: past it the count still
// grows (the search is then given up) but nothing is written.
struct UpdSearch {
  int32_t T;      // threshold rule: smallest old coreness passed
  int32_t D;      // window rule: window width (0: threshold rule)
  int32_t* flag;  // bit 1: in A
  int32_t* vis;   // window rule: reached window offsets
  int64_t cap;    // capacity of every queue
};

constexpr uint32_t kStateMask = (1u << 30) - 1;

// A vertex of Z (two or more inserted edges, counted in its flag word from bit 2).
__device__ __forceinline__ bool upd_heavy(int32_t f) { return (f >> 2) >= 2; }

// Vertex and window offset of a queued state (the threshold rule queues plain vertex ids).
__device__ __forceinline__ int32_t state_vertex(const UpdSearch& q, uint32_t st) {
  return q.D ? (int32_t)(st & kStateMask) : (int32_t)st;
}
__device__ __forceinline__ int32_t state_offset(const UpdSearch& q, uint32_t st) {
  return q.D ? (int32_t)(st >> 30) : 0;
}

// Marks state (y, offset j) reached; true when it was new.  Under the window
// rule the state of offset 0 also puts y in A.
__device__ __forceinline__ bool upd_reach(const UpdSearch& q, int32_t y, int32_t j) {
  if (q.D == 0) return (q.flag[y] & 2) == 0 && (atomicOr(&q.flag[y], 2) & 2) == 0;
  const int32_t bit = 1 << j;
  if ((q.vis[y] & bit) || (atomicOr(&q.vis[y], bit) & bit)) return false;
  if (j == 0) atomicOr(&q.flag[y], 2);
  return true;
}

// The search starts from the endpoints of the inserted edges: under the
// window rule from (u, c) for c_old(u) <= c <= min(c_old(u), K) + D - 1, K the
// edge's min(c_old(u), c_old(v)) (both endpoints lie in the new (c+1)-core).
__global__ __launch_bounds__(256) void k_upd_bfs_start(const int32_t* ins, int64_t ni, const int32_t* prev,
                                                       UpdSearch q, int32_t* queue, int32_t* qcnt) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 2 * ni; i += stride) {
    const int32_t u = ins[i];
    const int32_t lu = prev[u], k = min(lu, prev[ins[i ^ 1]]);
    const int32_t top = q.D ? k + q.D - 1 - lu : 0;  // largest window offset of u
    for (int32_t j = 0; j <= top; ++j)
      if (upd_reach(q, u, j)) {
        const int32_t pos = atomicAdd(qcnt, 1);
        if (pos < q.cap) queue[pos] = (int32_t)((uint32_t)u | (uint32_t)j << 30);
      }
  }
}

// One slice of kBfsSlice entries of a row, [j0, min(j0 + kBfsSlice, e)), seen
// from a state of window top c (threshold rule: c unused): the new states are
// appended to out_q.  Loads, gathers and flag updates of the slice are issued
// together, then one atomic reserves the wavefront's places in the queue.
// A wavefront's staging buffer in LDS for the states a search level finds: they
// go to the output queue up to kBfsBuf at a time, with one atomic on the queue's
// counter per flush, since the appends of every wavefront of a level meet on
// that counter's line (served one at a time, about 11 ns each).
constexpr int kBfsBuf = 1024;
struct StateBuf {
  int32_t* buf;  // kBfsBuf entries of LDS
  int32_t held;  // entries held (the same in every lane)
};

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The held states to the queue (the whole wavefront calls this).
__device__ __forceinline__ void bfs_flush(StateBuf& b, const UpdSearch& q, int32_t* out_q, int32_t* out_cnt) {
  if (b.held == 0) return;
  wave_lds_sync();
  int32_t base = 0;
  if (lane_id() == 0) base = atomicAdd(out_cnt, b.held);
  base = __shfl(base, 0);
  for (int32_t j = lane_id(); j < b.held; j += kWave) {
    const int64_t pos = (int64_t)base + j;
    if (pos < q.cap) out_q[pos] = b.buf[j];
  }
  wave_lds_sync();
  b.held = 0;
}

// With Src (the sources of the heavy-vertex search) every neighbour outside Z is
// taken, at window offset 0, whatever its old coreness.  The new states go to
// the wavefront's staging buffer sb.
template <bool Src = false, typename Off>
__device__ __forceinline__ void bfs_slice(const int32_t* col, const int32_t* prev, const UpdSearch& q, int32_t c,
                                          Off j0, Off e, int32_t* out_q, int32_t* out_cnt, StateBuf& sb) {
  static_assert(kBfsSlice <= kBfsBuf, "a slice's states fit an empty buffer");
  constexpr int K = kBfsSlice / kWave;
  const int lane = lane_id();
  const int32_t lo = q.D ? c + 1 - q.D : q.T, hi = q.D ? c : INT32_MAX;
  int32_t w[K], off[K];
  bool add[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const Off j = j0 + k * kWave + lane;
    w[k] = j < e ? col[j] : -1;
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    add[k] = false;
    off[k] = 0;
    if (w[k] >= 0) {
      if (Src) {
        add[k] = !upd_heavy(q.flag[w[k]]);
      } else {
        const int32_t cw = prev[w[k]];
        add[k] = cw >= lo && cw <= hi;
        off[k] = q.D ? c - cw : 0;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k) add[k] = add[k] && upd_reach(q, w[k], off[k]);
  uint64_t m[K];
  int32_t total = 0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    m[k] = ballot(add[k]);
    total += popc(m[k]);
  }
  if (total == 0) return;
  if (sb.held + total > kBfsBuf) bfs_flush(sb, q, out_q, out_cnt);
  int32_t at = sb.held;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if (add[k]) sb.buf[at + lanes_below(m[k])] = (int32_t)((uint32_t)w[k] | (uint32_t)off[k] << 30);
    at += popc(m[k]);
  }
  sb.held = at;
}

// One level of the search: one wavefront per queued state.  A row longer than
// kBfsLongRow is only registered in long_q as (state, first slice number), the
// row count and the slice count advancing together in one 64-bit counter so
// that the slice numbers increase along long_q; k_upd_bfs_long then shares out
// the slices evenly (on a skewed graph one hub row holds a large share of a
// level's entries).  The counters rotate: this level reads cnt[0], adds to
// cnt[1] and clears cnt[2] (the previous level's input, no longer read), and
// clears the previous level's long-row counter.  `reached` sums the levels'
// input counts (several levels run between two looks of the host).
template <typename Off>
__global__ __launch_bounds__(256) void k_upd_bfs_level(const Off* row_ptr, const int32_t* col, const int32_t* prev,
                                                       UpdSearch q, const int32_t* in_q, const int32_t* in_cnt,
                                                       int32_t* out_q, int32_t* out_cnt, int32_t* stale_cnt,
                                                       int32_t* long_q, unsigned long long* long_cnt,
                                                       unsigned long long* stale_long_cnt,
                                                       unsigned long long* reached) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *stale_cnt = 0;
    *stale_long_cnt = 0;
    *reached += (unsigned long long)*in_cnt;
  }
  __shared__ int32_t stage[(256 / kWave) * kBfsBuf];
  StateBuf sb{stage + (threadIdx.x / kWave) * kBfsBuf, 0};
  const int64_t nq = min((int64_t)*in_cnt, q.cap);
  const int64_t nw = (int64_t)gridDim.x * blockDim.x / kWave;
  for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; i < nq; i += nw) {
    const uint32_t st = (uint32_t)in_q[i];
    const int32_t u = state_vertex(q, st);
    const Off b = row_ptr[u], e = row_ptr[u + 1];
    if (e - b > kBfsLongRow) {
      if (lane_id() == 0) {
        const unsigned long long slices = (unsigned long long)((e - b + kBfsSlice - 1) / kBfsSlice);
        const unsigned long long old = atomicAdd(long_cnt, (1ull << 32) | slices);
        const int64_t r = (int64_t)(old >> 32);
        long_q[2 * r] = (int32_t)st;
        long_q[2 * r + 1] = (int32_t)(old & 0xffffffffull);
      }
      continue;
    }
    const int32_t c = prev[u] + state_offset(q, st);
    for (Off j0 = b; j0 < e; j0 += kBfsSlice) bfs_slice(col, prev, q, c, j0, e, out_q, out_cnt, sb);
  }
  bfs_flush(sb, q, out_q, out_cnt);
}

// Slices of the rows registered in long_q as (state, first slice number), the
// first slice numbers increasing along the list (lc: row count in the high 32
// bits, slice count S in the low ones), shared out evenly: wavefront g of W
// takes the slices [g * S / W, (g + 1) * S / W), finds the row of its first
// slice by binary search, and walks on, calling f(state, first entry, row end)
// on each slice.
template <typename Off, typename F>
__device__ __forceinline__ void for_long_slices(const Off* row_ptr, const UpdSearch& q, const int32_t* long_q,
                                                unsigned long long lc, F&& f) {
  const int64_t nl = (int64_t)(lc >> 32), S = (int64_t)(lc & 0xffffffffull);
  if (nl == 0) return;
  const int64_t W = (int64_t)gridDim.x * blockDim.x / kWave;
  const int64_t g = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t c0 = g * S / W, c1 = (g + 1) * S / W;
  if (c0 >= c1) return;
  int64_t lo = 0, hi = nl - 1;  // the last row whose first slice is <= c0
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) / 2;
    if (long_q[2 * mid + 1] <= c0) lo = mid;
    else hi = mid - 1;
  }
  int64_t i = lo;
  uint32_t st = (uint32_t)long_q[2 * i];
  int64_t first = long_q[2 * i + 1];
  Off b = row_ptr[state_vertex(q, st)], e = row_ptr[state_vertex(q, st) + 1];
  for (int64_t c = c0; c < c1; ++c) {
    while (c >= first + (int64_t)((e - b + kBfsSlice - 1) / kBfsSlice)) {
      ++i;
      st = (uint32_t)long_q[2 * i];
      first = long_q[2 * i + 1];
      b = row_ptr[state_vertex(q, st)];
      e = row_ptr[state_vertex(q, st) + 1];
    }
    f(st, b + (Off)((c - first) * kBfsSlice), e);
  }
}

// The long rows of one level.
template <typename Off>
__global__ __launch_bounds__(256) void k_upd_bfs_long(const Off* row_ptr, const int32_t* col, const int32_t* prev,
                                                      UpdSearch q, const int32_t* long_q,
                                                      const unsigned long long* long_cnt, int32_t* out_q,
                                                      int32_t* out_cnt) {
  __shared__ int32_t stage[(256 / kWave) * kBfsBuf];
  StateBuf sb{stage + (threadIdx.x / kWave) * kBfsBuf, 0};
  for_long_slices(row_ptr, q, long_q, *long_cnt, [&](uint32_t st, Off j0, Off e) {
    bfs_slice(col, prev, q, prev[state_vertex(q, st)] + state_offset(q, st), j0, e, out_q, out_cnt, sb);
  });
  bfs_flush(sb, q, out_q, out_cnt);
}

// Levels of the search inside one workgroup of kBfsSmallBlock threads, from
// `level` on, while a level holds at most kBfsSmallBlock states and
// kBfsSmallEntries adjacency entries: a search that has narrowed to a few states
// per level (a long path through one shell) then costs no launch and no look of
// the host per level.  A level's entries are shared out over all threads (an
// exclusive scan of the states' degrees in LDS, each thread finding its entry's
// state by binary search), the level's new states are counted in LDS, and stores
// become visible to the whole workgroup at each barrier.  The queues and
// counters rotate as in k_upd_bfs_level, `reached` grows by each level's input,
// and the kernel stops at an empty level, at a level larger than it takes, or
// where `reached` plus the level's input would pass `budget`; out[15] is the
// level it stopped at.  Both long-row counters are cleared on exit, so that
// later launches of k_upd_bfs_level start from empty lists.
template <typename Off>
__global__ __launch_bounds__(kBfsSmallBlock) void k_upd_bfs_small(const Off* row_ptr, const int32_t* col,
                                                                  const int32_t* prev, UpdSearch q, int32_t* q0,
                                                                  int32_t* q1, int32_t* cnt, int32_t level,
                                                                  int64_t budget, unsigned long long* reached,
                                                                  unsigned long long* long_cnt, int32_t* out) {
  __shared__ int32_t first[kBfsSmallBlock];  // first entry of each state (of the level's entries)
  __shared__ Off base[kBfsSmallBlock];       // its row start
  __shared__ int32_t top[kBfsSmallBlock];    // its window top (threshold rule: unused)
  __shared__ int32_t red[kBfsSmallBlock / kWave];
  __shared__ int32_t made;                   // states appended in the level
  const int tid = threadIdx.x;
  for (;; ++level) {
    const int32_t nin = ld_counter(&cnt[level % 3]);
    const unsigned long long done = __hip_atomic_load(reached, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (nin == 0 || nin > kBfsSmallBlock || (int64_t)done + nin > budget) break;
    const int32_t* in_q = (level & 1) ? q1 : q0;
    int32_t* out_q = (level & 1) ? q0 : q1;
    int32_t d = 0;
    if (tid < nin) {
      const uint32_t st = (uint32_t)in_q[tid];
      const int32_t u = state_vertex(q, st);
      const Off b = row_ptr[u];
      d = (int32_t)min((Off)(kBfsSmallEntries + 1), row_ptr[u + 1] - b);  // (the sum stays in range)
      base[tid] = b;
      top[tid] = prev[u] + state_offset(q, st);
    }
    int32_t E = 0;
    const int32_t f = block_excl_scan<kBfsSmallBlock>(d, E, red);
    if (E > kBfsSmallEntries) break;
    if (tid < nin) first[tid] = f;
    if (tid == 0) {
      made = 0;
      cnt[(level + 2) % 3] = 0;  // the previous level's input, no longer read
      __hip_atomic_store(reached, done + (unsigned long long)nin, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    for (int32_t j0 = 0; j0 < E; j0 += kBfsSmallBlock) {
      const int32_t j = j0 + tid;
      int32_t w = 0, off = 0;
      bool add = false;
      if (j < E) {
        int32_t lo = 0, hi = nin - 1;  // the last state whose first entry is <= j
        while (lo < hi) {
          const int32_t mid = (lo + hi + 1) / 2;
          if (first[mid] <= j) lo = mid;
          else hi = mid - 1;
        }
        w = col[base[lo] + (Off)(j - first[lo])];
        const int32_t c = top[lo], cw = prev[w];
        const bool in = q.D ? (cw >= c + 1 - q.D && cw <= c) : cw >= q.T;
        off = q.D ? c - cw : 0;
        add = in && upd_reach(q, w, off);
      }
      const uint64_t m = ballot(add);
      if (m) {
        int32_t pos = 0;
        if (lane_id() == 0) pos = atomicAdd(&made, popc(m));
        pos = __shfl(pos, 0) + lanes_below(m);
        if (add && pos < q.cap) out_q[pos] = (int32_t)((uint32_t)w | (uint32_t)off << 30);
      }
    }
    __syncthreads();
    if (tid == 0) cnt[(level + 1) % 3] = made;
    __syncthreads();
  }
  if (tid == 0) {
    out[15] = level;
    long_cnt[0] = 0;
    long_cnt[1] = 0;
  }
}

// The heavy-vertex rule (several inserted edges at few vertices, as when a
// vertex arrives with its edges).  Z is the set of vertices with two or more
// inserted edges and D' the largest, over the vertices outside Z, of their
// edges to Z plus their inserted edges to vertices outside Z.  When D' <= 1, let
// H be the new k-core of a vertex w outside Z: in the old graph H minus Z loses
// at most D' <= 1 neighbours per vertex (its edges to Z and its inserted edges),
// so c_old(w) >= c_new(w) - 1.  If w rises (c = c_old(w), N the new
// (c+1)-core), its component C among the vertices of N outside Z of old
// coreness <= c all have old coreness exactly c, and some vertex of C has a
// neighbour in Z or an inserted edge to a vertex of N outside Z (else C with the
// old (c+1)-core would have minimum degree c + 1 in the old graph); that edge's
// other endpoint lies in C or has old coreness above c, so the vertex is a lower
// (or equal) endpoint.  The search therefore starts from the neighbours of Z
// outside Z and the lower endpoints of the inserted edges outside Z, keeps to
// old shells (the window rule with width 1) and never enters Z; Z is in A with
// rise D, every other vertex rises by at most 1, and a search given up takes the
// vertices of old coreness >= T', the smallest old coreness of a source.
// Membership of Z is read from the counts that k_upd_edges leaves in the flags
// (upd_heavy); the counts of D' go to bits 8 and up of vis[y] (the window bits are 0..3),
// saturating near 2, since only whether a count exceeds 1 matters.

// One more count at y (outside Z); returns the count, or 2 once it is past 1.
__device__ __forceinline__ int32_t upd_zcount(int32_t* vis, int32_t y) {
  if ((vis[y] >> 8) >= 2) return 2;
  return (atomicAdd(&vis[y], 256) >> 8) + 1;
}

// Registers the rows of Z once each (claimed through bit 7 of vis) as long rows
// in long_q for for_long_slices, and resets out[6] (D') and out[7] (T').
template <typename Off>
__global__ __launch_bounds__(256) void k_upd_zreg(const Off* row_ptr, const int32_t* ins, int64_t ni,
                                                  const int32_t* flag, int32_t* vis, int32_t* long_q,
                                                  unsigned long long* long_cnt, int32_t* out) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    out[6] = 0;
    out[7] = INT32_MAX;
  }
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 2 * ni; i += stride) {
    const int32_t z = ins[i];
    if (!upd_heavy(flag[z]) || (atomicOr(&vis[z], 128) & 128)) continue;
    const unsigned long long slices =
        (unsigned long long)((row_ptr[z + 1] - row_ptr[z] + kBfsSlice - 1) / kBfsSlice);
    const unsigned long long old = atomicAdd(long_cnt, (1ull << 32) | slices);
    const int64_t r = (int64_t)(old >> 32);
    long_q[2 * r] = z;
    long_q[2 * r + 1] = (int32_t)(old & 0xffffffffull);
  }
}

// D' and T' (out[6], out[7]), and in out[14] the number of distinct neighbours
// of Z outside Z: the rows of Z, then the inserted edges outside Z.
template <typename Off>
__global__ __launch_bounds__(256) void k_upd_zcount(const Off* row_ptr, const int32_t* col, const int32_t* prev,
                                                    UpdSearch q, const int32_t* ins, int64_t ni,
                                                    const int32_t* long_q, const unsigned long long* long_cnt,
                                                    int32_t* out) {
  int32_t most = 0, low = INT32_MAX, fresh = 0;
  for_long_slices(row_ptr, q, long_q, *long_cnt, [&](uint32_t, Off j0, Off e) {
    for (Off j = j0 + lane_id(); j < min(e, j0 + (Off)kBfsSlice); j += kWave) {
      const int32_t y = col[j];
      if (upd_heavy(q.flag[y])) continue;
      const int32_t k = upd_zcount(q.vis, y);
      most = max(most, k);
      fresh += k == 1;
      low = min(low, prev[y]);
    }
  });
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ni; i += stride) {
    const int32_t u = ins[2 * i], v = ins[2 * i + 1];
    if (upd_heavy(q.flag[u]) || upd_heavy(q.flag[v])) continue;
    most = max(most, max(upd_zcount(q.vis, u), upd_zcount(q.vis, v)));
    low = min(low, min(prev[u], prev[v]));
  }
  most = wave_max(most);
  low = wave_min(low);
  fresh = wave_sum(fresh);
  if (lane_id() == 0) {
    if (most) atomicMax(&out[6], most);
    if (low != INT32_MAX) atomicMin(&out[7], low);
    if (fresh) atomicAdd(&out[14], fresh);
  }
}

// The sources of the heavy-vertex search: Z goes into A and is marked reached
// (so the search never enters it), and, unless the search is given up at once
// (sources == 0), every neighbour of Z outside Z is queued at window offset 0
// (q.D = 1).
template <typename Off>
__global__ __launch_bounds__(256) void k_upd_zsrc(const Off* row_ptr, const int32_t* col, const int32_t* prev,
                                                  UpdSearch q, const int32_t* long_q,
                                                  const unsigned long long* long_cnt, int32_t sources,
                                                  int32_t* queue, int32_t* qcnt) {
  const unsigned long long lc = *long_cnt;
  const int64_t nl = (int64_t)(lc >> 32);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nl; i += stride) {
    const int32_t z = long_q[2 * i];
    atomicOr(&q.vis[z], 1);
    atomicOr(&q.flag[z], 2);
  }
  if (!sources) return;
  __shared__ int32_t stage[(256 / kWave) * kBfsBuf];
  StateBuf sb{stage + (threadIdx.x / kWave) * kBfsBuf, 0};
  for_long_slices(row_ptr, q, long_q, lc, [&](uint32_t, Off j0, Off e) {
    bfs_slice<true>(col, prev, q, 0, j0, e, queue, qcnt, sb);
  });
  bfs_flush(sb, q, queue, qcnt);
}

// Start of an update run: estimates from the bounds above, classes and class
// populations from the new degrees, no pruned lists, slack 0, and the round
// stamp r on every frontier vertex (endpoints of removed edges, vertices of A
// whose bound is above c_old, neighbours of vertices left with degree 1); round
// r then builds its lists from the stamps (a compaction round) as a later round.
template <typename Off>
__global__ __launch_bounds__(256) void k_upd_init(Args<Off> a, const int32_t* prev, const int32_t* flag, int64_t rise,
                                                  int32_t heavy, int64_t cap, int32_t all_from, int32_t insert_only,
                                                  int32_t r, int32_t t0, int32_t t1, int32_t t2) {
  __shared__ uint32_t part[kClasses][256 / kWave];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.ctl->overflow[r % 3][0] = 1;
    a.ctl->rbase = r;
    a.ctl->dirty_from = r + 1;  // the seeds are not marked: round r reads every piece
  }
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  uint32_t p[kClasses] = {0, 0, 0, 0};
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += stride) {
    const Off beg = a.row_ptr[v];
    const int32_t d = (int32_t)(a.row_ptr[v + 1] - beg);
    const int32_t c = prev[v];
    const int32_t f = flag[v];
    int64_t x = c;
    // under the heavy-vertex rule only the vertices of Z rise by more than 1
    const int64_t up = heavy && !upd_heavy(f) ? 1 : rise;
    if ((f & 2) || c >= all_from) x = max((int64_t)c, min(min((int64_t)d, cap), (int64_t)c + up));
    // a vertex that kept its old coreness as its bound and lost no edge keeps at least
    // c_old neighbours of bound >= c_old (insertions only add neighbours), so it starts
    // out of the frontier
    bool seed = (f & 1) || x > c;
    if (d <= 1 && x > d) {
      x = d;  // the coreness of a vertex of degree 0 or 1 is its degree
      if (d == 1) a.stamp[a.col[beg]] = r;  // its neighbour lost support it had counted
    }
    if (d <= 1) seed = false;
    const uint8_t cl = d <= 1 ? kClasses : (d <= t0 ? 0 : (d <= t1 ? 1 : (d <= t2 ? 2 : 3)));
    a.est[v] = est_enc((int32_t)min(x, (int64_t)kEstMax), cl);
    if (cl == 2 || cl == 3) a.plen[v] = 0;
    a.cls[v] = cl;
    // with insertions only, a vertex out of the frontier keeps its old coreness, which is then its
    // new one (no bound of it lies above, none below): no loss of support can move it
    a.slack[v] = insert_only && !seed ? kSlackFinal : 0;
    if (seed) a.stamp[v] = r;
#pragma unroll
    for (int k = 0; k < kClasses; ++k) p[k] += cl == k;
  }
  const int wave = threadIdx.x / kWave;
#pragma unroll
  for (int k = 0; k < kClasses; ++k) {
    const uint32_t w = wave_sum(p[k]);
    if (lane_id() == 0) part[k][wave] = w;
  }
  __syncthreads();
  if (threadIdx.x == 0) add_pops(a.ctl, part);
}

// ------------------------------------------------------------------ degree relabelling
// On request, a graph is renumbered by decreasing degree (in buckets of
// kRelabelBuckets degrees, stable) before the decomposition, so that the
// estimates of the high-degree vertices, which most adjacency entries of a
// skewed graph point to, share cache lines.

// Rows of degree above kRelabelLongDeg (they come first after the renumbering) and their entries.
template <typename Off>
__global__ __launch_bounds__(256) void k_relabel_probe(int64_t n, const Off* row_ptr,
                                                       unsigned long long* out /* [2] */) {
  unsigned long long rows = 0, entries = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int64_t d = (int64_t)(row_ptr[v + 1] - row_ptr[v]);
    if (d > kRelabelLongDeg) {
      rows += 1;
      entries += (unsigned long long)d;
    }
  }
  rows = wave_sum(rows);
  entries = wave_sum(entries);
  if (lane_id() == 0 && (rows || entries)) {
    atomicAdd(&out[0], rows);
    atomicAdd(&out[1], entries);
  }
}

// Sort keys (smaller key = larger degree bucket) and the identity permutation.
template <typename Off>
__global__ __launch_bounds__(256) void k_relabel_keys(int64_t n, const Off* row_ptr, uint32_t* keys, int32_t* ids) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int64_t d = (int64_t)(row_ptr[v + 1] - row_ptr[v]);
    keys[v] = (uint32_t)(kRelabelBuckets - 1 - min(d, (int64_t)kRelabelBuckets - 1));
    ids[v] = (int32_t)v;
  }
}

// new_of[order[i]] = i, and the degree of every new row.
template <typename Off>
__global__ __launch_bounds__(256) void k_relabel_inverse(int64_t n, const Off* row_ptr, const int32_t* order,
                                                         int32_t* new_of, int64_t* new_deg) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += (int64_t)gridDim.x * blockDim.x) {
    if (i == n) {
      new_deg[n] = 0;
      continue;
    }
    const int32_t u = order[i];
    new_of[u] = (int32_t)i;
    new_deg[i] = (int64_t)(row_ptr[u + 1] - row_ptr[u]);
  }
}

// Rows [0, nlong) (the long ones come first) are copied by one wavefront each,
// the others by one lane each; entries are renamed through new_of.
template <typename Off>
__global__ __launch_bounds__(256) void k_relabel_rows(int64_t n, int64_t nlong, const Off* row_ptr,
                                                      const int32_t* col, const int32_t* order,
                                                      const int32_t* new_of, const int64_t* nrp, int32_t* ncol) {
  const int lane = lane_id();
  const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = (int64_t)gridDim.x * blockDim.x / kWave;
  for (int64_t i = gw; i < nlong; i += nw) {
    const int32_t u = order[i];
    const Off b = row_ptr[u];
    const int64_t d = (int64_t)(row_ptr[u + 1] - b), o = nrp[i];
    for (int64_t j = lane; j < d; j += kWave) ncol[o + j] = new_of[col[b + j]];
  }
  for (int64_t i = nlong + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = order[i];
    const Off b = row_ptr[u];
    const int64_t d = (int64_t)(row_ptr[u + 1] - b), o = nrp[i];
    for (int64_t j = 0; j < d; ++j) ncol[o + j] = new_of[col[b + j]];
  }
}

// Results back to the caller's numbering.
__global__ __launch_bounds__(256) void k_relabel_out(int64_t n, const int32_t* new_of, const int32_t* est_new,
                                                     int32_t* out) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    out[v] = est_new[new_of[v]];
}

}  // namespace kcore
