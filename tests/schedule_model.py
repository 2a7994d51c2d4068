"""CPU model of the round schedule the GPU kernels follow (test infrastructure).

It replays the rules of the round kernels on small graphs, with the reads,
writes and atomics of all vertices of a round interleaved at random:

* estimates start at the degree; a frontier vertex recomputes the h-index of
  the neighbour estimates it read, capped by its own (Sec. II-B, Alg. 1;
  FastK, Sec. IV, Alg. 4), and writes it in place (other vertices of the same
  round may read the old or the new value);
* it records its support slack: neighbours read at or above the new value,
  minus the value;
* a change from e to h makes neighbour v (estimate x as read) a candidate when
  x > h; in the first round every candidate is activated (one-sided rule);
  later, if v is updated in the same kernel of this round, the check is
  deferred: once the round's kernels are over, the drop is charged to v's
  slack if h < est(v) <= e, and v is activated when the slack goes negative
  (with defer=False, v is re-activated at once instead); v is skipped if it is
  updated by the kernel that runs after the current one, and otherwise charged
  against its slack when x <= e (the two-sided rule), activated when the slack
  goes negative;
* class-3 vertices (degree above `big_deg`) run before the others in a round
  (after them with big_first=False);
* in every round, a candidate of the other kernel (class 3 seen from classes
  0..2, or the reverse) read above the vertex's own old value is skipped: it
  was never counted at that level, and it is not updated concurrently;
* in the first round (class-3 kernel first), a class-3 vertex notifies no
  neighbour and puts itself in the next frontier instead, and class-0..2
  vertices skip every class-3 candidate; a class-3 vertex of degree above
  `delay_deg` is not even recomputed there (it keeps its degree and its
  meaningless slack until the second round).

`rule` selects deliberate mistakes, so that tests can show the model would
notice them: "no_frontier_clause" drops the re-activation (or the deferred
check) of same-kernel frontier vertices, "defer_strict_level" defers the check
but leaves out a level equal to e (a drop from e itself), "no_kernel_order" runs both classes interleaved while
keeping the rule that relies on their order, "skip_in_class3_kernel" applies
the class-3 skip inside the class-3 kernel too, where such a candidate may be
updated concurrently, "delay_unqueued" leaves a vertex that sits out the first
round out of the second round's frontier.
"""
import random


def _hindex(vals, cap):
    vals = sorted(vals, reverse=True)
    h = 0
    for i, x in enumerate(vals):
        if x >= i + 1:
            h = i + 1
    return min(h, cap)


def run_model(n, adj, rng: random.Random, big_deg: int, rule: str = "gpu", max_rounds: int = 10_000,
              big_first: bool = True, defer: bool = True, start=None, delay_deg: int | None = None):
    """Coreness of the graph (adjacency lists) under one random schedule; returns (estimates, rounds).

    start = (estimates, frontier[, slack]) begins instead from those estimates with that frontier as an
    ordinary later round and the given slacks, 0 by default (the start of an update after edge changes)."""
    est = [len(adj[u]) for u in range(n)]
    big = [len(adj[u]) > big_deg for u in range(n)]
    stamp = [0] * n
    slack = [rng.randint(-3, 3) for _ in range(n)]  # meaningless until a vertex's first recomputation
    r = 1
    first = True
    frontier = [u for u in range(n) if est[u] >= 2]
    if start is not None:
        est = list(start[0])
        slack = list(start[2]) if len(start) > 2 else [0] * n
        first = False
        frontier = [u for u in start[1] if len(adj[u]) >= 2]
        for u in frontier:
            stamp[u] = r
        rng.shuffle(frontier)
    rounds = 0
    deferred = []

    def proc(u, cur_big):
        e = est[u]
        if e < 2:
            return
        if first and big_first and cur_big and delay_deg is not None and len(adj[u]) > delay_deg:
            if rule != "delay_unqueued":
                stamp[u] = r + 1  # into the second round's frontier, unrecomputed
            return
        reads = []
        for v in adj[u]:
            reads.append((v, est[v]))
            yield
        xs = [x for _, x in reads]
        h = _hindex(xs, e)
        if h < e:
            est[u] = h
        slack[u] = sum(1 for x in xs if x >= h) - h
        yield
        if first and big_first and cur_big:
            stamp[u] = r + 1
            return
        if h == e:
            return
        for v, x in reads:
            other = big[v] != cur_big
            if ((other or (rule == "skip_in_class3_kernel" and cur_big)) and (x > e or (first and big_first and not cur_big))):
                yield
                continue
            if x > h and stamp[v] < r + 1:
                act = False
                if first:
                    act = True
                elif stamp[v] == r and big[v] == cur_big:
                    if rule == "no_frontier_clause":
                        act = False
                    elif defer:
                        deferred.append((v, e, h))
                    else:
                        act = True
                elif stamp[v] == r and cur_big == big_first:
                    act = False  # v is updated by the kernel that runs after the current one
                elif x <= e:
                    old = slack[v]
                    slack[v] = old - 1
                    act = old <= 0
                if act:
                    stamp[v] = r + 1
            yield

    while frontier:
        rounds += 1
        if rounds > max_rounds:
            raise RuntimeError("model did not converge")
        phases = [None] if rule == "no_kernel_order" else [big_first, not big_first]
        for ph in phases:
            gens = [proc(u, big[u]) for u in frontier if ph is None or big[u] == ph]
            live = list(range(len(gens)))
            while live:
                i = rng.choice(live)
                try:
                    next(gens[i])
                except StopIteration:
                    live.remove(i)
        # the deferred same-kernel checks, after the round's kernels
        rng.shuffle(deferred)
        for v, e, h in deferred:
            lv = est[v]
            crossed = h < lv < e if rule == "defer_strict_level" else h < lv <= e
            if crossed and stamp[v] < r + 1:
                old = slack[v]
                slack[v] = old - 1
                if old <= 0:
                    stamp[v] = r + 1
        deferred.clear()
        first = False
        r += 1
        frontier = [u for u in range(n) if stamp[u] == r]
        rng.shuffle(frontier)
    return est, rounds


def random_graph(rng: random.Random, nmax: int = 28):
    n = rng.randint(2, nmax)
    p = rng.uniform(0.05, 0.8)
    adj = [set() for _ in range(n)]
    for u in range(n):
        for v in range(u + 1, n):
            if rng.random() < p:
                adj[u].add(v)
                adj[v].add(u)
    return n, [sorted(a) for a in adj]
