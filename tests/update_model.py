"""CPU model of the start of an update run after edge changes (test infrastructure).

It restates, in plain Python, the bounds and the frontier that the update's
start kernels set (core maintenance, the paper's future work on dynamic
graphs, Sec. VI), so that tests can run the round schedule model from them and
compare with the oracle on the changed graph:

* every vertex starts at its old coreness c_old (removals only lower coreness);
* the endpoints of removed edges start in the frontier;
* with insertions, T = min over inserted edges of min(c_old(u), c_old(v)); the
  vertices reached from the inserted endpoints, in the changed graph, through
  vertices of old coreness >= T (the set A) start at
  max(c_old, min(degree, c_old + number of insertions)) and in the frontier;
* a vertex left with degree 0 or 1 starts at its degree, out of the frontier,
  and its neighbour joins the frontier.

`rule` selects deliberate mistakes that the tests must catch: "threshold_too_high"
(T one above that minimum), "endpoints_only" (A = the inserted
endpoints, no search), "clamp_to_degree" (removal endpoints start at
min(c_old, degree), which drops support unannounced), "no_neighbour_seed" (a
vertex left with degree 1 does not seed its neighbour).
"""


def update_start(adj, prev, removed, inserted, rule: str = "gpu"):
    """(estimates, frontier) of an update of the graph `adj` (after the changes) from coreness `prev`."""
    n = len(adj)
    nd, ni = len(removed), len(inserted)
    flag = [0] * n
    for u, v in removed:
        flag[u] |= 1
        flag[v] |= 1
    if ni:
        kmin = min(min(prev[u], prev[v]) for u, v in inserted)
        T = kmin + 1 if rule == "threshold_too_high" else kmin
        queue = []
        for u, v in inserted:
            for w in (u, v):
                if not flag[w] & 2:
                    flag[w] |= 2
                    queue.append(w)
        while queue and rule != "endpoints_only":
            q = queue.pop()
            for w in adj[q]:
                if prev[w] >= T and not flag[w] & 2:
                    flag[w] |= 2
                    queue.append(w)
    est = [0] * n
    frontier = set()
    for v in range(n):
        d, c = len(adj[v]), prev[v]
        x = max(c, min(d, c + ni)) if flag[v] & 2 else c
        if rule == "clamp_to_degree" and flag[v] & 1:
            x = min(x, d)
        seed = flag[v] != 0
        if d <= 1 and x > d:
            x = d
            if d == 1 and rule != "no_neighbour_seed":
                frontier.add(adj[v][0])
        if seed and d >= 2:
            frontier.add(v)
        est[v] = x
    return est, sorted(frontier)
