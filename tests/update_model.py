"""CPU model of the start of an update run after edge changes (test infrastructure).

It restates, in plain Python, the bounds and the frontier that the update's
start kernels set (core maintenance, the paper's future work on dynamic
graphs, Sec. VI), so that tests can run the round schedule model from them and
compare with the oracle on the changed graph:

* every vertex starts at its old coreness c_old (removals only lower coreness);
* the endpoints of removed edges start in the frontier;
* with insertions, T = min and K_max = max over inserted edges of
  min(c_old(u), c_old(v)), and D = the largest number of inserted edges at one
  vertex; the set A is found by a search in the changed graph.  While
  D <= window_max (4 on the GPU; the window rule) its states are (vertex x, window top c) with
  c_old(x) <= c <= c_old(x) + D - 1: it starts from (u, c) for each endpoint u
  of an inserted edge with c <= K + D - 1 (K = the edge's min(c_old(u),
  c_old(v))), moves to the neighbours y with c_old(y) in [c + 1 - D, c], and a
  vertex joins A when its state of window top c_old(y) is reached (for D = 1,
  the subcores of the lower endpoints).  Otherwise (the threshold rule) it
  moves from the inserted endpoints through vertices of old coreness >= T.  A
  search that reaches more than `budget` states is given up, and A is then
  every vertex of old coreness >= T (a superset); A starts at
  max(c_old, min(degree, c_old + D, K_max + D)), every other vertex at c_old;
* the heavy-vertex rule, tried first when D >= 2: Z = the vertices with two or
  more inserted edges, D' = the largest, over the other vertices, of their edges
  to Z plus their inserted edges to vertices outside Z.  When D' <= 1 a vertex
  outside Z rises by at most 1 and, if it rises, shares its old shell with a
  source: a neighbour of Z outside Z, or the lower endpoint of an inserted edge
  outside Z.  The search then starts from the sources, keeps to old shells and
  never enters Z; Z is in A with rise D, the rest of A with rise 1, and a
  search given up takes the vertices of old coreness >= the smallest old
  coreness of a source;
* a vertex left with degree 0 or 1 starts at its degree, out of the frontier,
  and its neighbour joins the frontier;
* every slack starts at 0, except, when nothing was removed, on the vertices
  out of the frontier (their old coreness is then final): SLACK_FINAL.

`rule` selects deliberate mistakes that the tests must catch: "threshold_too_high"
(T one above that minimum), "rise_by_one" (D taken as 1), "cap_too_low" (K_max + D - 1
in place of K_max + D), "z_no_neighbour_sources" (the heavy-vertex search
without the neighbours of Z as sources), "z_rise_one" (heavy vertices raised by
1 only), "z_threshold_too_high" (a heavy-vertex search given up takes one shell
too few), "no_removal_seed" (removal endpoints left out of the
frontier), "window_from_upper" (the window search started from each edge's
upper endpoints only), "window_narrow" (windows [c + 2 - D, c]),
"endpoints_only" (A = the inserted
endpoints, no search), "clamp_to_degree" (removal endpoints start at
min(c_old, degree), which drops support unannounced), "no_neighbour_seed" (a
vertex left with degree 1 does not seed its neighbour), "final_with_removals"
(the final slack given also when edges were removed).
"""

SLACK_FINAL = 1 << 30


def update_start(adj, prev, removed, inserted, rule: str = "gpu", budget=None, window_max: int = 4):
    """(estimates, frontier, slacks) of an update of the graph `adj` (after the changes) from coreness `prev`."""
    n = len(adj)
    nd, ni = len(removed), len(inserted)
    flag = [0] * n
    all_from = float("inf")
    for u, v in removed:
        flag[u] |= 1
        flag[v] |= 1
    if ni:
        kmin = min(min(prev[u], prev[v]) for u, v in inserted)
        T = kmin + 1 if rule == "threshold_too_high" else kmin
        kmax = max(min(prev[u], prev[v]) for u, v in inserted)
        hits = [0] * n
        for u, v in inserted:
            hits[u] += 1
            hits[v] += 1
        D = 1 if rule == "rise_by_one" else max(hits)
        cap = kmax + D - (1 if rule == "cap_too_low" else 0)
        window = D <= window_max
        seen = set()  # reached states
        queue = []
        # the heavy-vertex rule: Z = vertices with two or more inserted edges; if every other vertex has at
        # most one edge to Z or inserted edge to a vertex outside Z (D' <= 1), a vertex outside Z rises by
        # at most 1, the search keeps to old shells, starts from the lower endpoints of the inserted edges
        # outside Z and from every neighbour of Z, and never enters Z; Z itself is in A
        Z = {x for x in range(n) if hits[x] >= 2}
        zrule = False
        if Z and rule != "no_z_rule":
            cnt = [0] * n
            for z in Z:
                for y in adj[z]:
                    if y not in Z:
                        cnt[y] += 1
            for u, v in inserted:
                if u not in Z and v not in Z:
                    cnt[u] += 1
                    cnt[v] += 1
            zrule = max(cnt) <= 1
        if zrule:
            # a vertex outside Z that rises shares its old shell with a source, so a search given up
            # takes the vertices of old coreness >= the smallest old coreness of a source
            T = min([prev[y] for z in Z for y in adj[z] if y not in Z]
                    + [min(prev[u], prev[v]) for u, v in inserted if u not in Z and v not in Z], default=T)
            T += 1 if rule == "z_threshold_too_high" else 0

        def reach(x, j):
            if (x, j) in seen:
                return
            seen.add((x, j))
            if j == 0:
                flag[x] |= 2
            queue.append((x, j))

        if zrule:
            for z in Z:
                flag[z] |= 2
                if rule != "z_no_neighbour_sources":
                    for y in adj[z]:
                        if y not in Z:
                            reach(y, 0)
            for u, v in inserted:
                if u in Z or v in Z:
                    continue
                for w, o in ((u, v), (v, u)):
                    if prev[w] <= prev[o]:
                        reach(w, 0)
        else:
            for u, v in inserted:
                for w, o in ((u, v), (v, u)):
                    if rule == "window_from_upper" and prev[w] < prev[o]:
                        continue
                    if window:
                        for j in range(min(prev[w], prev[o]) + D - prev[w]):
                            reach(w, j)
                    else:
                        reach(w, 0)
        while queue and rule != "endpoints_only":
            if budget is not None and len(seen) > budget:
                all_from = T
                break
            q, j = queue.pop()
            c = prev[q] + j
            if zrule:
                for y in adj[q]:
                    if prev[y] == c and y not in Z:
                        reach(y, 0)
                continue
            lo = (c + 1 - D + (1 if rule == "window_narrow" else 0)) if window else T
            hi = c if window else float("inf")
            for y in adj[q]:
                if lo <= prev[y] <= hi:
                    reach(y, c - prev[y] if window else 0)
    est = [0] * n
    slack = [0] * n
    frontier = set()
    for v in range(n):
        d, c = len(adj[v]), prev[v]
        rise = D if ni else 0
        if ni and zrule:
            rise = 1 if (v not in Z or rule == "z_rise_one") else D
        x = max(c, min(d, c + rise, cap)) if flag[v] & 2 or c >= all_from else c
        if rule == "clamp_to_degree" and flag[v] & 1:
            x = min(x, d)
        seed = (flag[v] & 1 and rule != "no_removal_seed") or x > c
        if d <= 1 and x > d:
            x = d
            if d == 1 and rule != "no_neighbour_seed":
                frontier.add(adj[v][0])
        if seed and d >= 2:
            frontier.add(v)
        elif nd == 0 or rule == "final_with_removals":
            slack[v] = SLACK_FINAL
        est[v] = x
    return est, sorted(frontier), slack
