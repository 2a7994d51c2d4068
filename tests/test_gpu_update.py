"""Core maintenance (kcore_update): coreness after edge removals and insertions, started from the
coreness before them, equals the oracle's coreness of the changed graph, bit for bit."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from tests import small_graphs as sg

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def kc():
    import paper_2512_00233_amd as kc
    return kc


def edges_of(g):
    """Undirected edges (u < v) of a CSR graph."""
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))
    m = src < g.col_idx
    return np.stack([src[m], g.col_idx[m].astype(np.int64)], axis=1)


def change(g, n_remove, n_insert, seed):
    """Graph g with n_remove of its edges removed and n_insert new edges added (seeded)."""
    rng = np.random.default_rng(seed)
    e = edges_of(g)
    rem_idx = rng.choice(e.shape[0], size=min(n_remove, e.shape[0]), replace=False)
    removed = e[rem_idx]
    keep = np.ones(e.shape[0], bool)
    keep[rem_idx] = False
    ins = set()
    while len(ins) < n_insert:
        u, v = (int(x) for x in rng.integers(0, g.n, 2))
        a, b = min(u, v), max(u, v)
        # rows are sorted: an existing edge is found by binary search in row a
        row = g.col_idx[g.row_ptr[a]:g.row_ptr[a + 1]]
        j = int(np.searchsorted(row, b))
        if a != b and not (j < row.size and row[j] == b) and (a, b) not in ins:
            ins.add((a, b))
    inserted = np.array(sorted(ins), np.int64).reshape(-1, 2)
    new_e = np.concatenate([e[keep], inserted])
    g2 = gg.from_edges(g.n, new_e[:, 0], new_e[:, 1])
    return g2, removed, inserted


def run_update(g_new, prev, removed, inserted, in_place=False, tuning=None, stats=None):
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(g_new.row_ptr).to(dev)
    ci = torch.from_numpy(g_new.col_idx).to(dev)
    pv = torch.from_numpy(np.ascontiguousarray(prev, np.int32)).to(dev)
    rm = torch.from_numpy(np.ascontiguousarray(removed, np.int32).reshape(-1, 2)).to(dev)
    ins = torch.from_numpy(np.ascontiguousarray(inserted, np.int32).reshape(-1, 2)).to(dev)
    out = kc().update(rp, ci, pv, rm, ins, out=pv if in_place else None, tuning=tuning, stats=stats)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def check(name, g, n_remove, n_insert, seed, **kw):
    g2, removed, inserted = change(g, n_remove, n_insert, seed)
    prev = oracle.coreness(g.row_ptr, g.col_idx)
    ref = oracle.coreness(g2.row_ptr, g2.col_idx)
    print(f"[update] {name}: n={g.n} -{len(removed)} +{len(inserted)} changed={(prev != ref).sum()} {kw}",
          flush=True)
    got = run_update(g2, prev, removed, inserted, **kw)
    if not np.array_equal(got, ref):
        bad = np.nonzero(got != ref)[0]
        raise AssertionError(f"{name}: {bad.size} mismatches, first v={bad[0]} gpu={got[bad[0]]} ref={ref[bad[0]]} "
                             f"prev={prev[bad[0]]}")


@pytest.mark.parametrize("name", ["rmat20", "road_512", "rmat16", "er_small"])
@pytest.mark.parametrize("n_remove,n_insert", [(1, 0), (1000, 0), (0, 1), (0, 1000), (500, 500), (20000, 0)])
def test_update_matches_oracle(name, n_remove, n_insert):
    g = gg.workload(name)
    check(name, g, n_remove, n_insert, seed=n_remove * 7 + n_insert)


@pytest.mark.parametrize("tuning", [dict(activation=1), dict(activation=2, deferred=1), dict(tail_threshold=-1),
                                    dict(no_prune=1, list_cap=1), dict(thread_max_deg=1, group_max_deg=1,
                                                                       wave_max_deg=1),
                                    dict(tail_order=1, tail_big=1, tail_threshold=1 << 30)])
def test_update_tunings_and_in_place(tuning):
    g = gg.workload("rmat16")
    t = kc().Tuning(**tuning)
    check("rmat16", g, 300, 300, seed=5, tuning=t)
    check("rmat16/in place", g, 300, 300, seed=6, tuning=t, in_place=True)


@pytest.mark.parametrize("name", ["rmat24", "road"])
def test_update_at_full_size(name):
    # the full 16.8M-vertex workloads: a mixed batch of 1,000 removals and 1,000 insertions, against the
    # oracle on the changed graph (element by element) and the device certificate
    g = gg.workload(name)
    g2, removed, inserted = change(g, 1000, 1000, seed=77)
    prev = oracle.coreness_bz(g.row_ptr, g.col_idx)
    ref = oracle.coreness_bz(g2.row_ptr, g2.col_idx)
    print(f"[update] {name} full size: -{len(removed)} +{len(inserted)} changed={(prev != ref).sum()}", flush=True)
    got = run_update(g2, prev, removed, inserted)
    assert np.array_equal(got, ref)
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(g2.row_ptr).to(dev)
    ci = torch.from_numpy(g2.col_idx).to(dev)
    assert kc().certify(rp, ci, torch.from_numpy(got).to(dev)) == (0, -1)


def test_update_and_certificate_with_int32_offsets():
    # kcore_update32 / kcore_certify32: the int32-offset graph of ER small, removals and insertions
    g = gg.workload("er_small")
    dev = torch.device("cuda:0")
    for n_remove, n_insert, seed in ((50, 0, 1), (0, 50, 2), (300, 300, 3)):
        g2, removed, inserted = change(g, n_remove, n_insert, seed)
        prev = oracle.coreness(g.row_ptr, g.col_idx)
        ref = oracle.coreness(g2.row_ptr, g2.col_idx)
        rp = torch.from_numpy(g2.row_ptr.astype(np.int32)).to(dev)
        ci = torch.from_numpy(g2.col_idx).to(dev)
        pv = torch.from_numpy(prev).to(dev)
        rm = torch.from_numpy(removed.astype(np.int32).reshape(-1, 2)).to(dev)
        it = torch.from_numpy(inserted.astype(np.int32).reshape(-1, 2)).to(dev)
        got = kc().update(rp, ci, pv, rm, it)
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), ref), (n_remove, n_insert)
        assert kc().certify(rp, ci, got) == (0, -1)
        bad = got.clone()
        v = int(np.argmax(ref))
        bad[v] += 1  # above its support
        code, vertex = kc().certify(rp, ci, bad)
        assert code != 0 and vertex <= v


def test_update_degenerate_changes():
    # no change at all: the old coreness comes back
    g = gg.workload("road_512")
    prev = oracle.coreness(g.row_ptr, g.col_idx)
    none = np.zeros((0, 2), np.int32)
    assert np.array_equal(run_update(g, prev, none, none), prev)
    # a clique losing edges down to a path-like remainder, vertices left isolated or with one neighbour
    n, edges = sg.complete(30)
    rp, ci = sg.to_csr(n, edges)
    full = gg.Graph(rp, ci)
    e = edges_of(full)
    rng = np.random.default_rng(3)
    for k in (1, 50, 300, 420, 435):
        keep = np.ones(e.shape[0], bool)
        keep[rng.choice(e.shape[0], k, replace=False)] = False
        g2 = gg.from_edges(n, e[keep, 0], e[keep, 1])
        ref = oracle.coreness(g2.row_ptr, g2.col_idx)
        got = run_update(g2, oracle.coreness(rp, ci), e[~keep], none)
        assert np.array_equal(got, ref), k
        # and back: insert the same edges into the reduced graph
        back = run_update(full, ref, none, e[~keep])
        assert np.array_equal(back, oracle.coreness(rp, ci)), k
    # a path grown edge by edge from isolated vertices, then the middle edge removed
    n = 1000
    cur = gg.from_edges(n, np.zeros(0, np.int32), np.zeros(0, np.int32))
    core = np.zeros(n, np.int32)
    for i in range(0, n - 1, 97):
        src = np.arange(0, i + 1)
        nxt = gg.from_edges(n, src, src + 1)
        new_edges = edges_of(nxt)
        old_edges = set(map(tuple, edges_of(cur).tolist()))
        added = np.array([x for x in new_edges.tolist() if tuple(x) not in old_edges], np.int64).reshape(-1, 2)
        core = run_update(nxt, core, none, added)
        assert np.array_equal(core, oracle.coreness(nxt.row_ptr, nxt.col_idx)), i
        cur = nxt


def test_update_insertions_into_dense_cores():
    # insertions that raise cores: edges added inside and between dense parts of a power-law graph
    g = gg.chung_lu(100_000, 2.1, 16, seed=91)
    for k, seed in ((1, 1), (10, 2), (5000, 3)):
        check("chung_lu", g, 0, k, seed=seed)
        check("chung_lu mixed", g, k, k, seed=seed + 10)


def local_insertions(g, k, seed):
    """k new edges, each closing a triangle (a vertex joined to a neighbour of a neighbour), so that both
    ends lie in the same dense region; returns (new graph, inserted edges)."""
    rng = np.random.default_rng(seed)
    e = edges_of(g)
    existing = set(map(tuple, e.tolist()))
    ins = set()
    while len(ins) < k:
        u = int(rng.integers(0, g.n))
        nb = g.col_idx[g.row_ptr[u]:g.row_ptr[u + 1]]
        if nb.size == 0:
            continue
        x = int(rng.choice(nb))
        v = int(rng.choice(g.col_idx[g.row_ptr[x]:g.row_ptr[x + 1]]))
        a, b = min(u, v), max(u, v)
        if a != b and (a, b) not in existing:
            ins.add((a, b))
    inserted = np.array(sorted(ins), np.int64).reshape(-1, 2)
    new_e = np.concatenate([e, inserted])
    return gg.from_edges(g.n, new_e[:, 0], new_e[:, 1]), inserted


@pytest.mark.parametrize("name,k", [("rmat20", 1), ("rmat20", 10), ("rmat20", 300), ("rmat20", 3000),
                                    ("road_512", 1), ("road_512", 1000), ("rmat16", 100)])
def test_update_local_insertions(name, k):
    # triangle-closing insertions: with one inserted edge per vertex (D = 1) the search follows the
    # subcores of the lower endpoints, which on a skewed graph cross hub rows of many thousand entries
    g = gg.workload(name)
    g2, inserted = local_insertions(g, k, seed=k + 17)
    D = int(np.bincount(inserted.ravel(), minlength=g.n).max())
    prev = oracle.coreness(g.row_ptr, g.col_idx)
    ref = oracle.coreness(g2.row_ptr, g2.col_idx)
    print(f"[update] {name} +{k} local: D={D} changed={(prev != ref).sum()}", flush=True)
    st = kc().Stats()
    got = run_update(g2, prev, np.zeros((0, 2), np.int64), inserted, stats=st)
    assert np.array_equal(got, ref)


def test_update_search_keeps_to_the_touched_component():
    # one graph made of 40 disjoint power-law parts; six insertions inside one part, with D = 1, 3, 4, 5, 6:
    # the search stays inside that part, so the run recomputes a small share of the vertices, and the
    # result is exact
    parts = [gg.chung_lu(5000, 2.3, 12, seed=300 + i) for i in range(40)]
    src, dst, off = [], [], 0
    for p in parts:
        e = edges_of(p)
        src.append(e[:, 0] + off)
        dst.append(e[:, 1] + off)
        off += p.n
    g = gg.from_edges(off, np.concatenate(src), np.concatenate(dst))
    prev = oracle.coreness(g.row_ptr, g.col_idx)
    e = edges_of(g)
    existing = set(map(tuple, e.tolist()))
    rng = np.random.default_rng(8)
    base = 7 * 5000  # part 7
    # D = 1, 3 and 4 take the window rule, D = 5 and 6 the threshold rule
    for star in (1, 3, 4, 5, 6):
        ins = []
        hub = base + int(rng.integers(0, 5000))
        while len(ins) < 6:
            u = hub if len(ins) < star and star > 1 else base + int(rng.integers(0, 5000))
            v = base + int(rng.integers(0, 5000))
            a, b = min(u, v), max(u, v)
            used = [x for pair in ins for x in pair if x != hub or star == 1]
            if a != b and (a, b) not in existing and (a, b) not in ins and not (
                    (a in used and a != hub) or (b in used and b != hub) or (star == 1 and hub in (a, b))):
                ins.append((a, b))
        inserted = np.array(ins, np.int64)
        D = int(np.bincount(inserted.ravel(), minlength=g.n).max())
        assert D == star, (D, star)
        new_e = np.concatenate([e, inserted])
        g2 = gg.from_edges(g.n, new_e[:, 0], new_e[:, 1])
        ref = oracle.coreness(g2.row_ptr, g2.col_idx)
        st = kc().Stats()
        got = run_update(g2, prev, np.zeros((0, 2), np.int64), inserted, stats=st)
        print(f"[update] 40 parts, +6 in one part (D={D}): vertex updates {st.vertex_updates} of n={g.n}",
              flush=True)
        assert np.array_equal(got, ref)
        assert st.vertex_updates < g.n // 4  # a search abandoned for all of old coreness >= T would exceed it


def test_update_time_against_full_recompute():
    # the point of an update: a small change costs far less than a full decomposition
    import time
    g = gg.workload("rmat20")
    dev = torch.device("cuda:0")
    for n_remove, n_insert in ((100, 0), (0, 100)):
        g2, removed, inserted = change(g, n_remove, n_insert, seed=42)
        prev = oracle.coreness(g.row_ptr, g.col_idx)
        rp = torch.from_numpy(g2.row_ptr).to(dev)
        ci = torch.from_numpy(g2.col_idx).to(dev)
        pv = torch.from_numpy(prev).to(dev)
        rm = torch.from_numpy(removed.astype(np.int32).reshape(-1, 2)).to(dev)
        ins = torch.from_numpy(inserted.astype(np.int32).reshape(-1, 2)).to(dev)
        out = torch.empty_like(pv)
        for _ in range(2):
            kc().update(rp, ci, pv, rm, ins, out=out)
            kc().decompose(rp, ci, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            kc().update(rp, ci, pv, rm, ins, out=out)
        torch.cuda.synchronize()
        t_upd = (time.perf_counter() - t0) / 5
        got = out.cpu().numpy()
        t0 = time.perf_counter()
        for _ in range(5):
            kc().decompose(rp, ci, out=out)
        torch.cuda.synchronize()
        t_full = (time.perf_counter() - t0) / 5
        print(f"[update] rmat20 -{n_remove} +{n_insert}: update {t_upd * 1e3:.3f} ms, full {t_full * 1e3:.3f} ms",
              flush=True)
        assert np.array_equal(got, out.cpu().numpy())
        assert np.array_equal(got, oracle.coreness(g2.row_ptr, g2.col_idx))


def arrivals(g, m, k, seed, prop=True, off=False):
    """m vertices arrive (isolated vertices where the graph has them) with k edges each, to targets drawn in
    proportion to degree (prop) or uniformly.  With `off`, a vertex w of the graph also gains two edges and
    the first arrival an edge to a neighbour y of w: y, outside Z, then has two edges to Z (D' = 2).
    Returns (new graph, inserted edges)."""
    rng = np.random.default_rng(seed)
    deg = np.diff(g.row_ptr)
    iso = np.flatnonzero(deg == 0)
    zs = [int(z) for z in (rng.choice(iso, m, replace=False) if iso.size >= m else rng.choice(g.n, m, replace=False))]

    def row(x):
        return set(g.col_idx[g.row_ptr[x]:g.row_ptr[x + 1]].tolist())

    ins = set()
    for z in zs:
        rz, targets = row(z), set()
        while len(targets) < k:
            t = int(g.col_idx[rng.integers(0, g.col_idx.size)]) if prop else int(rng.integers(0, g.n))
            if t != z and t not in rz:
                targets.add(t)
        ins |= {(min(z, t), max(z, t)) for t in targets}
    if off:
        busy = {x for pair in ins for x in pair}
        while True:
            w = int(g.col_idx[rng.integers(0, g.col_idx.size)])
            y = int(rng.choice(g.col_idx[g.row_ptr[w]:g.row_ptr[w + 1]]))
            if w not in busy and y not in busy and y not in row(zs[0]):
                break
        rw, extra = row(w), set()
        while len(extra) < 2:
            t = int(rng.integers(0, g.n))
            if t not in rw and t not in busy and t not in (w, y):
                extra.add(t)
        ins |= {(min(w, t), max(w, t)) for t in extra} | {(min(zs[0], y), max(zs[0], y))}
    inserted = np.array(sorted(ins), np.int64).reshape(-1, 2)
    e = edges_of(g)
    new_e = np.concatenate([e, inserted])
    return gg.from_edges(g.n, new_e[:, 0], new_e[:, 1]), inserted


def heavy_rule_applies(g2, inserted):
    """D' <= 1: every vertex outside Z (two or more inserted edges) has at most one edge to Z plus inserted
    edge to a vertex outside Z."""
    hits = np.bincount(inserted.ravel(), minlength=g2.n)
    z = hits >= 2
    if not z.any():
        return False
    src = np.repeat(np.arange(g2.n), np.diff(g2.row_ptr))
    cnt = np.bincount(g2.col_idx[z[src]], minlength=g2.n)
    out = inserted[~z[inserted[:, 0]] & ~z[inserted[:, 1]]]
    cnt += np.bincount(out.ravel(), minlength=g2.n)
    return int(cnt[~z].max()) <= 1


@pytest.mark.parametrize("name", ["rmat20", "road_512", "rmat16", "er_small"])
@pytest.mark.parametrize("m,k,prop,off", [(1, 2, True, False), (1, 8, True, False), (1, 64, False, False),
                                          (3, 8, True, False), (20, 5, False, False), (2, 4, True, True)])
def test_update_vertex_arrivals(name, m, k, prop, off):
    # vertices that arrive with several edges each (D = k): the heavy-vertex rule where it applies, and
    # left off where a vertex outside Z has two edges to Z; exact either way
    g = gg.workload(name)
    g2, inserted = arrivals(g, m, k, seed=m * 100 + k, prop=prop, off=off)
    prev = oracle.coreness(g.row_ptr, g.col_idx)
    ref = oracle.coreness(g2.row_ptr, g2.col_idx)
    rule = heavy_rule_applies(g2, inserted)
    st = kc().Stats()
    got = run_update(g2, prev, np.zeros((0, 2), np.int64), inserted, stats=st)
    print(f"[update] {name}: {m} arrivals x {k} edges (prop={prop}, off={off}): heavy rule {rule}, "
          f"changed {(prev != ref).sum()}, vertex updates {st.vertex_updates} of n={g.n}", flush=True)
    if off:
        assert not rule
    assert np.array_equal(got, ref)
    # 300 removals mixed in (edges of the old graph, or arrivals' edges, which are then not inserted)
    g3, removed, _ = change(g2, 300, 0, seed=5)
    key_rem = removed[:, 0] * g.n + removed[:, 1]
    key_ins = inserted[:, 0] * g.n + inserted[:, 1]
    got3 = run_update(g3, prev, removed[~np.isin(key_rem, key_ins)], inserted[~np.isin(key_ins, key_rem)])
    assert np.array_equal(got3, oracle.coreness(g3.row_ptr, g3.col_idx))


def test_update_vertex_arrival_is_local():
    # one vertex arriving with 16 edges to high-degree vertices of R-MAT scale 20: with the heavy-vertex rule
    # the bounds rise by 1 on the targets' shells only, so the run recomputes a small share of the vertices
    g = gg.workload("rmat20")
    g2, inserted = arrivals(g, 1, 16, seed=4, prop=True)
    assert heavy_rule_applies(g2, inserted)
    prev = oracle.coreness(g.row_ptr, g.col_idx)
    ref = oracle.coreness(g2.row_ptr, g2.col_idx)
    st = kc().Stats()
    got = run_update(g2, prev, np.zeros((0, 2), np.int64), inserted, stats=st)
    print(f"[update] rmat20, one arrival x 16: vertex updates {st.vertex_updates} of n={g.n}", flush=True)
    assert np.array_equal(got, ref)
    assert st.vertex_updates < g.n // 8  # D = 16 by the threshold rule would restart every vertex


def test_update_window_search_on_small_dense_graphs():
    # dense graphs of 12 to 80 vertices with D = 2, 3 or 4 inserted edges at one vertex (the window rule, whose
    # states are vertex and window offset, so one level can hold more states than there are vertices) and
    # further single insertions: exact, with the search given up where it would overflow its queues
    rng = np.random.default_rng(21)
    for case in range(60):
        n = int(rng.integers(12, 81))
        a = np.triu(rng.random((n, n)) < rng.uniform(0.3, 0.85), 1)
        u, v = np.nonzero(a)
        full = gg.from_edges(n, u, v)
        e = edges_of(full)
        D = int(rng.integers(2, 5))
        hub = int(rng.integers(0, n))
        at_hub = np.flatnonzero((e[:, 0] == hub) | (e[:, 1] == hub))
        if at_hub.size < D:
            continue
        pick = set(rng.choice(at_hub, D, replace=False).tolist())
        used = {hub} | {int(x) for i in pick for x in e[i]}
        for i in rng.permutation(e.shape[0])[:40]:
            if len(pick) >= D + 6:
                break
            if int(e[i, 0]) not in used and int(e[i, 1]) not in used:
                pick.add(int(i))
                used |= {int(e[i, 0]), int(e[i, 1])}
        ins = np.zeros(e.shape[0], bool)
        ins[sorted(pick)] = True
        old = gg.from_edges(n, e[~ins, 0], e[~ins, 1])
        prev = oracle.coreness(old.row_ptr, old.col_idx)
        got = run_update(full, prev, np.zeros((0, 2), np.int32), e[ins])
        assert np.array_equal(got, oracle.coreness(full.row_ptr, full.col_idx)), (case, n, D)
