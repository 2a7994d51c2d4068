"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, bit-exact.

Coreness is integer, so the bar is equality on every vertex (tolerance 0).
Every GPU result is also run through the oracle's local certificate.
"""
import os

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


def run_gpu(row_ptr, col_idx, int32_rows=False, tuning=None, stats=None):
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(np.ascontiguousarray(row_ptr, dtype=np.int32 if int32_rows else np.int64)).to(dev)
    ci = torch.from_numpy(np.ascontiguousarray(col_idx, dtype=np.int32)).to(dev)
    out = kc().decompose(rp, ci, tuning=tuning, stats=stats)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def certify_gpu(row_ptr, col_idx, core):
    """The device certificate (kcore_certify) of a coreness vector."""
    dev = torch.device("cuda:0")
    return kc().certify(torch.from_numpy(np.ascontiguousarray(row_ptr, dtype=np.int64)).to(dev),
                        torch.from_numpy(np.ascontiguousarray(col_idx, dtype=np.int32)).to(dev),
                        torch.from_numpy(np.ascontiguousarray(core, dtype=np.int32)).to(dev))


def assert_parity(name, row_ptr, col_idx, **kw):
    print(f"[parity] {name}: n={len(row_ptr) - 1} nnz={len(col_idx)} {kw}", flush=True)
    got = run_gpu(row_ptr, col_idx, **kw)
    ref = oracle.coreness(row_ptr, col_idx)
    if not np.array_equal(got, ref):
        bad = np.nonzero(got != ref)[0]
        raise AssertionError(f"{name}: {bad.size} mismatches, first v={bad[0]} gpu={got[bad[0]]} ref={ref[bad[0]]}")
    assert oracle.check(row_ptr, col_idx, got)[0] == 0
    assert certify_gpu(row_ptr, col_idx, got) == (0, -1)
    return got


def test_device_certificate_agrees_with_the_cpu_one():
    # the device certificate and the oracle's certificate give the same verdict on planted mistakes
    g = gg.workload("rmat16")
    core = oracle.coreness(g.row_ptr, g.col_idx)
    assert certify_gpu(g.row_ptr, g.col_idx, core) == (0, -1)
    deg = np.diff(g.row_ptr)
    rng = np.random.default_rng(4)
    cases = []
    bad = core.copy()
    v = int(np.argmax(deg > 3))
    bad[v] = deg[v] + 1
    cases.append(bad)                      # above the degree
    bad = core.copy()
    bad[int(np.argmax(deg == 0))] = 1
    cases.append(bad)                      # isolated vertex with a core
    bad = core.copy()
    v = int(np.argmax(core == core.max()))
    bad[v] = core.max() + 1
    cases.append(bad)                      # support too small at the raised level
    bad = np.where(core == core.max(), core - 1, core).astype(np.int32)
    cases.append(bad)                      # passes locally although it is not the coreness (not maximal)
    bad = core.copy()
    bad[rng.integers(0, g.n, 50)] += 3
    cases.append(bad)
    for c in cases:
        code_cpu, v_cpu = oracle.check(g.row_ptr, g.col_idx, c)
        code_gpu, v_gpu = certify_gpu(g.row_ptr, g.col_idx, c)
        assert code_gpu == code_cpu, (code_gpu, code_cpu)
        if code_cpu in (1, 2, 3):
            assert v_gpu == v_cpu, (v_gpu, v_cpu)


# ---------------------------------------------------------------- small fixtures
def test_golden_small_graphs():
    from tests.golden.load import small_graphs
    for name, n, edges, core in small_graphs():
        rp, ci = sg.to_csr(n, edges)
        got = run_gpu(rp, ci)
        assert got.tolist() == core, name


def test_closed_forms():
    cases = [
        ("K40", sg.complete(40), 39),
        ("C1000", sg.cycle(1000), 2),
        ("grid64x80", sg.grid(64, 80), 2),
        ("Q8", sg.hypercube(8), 8),
        ("K30,50", sg.complete_bipartite(30, 50), 30),
        ("petersen", sg.petersen(), 3),
        ("wheel50", sg.wheel(50), 3),
    ]
    for name, (n, edges), k in cases:
        rp, ci = sg.to_csr(n, edges)
        assert run_gpu(rp, ci).tolist() == [k] * n, name


# ---------------------------------------------------------------- edge cases
def test_empty_and_degenerate():
    assert run_gpu(np.zeros(1, np.int64), np.zeros(0, np.int32)).size == 0          # n = 0
    assert run_gpu(np.zeros(2, np.int64), np.zeros(0, np.int32)).tolist() == [0]   # n = 1
    assert run_gpu(np.zeros(1001, np.int64), np.zeros(0, np.int32)).tolist() == [0] * 1000  # no edges
    rp, ci = sg.to_csr(2, [(0, 1)])
    assert run_gpu(rp, ci).tolist() == [1, 1]


def test_star_with_a_million_leaves():
    n, edges = sg.star(1_000_000)
    g = gg.from_edges(n, [e[0] for e in edges], [e[1] for e in edges])
    got = run_gpu(g.row_ptr, g.col_idx)
    assert (got == 1).all()


@pytest.mark.parametrize("k", [200, 1500, 3000])
def test_large_cliques(k):
    # wavefront path (k-1 <= 512), workgroup register path (<= 2048), LDS histogram path (> 2048)
    n, edges = sg.complete(k)
    rp, ci = sg.to_csr(n, edges)
    assert (run_gpu(rp, ci) == k - 1).all()


def clique_csr(k):
    """K_k as a CSR built directly (k*(k-1) entries)."""
    ids = np.broadcast_to(np.arange(k, dtype=np.int32), (k, k))
    col = ids[~np.eye(k, dtype=bool)]
    return np.arange(k + 1, dtype=np.int64) * (k - 1), np.ascontiguousarray(col)


def dense_random_csr(n, seed):
    """G(n, 1/2) as a CSR: each pair u < v joined with probability 1/2 (rows sorted)."""
    rng = np.random.default_rng(seed)
    a = rng.integers(0, 2, size=(n, n), dtype=np.uint8).astype(bool)
    a = np.triu(a, 1)
    a |= a.T
    rp = np.zeros(n + 1, np.int64)
    np.cumsum(a.sum(axis=1), out=rp[1:])
    ci = np.nonzero(a)[1].astype(np.int32)
    return rp, ci


def test_cores_above_the_histogram_bins():
    # coreness above the 4096 LDS histogram bins: the one-pass search hands over to the
    # multi-pass search over the global list (every value of a K_4500 lies above the bins)
    rp, ci = clique_csr(4500)
    assert_parity("K4500", rp, ci)
    # a 4200-clique whose first ten vertices also carry 20,000 pendant leaves each (lists
    # longer than the kept-values buffer, cores above the bins)
    k, hubs, leaves = 4200, 10, 20_000
    cr, cc = clique_csr(k)
    src = [np.repeat(np.arange(k, dtype=np.int32), k - 1), np.repeat(np.arange(hubs, dtype=np.int32), leaves)]
    dst = [cc, (k + np.arange(hubs * leaves)).astype(np.int32)]
    g = gg.from_edges(k + hubs * leaves, np.concatenate(src), np.concatenate(dst))
    assert_parity("K4200+pendant hubs", g.row_ptr, g.col_idx)
    # dense G(12000, 1/2): degrees about 6000, cores above 4096 (pruned lists of thousands)
    rp, ci = dense_random_csr(12_000, seed=17)
    got = assert_parity("G(12000,1/2)", rp, ci)
    assert got.min() > 4096


def test_long_path_through_resumed_tails():
    # a path needs about n/2 rounds (one vertex from each end per round); the tail hands its
    # frontier back to the round launches every tail_round_cap rounds
    n = 1_000_000
    g = gg.from_edges(n, np.arange(n - 1), np.arange(1, n))
    st = kc().Stats()
    assert (run_gpu(g.row_ptr, g.col_idx, stats=st) == 1).all()
    print(f"[parity] path 1e6: rounds={st.rounds} tail={st.tail_rounds} launches={st.launches}", flush=True)
    assert st.rounds >= n // 2 - 2
    n = 10_000
    g = gg.from_edges(n, np.arange(n - 1), np.arange(1, n))
    for extra in ({}, dict(tail_order=1), dict(tail_big=1)):
        st = kc().Stats()
        t = kc().Tuning(tail_round_cap=1000, **extra)
        assert (run_gpu(g.row_ptr, g.col_idx, tuning=t, stats=st) == 1).all(), extra
        assert st.tail_rounds >= 4000 and st.launches >= 5, (extra, st.tail_rounds, st.launches)
    # a chain of cliques of growing size joined by single edges: long drop chains with several levels
    sizes = [3 + (i % 7) for i in range(3000)]
    n, edges = sg.onion(sizes)
    rp, ci = sg.to_csr(n, edges)
    for extra in ({}, dict(tail_order=1), dict(tail_order=1, tail_big=1, tail_threshold=1 << 20)):
        t = kc().Tuning(tail_round_cap=7, **extra)
        assert np.array_equal(run_gpu(rp, ci, tuning=t), oracle.coreness(rp, ci)), extra


def test_timing_with_long_first_chunk():
    # more rounds in the first chunk than the timing mode keeps events for: the chunk is clamped
    kc_ = kc()
    g = gg.workload("rmat16")
    st = kc_.Stats()
    got = run_gpu(g.row_ptr, g.col_idx, tuning=kc_.Tuning(timing=1, rounds_per_poll=100), stats=st)
    assert np.array_equal(got, oracle.coreness(g.row_ptr, g.col_idx))
    assert st.total_ms > 0


def test_long_path_and_onion():
    n = 200_000
    g = gg.from_edges(n, np.arange(n - 1), np.arange(1, n))
    assert (run_gpu(g.row_ptr, g.col_idx) == 1).all()
    sizes = [3, 50, 7, 600, 9, 2200, 4]
    n, edges = sg.onion(sizes)
    rp, ci = sg.to_csr(n, edges)
    assert_parity("onion", rp, ci)


def test_hubs_over_a_core():
    # a dense core (ER) plus hubs with tens of thousands of pendant leaves
    rng = np.random.default_rng(7)
    core_n, leaves = 3000, 60000
    src = list(rng.integers(0, core_n, 40000))
    dst = list(rng.integers(0, core_n, 40000))
    for h in range(5):
        src += [h] * (leaves // 5)
        dst += list(range(core_n + h * (leaves // 5), core_n + (h + 1) * (leaves // 5)))
    g = gg.from_edges(core_n + leaves, src, dst)
    assert_parity("hubs", g.row_ptr, g.col_idx)


# ---------------------------------------------------------------- workloads
def test_er_small_int32_and_int64_rows():
    g = gg.workload("er_small")
    a = assert_parity("er_small/int64", g.row_ptr, g.col_idx)
    b = run_gpu(g.row_ptr, g.col_idx, int32_rows=True)
    assert np.array_equal(a, b)
    st = kc().Stats()
    c = run_gpu(g.row_ptr, g.col_idx, int32_rows=True, tuning=kc().Tuning(no_graph=1), stats=st)
    assert np.array_equal(a, c) and st.rounds >= 1 and st.edge_visits > 0


@pytest.mark.parametrize("name", ["road_512", "rmat16", "rmat20"])
def test_medium_workloads(name):
    g = gg.workload(name)
    assert_parity(name, g.row_ptr, g.col_idx)


def test_chung_lu_and_batch_members():
    for gamma in (2.1, 2.5):
        g = gg.chung_lu(200_000, gamma, 16, seed=11)
        assert_parity(f"chung_lu{gamma}", g.row_ptr, g.col_idx)
    b = gg.batch(6, seed=4, nmin=1000, nmax=100_000)
    for i in range(b.num_graphs):
        sub = b.graph(i)
        assert_parity(f"batch[{i}]", sub.row_ptr, sub.col_idx)


@pytest.mark.parametrize("name", ["road", "rmat24"])
def test_full_size_workloads(name):
    g = gg.workload(name)
    kc_ = kc()
    st = kc_.Stats()
    got = run_gpu(g.row_ptr, g.col_idx, stats=st)
    ref = oracle.coreness(g.row_ptr, g.col_idx)
    print(f"[parity] {name}: rounds={st.rounds} tail={st.tail_rounds} visits={st.edge_visits}", flush=True)
    assert np.array_equal(got, ref)
    assert oracle.check(g.row_ptr, g.col_idx, got)[0] == 0
    assert certify_gpu(g.row_ptr, g.col_idx, got) == (0, -1)


# ---------------------------------------------------------------- schedule independence
TUNINGS = {
    "defaults": {},
    "no_tail": dict(tail_threshold=-1),
    "tail_everything": dict(tail_threshold=1 << 30),
    "one_sided": dict(activation=1),
    "deferred": dict(deferred=1),
    "deferred_no_tail_small_cap": dict(deferred=1, tail_threshold=-1, list_cap=256),
    "not_deferred": dict(deferred=2),
    "two_sided": dict(activation=2),
    "two_sided_no_tail": dict(activation=2, tail_threshold=-1, list_cap=256),
    "tiny_grid": dict(grid_blocks=8, big_grid_blocks=1),
    "lane_only_small": dict(thread_max_deg=2, group_max_deg=16, wave_max_deg=64),
    "all_workgroup": dict(thread_max_deg=1, group_max_deg=1, wave_max_deg=1),
    "all_wavefront": dict(thread_max_deg=1, group_max_deg=1),
    "poll_every_round": dict(rounds_per_poll=1, timing=1),
    "always_compact": dict(list_cap=1, tail_threshold=-1),
    "never_compact": dict(list_cap=1 << 30),
    "no_prune": dict(no_prune=1),
    "no_prune_one_sided": dict(no_prune=1, activation=1, list_cap=64),
    "relabel_always": dict(relabel=2),
    "relabel_always_no_tail": dict(relabel=2, tail_threshold=-1, list_cap=256),
    "tail_lowest_first": dict(tail_order=1, tail_threshold=1 << 30),
    "tail_lowest_first_default_threshold": dict(tail_order=1),
    "tail_with_class3": dict(tail_big=1, tail_threshold=4096),
    "tail_with_class3_lowest_first": dict(tail_big=1, tail_order=1, tail_threshold=1 << 30),
    "tail_cap_3": dict(tail_round_cap=3, tail_threshold=1 << 30),
    "tail_cap_1_lowest_first": dict(tail_round_cap=1, tail_order=1, tail_big=1, tail_threshold=1 << 30),
    "full_dense_sweep": dict(dense_sweep=2),
    "full_dense_sweep_small_cap": dict(dense_sweep=2, list_cap=64, tail_threshold=-1),
    "class3_wave_pass": dict(big_wave=1),
    "class3_wave_pass_deferred": dict(big_wave=1, deferred=1, list_cap=512),
    "class3_wave_pass_everything": dict(thread_max_deg=1, group_max_deg=1, wave_max_deg=1, deferred=1, big_wave=1),
    "renumber_often": dict(round_renorm=1024, rounds_per_poll=1),
    "renumber_often_deferred": dict(round_renorm=1024, deferred=1, no_graph=1),
}


@pytest.mark.parametrize("tname", list(TUNINGS))
def test_results_do_not_depend_on_tuning(tname):
    kc_ = kc()
    t = kc_.Tuning(**TUNINGS[tname])
    for name in ["rmat16", "road_512"]:
        g = gg.workload(name)
        st = kc_.Stats()
        got = run_gpu(g.row_ptr, g.col_idx, tuning=t, stats=st)
        assert np.array_equal(got, oracle.coreness(g.row_ptr, g.col_idx)), (tname, name)
        assert st.rounds >= 1


def test_relabel_on_degenerate_and_int32_rows():
    kc_ = kc()
    t = kc_.Tuning(relabel=2)
    # star (one long row), a clique (all rows equal), isolated vertices, int32 row offsets
    for n, edges in [sg.star(3000), sg.complete(70), (50, [])]:
        rp, ci = sg.to_csr(n, edges)
        assert np.array_equal(run_gpu(rp, ci, tuning=t), oracle.coreness(rp, ci))
    g = gg.workload("er_small")
    dev = torch.device("cuda:0")
    out = kc_.decompose(torch.from_numpy(g.row_ptr.astype(np.int64)).to(dev), torch.from_numpy(g.col_idx).to(dev),
                        tuning=t)
    assert np.array_equal(out.cpu().numpy(), oracle.coreness(g.row_ptr, g.col_idx))


def test_workspace_reuse_across_sizes():
    seq = ["rmat16", "er_small", "road_512", "rmat16", "er_small"]
    for name in seq:
        g = gg.workload(name)
        assert_parity(f"reuse/{name}", g.row_ptr, g.col_idx)


# ---------------------------------------------------------------- errors
def test_invalid_arguments_raise():
    kc_ = kc()
    lib = kc_.load()
    assert lib.kcore_decompose(-1, None, None, None, None) == -1
    assert lib.kcore_decompose(10, None, None, None, None) == -1
    assert "null" in lib.kcore_last_error().decode()
    with pytest.raises(TypeError):
        kc_.decompose(torch.zeros(3, dtype=torch.int64, device="cuda"), torch.zeros(2, dtype=torch.int64,
                                                                                     device="cuda"))


def test_validation_mode_rejects_bad_csr(monkeypatch):
    kc_ = kc()
    monkeypatch.setenv("KCORE_VALIDATE", "1")
    rp, ci = sg.to_csr(4, [(0, 1), (1, 2), (2, 3)])
    assert run_gpu(rp, ci).tolist() == [1, 1, 1, 1]
    asym_rp = np.array([0, 1, 1, 1, 1], np.int64)
    asym_ci = np.array([1], np.int32)
    with pytest.raises(kc_.KcoreError, match="symmetric"):
        run_gpu(asym_rp, asym_ci)
    loop_rp = np.array([0, 1, 2], np.int64)
    loop_ci = np.array([0, 1], np.int32)
    with pytest.raises(kc_.KcoreError, match="self-loop"):
        run_gpu(loop_rp, loop_ci)
    oob_ci = np.array([1, 7], np.int32)
    with pytest.raises(kc_.KcoreError, match="range"):
        run_gpu(np.array([0, 1, 2], np.int64), oob_ci)


# ---------------------------------------------------------------- convergence instrumentation
def test_runs_stopped_early_give_upper_bounds():
    # estimates only decrease and never drop below the coreness (Sec. III; Montresor et al.)
    kc_ = kc()
    g = gg.workload("rmat16")
    ref = oracle.coreness(g.row_ptr, g.col_idx)
    deg = np.diff(g.row_ptr)
    for r in (1, 2, 3, 5, 8):
        st = kc_.Stats()
        est = run_gpu(g.row_ptr, g.col_idx, tuning=kc_.Tuning(max_rounds=r), stats=st)
        assert (est >= ref).all() and (est <= deg).all(), r
        assert st.rounds <= r and st.tail_rounds == 0
    assert np.array_equal(run_gpu(g.row_ptr, g.col_idx, tuning=kc_.Tuning(max_rounds=1 << 20)), ref)


def test_convergence_profile_reaches_the_coreness():
    from paper_2512_00233_amd import convergence
    g = gg.workload("road_512")
    dev = torch.device("cuda:0")
    ref = oracle.coreness(g.row_ptr, g.col_idx)
    rows, total = convergence.profile(torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col_idx).to(dev),
                                      reference=ref)
    assert len(rows) == total and total >= 2
    assert rows[0]["active"] > 0 and rows[-1]["exact_share"] == 1.0
    errs = [r["mean_abs_err"] for r in rows]
    assert errs[-1] == 0.0 and errs[0] > 0


@pytest.mark.parametrize("name,tuning", [("rmat16", {}), ("rmat20", {}), ("rmat20", dict(tail_threshold=-1)),
                                         ("rmat20", dict(deferred=1)), ("road_512", {})])
def test_round_by_round_records(name, tuning):
    kc_ = kc()
    g = gg.workload(name)
    dev = torch.device("cuda:0")
    rp, ci = torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col_idx).to(dev)
    out, recs = kc_.decompose_rounds(rp, ci, tuning=kc_.Tuning(**tuning))
    assert np.array_equal(out.cpu().numpy(), oracle.coreness(g.row_ptr, g.col_idx))
    assert len(recs) >= 2 and [r["round"] for r in recs] == list(range(1, len(recs) + 1))
    # the first round recomputes every vertex of degree >= 2 except the class-3 ones above degree 16384,
    # which wait for the second round
    deg = np.diff(g.row_ptr)
    assert recs[0]["vertex_updates"] == int((deg >= 2).sum() - (deg > 16384).sum())
    if (deg > 16384).any():
        assert recs[1]["vertex_updates"] >= int((deg > 16384).sum())
    for r in recs:
        assert r["vertex_updates"] > 0 and r["ms"] > 0, r
        for key in ("vertex_updates", "edge_visits", "changes", "activations"):
            assert r[key] >= 0, (key, r)
        assert r["changes"] <= r["vertex_updates"] <= r["edge_visits"], r
