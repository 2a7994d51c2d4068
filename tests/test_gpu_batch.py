"""Batched form: every graph's coreness in the batch equals the oracle, the same
graph decomposed alone, and does not depend on the order of the batch."""
import os
import time

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def kc():
    import paper_2512_00233_amd as kc
    return kc


def to_dev(b):
    dev = torch.device("cuda:0")
    return (torch.from_numpy(b.graph_vtx_off).to(dev), torch.from_numpy(b.row_ptr).to(dev),
            torch.from_numpy(b.col_idx).to(dev))


def run_batch(b, **kw):
    vo, rp, ci = to_dev(b)
    out = kc().decompose_batch(vo, rp, ci, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_batch_matches_oracle_and_plain():
    b = gg.batch(48, seed=4, nmin=1000, nmax=60_000)
    print(f"[batch] G={b.num_graphs} N={b.graph_vtx_off[-1]} nnz={b.col_idx.size}", flush=True)
    got = run_batch(b)
    ref = oracle.coreness_batch(b.graph_vtx_off, b.row_ptr, b.col_idx, threads=8)
    assert np.array_equal(got, ref)
    for g in range(0, b.num_graphs, 7):
        sub = b.graph(g)
        dev = torch.device("cuda:0")
        alone = kc().decompose(torch.from_numpy(sub.row_ptr).to(dev), torch.from_numpy(sub.col_idx).to(dev))
        v0, v1 = b.graph_vtx_off[g], b.graph_vtx_off[g + 1]
        assert np.array_equal(alone.cpu().numpy(), got[v0:v1])


def test_full_batch_workload_above_2_31_entries():
    # the batched workload itself: 2048 graphs (seed 4), 4.08e9 entries, so the row offsets pass
    # 2^31 and the automatic small-class grid grows to its largest size
    t0 = time.time()
    b = gg.batch(2048, seed=4, nmin=1000, nmax=1_000_000)
    nnz = int(b.col_idx.size)
    print(f"[batch] full workload generated in {time.time() - t0:.1f} s: N={int(b.graph_vtx_off[-1])} "
          f"entries={nnz}", flush=True)
    assert nnz > 2**31
    st = kc().Stats()
    got = run_batch(b, stats=st)
    print(f"[batch] GPU done: rounds={st.rounds} tail={st.tail_rounds}", flush=True)
    ref = oracle.coreness_batch(b.graph_vtx_off, b.row_ptr, b.col_idx, threads=min(16, os.cpu_count() or 1))
    print(f"[batch] oracle done at {time.time() - t0:.1f} s", flush=True)
    if not np.array_equal(got, ref):
        bad = np.nonzero(got != ref)[0]
        raise AssertionError(f"{bad.size} mismatches, first v={bad[0]} gpu={got[bad[0]]} ref={ref[bad[0]]}")


def test_batch_order_does_not_matter():
    b = gg.batch(20, seed=9, nmin=500, nmax=20_000)
    got = run_batch(b)
    perm = np.random.default_rng(3).permutation(b.num_graphs)
    graphs = [b.graph(int(g)) for g in perm]
    b2 = gg.concat(graphs)
    got2 = run_batch(b2)
    for j, g in enumerate(perm):
        a0, a1 = b.graph_vtx_off[g], b.graph_vtx_off[g + 1]
        c0, c1 = b2.graph_vtx_off[j], b2.graph_vtx_off[j + 1]
        assert np.array_equal(got[a0:a1], got2[c0:c1])


def test_batch_edge_cases():
    from tests import small_graphs as sg
    graphs = []
    for n, edges in [sg.complete(7), (1, []), sg.cycle(5), (3, []), sg.star(40), sg.complete(600), sg.path(9)]:
        rp, ci = sg.to_csr(n, edges)
        graphs.append(gg.Graph(rp, ci))
    b = gg.concat(graphs)
    got = run_batch(b)
    ref = oracle.coreness_batch(b.graph_vtx_off, b.row_ptr, b.col_idx, threads=2)
    assert np.array_equal(got, ref)
    # no graphs at all
    empty = gg.Batch(np.zeros(1, np.int64), np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32))
    vo, rp, ci = to_dev(empty)
    assert kc().load().kcore_decompose_batch(0, vo.data_ptr(), rp.data_ptr(), 0, 0, None, None, None) == 0


@pytest.mark.parametrize("tuning", [dict(), dict(no_graph=1), dict(list_cap=1, tail_threshold=-1),
                                    dict(thread_max_deg=1, group_max_deg=1, wave_max_deg=1),
                                    dict(activation=1, no_prune=1), dict(activation=2), dict(deferred=1),
                                    dict(tail_order=1, tail_big=1, tail_threshold=1 << 30),
                                    dict(tail_round_cap=2, tail_threshold=1 << 30),
                                    dict(round_renorm=1024, rounds_per_poll=1), dict(big_wave=1),
                                    dict(thread_max_deg=1, group_max_deg=1, wave_max_deg=1, big_wave=1)])
def test_batch_tunings(tuning):
    b = gg.batch(16, seed=5, nmin=1000, nmax=30_000)
    got = run_batch(b, tuning=kc().Tuning(**tuning))
    ref = oracle.coreness_batch(b.graph_vtx_off, b.row_ptr, b.col_idx, threads=8)
    assert np.array_equal(got, ref)


def test_autotuner_records_a_correct_choice(tmp_path):
    from paper_2512_00233_amd import autotune
    b = gg.batch(12, seed=6, nmin=1000, nmax=20_000)
    vo, rp, ci = to_dev(b)
    path = str(tmp_path / "tune.json")
    entry = autotune.tune_and_save(vo, rp, ci, path, reps=1)
    assert entry["ms"] > 0
    assert autotune.load_file(path) == 1
    t = kc().tuning_cache_get(b.num_graphs, int(b.graph_vtx_off[-1]), int(b.col_idx.size))
    assert t is not None
    got = run_batch(b)  # uses the cached tuning
    ref = oracle.coreness_batch(b.graph_vtx_off, b.row_ptr, b.col_idx, threads=8)
    assert np.array_equal(got, ref)


def test_batch_validation(monkeypatch):
    monkeypatch.setenv("KCORE_VALIDATE", "1")
    b = gg.batch(4, seed=7, nmin=100, nmax=1000)
    run_batch(b)  # valid
    bad = gg.Batch(b.graph_vtx_off.copy(), b.row_ptr.copy(), b.col_idx.copy(), b.kind.copy())
    v0 = int(b.graph_vtx_off[1])
    e0 = int(b.row_ptr[v0])
    bad.col_idx[e0] = int(b.graph_vtx_off[2] - b.graph_vtx_off[1]) + 5  # outside graph 1
    with pytest.raises(kc().KcoreError, match="outside"):
        run_batch(bad)
