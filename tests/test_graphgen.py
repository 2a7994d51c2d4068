"""Input generators: determinism, thread-count independence, CSR preconditions."""
import os

import numpy as np
import pytest

import graphgen as gg


def _same(a, b):
    return np.array_equal(a.row_ptr, b.row_ptr) and np.array_equal(a.col_idx, b.col_idx)


@pytest.mark.parametrize("make", [
    lambda: gg.erdos_renyi(3000, 12000, seed=9),
    lambda: gg.lattice(300, 200, seed=5),
    lambda: gg.rmat(14, seed=3),
    lambda: gg.chung_lu(30000, 2.5, 10, seed=8),
], ids=["er", "lattice", "rmat", "chung_lu"])
def test_deterministic_and_thread_independent(make, monkeypatch):
    monkeypatch.setenv("GG_THREADS", "1")
    a = make()
    monkeypatch.setenv("GG_THREADS", "7")
    b = make()
    assert _same(a, b)
    assert gg.validate(a) == 0


def test_seed_changes_graph():
    assert not _same(gg.rmat(12, seed=1), gg.rmat(12, seed=2))


def test_er_has_exactly_m_edges():
    g = gg.workload("er_small", cache=False)
    assert g.n == 10_000 and g.nnz == 100_000


def test_lattice_shape():
    g = gg.lattice(64, 64, p=1.0, chord_prob=0.0)
    assert g.nnz == 2 * (2 * 64 * 63)
    assert gg.validate(g) == 0
    g = gg.lattice(400, 400)
    expect = 2 * (0.6 * 2 * 400 * 399 + 0.01 * 400 * 400)
    assert abs(g.nnz - expect) / expect < 0.02


def test_from_edges_cleans_input():
    g = gg.from_edges(5, [0, 1, 1, 2, 3, 3], [1, 0, 1, 3, 2, 4])
    assert g.row_ptr.tolist() == [0, 1, 2, 3, 5, 6]
    assert g.col_idx.tolist() == [1, 0, 3, 2, 4, 3]


def test_validate_rejects_bad_csr():
    g = gg.from_edges(4, [0, 1, 2], [1, 2, 3])
    assert gg.validate(g) == 0
    bad = gg.Graph(g.row_ptr.copy(), g.col_idx.copy())
    bad.col_idx[0] = 9
    assert gg.validate(bad) == 3
    loop = gg.Graph(g.row_ptr.copy(), g.col_idx.copy())
    loop.col_idx[0] = 0
    assert gg.validate(loop) == 4
    asym = gg.Graph(np.array([0, 1, 1, 1, 1]), np.array([1], np.int32))
    assert gg.validate(asym) == 6


def test_batch_layout():
    b = gg.batch(16, seed=4, nmin=1000, nmax=5000)
    assert b.num_graphs == 16
    for g in range(16):
        kind, n = gg.batch_spec(4, g, 1000, 5000)
        sub = b.graph(g)
        assert sub.n == n and kind == int(b.kind[g])
        assert gg.validate(sub) == 0
    b2 = gg.batch(4, seed=4, nmin=1000, nmax=5000, first=3)
    assert np.array_equal(b2.graph(0).col_idx, b.graph(3).col_idx)
