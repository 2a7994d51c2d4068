"""kcore_decompose_noalloc (the entry point for callers that cannot allocate) against
kcore_decompose and the oracle, through the C ABI, on calls in a row that share the
fixed device workspace."""
import ctypes

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def kc():
    import paper_2512_00233_amd as kc
    return kc


def dev_csr(g):
    dev = torch.device("cuda:0")
    return torch.from_numpy(np.ascontiguousarray(g.row_ptr)).to(dev), torch.from_numpy(g.col_idx).to(dev)


def noalloc(rp, ci, n):
    lib = kc().load()
    out = torch.full((n,), -3, dtype=torch.int32, device=rp.device)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    status = lib.kcore_decompose_noalloc(n, rp.data_ptr(), ci.data_ptr(), out.data_ptr(), st)
    assert status == 0, lib.kcore_last_error().decode()
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_noalloc_matches_decompose_on_calls_in_a_row():
    # a larger graph, then a smaller one: the second call meets the first call's leftovers
    for name in ["rmat16", "er_small", "road_512", "er_small"]:
        g = gg.workload(name)
        rp, ci = dev_csr(g)
        print(f"[noalloc] {name}: n={g.n} nnz={g.nnz}", flush=True)
        got = noalloc(rp, ci, g.n)
        ref = kc().decompose(rp, ci).cpu().numpy()
        assert np.array_equal(got, ref), name
        assert np.array_equal(got, oracle.coreness(g.row_ptr, g.col_idx)), name


def test_noalloc_at_its_limits_and_beyond():
    lib = kc().load()
    # a graph of exactly the vertex limit with many entries
    g = gg.chung_lu(1 << 20, 2.3, 7.5, seed=81)
    assert g.n == 1 << 20 and g.nnz <= 1 << 23, (g.n, g.nnz)
    rp, ci = dev_csr(g)
    got = noalloc(rp, ci, g.n)
    assert np.array_equal(got, oracle.coreness(g.row_ptr, g.col_idx))
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    # one vertex too many: refused before any device access
    assert lib.kcore_decompose_noalloc((1 << 20) + 1, rp.data_ptr(), ci.data_ptr(), ci.data_ptr(), st) == -4
    assert b"exceeds" in lib.kcore_last_error()
    # too many entries: row_ptr[n] is read, nothing else
    dev = torch.device("cuda:0")
    big_rp = torch.tensor([0, 0, (1 << 23) + 1], dtype=torch.int64, device=dev)
    out = torch.zeros(2, dtype=torch.int32, device=dev)
    assert lib.kcore_decompose_noalloc(2, big_rp.data_ptr(), out.data_ptr(), out.data_ptr(), st) == -4
    # and the next call is still right
    g2 = gg.workload("rmat16")
    rp2, ci2 = dev_csr(g2)
    assert np.array_equal(noalloc(rp2, ci2, g2.n), oracle.coreness(g2.row_ptr, g2.col_idx))
    assert lib.kcore_decompose_noalloc(0, None, None, None, st) == 0
