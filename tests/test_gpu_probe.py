"""The gather-rate probe used by the benchmark computes what it claims (sum of
vals[idx[j]]), on a graph's adjacency and on an empty one."""
import numpy as np
import pytest

import graphgen as gg

pytestmark = pytest.mark.gpu


def test_probe_sum_matches_numpy():
    import torch
    import paper_2512_00233_amd as kc
    dev = torch.device("cuda:0")
    g = gg.workload("rmat16")
    rng = np.random.default_rng(3)
    vals = rng.integers(-1000, 1000, size=g.n, dtype=np.int32)
    idx_t = torch.from_numpy(g.col_idx).to(dev)
    vals_t = torch.from_numpy(vals).to(dev)
    out = torch.full((1,), 77, dtype=torch.int64, device=dev)
    kc.probe_gather(idx_t, vals_t, out)
    assert int(out.item()) == int(vals[g.col_idx].astype(np.int64).sum())
    # a ragged length (not a multiple of the unrolled stride) and an empty pass
    kc.probe_gather(idx_t[:12345], vals_t, out)
    assert int(out.item()) == int(vals[g.col_idx[:12345]].astype(np.int64).sum())
    kc.probe_gather(idx_t[:0], vals_t, out)
    assert int(out.item()) == 0
