"""Host logic of the measurement tools, on synthetic inputs (no GPU): the counter summary's derived figures
and the bench's algorithmic byte count."""
import csv
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def write_counter_csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_counter_summary_derived_figures(tmp_path):
    from paper_2512_00233_amd import profiling
    k = "void kcore::k_big<false, false, long>(kcore::Args<long>, int, int)"
    # two dispatches per counter; means: 32B 10, 64B 20, 128B 30 read requests; 100 writes of which 40 are 64 B
    reads = [dict(Dispatch_Id=d, Kernel_Name=k, Counter_Name=c, Counter_Value=v)
             for d, vals in ((1, (8, 18, 28)), (2, (12, 22, 32)))
             for c, v in zip(("TCC_EA0_RDREQ_32B", "TCC_EA0_RDREQ_64B", "TCC_EA0_RDREQ_128B"), vals)]
    other = [dict(Dispatch_Id=1, Kernel_Name=k, Counter_Name=c, Counter_Value=v) for c, v in (
        ("TCC_EA0_WRREQ", 100), ("TCC_EA0_WRREQ_64B", 40), ("TCC_HIT", 30), ("TCC_MISS", 70),
        ("SQ_WAVE_CYCLES", 256 * 1000), ("GRBM_GUI_ACTIVE", 8 * 4000), ("SQ_WAIT_INST_ANY", 128 * 1000),
        ("SQ_WAIT_ANY", 64 * 1000), ("SQ_ACTIVE_INST_VALU", 32 * 1000))]
    a, b = tmp_path / "a.csv", tmp_path / "b.csv"
    write_counter_csv(a, reads)
    write_counter_csv(b, other)
    out = profiling.counters([str(a), str(b)], "synthetic", ["cmd"], ["k_big<false, false, long>"], "h",
                             str(tmp_path / "o.json"), str(tmp_path / "o.md"))
    d = out["kernels"]["k_big<false, false, long>"]
    assert d["read_bytes"] == 32 * 10 + 64 * 20 + 128 * 30
    assert d["write_bytes"] == 32 * 60 + 64 * 40
    assert d["l2_hit_rate"] == 0.3
    # 4 * wave cycles / (busy cycles of one XCD) / 256 compute units: 4 * 256000 / 4000 / 256 = 1.0
    assert d["mean_waves_per_cu"] == 1.0
    assert d["wait_inst_share"] == 0.5 and d["wait_any_share"] == 0.25 and d["valu_share"] == 0.125
    assert json.load(open(tmp_path / "o.json"))["source_hash"] == "h"
    assert "k_big<false, false, long>" in open(tmp_path / "o.md").read()


def test_algorithmic_bytes_per_unit():
    import bench
    # per recomputed vertex: two row offsets, its own estimate and its frontier entry; per visit the
    # neighbour id and its estimate; 4 B per change and per activation
    assert bench.algorithmic_bytes(1, 0, 0, 0) == 2 * 8 + 8
    assert bench.algorithmic_bytes(0, 1, 0, 0) == 8
    assert bench.algorithmic_bytes(0, 0, 1, 1) == 8
    assert bench.algorithmic_bytes(1, 0, 0, 0, off_bytes=4) == 2 * 4 + 8


def test_kernel_source_hash_is_stable():
    import bench
    h = bench.kernel_source_hash()
    assert h == bench.kernel_source_hash() and len(h) == 12 and all(c in "0123456789abcdef" for c in h)
