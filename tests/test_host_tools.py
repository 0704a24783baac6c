"""Host-side logic that needs no GPU: the rocprofv3 summary arithmetic, the regrid size
cap of the driver, and the one-at-a-time serving timeline."""
import csv
import json

import pytest

from paper_2404_02950_amd import driver, rocprof_summary, serve


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, value in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_traffic_summary_scales_by_the_copy_kernel(tmp_path):
    n = 8
    ref = 4 * n ** 3 * 8  # k_xfer: dense FP64 state in, FP64 boxes out
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    # the read counter sees half of what is read; the write counter is exact
    _counter_csv(fetch, "FETCH_SIZE", [("void k_xfer<double, true>(...)", ref / 2 / 1024),
                                       ("void k_fused_step<double, ...>(...)", 3000.0),
                                       ("void k_fused_step<double, ...>(...)", 3200.0),
                                       ("other", 1.0)])
    _counter_csv(write, "WRITE_SIZE", [("void k_xfer<double, true>(...)", ref / 1024),
                                       ("void k_fused_step<double, ...>(...)", 4000.0),
                                       ("void k_fused_step<double, ...>(...)", 4000.0)])
    out_json, out_md = tmp_path / "t.json", tmp_path / "t.md"
    rocprof_summary.main(["traffic", str(fetch), str(write), str(out_json), str(out_md), "--kernel", "k_fused_step",
                          "--n", str(n), "--prec", "f64", "--alg-bytes", "64", "--cmd-fetch", "a", "--cmd-write", "b"])
    rec = json.load(open(out_json))
    assert rec["calibration"]["fetch_factor"] == pytest.approx(2.0)
    assert rec["calibration"]["write_factor"] == pytest.approx(1.0)
    assert rec["hbm_read_bytes_per_launch"] == pytest.approx(3100.0 * 1024 * 2)
    assert rec["hbm_write_bytes_per_launch"] == pytest.approx(4000.0 * 1024)
    assert rec["algorithmic_bytes_per_launch"] == 64 * n ** 3
    assert rec["dispatches"] == 2
    assert len(rec["kernel_source_sha256"]) == 64
    assert "k_fused_step" in open(out_md).read()


def test_traffic_summary_fp32_reference_reads_fp64(tmp_path):
    # in FP32 mode k_xfer still reads the dense FP64 state but writes FP32 boxes
    n = 4
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    _counter_csv(fetch, "FETCH_SIZE", [("k_xfer<float>", 4 * n ** 3 * 8 / 1024), ("k_fused_step<float>", 10.0)])
    _counter_csv(write, "WRITE_SIZE", [("k_xfer<float>", 4 * n ** 3 * 4 / 1024), ("k_fused_step<float>", 10.0)])
    out_json = tmp_path / "t.json"
    rocprof_summary.main(["traffic", str(fetch), str(write), str(out_json), str(tmp_path / "t.md"), "--kernel",
                          "k_fused_step", "--n", str(n), "--prec", "f32", "--alg-bytes", "32", "--cmd-fetch", "a",
                          "--cmd-write", "b"])
    rec = json.load(open(out_json))
    assert rec["calibration"]["fetch_factor"] == pytest.approx(1.0)
    assert rec["calibration"]["write_factor"] == pytest.approx(1.0)


def test_ambiguous_kernel_name_is_an_error(tmp_path):
    fetch = tmp_path / "f.csv"
    _counter_csv(fetch, "FETCH_SIZE", [("k_xfer", 1.0), ("k_fused_step<a>", 1.0), ("k_fused_step<b>", 1.0)])
    with pytest.raises(SystemExit):
        rocprof_summary.main(["traffic", str(fetch), str(fetch), str(tmp_path / "t.json"), str(tmp_path / "t.md"),
                              "--kernel", "k_fused_step", "--n", "4", "--prec", "f64", "--alg-bytes", "64",
                              "--cmd-fetch", "a", "--cmd-write", "b"])


class _FakeHierarchy:
    """Stands in for shamr.Hierarchy: level lev+1 gets `boxes[lev]`, each box costs 1 byte
    per cell."""

    def __init__(self, boxes):
        self._boxes = boxes
        self.levels = 1
        self.layouts = []

    def num_levels(self):
        return self.levels

    params = type("P", (), {"n_error_buf": 2})()

    def tag(self, lev):
        return 10 * (lev + 1), None

    def tag_blocks(self, lev, r, halve=False, bits=None):
        return (0, None) if halve else (10 * (lev + 1), None)

    def cluster(self, lev, idx, efficiency, carried=None):
        return self._boxes[lev]

    def cluster_blocks(self, lev, bits, efficiency):
        return self._boxes[lev]

    def arena_bytes(self, lev, boxes):
        return sum((b[3] - b[0] + 1) * (b[4] - b[1] + 1) * (b[5] - b[2] + 1) for b in boxes)

    def set_layout(self, lev, boxes):
        self.layouts.append((lev, list(boxes)))
        self.levels = lev + 1 if boxes else lev


def test_regrid_removes_a_level_above_the_size_cap():
    small = [(0, 0, 0, 7, 7, 7)]             # 512 cells
    big = [(0, 0, 0, 63, 63, 63)]            # 262144 cells
    h = _FakeHierarchy([small, big, small])
    msgs, timing = [], {}
    counts = driver.regrid(h, 3, max_level_bytes=10000, log=msgs.append, timing=timing)
    # level 1 is built, level 2 would exceed the cap: it and everything finer is removed
    assert h.layouts == [(1, small), (2, [])]
    assert counts == [10, 20]
    assert len(msgs) == 1 and "level 2" in msgs[0]
    assert set(timing) == {"tag", "cluster", "layout"}
    h2 = _FakeHierarchy([small, big, small])
    driver.regrid(h2, 3)                      # no cap: every level is built
    assert h2.layouts == [(1, small), (2, big), (3, small)]


def test_serving_report_percentiles_and_rate():
    jobs = [serve.Job(jid=i, n=32, steps=10, prec=0, seed=0, arrival=a) for i, a in enumerate((0.0, 0.5, 1.0, 1.5))]
    for j, lat in zip(jobs, (0.1, 0.2, 0.3, 1.3)):
        j.t_done = j.arrival + lat
    r = serve._report(jobs, 2.8)
    assert r["p50_s"] == pytest.approx(0.25)
    assert r["p99_s"] == pytest.approx(0.3 + 0.97 * 1.0)
    assert r["cell_updates_per_s"] == pytest.approx(4 * 32 ** 3 * 4 * 10 / 2.8)
