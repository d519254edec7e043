"""Host-side measurement tools (no GPU): the kernel-source hash that ties a
counter summary to the code it measured, the counter scaling of the traffic
summary, the benchmark's use of a stale summary, and its one-GPU guard."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_0809_4958_amd import prof_summary  # noqa: E402


def test_code_only_ignores_comments_and_blank_lines():
    a = "int a = 1;  // one\n\n/* block\n   comment */ int b = 2;\n// whole line\nint c;\n"
    b = "int a = 1;\nint b = 2;\nint c;  // edited comment\n"
    assert prof_summary._code_only(a) == "int a = 1;\n int b = 2;\nint c;"
    assert prof_summary._code_only(b) == "int a = 1;\nint b = 2;\nint c;"
    # a change of code is a change
    assert prof_summary._code_only("int a = 1;") != prof_summary._code_only("int a = 2;")


def test_short_kernel_names():
    """The summaries name kernels as the trace gives them, shortened: template
    arguments of the step kernels kept, namespaces and argument lists
    dropped, and a name the tool left mangled reduced to its last component."""
    sn = prof_summary.short_name
    assert sn("void k_lb<2, 1, false, 256, false, false>(LbArgs)") == "k_lb<2, 1, false, 256, false, false>"
    assert sn("void lbnet::k_conv<64, 64, 2>(bool _Accum const*, _P, float const, bool _Accum const*)") == \
        "k_conv<64, 64, 2>"
    assert sn("lbnet::k_reduce_parts(float const*, int, int, float*)") == "k_reduce_parts"
    assert sn("_ZN5lbnet6k_headEPKfS1_NS_10LiftWindowEiPKDF16bS1_PDF16bS5_PfS6_i") == "k_head"


def test_kernel_source_hash_is_stable():
    h = prof_summary.kernel_source_hash()
    assert len(h) == 16 and all(ch in "0123456789abcdef" for ch in h)
    assert h == prof_summary.kernel_source_hash()


def _write_counters(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (k, c, v) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})


def test_traffic_scaling_by_the_copy_probe(tmp_path):
    """Each counter is scaled by its own reading for the copy probe: a copy of
    C bytes reads C and writes C, so FETCH_SIZE reading C/2 KiB-units gives a
    factor 2 and WRITE_SIZE reading C gives 1 (the values seen on this GPU)."""
    C = 1 << 28
    fetch = tmp_path / "f.csv"
    write = tmp_path / "w.csv"
    lb = "void lbdev::k_lb<2, 2, false, 256>(lbdev::LbArgs)"
    cp = "lbdev::k_copy(HIP_vector_type<unsigned int, 4u> const*, unsigned long)"
    _write_counters(fetch, [(cp, "FETCH_SIZE", C / 2 / 1024), (cp, "FETCH_SIZE", C / 2 / 1024),
                            (lb, "FETCH_SIZE", 3e9 / 2 / 1024)])
    _write_counters(write, [(cp, "WRITE_SIZE", C / 1024), (lb, "WRITE_SIZE", 2e9 / 1024)])
    out = tmp_path / "t.txt"
    prof_summary.traffic(str(fetch), str(write), str(out), C, "cmd f", "cmd w", "test", "f16", 4e9)
    vals = dict(ln.split(":", 1) for ln in out.read_text().splitlines() if ":" in ln and not ln.startswith("#"))
    assert float(vals["fetch_scale"]) == pytest.approx(2.0)
    assert float(vals["write_scale"]) == pytest.approx(1.0)
    assert float(vals["hbm_read_bytes_per_launch"]) == pytest.approx(3e9)
    assert float(vals["hbm_write_bytes_per_launch"]) == pytest.approx(2e9)
    assert float(vals["traffic_over_algorithmic"]) == pytest.approx(5e9 / 4e9, rel=1e-4)
    assert vals["kernel_sources_sha1"].strip() == prof_summary.kernel_source_hash()


def test_bench_ignores_a_summary_of_other_kernel_sources(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "profiles")
    path = bench.traffic_file("f16", 256)
    assert bench.committed_traffic("f16", 256) is None          # no summary
    with open(path, "w") as fh:
        fh.write(f"kernel_sources_sha1: {prof_summary.kernel_source_hash()}\nhbm_bytes_per_launch: 123.5\n")
    assert bench.committed_traffic("f16", 256) == 123.5
    with open(path, "w") as fh:
        fh.write("kernel_sources_sha1: 0000000000000000\nhbm_bytes_per_launch: 123.5\n")
    assert bench.committed_traffic("f16", 256) is None          # stale summary


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_long_run_sites_and_subset():
    """Sites of the long-run comparisons are unique interior nodes that include
    the rows next to every face and the cube around each anchor; the 16-box
    subset holds four boxes of every edge, and building only those boxes
    gives the inputs the whole batch gives them."""
    import numpy as np

    import bench
    import longrun
    for n in (32, 48, 96):
        anc = [np.array([n / 3.0, n / 2.0 + 0.3, 2 * n / 3.0])]
        s = longrun.sites(n, anc, 7)
        assert s.min() >= 1 and s.max() <= n - 2
        lin = (s[:, 2].astype(np.int64) * n + s[:, 1]) * n + s[:, 0]
        assert np.all(np.diff(lin) > 0)
        have = set(map(tuple, s.tolist()))
        for y, z in ((1, 1), (n - 2, n - 2), (1, n - 2)):
            assert all((x, y, z) in have for x in range(1, n - 1))
        c = np.floor(anc[0]).astype(int)
        assert all((c[0] + dx, c[1] + dy, c[2] + dz) in have
                   for dx in range(-3, 5) for dy in range(-3, 5) for dz in range(-3, 5))
    idx = longrun.batch16_indices()
    sizes = bench.batch_inputs(256, 1, 0.6, only=set())
    assert sizes == []
    sub = bench.batch_inputs(256, 40, 0.6, only=set(idx[:2] + idx[-2:]))
    full = bench.batch_inputs(256, 40, 0.6)
    assert len(idx) == 16 and sorted(b["n"] for b in bench.batch_inputs(256, 20, 0.6, only=set(idx))) \
        == [32] * 4 + [48] * 4 + [64] * 4 + [96] * 4
    for b in sub:
        f = full[b["index"]]
        assert f["n"] == b["n"] and np.array_equal(f["faces"], b["faces"])
        assert np.array_equal(f["u0"], b["u0"]) and np.array_equal(f["pos"], b["pos"])
