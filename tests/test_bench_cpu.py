"""CPU checks of bench.py's host logic: the single-GPU guard and the rule that measured HBM
traffic is reported only for the kernel source and workload it was measured on."""
import hashlib
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=300)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and p.stdout == ""


def test_traffic_only_for_the_measured_source_and_workload(tmp_path):
    src = tmp_path / "kernel.hip"
    src.write_bytes(b"kernel source v1")
    sha = hashlib.sha256(b"kernel source v1").hexdigest()
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps({"k_x": {"sources_sha256": sha, "tag": "wl|all|a*", "bytes_per_launch": 1234}}))
    rel = os.path.relpath(str(src), bench.ROOT)
    assert bench.load_traffic(str(f), "k_x", [rel], "wl|all|a*") == 1234
    assert bench.load_traffic(str(f), "k_x", [rel], "wl|64|a*") is None        # another workload
    assert bench.load_traffic(str(f), "k_y", [rel], "wl|all|a*") is None       # another kernel
    assert bench.load_traffic(str(tmp_path / "none.json"), "k_x", [rel], "wl|all|a*") is None
    src.write_bytes(b"kernel source v2")                                       # the kernel changed
    assert bench.load_traffic(str(f), "k_x", [rel], "wl|all|a*") is None


def test_committed_traffic_files_name_their_workload():
    pdir = os.path.join(ROOT, "profiles")
    for name in os.listdir(pdir):
        if name.startswith("traffic_") and name.endswith(".json"):
            d = json.load(open(os.path.join(pdir, name)))
            for kernel, ent in d.items():
                assert ent["tag"].startswith(name[len("traffic_"):-len(".json")] + "|"), (name, kernel)
                assert len(ent["sources_sha256"]) == 64 and ent["bytes_per_launch"] > 0


def test_expand_roofline_counts_one_visited_word_read_per_item_word():
    # tallies of one R-MAT 18 step (per launch): items, segments, frontier words, visited-word
    # reads, ORs; the method's bytes charge 8 B per visited-word read; the two-read kernel also
    # reads the Next word beside each (its extra words are the visited-word reads)
    prof = dict(expand_launches=2, expand_ms=2 * 1.4714, edge_items=2 * 13_070_000, descriptors=2 * 1_414_000,
                row_words=2 * 45_260_000, word_reads=2 * 275_400_000, word_updates=2 * 56_380_000,
                expand_extra_words=2 * 275_400_000)
    method, impl, avg_ms = bench.expand_roofline(prof)
    assert method == 4 * 13_070_000 + 16 * 1_414_000 + 8 * 45_260_000 + 8 * 275_400_000 + 8 * 56_380_000
    assert impl - method == 8 * 275_400_000
    # seen OR: the kernel makes the method's accesses only
    method2, impl2, _ = bench.expand_roofline(dict(prof, expand_extra_words=0))
    assert method2 == method and impl2 == method2
    assert abs(avg_ms - 1.4714) < 1e-12
    assert abs(method / (avg_ms / 1e3) / 8e12 - 0.2626) < 5e-4


def test_finalize_and_extract_rooflines_from_their_tallies():
    # two finalize launches over 1,000 rows of 64 words, 30,000 of them non-zero and 5,000 of those in
    # final-state rows; one extraction count pass over 1,000,000 answer words
    prof = dict(finalize_launches=2, finalize_ms=2 * 0.5, finalize_rows=2000, finalize_row_words=128_000,
                finalize_words=60_000, finalize_vis_words=2 * 60_000, finalize_ans_words=10_000, extract_launches=1,
                extract_ms=0.25, extract_words=1_000_000)
    out = bench.other_rooflines(prof)
    fin_bytes = (8 * 2000 + 16 * 128_000 + 24 * 60_000 + 16 * 10_000) / 2
    assert out["finalize"]["alg_bytes_per_launch"] == round(fin_bytes, 1)
    assert abs(out["finalize"]["achieved"] - round(fin_bytes / 0.5e-3 / 1e9, 2)) < 1e-9
    assert abs(out["extract"]["achieved"] - 8e6 / 0.25e-3 / 1e9) < 1e-6
    assert abs(out["extract"]["frac"] - round(8e6 / 0.25e-3 / 1e9 / 8000, 5)) < 1e-9
    # seen OR: finalize reads the visited word of every row word and writes none
    fin2 = (8 * 2000 + 16 * 128_000 + 8 * 60_000 + 8 * 128_000 + 16 * 10_000) / 2
    assert bench.other_rooflines(dict(prof, finalize_vis_words=128_000))["finalize"]["alg_bytes_per_launch"] == round(fin2, 1)
    # no launches, no entry
    assert bench.other_rooflines(dict(prof, finalize_launches=0, extract_launches=0)) == {}
