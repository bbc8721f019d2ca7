"""Host logic of bench.py: the HBM-traffic figure is read from the committed
counter summary only while the kernel sources still hash to the value
recorded beside it, and the edge and op counts behind the roofline."""
import json
import os
import shutil

import pytest

import bench


def _recorded(kernel):
    import hashlib
    import re
    text = open(os.path.join(bench.ROOT, "profiles", "hbm_traffic_large.md")).read()
    entry = json.loads(re.search(r"```json\n(.*?)\n```", text, flags=re.S).group(1)).get(bench.KERNEL_NAMES[kernel])
    h = hashlib.sha256()
    for f in bench.KERNEL_SOURCES[bench.KERNEL_NAMES[kernel].split("<")[0]]:
        with open(os.path.join(bench.ROOT, f), "rb") as fh:
            h.update(fh.read())
    return entry, h.hexdigest()[:16]


def test_traffic_is_read_while_the_source_hash_matches():
    """The committed figure is reported exactly while the sources it was taken
    on are unchanged (and dropped, not reused, once they change)."""
    for k in ("forward", "adjoint", "filter"):
        entry, digest = _recorded(k)
        t = bench.measured_traffic(k)
        if entry is None:          # no counters taken on this kernel yet
            assert t is None, k
        elif digest == entry["source_hash"]:
            assert t == entry["read_bytes"] + entry["write_bytes"] and t > 0, k
        else:
            assert t is None, k


def test_traffic_is_dropped_once_a_kernel_source_changes(tmp_path, monkeypatch):
    root = tmp_path / "repo"
    (root / "profiles").mkdir(parents=True)
    for srcs in bench.KERNEL_SOURCES.values():
        for f in srcs:
            (root / os.path.dirname(f)).mkdir(parents=True, exist_ok=True)
            shutil.copy(os.path.join(bench.ROOT, f), root / f)
    # a summary taken on exactly these sources
    entries = {}
    for k in ("forward", "adjoint", "filter"):
        _, digest = _recorded(k)
        entries[bench.KERNEL_NAMES[k]] = {"read_bytes": 1000, "write_bytes": 24, "source_hash": digest}
    (root / "profiles" / "hbm_traffic_large.md").write_text("```json\n" + json.dumps(entries) + "\n```\n")
    monkeypatch.setattr(bench, "ROOT", str(root))
    assert bench.measured_traffic("forward") == 1024
    with open(root / "paper_2601_00551_amd/csrc/forward.hip", "a") as fh:
        fh.write("\n// edited\n")
    assert bench.measured_traffic("forward") is None
    assert bench.measured_traffic("adjoint") is not None      # its own sources are unchanged
    with open(root / "paper_2601_00551_amd/csrc/sbp_internal.hpp", "a") as fh:
        fh.write("\n// edited\n")
    assert bench.measured_traffic("adjoint") is None and bench.measured_traffic("filter") is None


def test_edges_per_pair():
    # a 0.15 mm GAUSS ball (support 5 a) at 40 MHz and 1.5 mm/us: 40 bins, 41 edges
    assert bench.edges_per_pair(0.75, 1.5 * 0.025) == pytest.approx(40.0)


def test_more_than_one_gpu_is_refused():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in (r.stdout + r.stderr)
