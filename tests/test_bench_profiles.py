"""The benchmark's traffic figure comes only from a whole, self-consistent
rocprofv3 counter summary taken on the current kernel sources."""
import re

import bench


def _with_current_hash(text):
    return re.sub(r"kernel_hash: \w+", "kernel_hash: " + bench.kernel_hash(), text)


def _read(tmp_path, text, key="hbm_bytes_per_launch"):
    p = tmp_path / "traffic.txt"
    p.write_text(text)
    saved = bench.TRAFFIC_FILE
    bench.TRAFFIC_FILE = str(p)
    try:
        return bench.read_traffic(key)
    finally:
        bench.TRAFFIC_FILE = saved


def test_committed_summary_is_consistent(tmp_path):
    text = _with_current_hash(open(bench.TRAFFIC_FILE).read())
    got = _read(tmp_path, text)
    assert got is not None and got > 0
    assert _read(tmp_path, text, "lookup_hbm_bytes_per_launch") > 0


def test_incomplete_or_inconsistent_summary_rejected(tmp_path):
    text = _with_current_hash(open(bench.TRAFFIC_FILE).read())
    lines = text.split("\n")
    drop = next(i for i, l in enumerate(lines) if l.startswith("  eq "))
    assert _read(tmp_path, "\n".join(lines[:drop] + lines[drop + 1:])) is None      # a PP-VBS row missing
    stated = re.search(r"hbm_bytes_per_launch: (\d+)", text).group(1)
    off = text.replace("hbm_bytes_per_launch: " + stated, "hbm_bytes_per_launch: %d" % (int(stated) + 10**6), 1)
    assert _read(tmp_path, off) is None                                              # average not from the rows
    assert _read(tmp_path, re.sub(r"kernel_hash: \w+", "kernel_hash: 0000", text)) is None   # other kernels
