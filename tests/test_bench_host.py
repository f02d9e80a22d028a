"""Host-side checks of bench.py's bookkeeping (no GPU): the HBM-traffic
record lookup and the algorithmic byte and flop counts it reports against.
"""
import hashlib
import os

import pytest

import bench
from workloads import layout


def _record(tmp_path, lines):
    p = tmp_path / "traffic.md"
    p.write_text("# traffic\n\n" + "\n".join(lines) + "\n")
    return str(p)


def _digest():
    h = hashlib.sha256()
    for f in bench.TRAFFIC_SOURCES:
        h.update(open(os.path.join(bench.ROOT, "paper_1402_5168_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def test_traffic_record_is_the_mean_of_the_listed_kernels(tmp_path, monkeypatch):
    d = _digest()
    monkeypatch.setattr(bench, "TRAFFIC_RECORD", _record(tmp_path, [
        f'    traffic-record kernel="k<a>" fetch_bytes=100 write_bytes=10 sources_sha256={d}',
        f'    traffic-record kernel="k<b>" fetch_bytes=300 write_bytes=30 sources_sha256={d}',
    ]))
    tr = bench.measured_traffic(["k<a>", "k<b>"])
    assert tr["read"] == 200 and tr["written"] == 20
    assert tr["per_launch"]["k<b>"] == {"read": 300, "written": 30}


def test_traffic_record_is_void_for_other_sources_or_kernels(tmp_path, monkeypatch):
    d = _digest()
    monkeypatch.setattr(bench, "TRAFFIC_RECORD", _record(tmp_path, [
        f'    traffic-record kernel="k<a>" fetch_bytes=100 write_bytes=10 sources_sha256={d}',
        '    traffic-record kernel="k<b>" fetch_bytes=300 write_bytes=30 sources_sha256=' + "0" * 64,
    ]))
    assert bench.measured_traffic(["k<a>"]) is not None
    assert bench.measured_traffic(["k<b>"]) is None            # sources changed since
    assert bench.measured_traffic(["k<a>", "k<c>"]) is None    # a kernel not recorded
    assert bench.measured_traffic([]) is None
    monkeypatch.setattr(bench, "TRAFFIC_RECORD", str(tmp_path / "missing.md"))
    assert bench.measured_traffic(["k<a>"]) is None


@pytest.mark.parametrize("nex,ney,p,walls", [(1, 1, 8, False), (2, 1, 6, False), (4, 4, 10, False),
                                             (2, 2, 8, True), (1, 1, 6, True)])
def test_interface_node_count(nex, ney, p, walls):
    """Sum over elements of their edge nodes that are unknowns: every
    interior edge counts once for each of its two elements; with walls each
    boundary edge counts once for its element."""
    m = layout.Mesh(nex, ney, p)
    q = p - 2
    count = 0
    for ey in range(ney):
        for ex in range(nex):
            for inside in (ex > 0, ex < nex - 1, ey > 0, ey < ney - 1):
                count += q if (inside or walls) else 0
    assert bench.interface_nodes(m, walls) == count


def test_leaf_up_flops_counts_complex_products():
    """8 real flops per complex multiply-add, q^4 per element and column."""
    m = layout.Mesh(4, 2, 10)
    assert bench.leaf_up_flops(m, 66, 32) == 8.0 * 8 * 64 * 64 * 66 * 32
