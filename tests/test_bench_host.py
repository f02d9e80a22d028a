"""Host-side checks of bench.py's bookkeeping (no GPU): the HBM-traffic
record lookup and the algorithmic byte and flop counts it reports against.
"""
import numpy as np
import pytest

import bench
from workloads import layout


def _record(tmp_path, lines):
    p = tmp_path / "traffic.md"
    p.write_text("# traffic\n\n" + "\n".join(lines) + "\n")
    return str(p)


def _step(cls, launches, tiles, variants, fetch, write, digest):
    return (f'    traffic-step class="{cls}" launches={launches} tiles={tiles} '
            f'variants={variants} fetch_bytes={fetch} write_bytes={write} sources_sha256={digest}')


def test_step_traffic_record_is_read_per_class(tmp_path, monkeypatch):
    d = bench.sources_digest()
    monkeypatch.setattr(bench, "TRAFFIC_RECORD", _record(tmp_path, [
        _step("k_merge_up", 24, "2,1,2,1,1", "1,0,0,0,0", 300, 30, d),
        _step("k_leaf_up", 2, "2,1,2,1,1", "1,0,0,0,0", 100, 10, d),
    ]))
    tr = bench.measured_step_traffic([2, 1, 2, 1, 1], [1, 0, 0, 0, 0])
    assert tr == {"k_merge_up": {"read": 300, "written": 30, "launches": 24},
                  "k_leaf_up": {"read": 100, "written": 10, "launches": 2}}


def test_step_traffic_record_is_void_for_other_sources_or_shapes(tmp_path, monkeypatch):
    d = bench.sources_digest()
    monkeypatch.setattr(bench, "TRAFFIC_RECORD", _record(tmp_path, [
        _step("k_merge_up", 24, "2,1,2,1,1", "1,0,0,0,0", 300, 30, "0" * 64),
        _step("k_leaf_up", 2, "2,1,2,1,1", "1,0,0,0,0", 100, 10, d),
    ]))
    assert list(bench.measured_step_traffic([2, 1, 2, 1, 1], [1, 0, 0, 0, 0])) == ["k_leaf_up"]
    assert bench.measured_step_traffic([1, 1, 2, 1, 1], [1, 0, 0, 0, 0]) == {}   # other tiles
    assert bench.measured_step_traffic([2, 1, 2, 1, 1], [0, 0, 0, 0, 0]) == {}   # other variants
    monkeypatch.setattr(bench, "TRAFFIC_RECORD", str(tmp_path / "missing.md"))
    assert bench.measured_step_traffic([2, 1, 2, 1, 1], [1, 0, 0, 0, 0]) == {}


def test_committed_record_matches_these_sources():
    """The committed counter record was taken with the current kernel and
    plan sources (else the benchmark reports no traffic)."""
    tr = bench.measured_step_traffic([2, 1, 2, 1, 1], [1, 0, 0, 0, 0])
    assert set(tr) == {"k_leaf_up", "k_merge_up", "k_merge_down", "k_leaf_down", "k_residual"}


def _tree_by_sets(nex, ney, q, walls):
    """Merge tree from explicit node sets: every element side owns q node
    ids (shared by the two elements of an interior side; on the outer
    boundary only with walls); a merge's n3 is the intersection of its
    children's sets, n1 and n2 the rest of each, the parent keeps the
    symmetric difference."""
    ids = {}

    def side(key):
        return ids.setdefault(key, [len(ids) * q + t for t in range(q)])

    sets = []
    for ey in range(ney):
        for ex in range(nex):
            s = set()
            for key, outer in ((("v", ex, ey), ex == 0), (("v", ex + 1, ey), ex + 1 == nex),
                               (("h", ex, ey), ey == 0), (("h", ex, ey + 1), ey + 1 == ney)):
                if walls or not outer:
                    s |= set(side(key))
            sets.append(s)
    nbx, nby, w, h = nex, ney, 1, 1
    levels = []
    while nbx * nby > 1:
        in_x = nbx > 1 and (w <= h or nby == 1)
        nbx2, nby2 = (nbx // 2, nby) if in_x else (nbx, nby // 2)
        nxt, lev = [], []
        for by in range(nby2):
            for bx in range(nbx2):
                a = sets[2 * bx + nbx * by] if in_x else sets[bx + nbx * 2 * by]
                b = sets[2 * bx + 1 + nbx * by] if in_x else sets[bx + nbx * (2 * by + 1)]
                lev.append((len(a - b), len(b - a), len(a & b)))
                nxt.append(a ^ b)
        levels.append(lev)
        sets, nbx, nby = nxt, nbx2, nby2
        w, h = (2 * w, h) if in_x else (w, 2 * h)
    return levels


@pytest.mark.parametrize("nex,ney,p,walls", [(2, 1, 4, False), (2, 2, 6, False), (4, 2, 8, False),
                                             (4, 4, 10, False), (8, 4, 6, False), (4, 4, 6, True),
                                             (8, 8, 5, True), (2, 4, 7, True)])
def test_merge_levels_match_explicit_node_sets(nex, ney, p, walls):
    m = layout.Mesh(nex, ney, p)
    lv = bench.merge_levels(m, walls)
    assert lv == _tree_by_sets(nex, ney, m.q, walls)
    # every interface node is shared at exactly one merge; the root keeps
    # only wall nodes
    n3 = sum(b[2] for lev in lv for b in lev)
    walls_nodes = 2 * (nex + ney) * m.q if walls else 0
    assert 2 * n3 == bench.interface_nodes(m, walls) - walls_nodes
    assert lv[-1] == [(lv[-1][0][0], lv[-1][0][1], lv[-1][0][2])]
    assert lv[-1][0][0] + lv[-1][0][1] == walls_nodes


def test_stage_work_by_hand():
    """Two elements of p = 4 (2 x 2 interior nodes, one shared edge of 2
    nodes), one pole, one RHS, FP64 (16 B per complex), one sweep.
    Element up: W 2 x 16 entries, w 2 x 4 and h 4 entries written, the
    (u, v) state (2 x 2 x 4 doubles) read.  The one merge: Y is empty
    (no exterior), Z is 2 x 2, vectors 2 ext + 3 n3 = 6 rows.  Element
    down: S 4 x 4 (interior x edge slots, summed over both), u_e (4) and
    w (8) read, state read and written."""
    m = layout.Mesh(2, 1, 4)
    w = bench.stage_work(m, 1, 1, False)
    assert w["k_leaf_up"][:2] == (16 * 32 + 16 * 12 + 128, 8.0 * 32)
    assert w["k_merge_up"][:2] == (16 * 6, 0.0)
    assert w["k_merge_down"][:2] == (16 * 4 + 16 * 6, 8.0 * 4)
    assert w["k_leaf_down"][:2] == (16 * 16 + 16 * 12 + 2 * 128, 8.0 * 16)
    assert "k_residual" not in w
    w32 = bench.stage_work(m, 1, 1, True)   # two sweeps, 8 B per complex
    assert w32["k_merge_down"][:2] == (2 * (8 * 4 + 8 * 6), 2 * 8.0 * 4)
    # correction sweep: the FP64 flux residual of the 4 edge slots
    assert w32["k_merge_up"][0] == 2 * 8 * 6 + 16 * 4


def test_stage_rooflines_take_the_longer_bound():
    work = {"k_leaf_up": (8e9, 1e12, 100.0),      # 1 ms of bytes, 10 ms of flops
            "k_merge_up": (16e9, 1e9, 100.0),     # 2 ms of bytes
            "k_residual": (1e6, 1e12, 78.6)}
    st = bench.stage_rooflines(work, {"k_leaf_up": 20.0, "k_merge_up": 4.0, "k_residual": 50.0})
    assert st["k_leaf_up"]["bound"] == "mfma" and st["k_leaf_up"]["frac"] == pytest.approx(0.5)
    assert st["k_merge_up"]["bound"] == "hbm" and st["k_merge_up"]["frac"] == pytest.approx(0.5)
    assert st["k_merge_up"]["GBps"] == pytest.approx(4000.0)
    assert st["k_residual"]["bound"] == "alu"
    assert "k_leaf_down" not in bench.stage_rooflines(work, {"k_leaf_down": 1.0})


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


def test_trace_step_lists_the_last_step(tmp_path, capsys):
    """A kernel trace of two steps (element up, merge up x2, merge down x2,
    element down) plus a foreign kernel: the last step alone is listed and
    summed per class."""
    import sqlite3

    db = tmp_path / "trace.db"
    con = sqlite3.connect(db)
    con.execute("create table kernels (name text, start int, end int, grid_x int, workgroup_x int)")
    step = [("void hx::k_leaf_up_mm<float, 2, true>(args)", 1000),
            ("void hx::k_merge_up_mm<float, 1, 4>(args)", 300),
            ("void hx::k_merge_up_mm<float, 1, 1>(args)", 100),
            ("void hx::k_merge_down_mm<float, 1, 4>(args)", 200),
            ("void hx::k_merge_down_mm<float, 1, 1>(args)", 200),
            ("void hx::k_leaf_down_sum_mm<float, 1>(args)", 500)]
    t = 0
    for rep in range(2):
        for name, dur in step:
            scale = 1 + rep          # the second step takes twice as long
            con.execute("insert into kernels values (?, ?, ?, ?, ?)",
                        (name, t, t + dur * scale * 1000, 256 * 64, 256))
            t += dur * scale * 1000 + 10
        con.execute("insert into kernels values ('copyBuffer', ?, ?, 1, 1)", (t, t + 5))
        t += 10
    con.commit()
    con.close()
    bench.trace_step(str(db))
    out = capsys.readouterr().out
    assert "| k_merge_up | 2 | 0.800 | 0.400 |" in out
    assert "| k_merge_down | 2 | 0.800 | 0.400 |" in out
    assert "| k_leaf_up | 1 | 2.000 | 2.000 |" in out
    assert "| k_leaf_down | 1 | 1.000 | 1.000 |" in out
    assert "step: 6 launches, 4.600 ms of kernels" in out


@pytest.mark.parametrize("nex,ney,walls", [(1, 1, False), (2, 1, False), (4, 4, False),
                                           (16, 8, False), (2, 8, False), (4, 2, True),
                                           (8, 8, True)])
def test_library_operator_storage_equals_tree_counts(nex, ney, walls):
    """The library's stored operator entries per pole (its plan query, no
    GPU) equal the counts the benchmark derives from the mesh: W (q^4) and
    S (q^2 e) per element, Y (ext n3) and Z (n3 (ext + n3)) per merge box,
    and with slip walls the root's dense wall system (n_wall^2).  p = 10
    (q = 8) keeps every block a multiple of the library's 8-entry
    alignment, so the counts agree exactly."""
    from paper_1402_5168_amd import hpsexp as hx
    from workloads.rational import calibrated_fit

    m = layout.Mesh(nex, ney, 10)
    fit = calibrated_fit(21)
    plan = hx.Plan()
    nrhs = 3
    if walls:
        plan.add_sw(nex, ney, m.p, 1.0, 1.0, 0.5, 1e-10, fit.alpha, fit.b, nrhs=nrhs)
    else:
        plan.add(nex, ney, m.p, np.ones(m.n_el * m.p * m.p), 0.5, 1e-10, fit.alpha, fit.b,
                 nrhs=nrhs)
    info = plan.query()
    plan.close()
    q2 = m.q * m.q
    boxes = [b for lev in bench.merge_levels(m, walls) for b in lev]
    entries = (m.n_el * q2 * q2 + q2 * bench.interface_nodes(m, walls)
               + sum((n1 + n2) * n3 + n3 * (n1 + n2 + n3) for n1, n2, n3 in boxes))
    if walls:
        entries += (2 * (nex + ney) * m.q) ** 2
    npole = info["folded_poles"]
    assert info["operator_bytes"] == 16 * npole * entries
    if not walls:
        # one batched FP64 sweep: 8 flops per stored entry and column
        assert info["flops_per_step"] == 8.0 * npole * nrhs * entries
