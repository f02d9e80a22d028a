#!/usr/bin/env python3
"""Throughput of the rational time stepper on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

One step applies exp(tau L) ~ sum_m b_m (tau L - alpha_m)^{-1} to the state
(all folded poles, the sweeps of the hierarchical solver, the FP64 pole
sum).  The default run is the precision form (FP32 operators and sweeps on
the matrix cores, one FP64 residual correction per step) with 32 batched
right-hand sides on 64x64 elements x 10^2 nodes and 131 poles; the same
inputs are then run in FP64 (batched, and with one right-hand side) for
the comparison and the accuracy of the precision form.  The timed region
is K steps replayed from the library's hipGraph, with the state and every
operator already resident in HBM; the build stage is timed separately.
Prints one JSON line.

Roofline: the same K steps are run again through hx_step_profile, which
brackets every kernel with HIP events on its launch stream.  Batched wave
runs put every kernel class (all its launches in a step) against its own
roofline, from its algorithmic bytes and flops per step (`stages`), and
report the class with the most time per step as the roofline object; with
one right-hand side the element upward sweep's bytes per launch over its
mean duration are compared with the HBM peak.
cpu_baseline: the FP64 CPU oracle (sparse LU of the assembled collocation
system) timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DOF·steps/s applying exp(τL), FP32-MFMA batched vs FP64, at rel err ≤1e-7"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6       # MI355X dense FP64 (vector and matrix)
FP32_PEAK_TFLOPS = 157.3      # MI355X dense FP32 (vector and matrix)


TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "traffic_wave_64x64_p10_fp32refine_r32.md")
TRAFFIC_SOURCES = ("apply_mm.hip", "residual.hip", "plan.hip", "hx_kernels.h", "hx_internal.h")


def sources_digest() -> str:
    """SHA-256 over the kernel and launch-plan sources the record depends on."""
    import hashlib

    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1402_5168_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def measured_step_traffic(tiles, variants) -> dict:
    """HBM bytes of one step per kernel class of the default workload, from
    the committed counter record: {class: {"read", "written", "launches"}},
    only for records taken with these sources and with the plan's tuned
    tiles and variants (empty otherwise)."""
    import re

    if not os.path.exists(TRAFFIC_RECORD):
        return {}
    want = (",".join(map(str, tiles)), ",".join(map(str, variants)))
    out = {}
    digest = None
    for m in re.finditer(r'traffic-step class="([^"]+)" launches=(\d+) tiles=([0-9,]+) '
                         r'variants=([0-9,]+) fetch_bytes=(\d+) write_bytes=(\d+) '
                         r'sources_sha256=([0-9a-f]+)', open(TRAFFIC_RECORD).read()):
        if (m.group(3), m.group(4)) != want:
            continue
        digest = digest or sources_digest()
        if m.group(7) != digest:
            continue
        out[m.group(1)] = {"read": int(m.group(5)), "written": int(m.group(6)),
                           "launches": int(m.group(2))}
    return out


def interface_nodes(mesh, walls: bool = False) -> int:
    """Sum over elements of their edge nodes that are unknowns (interfaces;
    with slip walls also the wall nodes)."""
    sides = 2 * ((mesh.nex - 1) * mesh.ney + mesh.nex * (mesh.ney - 1))
    if walls:
        sides += 2 * (mesh.nex + mesh.ney)
    return sides * mesh.q


def leaf_up_flops(mesh, npole: int, nrhs: int) -> float:
    """W g for every element, folded pole and right-hand side: 8 flops per
    complex multiply-add, q^4 of them per element and column."""
    q2 = mesh.q * mesh.q
    return 8.0 * mesh.n_el * q2 * q2 * npole * nrhs


def algorithmic_bytes(mesh, npole: int, nrhs: int, sw: bool = False) -> dict:
    """Bytes each kernel class must move per launch (all columns).

    k_leaf_up: W (q^4 complex) per element and column, the state read once
    per element and right-hand side (u0, v0), w (q^2) and h (edge nodes)
    written per column.  k_leaf_down: S (q^2 x e) per element and column,
    u_e read, w read and y written.  k_pole_sum: y read per column, state
    read and written once."""
    q2 = mesh.q * mesh.q
    ncol = npole * nrhs
    E = interface_nodes(mesh, sw)
    c16, d8 = 16, 8
    leaf_up = ncol * (mesh.n_el * q2 * q2 * c16 + mesh.n_el * q2 * c16 + E * c16) \
        + nrhs * 2 * mesh.n_el * q2 * d8
    leaf_down = ncol * (q2 * E * c16 + E * c16 + 2 * mesh.n_el * q2 * c16)
    pole_sum = ncol * mesh.n_el * q2 * c16 + nrhs * 3 * mesh.n_el * q2 * d8
    return {"k_leaf_up": leaf_up, "k_leaf_down": leaf_down, "k_pole_sum": pole_sum}


def merge_levels(mesh, walls: bool = False) -> list:
    """Boxes of each merge level, from the elements up: (n1, n2, n3) per box.

    Boxes are rectangles of elements; a level pairs neighbouring boxes along
    x while the boxes are no wider than tall (or only one row of boxes is
    left), else along y.  n3 counts the unknowns on the pair's shared edge,
    n1 and n2 those on the rest of each child's boundary: interface nodes,
    and wall nodes with slip walls (a Dirichlet boundary has none)."""
    q = mesh.q

    def ext(x0, y0, w, h):
        n = 0
        for length, outer in ((h, x0 == 0), (h, x0 + w == mesh.nex),
                              (w, y0 == 0), (w, y0 + h == mesh.ney)):
            if walls or not outer:
                n += length * q
        return n

    nbx, nby = mesh.nex, mesh.ney
    boxes = [(ex, ey, 1, 1) for ey in range(mesh.ney) for ex in range(mesh.nex)]
    levels = []
    while nbx * nby > 1:
        w, h = boxes[0][2], boxes[0][3]
        in_x = nbx > 1 and (w <= h or nby == 1)
        nbx2, nby2 = (nbx // 2, nby) if in_x else (nbx, nby // 2)
        nxt, lev = [], []
        for by in range(nby2):
            for bx in range(nbx2):
                a = boxes[2 * bx + nbx * by] if in_x else boxes[bx + nbx * 2 * by]
                b = boxes[2 * bx + 1 + nbx * by] if in_x else boxes[bx + nbx * (2 * by + 1)]
                n3 = (a[3] if in_x else a[2]) * q
                lev.append((ext(*a) - n3, ext(*b) - n3, n3))
                nxt.append((a[0], a[1], a[2] * 2, a[3]) if in_x else (a[0], a[1], a[2], a[3] * 2))
        levels.append(lev)
        boxes, nbx, nby = nxt, nbx2, nby2
    return levels


def stage_work(mesh, npole: int, nrhs: int, fp32: bool) -> dict:
    """Algorithmic HBM bytes and flops of one step of the batched wave
    problem, per kernel class: (bytes, flops, flop peak in TFLOP/s).

    Operators are read once per pole and serve all nrhs columns; vectors
    are read and written once per column (pole x RHS); c bytes per complex
    entry (8 FP32, 16 FP64).  The precision form runs two sweeps (the first
    and the correction), the FP64 form one; per sweep:
      k_leaf_up     W (q^4 per element and pole); w and h written
                    (q^2 + e per element and column); first sweep: the
                    FP64 sources (2 q^2 per element and RHS); correction:
                    the FP32 interior residual g (q^2 per element and column)
      k_merge_up    Y (ext x n3 per box and pole); children's h read
                    (ext + 2 n3), g3 and the box's h written (n3 + ext);
                    correction: the FP64 flux residual at both sides of
                    each shared edge node (16 B, e per element and column)
      k_merge_down  Z (n3 x (ext + n3)); u_ext and g3 read (ext + n3),
                    the children's u written (ext + 2 n3)
      k_leaf_down   S (q^2 x e per element and pole); u_e and w read; the
                    first sweep writes y (q^2); the last reads y (precision
                    form) and reads and writes the FP64 state (2 q^2 per
                    element and RHS) for the pole sum and post-map
      k_residual    (precision form) y and u_e read (FP32), the sources and
                    c^2 read (FP64), the FP32 interior residual and the FP64
                    flux values written; FP64 vector flops: 8 p per interior
                    node and column, 4 p per edge node
    Flops: 8 per complex multiply-add of the products."""
    q2 = mesh.q * mesh.q
    nel = mesh.n_el
    E = interface_nodes(mesh)
    ncol = npole * nrhs
    c = 8 if fp32 else 16
    sweeps = 2 if fp32 else 1
    boxes = [b for lev in merge_levels(mesh) for b in lev]
    Y = sum((n1 + n2) * n3 for n1, n2, n3 in boxes)
    Z = sum(n3 * (n1 + n2 + n3) for n1, n2, n3 in boxes)
    V = sum(2 * (n1 + n2) + 3 * n3 for n1, n2, n3 in boxes)
    peak = FP32_PEAK_TFLOPS if fp32 else FP64_PEAK_TFLOPS
    state = 2 * nel * q2 * 8 * nrhs           # the FP64 (u, v) of all RHS
    leaf_up = sweeps * (c * npole * nel * q2 * q2 + c * ncol * (nel * q2 + E)) + state
    merge_up = sweeps * (c * npole * Y + c * ncol * V)
    merge_down = sweeps * (c * npole * Z + c * ncol * V)
    leaf_down = sweeps * (c * npole * q2 * E + c * ncol * (E + nel * q2)) + 2 * state
    out = {
        "k_leaf_up": (leaf_up, 8.0 * sweeps * ncol * nel * q2 * q2, peak),
        "k_merge_up": (merge_up, 8.0 * sweeps * ncol * Y, peak),
        "k_merge_down": (merge_down, 8.0 * sweeps * ncol * Z, peak),
    }
    if fp32:
        out["k_leaf_up"] = (leaf_up + 8 * ncol * nel * q2, *out["k_leaf_up"][1:])
        out["k_merge_up"] = (merge_up + 16 * ncol * E, *out["k_merge_up"][1:])
        leaf_down += 2 * 8 * ncol * nel * q2
        p = mesh.p
        res = 8 * ncol * (nel * q2 + E) + state + 8 * nel * p * p + 8 * ncol * nel * q2 \
            + 16 * ncol * E
        out["k_residual"] = (res, float(ncol * (8 * p * nel * q2 + 4 * p * E)),
                             FP64_PEAK_TFLOPS)
    out["k_leaf_down"] = (leaf_down, 8.0 * sweeps * ncol * q2 * E, peak)
    return out


def stage_rooflines(work: dict, ms_per_step: dict) -> dict:
    """Each kernel class against its own roofline: the time its bytes take
    at the HBM peak or its flops at the flop peak, whichever is longer,
    over its measured time per step."""
    out = {}
    for name, (nbytes, flops, peak) in work.items():
        ms = ms_per_step.get(name)
        if not ms:
            continue
        t_hbm = nbytes / (HBM_PEAK_GBS * 1e9)
        t_flop = flops / (peak * 1e12)
        out[name] = {"ms_per_step": ms, "bytes_per_step": nbytes, "flops_per_step": flops,
                     "GBps": nbytes / (ms * 1e-3) / 1e9,
                     "TFLOPs": flops / (ms * 1e-3) / 1e12,
                     "bound": "hbm" if t_hbm >= t_flop else
                              ("mfma" if name != "k_residual" else "alu"),
                     "frac": max(t_hbm, t_flop) / (ms * 1e-3)}
    return out


def cpu_baseline_sw(recipe, npole_folded: int, sub: int = 8, poles: int = 4,
                    min_seconds: float = 10.0):
    """As cpu_baseline, for shallow water: the oracle's resolvent (sources,
    sparse solve of the eta system, velocity recovery) for `poles` of the
    folded shifts on a sub-mesh, scaled to all folded poles."""
    import numpy as np

    from oracle import shallow_water as osw
    from workloads import configs

    rec = configs.scaled_sw(recipe, sub, sub)
    w = configs.make_sw(rec, n_rhs=1)
    m = w.mesh
    g = osw.SWGrid(m.nex, m.ney, m.p)
    M = w.fit.M
    picks = np.linspace(0, M, poles).round().astype(int)
    steppers = [osw.SWStepper(g, rec.f, rec.gH, w.tau, w.fit.alpha[M + k:M + k + 1],
                              w.fit.b[M + k:M + k + 1]) for k in picks]
    reps = 0
    t0 = time.perf_counter()
    while True:
        for st in steppers:
            st.resolvent(0, w.v1[0], w.v2[0], w.eta[0])
        reps += 1
        if time.perf_counter() - t0 >= min_seconds or reps >= 100000:
            break
    dt = (time.perf_counter() - t0) / (reps * poles)
    step_s = dt * npole_folded
    dof = 3 * m.n_el * m.q * m.q
    return {"value": dof / step_s, "unit": "DOF·steps/s", "cores": 1, "kind": "oracle",
            "sample": (f"{sub}x{sub}-element sub-mesh, same p, f and gH, {poles} of "
                       f"{npole_folded} folded poles (sparse LU factorisation excluded), "
                       f"{reps} resolvent applications each ({dt * 1e3:.2f} ms each), scaled "
                       f"to {npole_folded} poles and one right-hand side; the SuperLU solve "
                       f"is single-threaded"),
            "step_seconds_sample": step_s}


def cpu_baseline(recipe, npole_folded: int, sub: int = 8, poles: int = 4,
                 min_seconds: float = 10.0):
    """The oracle's step rate on a sub-mesh of the same workload: `poles` of
    the folded shifts factored (factorisation excluded), their resolvent
    solves repeated for at least `min_seconds`, scaled to all folded poles."""
    import numpy as np

    from oracle import collocation as col
    from workloads import configs

    rec = configs.scaled(recipe, sub, sub)
    w = configs.make(rec, n_rhs=1)
    m = w.mesh
    grid = col.make_grid(m.nex, m.ney, m.p)
    K, P = col.assemble(grid, w.c2)
    M = w.fit.M
    picks = np.linspace(0, M, poles).round().astype(int)
    solvers = [col.ShiftedSolver(K, P, (w.fit.alpha[M + k] / w.tau) ** 2, grid.n_int)
               for k in picks]
    u0, v0 = w.u0[0], w.v0[0]
    reps = 0
    t0 = time.perf_counter()
    while True:
        for k, s in zip(picks, solvers):
            a = w.fit.alpha[M + k]
            y = s.solve_interior((a * u0 + w.tau * v0) / w.tau ** 2)
            _ = (a * y + u0) / w.tau
        reps += 1
        if time.perf_counter() - t0 >= min_seconds or reps >= 100000:
            break
    dt = (time.perf_counter() - t0) / (reps * poles)
    step_s = dt * npole_folded
    dof = 2 * m.n_el * m.q * m.q
    return {"value": dof / step_s, "unit": "DOF·steps/s", "cores": 1, "kind": "oracle",
            "sample": (f"{sub}x{sub}-element sub-mesh of the same field and p, "
                       f"{poles} of {npole_folded} folded poles (sparse LU factorisation "
                       f"excluded), {reps} resolvent solves each ({dt * 1e3:.2f} ms per "
                       f"solve), scaled to {npole_folded} poles and one right-hand side; "
                       f"the SuperLU solve is single-threaded"),
            "step_seconds_sample": step_s}


def run(w, precision: str, unbatched: bool, steps: int, warmup: int, profile: bool = True,
        autotune: bool = True):
    """Build one plan for the inputs w, time `steps` graph-replayed steps
    after `warmup` untimed ones, optionally profile the kernels.  Returns the
    measurements and the final state (host)."""
    import torch

    from paper_1402_5168_amd import hpsexp
    from workloads import configs

    m = w.mesh
    sw = isinstance(w, configs.SWInputs)
    nrhs = w.state().shape[0]
    fp32 = precision == "fp32-refine"
    batched = fp32 or sw or (nrhs > 1 and not unbatched)
    flags = (hpsexp.HX_FLAG_UNBATCHED if unbatched else 0) | (
        hpsexp.HX_FLAG_AUTOTUNE if autotune else 0)
    plan = hpsexp.Plan(device=0, flags=flags,
                       precision=hpsexp.HX_FP32_REFINE if fp32 else hpsexp.HX_FP64)
    if sw:
        plan.add_sw(m.nex, m.ney, m.p, w.recipe.f, w.recipe.gH, w.tau, configs.DELTA,
                    w.fit.alpha, w.fit.b, nrhs=nrhs)
    else:
        plan.add(m.nex, m.ney, m.p, w.c2, w.tau, configs.DELTA, w.fit.alpha, w.fit.b,
                 nrhs=nrhs)
    info = plan.query()
    plan.bind()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.build()
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    stream = torch.cuda.Stream(device=0)
    state = torch.tensor(w.state(), device="cuda:0")
    kms = nl = None
    with torch.cuda.stream(stream):
        plan.step([state], warmup, stream=stream)
        stream.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        plan.step([state], steps, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        if not bool(torch.isfinite(state).all()):
            raise RuntimeError("non-finite state after the timed steps")
        if profile:
            # roofline pass: same kernels, event pairs around each launch
            state2 = torch.tensor(w.state(), device="cuda:0")
            kms, nl = plan.step_profile([state2], steps, stream=stream)
            del state2
    final = state.cpu().numpy()
    tiles, variants = plan.tiles(0), plan.variants(0)
    plan.close()
    del plan, state
    torch.cuda.empty_cache()
    ms_step = ms / max(steps, 1)
    out = {"value": info["dof_state"] * steps / (ms / 1e3), "ms_per_step": ms_step,
           "build_s": build_s, "batched": batched, "info": info, "tiles": tiles,
           "variants": variants}
    if profile:
        kernels = {}
        ab = algorithmic_bytes(m, info["folded_poles"], nrhs, sw)
        for k, name in enumerate(hpsexp.KERNEL_NAMES):
            if nl[k] == 0:
                continue
            avg = kms[k] / nl[k]
            entry = {"launches": nl[k], "ms_total": kms[k], "ms_avg": avg}
            if name in ab and not batched:
                entry["bytes_per_launch"] = ab[name]
                entry["GBps"] = ab[name] / (avg * 1e-3) / 1e9
            kernels[name] = entry
        out["kernels"] = kernels
        if batched and not sw:
            # every kernel class against its roofline; the class with the
            # most time per step is the roofline object
            work = stage_work(m, info["folded_poles"], nrhs, fp32)
            st = stage_rooflines(work, {k: v["ms_total"] / steps for k, v in kernels.items()})
            meas = {}
            if fp32 and w.recipe.name == "wave_64x64_p10" and nrhs == 32:
                meas = measured_step_traffic(tiles, variants)
            for name, e in st.items():
                e["launches_per_step"] = kernels[name]["launches"] / steps
                t = meas.get(name)
                ok = t is not None and t["launches"] == e["launches_per_step"]
                e["traffic"] = t["read"] + t["written"] if ok else None
                e["traffic_split"] = {"read": t["read"], "written": t["written"]} if ok else None
            dom = max(st, key=lambda k: st[k]["ms_per_step"])
            d = st[dom]
            n = d["launches_per_step"]
            hbm = d["bound"] == "hbm"
            achieved = d["GBps"] if hbm else d["TFLOPs"]
            peak = HBM_PEAK_GBS if hbm else work[dom][2]
            out["roofline"] = {
                "bound": d["bound"], "kernel": dom, "launches_per_step": n,
                "achieved": achieved, "peak": peak, "unit": "GB/s" if hbm else "TFLOP/s",
                "frac": achieved / peak,
                "algorithmic_per_launch": (d["bytes_per_step"] if hbm else d["flops_per_step"]) / n,
                "ms_per_launch": d["ms_per_step"] / n,
                "traffic": None if d["traffic"] is None else d["traffic"] / n,
                "step_TFLOPs": info["flops_per_step"] / (ms_step * 1e-3) / 1e12}
            out["stages"] = st
        elif batched:
            # shallow water: the element upward sweep on the matrix cores
            dom = kernels["k_leaf_up"]
            flops = leaf_up_flops(m, info["folded_poles"], nrhs)
            tf = flops / (dom["ms_avg"] * 1e-3) / 1e12
            dom["flops_per_launch"] = flops
            dom["TFLOPs"] = tf
            peak = FP32_PEAK_TFLOPS if fp32 else FP64_PEAK_TFLOPS
            out["roofline"] = {"bound": "mfma", "kernel": "k_leaf_up", "achieved": tf,
                               "peak": peak, "unit": "TFLOP/s", "frac": tf / peak,
                               "traffic": None,
                               "step_TFLOPs": info["flops_per_step"] / (ms_step * 1e-3) / 1e12}
        else:
            dom = kernels["k_leaf_up"]
            out["roofline"] = {"bound": "hbm", "kernel": "k_leaf_up", "achieved": dom["GBps"],
                               "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": dom["GBps"] / HBM_PEAK_GBS, "traffic": None,
                               "step_op_bytes_GBps":
                                   info["op_bytes_per_step"] / (ms_step * 1e-3) / 1e9}
    return out, final


def run_batch(args):
    """Batching form: instances of the batch recipe, in order, as many as
    fit the arena budget, stepped as ONE plan (one fused launch per stage
    over all instances, replayed from a hipGraph), then each instance in a
    plan of its own, stepped one after the other, for the comparison."""
    import numpy as np
    import torch

    from paper_1402_5168_amd import hpsexp
    from workloads import configs

    rec = configs.BATCH_RECIPES[args.workload]
    prec = hpsexp.HX_FP32_REFINE if args.precision == "fp32-refine" else hpsexp.HX_FP64
    flags = hpsexp.HX_FLAG_AUTOTUNE if args.autotune else 0
    budget = args.budget_gb * 2 ** 30

    def add(plan, w):
        m = w.mesh
        return plan.add(m.nex, m.ney, m.p, w.c2, w.tau, configs.DELTA, w.fit.alpha, w.fit.b,
                        nrhs=w.u0.shape[0])

    ws, total = [], 0
    for i in range(args.max_instances or rec.n_instances):
        w = configs.batch_instance(rec, i)
        probe = hpsexp.Plan(device=0, precision=prec)
        add(probe, w)
        need = probe.query()["arena_bytes"]
        probe.close()
        if total + need > budget:
            break
        ws.append(w)
        total += need

    def timed(plans, states, steps, warmup):
        stream = torch.cuda.Stream(device=0)
        with torch.cuda.stream(stream):
            for pl, st in zip(plans, states):
                pl.step(st, warmup, stream=stream)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(steps):
                for pl, st in zip(plans, states):
                    pl.step(st, 1, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
        return e0.elapsed_time(e1), stream

    plan = hpsexp.Plan(device=0, precision=prec, flags=flags)
    for w in ws:
        add(plan, w)
    info = plan.query()
    plan.bind()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.build()
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    states = [torch.tensor(w.state(), device="cuda:0") for w in ws]
    ms, stream = timed([plan], [states], args.steps, args.warmup)
    finals = [x.cpu().numpy() for x in states]
    kms, nl = plan.step_profile(states, max(args.steps // 2, 1), stream=stream)
    tiles = [plan.tiles(k) for k in range(len(ws))]
    plan.close()
    del states
    torch.cuda.empty_cache()
    ms_step = ms / args.steps
    value = info["dof_state"] * 1e3 / ms_step
    kernels = {}
    for k, name in enumerate(hpsexp.KERNEL_NAMES):
        if nl[k]:
            kernels[name] = {"launches": nl[k], "ms_total": kms[k], "ms_avg": kms[k] / nl[k]}
    flops = sum(8.0 * w.mesh.n_el * w.mesh.q ** 4 * (w.fit.M + 1) * w.u0.shape[0] for w in ws)
    lu = kernels["k_leaf_up"]
    tf = flops / (lu["ms_avg"] * 1e-3) / 1e12
    peak = FP32_PEAK_TFLOPS if prec == hpsexp.HX_FP32_REFINE else FP64_PEAK_TFLOPS
    # the same instances, each in its own plan, stepped one after the other
    seq_ms = None
    if not args.no_compare:
        plans, sts = [], []
        for w in ws:
            pl = hpsexp.Plan(device=0, precision=prec)
            add(pl, w)
            pl.bind()
            pl.build()
            plans.append(pl)
            sts.append([torch.tensor(w.state(), device="cuda:0")])
        seq, _ = timed(plans, sts, args.steps, args.warmup)
        seq_ms = seq / args.steps
        err = 0.0
        for k, st in enumerate(sts):
            err = max(err, float(np.abs(st[0].cpu().numpy() - finals[k]).max()))
        for pl in plans:
            pl.close()
        del sts
    sides = {}
    for w in ws:
        sides[w.mesh.nex] = sides.get(w.mesh.nex, 0) + 1
    out = {
        "metric": METRIC, "value": value, "unit": "DOF·steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if prec == hpsexp.HX_FP32_REFINE else "f64", "data": "synthetic",
        "config": {"workload": f"{rec.name}: first {len(ws)} of {rec.n_instances} instances "
                               f"(arena budget {args.budget_gb} GiB)",
                   "instances": len(ws), "elements_per_side": sides, "p": rec.p,
                   "rhs_total": int(sum(w.u0.shape[0] for w in ws)),
                   "folded_poles_total": int(sum(w.fit.M + 1 for w in ws)),
                   "precision": args.precision, "autotune": bool(args.autotune),
                   "dof_state": info["dof_state"], "operator_GiB": info["operator_bytes"] / 2 ** 30,
                   "arena_GiB": info["arena_bytes"] / 2 ** 30},
        "build_s": build_s,
        "roofline": {"bound": "mfma", "kernel": "k_leaf_up", "achieved": tf, "peak": peak,
                     "unit": "TFLOP/s", "frac": tf / peak, "traffic": None},
        "kernels": kernels,
        "tiles_first_instances": {"stages": "leaf_up, merge_up, root, merge_down, leaf_down",
                                  "tiles": tiles[:6]},
    }
    if seq_ms is not None:
        out["compare"] = {"separate_plans_ms_per_step": seq_ms,
                          "speedup_fused_vs_separate": seq_ms / ms_step,
                          "max_abs_diff_fused_vs_separate": err}
    print(json.dumps(out), flush=True)


def trace_step(db: str) -> None:
    """The last step of a kernel trace of this benchmark: its dispatches
    from the last upward element sweep that follows a downward one (the
    step's first launch) to the end of the trace, with their durations,
    and the sums per kernel class.  With --steps K the trace ends with the
    per-kernel timing pass, whose steps launch the same kernels as the
    timed graph replays."""
    import sqlite3

    rows = list(sqlite3.connect(db).execute(
        "select name, start, end, grid_x, workgroup_x from kernels order by start"))
    rows = [r for r in rows if "hx::k_" in r[0]]
    starts = [i for i in range(1, len(rows))
              if "k_leaf_up" in rows[i][0] and "k_leaf_down" in rows[i - 1][0]]
    if not starts:
        raise SystemExit("no complete step in the trace")
    step = rows[starts[-1]:]
    classes = {}
    print("| # | kernel | blocks | us |\n|---:|---|---:|---:|")
    for i, (name, t0, t1, gx, wx) in enumerate(step):
        k = name.split("(")[0].replace("void ", "")
        us = (t1 - t0) / 1e3
        print(f"| {i} | {k} | {gx // max(wx, 1)} | {us:.1f} |")
        cls = k.replace("hx::", "").split("<")[0].replace("_sum_mm", "").replace("_mm", "")
        c = classes.setdefault(cls, [0, 0.0])
        c[0] += 1
        c[1] += us
    print("\n| class | launches | ms per step | ms per launch |\n|---|---:|---:|---:|")
    for cls, (n, us) in classes.items():
        print(f"| {cls} | {n} | {us / 1e3:.3f} | {us / 1e3 / n:.3f} |")
    print(f"\nstep: {len(step)} launches, {sum(c[1] for c in classes.values()) / 1e3:.3f} ms of kernels")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="wave_64x64_p10",
                    help="wave_4x4_p12, wave_32x32_p16, wave_64x64_p10, sw_32x32_p12 or batch_512")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the FP64 runs of the same workload")
    ap.add_argument("--nrhs", type=int, default=None,
                    help="right-hand sides (default: the workload's own count)")
    ap.add_argument("--unbatched", action="store_true",
                    help="one pass per right-hand side (reference for the batching speedup)")
    ap.add_argument("--precision", choices=["fp64", "fp32-refine"], default="fp32-refine")
    ap.add_argument("--budget-gb", type=float, default=120.0,
                    help="batch workloads: arena budget for the instances taken")
    ap.add_argument("--max-instances", type=int, default=None,
                    help="batch workloads: at most this many instances")
    ap.add_argument("--autotune", type=int, default=1,
                    help="tune the block shapes per stage at build (1, outside the timed region) "
                         "or use the default rule (0)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 1 GiB device to device once (calibrates HBM byte counters)")
    ap.add_argument("--trace-step", metavar="DB", default=None,
                    help="only print the last step's kernels from a rocprofv3 --kernel-trace "
                         "database (launch order, durations, per-class sums)")
    args = ap.parse_args()
    if args.trace_step:
        trace_step(args.trace_step)
        return
    if args.copy_probe:
        import torch
        x = torch.ones(2 ** 28, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": x.numel() * 4, "copy_bytes_written": y.numel() * 4}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(pole-sharded multi-GPU stepping is not part of this build)", file=sys.stderr)
        sys.exit(2)

    import numpy as np

    from workloads import configs

    if args.workload in configs.BATCH_RECIPES:
        run_batch(args)
        return
    sw = args.workload in configs.SW_RECIPES
    if sw:
        rec = configs.SW_RECIPES[args.workload]
        w = configs.make_sw(rec, n_rhs=args.nrhs)
    else:
        rec = configs.RECIPES[args.workload]
        w = configs.make(rec, n_rhs=args.nrhs)
    m = w.mesh
    nrhs = w.state().shape[0]
    nfield = 3 if sw else 2
    head, final = run(w, args.precision, args.unbatched, args.steps, args.warmup,
                      autotune=bool(args.autotune))
    info = head["info"]
    out = {
        "metric": METRIC, "value": head["value"], "unit": "DOF·steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "fp32-refine" else "f64",
        "data": "synthetic",
        "config": {"workload": rec.name, "problem": "shallow water, slip walls" if sw else
                   "wave, Dirichlet", "elements": f"{m.nex}x{m.ney}", "p": m.p,
                   "poles": rec.npoles, "folded_poles": info["folded_poles"], "nrhs": nrhs,
                   "precision": args.precision, "batched_rhs": head["batched"],
                   "tau": w.tau, "dof_state": info["dof_state"],
                   "dof_nodes": info["dof_nodes"], "fit_X": info["fit_X"],
                   "max_abs_R": info["max_abs_R"], "autotune": bool(args.autotune),
                   "tiles_per_stage": head["tiles"], "variants_per_stage": head["variants"],
                   "operator_GiB": info["operator_bytes"] / 2 ** 30},
        "dof_nodes_steps_per_s": info["dof_nodes"] * args.steps * 1e3 /
                                 (head["ms_per_step"] * args.steps),
        "build_s": head["build_s"],
        "roofline": head["roofline"],
        "kernels": head["kernels"],
    }
    if "stages" in head:
        out["stages"] = head["stages"]
    if not args.no_compare and args.precision == "fp32-refine":
        # the same inputs in FP64: batched, and one right-hand side
        ref, ref_final = run(w, "fp64", False, args.steps, args.warmup, profile=False,
                             autotune=bool(args.autotune))
        err = 0.0
        for r in range(nrhs):
            for f in range(nfield):
                x, y = final[r, f], ref_final[r, f]
                err = max(err, float(np.abs(x - y).max() / np.abs(y).max()))
        w1 = configs.make_sw(rec, n_rhs=1) if sw else configs.make(rec, n_rhs=1)
        one, _ = run(w1, "fp64", False, max(args.steps // 2, 1), 1, profile=False,
                     autotune=bool(args.autotune))
        out["compare"] = {
            "rel_err_vs_fp64": err,
            "fp64_batched": {"value": ref["value"], "ms_per_step": ref["ms_per_step"]},
            "fp64_1rhs": {"value": one["value"], "ms_per_step": one["ms_per_step"]},
            "speedup_vs_fp64_1rhs": head["value"] / one["value"],
            "speedup_vs_fp64_batched": head["value"] / ref["value"],
        }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = (cpu_baseline_sw if sw else cpu_baseline)(rec, info["folded_poles"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
