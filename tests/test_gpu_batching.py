"""GPU checks of the batching form: instances of uneven size in one plan run
as fused launches (one launch per stage over every instance), and must give
bit-identical results to each instance alone in its own plan (summation
order is the same per block), in FP64 and in the precision form, for wave
and shallow-water instances mixed.  Together with the per-instance parity
tests against the oracle this pins the fused path to the oracle."""
import dataclasses

import numpy as np
import pytest

from workloads import configs, layout

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def wave(nex, ney, p, npoles, nrhs, seed=0):
    rec = dataclasses.replace(configs.RECIPES["wave_4x4_p12"], mesh=layout.Mesh(nex, ney, p),
                              npoles=npoles, speed="clipped_lognormal", speed_seed=seed,
                              pulse_seeds=tuple(range(seed, seed + nrhs)))
    w = configs.make(rec)
    w.v0[:] = 0.25 * np.roll(w.u0, 1, axis=0)     # nonzero velocities
    return w


def sw(nex, ney, p, npoles, nrhs, f=1.0):
    rec = dataclasses.replace(configs.SW_RECIPES["sw_32x32_p12"], mesh=layout.Mesh(nex, ney, p),
                              npoles=npoles, f=f, kmax=4.0, seeds=tuple(range(nrhs)))
    return configs.make_sw(rec)


def run(ws, n_steps, precision, flags=0):
    torch = _torch()
    from paper_1402_5168_amd import hpsexp
    plan = hpsexp.Plan(device=0, precision=precision, flags=flags)
    for w in ws:
        m = w.mesh
        if isinstance(w, configs.SWInputs):
            plan.add_sw(m.nex, m.ney, m.p, w.recipe.f, w.recipe.gH, w.tau, 1e-10, w.fit.alpha,
                        w.fit.b, nrhs=w.state().shape[0])
        else:
            plan.add(m.nex, m.ney, m.p, w.c2, w.tau, 1e-10, w.fit.alpha, w.fit.b,
                     nrhs=w.state().shape[0])
    plan.bind()
    plan.build()
    states = [torch.tensor(w.state(), device="cuda:0") for w in ws]
    stream = torch.cuda.Stream(device=0)
    with torch.cuda.stream(stream):
        plan.step(states, n_steps, stream=stream)
    stream.synchronize()
    out = [x.cpu().numpy() for x in states]
    plan.close()
    return out


def batch():
    return [wave(4, 4, 8, 21, 3), wave(8, 8, 6, 41, 17, seed=3), wave(2, 4, 12, 21, 2, seed=5),
            sw(4, 4, 8, 21, 5), sw(2, 1, 10, 41, 18, f=0.5), wave(1, 1, 8, 21, 33, seed=7)]


@pytest.mark.parametrize("precision", [0, 1])
def test_fused_instances_equal_separate_plans(precision):
    say(f"6 instances (wave and shallow water, uneven meshes, 2..33 RHS), precision {precision}")
    ws = batch()
    both = run(ws, 3, precision)
    for k, w in enumerate(ws):
        alone = run([w], 3, precision)[0]
        assert np.isfinite(both[k]).all()
        assert np.array_equal(both[k], alone), (k, np.abs(both[k] - alone).max())


def test_fused_graph_equals_eager():
    say("6 instances, precision form, graph replay vs eager launches")
    from paper_1402_5168_amd import hpsexp
    ws = batch()
    g = run(ws, 4, 1)
    e = run(ws, 4, 1, flags=hpsexp.HX_FLAG_NO_GRAPH)
    for a, b in zip(g, e):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("precision", [0, 1])
def test_fused_merge_pairs_equal_per_level_merges(precision):
    """Fused pairs of low merge levels (the level between them kept in LDS)
    perform the same products, stagings and roundings as one launch per
    level: the results are bit-identical."""
    say(f"6 instances, precision {precision}, fused merge pairs vs one launch per level")
    from paper_1402_5168_amd import hpsexp
    ws = batch()
    fused = run(ws, 3, precision, flags=hpsexp.HX_FLAG_FUSED_MERGES)
    ref = run(ws, 3, precision)
    for a, b in zip(fused, ref):
        assert np.array_equal(a, b)


def test_autotuned_plan_equals_default_plan():
    """The autotuner only changes kernel shapes (16-column tiles per block,
    source staging, waves per block, pole groups, fused merge pairs); every
    column's arithmetic and order stay the same, so the results are
    bit-identical to the default shapes."""
    say("6 instances, precision form, autotuned shapes vs default shapes")
    torch = _torch()
    from paper_1402_5168_amd import hpsexp
    ws = batch()
    tuned = hpsexp.Plan(device=0, precision=1, flags=hpsexp.HX_FLAG_AUTOTUNE)
    for w in ws:
        m = w.mesh
        if isinstance(w, configs.SWInputs):
            tuned.add_sw(m.nex, m.ney, m.p, w.recipe.f, w.recipe.gH, w.tau, 1e-10, w.fit.alpha,
                         w.fit.b, nrhs=w.state().shape[0])
        else:
            tuned.add(m.nex, m.ney, m.p, w.c2, w.tau, 1e-10, w.fit.alpha, w.fit.b,
                      nrhs=w.state().shape[0])
    tuned.bind()
    tuned.build()
    tiles = [tuned.tiles(k) for k in range(len(ws))]
    say(f"tiles per instance: {tiles}")
    for k, w in enumerate(ws):
        assert all(t in (1, 2) for t in tiles[k])
        if w.state().shape[0] <= 16:
            assert tiles[k] == [1] * hpsexp.HX_STAGES
    states = [torch.tensor(w.state(), device="cuda:0") for w in ws]
    stream = torch.cuda.Stream(device=0)
    with torch.cuda.stream(stream):
        tuned.step(states, 3, stream=stream)
    stream.synchronize()
    got = [x.cpu().numpy() for x in states]
    tuned.close()
    ref = run(ws, 3, 1)
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)
