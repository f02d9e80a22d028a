"""GPU parity for shallow water with slip walls: the HIP stepper against the
CPU oracle (oracle/shallow_water.py), through the C-ABI.

Tolerance: relative L-infinity error per field <= 1e-10 after the stated
number of steps (FP64 form), <= 1e-7 for the precision form (FP32 sweeps
with one FP64 residual correction per step).  The cases cover square and ragged meshes,
f = 0 and f != 0, several right-hand sides (one and two tiles of 16), a
stretched domain, and a plan holding a wave and a shallow-water instance.
"""
import dataclasses

import numpy as np
import pytest

from oracle import shallow_water as osw
from workloads import configs, layout

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def rel_err(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def make(nex, ney, p, npoles=21, n_rhs=1, f=1.0, gH=1.0, kmax=4.0):
    rec = dataclasses.replace(configs.SW_RECIPES["sw_32x32_p12"],
                              mesh=layout.Mesh(nex, ney, p), npoles=npoles, f=f, gH=gH,
                              kmax=kmax, seeds=tuple(range(n_rhs)))
    return configs.make_sw(rec)


def oracle_run(w, n_steps):
    m, r = w.mesh, w.recipe
    g = osw.SWGrid(m.nex, m.ney, m.p, m.x0, m.x1, m.y0, m.y1)
    st = osw.SWStepper(g, r.f, r.gH, w.tau, w.fit.alpha, w.fit.b, folded=True)
    return [st.run(w.v1[k], w.v2[k], w.eta[k], n_steps) for k in range(w.v1.shape[0])]


def gpu_run(ws, n_steps, extra_wave=None, precision=0):
    torch = _torch()
    from paper_1402_5168_amd import hpsexp
    plan = hpsexp.Plan(device=0, precision=precision)
    for w in ws:
        m, r = w.mesh, w.recipe
        plan.add_sw(m.nex, m.ney, m.p, r.f, r.gH, w.tau, 1e-10, w.fit.alpha, w.fit.b,
                    nrhs=w.v1.shape[0], domain=(m.x0, m.x1, m.y0, m.y1))
    if extra_wave is not None:
        m = extra_wave.mesh
        plan.add(m.nex, m.ney, m.p, extra_wave.c2, extra_wave.tau, 1e-10, extra_wave.fit.alpha,
                 extra_wave.fit.b, nrhs=extra_wave.u0.shape[0])
    plan.bind()
    plan.build()
    host = [w.state() for w in ws] + ([extra_wave.state()] if extra_wave is not None else [])
    states = [torch.tensor(x, device="cuda:0") for x in host]
    stream = torch.cuda.Stream(device=0)
    with torch.cuda.stream(stream):
        plan.step(states, n_steps, stream=stream)
    stream.synchronize()
    out = [s.cpu().numpy() for s in states]
    plan.close()
    return out


def check(w, got, n_steps, tol=TOL):
    ref = oracle_run(w, n_steps)
    worst = 0.0
    for k, fields in enumerate(ref):
        for fi, x in enumerate(fields):
            e = rel_err(got[k, fi], x)
            worst = max(worst, e)
            assert e <= tol, (k, fi, e)
    say(f"max rel err {worst:.3e} (tol {tol:.0e})")


@pytest.mark.parametrize("nex,ney,p,f", [(2, 2, 8, 1.0), (1, 1, 6, 1.0), (2, 1, 10, 0.0),
                                         (4, 2, 6, 2.0), (4, 4, 12, 1.0)])
def test_sw_meshes(nex, ney, p, f):
    say(f"sw {nex}x{ney} p={p} f={f}, 21 poles, 3 steps")
    w = make(nex, ney, p, f=f)
    got = gpu_run([w], 3)[0]
    check(w, got, 3)


def test_sw_more_poles_several_rhs():
    say("sw 4x4 p=8, 41 poles, 3 right-hand sides, 4 steps")
    w = make(4, 4, 8, npoles=41, n_rhs=3)
    got = gpu_run([w], 4)[0]
    check(w, got, 4)


def test_sw_two_rhs_tiles():
    say("sw 2x2 p=8, 21 poles, 20 right-hand sides (two tiles of 16), 2 steps")
    w = make(2, 2, 8, n_rhs=20)
    got = gpu_run([w], 2)[0]
    check(w, got, 2)


def test_sw_beside_wave_instance():
    say("sw 2x4 p=8 and wave 4x4 p=8 in one plan vs separate plans")
    w = make(2, 4, 8, n_rhs=2)
    rec = dataclasses.replace(configs.RECIPES["wave_4x4_p12"], mesh=layout.Mesh(4, 4, 8))
    wv = configs.make(rec)
    both = gpu_run([w], 3, extra_wave=wv)
    alone = gpu_run([w], 3)[0]
    assert np.array_equal(both[0], alone)
    check(w, alone, 3)


@pytest.mark.parametrize("nex,ney,p,npoles,n_rhs,f,steps",
                         [(2, 2, 8, 21, 1, 1.0, 5), (4, 4, 12, 21, 3, 1.0, 5),
                          (1, 1, 6, 21, 2, 0.0, 5), (4, 2, 10, 41, 20, 2.0, 3),
                          (8, 8, 6, 21, 5, 1.0, 3)])
def test_sw_precision_form(nex, ney, p, npoles, n_rhs, f, steps):
    say(f"sw fp32+refine {nex}x{ney} p={p} {npoles} poles nrhs={n_rhs} f={f} steps={steps}")
    w = make(nex, ney, p, npoles=npoles, n_rhs=n_rhs, f=f)
    got = gpu_run([w], steps, precision=1)[0]
    check(w, got, steps, tol=1e-7)
