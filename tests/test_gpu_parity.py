"""GPU parity: the HIP time stepper against the CPU oracle, through the C-ABI.

Tolerance: relative L-infinity error per field <= 1e-10 after the stated
number of steps (FP64 form), at sizes the oracle solves in seconds; the
meshes span several elements, ragged shapes (nex != ney, 1 x 1, 1 x n), the
smallest and largest p, several right-hand sides and several instances.
"""
import numpy as np
import pytest

from oracle import collocation as col
from workloads import configs, fields, layout
from workloads.rational import calibrated_fit

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


def oracle_run(w, n_steps):
    m = w.mesh
    st = col.WaveStepper(col.make_grid(m.nex, m.ney, m.p, m.x0, m.x1, m.y0, m.y1), w.c2,
                         w.tau, w.fit.alpha, w.fit.b, folded=True)
    return [st.run(w.u0[r], w.v0[r], n_steps) for r in range(w.u0.shape[0])]


def gpu_run(ws, n_steps, flags=0, split=None, workspace=None, precision=0):
    torch = _torch()
    from paper_1402_5168_amd import hpsexp
    plan = hpsexp.Plan(device=0, flags=flags, precision=precision)
    for w in ws:
        m = w.mesh
        plan.add(m.nex, m.ney, m.p, w.c2, w.tau, 1e-10, w.fit.alpha, w.fit.b,
                 nrhs=w.u0.shape[0], domain=(m.x0, m.x1, m.y0, m.y1))
    plan.bind()
    plan.build(workspace_bytes=workspace)
    states = [torch.tensor(w.state(), device="cuda:0") for w in ws]
    stream = torch.cuda.Stream(device=0)
    with torch.cuda.stream(stream):
        for n in (split or [n_steps]):
            plan.step(states, n, stream=stream)
    stream.synchronize()
    out = [s.cpu().numpy() for s in states]
    plan.close()
    return out


def check(w, got, n_steps, tol=TOL):
    ref = oracle_run(w, n_steps)
    worst = 0.0
    for r, (u, v) in enumerate(ref):
        eu, ev = rel_err(got[r, 0], u), rel_err(got[r, 1], v)
        worst = max(worst, eu, ev)
        assert eu <= tol and ev <= tol, (r, eu, ev)
    say(f"max rel err {worst:.3e} (tol {tol:.0e})")
    return ref


def make(nex, ney, p, npoles=21, n_rhs=1, speed="smooth", tau=0.5, domain=(0, 1, 0, 1)):
    rec = configs.RECIPES["wave_4x4_p12"]
    import dataclasses
    rec = dataclasses.replace(rec, mesh=layout.Mesh(nex, ney, p, *domain), npoles=npoles,
                              speed=speed, tau=tau, pulse_seeds=tuple(range(n_rhs)))
    return configs.make(rec)


def test_wave_4x4_p12_ten_steps():
    say("wave_4x4_p12, 21 poles, 10 steps")
    w = configs.make("wave_4x4_p12")
    got = gpu_run([w], 10)[0]
    check(w, got, 10)


@pytest.mark.parametrize("nex,ney,p", [(1, 1, 8), (2, 1, 6), (1, 4, 10), (8, 2, 8),
                                       (2, 2, 4), (2, 2, 18), (4, 8, 12)])
def test_ragged_meshes(nex, ney, p):
    say(f"ragged mesh {nex}x{ney} p={p}")
    w = make(nex, ney, p)
    got = gpu_run([w], 3)[0]
    check(w, got, 3)


def test_stretched_domain_and_more_poles():
    say("2x4 on [0,2]x[-1,0], p=10, 41 poles")
    w = make(2, 4, 10, npoles=41, domain=(0.0, 2.0, -1.0, 0.0))
    got = gpu_run([w], 3)[0]
    check(w, got, 3)


def test_several_rhs():
    say("4x2 p=8, 3 right-hand sides")
    w = make(4, 2, 8, n_rhs=3)
    w.v0[1] = 0.3 * w.u0[2]                 # one RHS with nonzero velocity
    got = gpu_run([w], 4)[0]
    check(w, got, 4)


def test_several_instances_match_single_instance_plans():
    say("two instances in one plan vs separate plans")
    w1 = make(4, 4, 8)
    w2 = make(2, 4, 10, npoles=41, n_rhs=2)
    both = gpu_run([w1, w2], 3)
    one = gpu_run([w1], 3)[0]
    two = gpu_run([w2], 3)[0]
    assert np.array_equal(both[0], one)
    assert np.array_equal(both[1], two)
    check(w2, two, 3)


def test_graph_replay_equals_eager_and_resume():
    say("graph vs eager, 6 = 3 + 3 steps")
    from paper_1402_5168_amd import hpsexp
    w = make(4, 4, 10)
    g = gpu_run([w], 6)[0]
    e = gpu_run([w], 6, flags=hpsexp.HX_FLAG_NO_GRAPH)[0]
    s = gpu_run([w], 6, split=[3, 0, 3])[0]
    assert np.array_equal(g, e)
    assert np.array_equal(g, s)


def test_pole_chunked_build_matches():
    say("build with a workspace for one pole at a time")
    from paper_1402_5168_amd import hpsexp
    w = make(4, 4, 8)
    plan = hpsexp.Plan()
    plan.add(4, 4, 8, w.c2, w.tau, 1e-10, w.fit.alpha, w.fit.b)
    small = plan.query()["workspace_min_bytes"]
    plan.close()
    a = gpu_run([w], 2, workspace=small)[0]
    b = gpu_run([w], 2)[0]
    assert rel_err(a, b) <= 1e-13


def test_nonfinite_state_is_rejected():
    say("NaN state with the check flag")
    torch = _torch()
    from paper_1402_5168_amd import hpsexp
    w = make(2, 2, 6)
    plan = hpsexp.Plan(flags=hpsexp.HX_FLAG_CHECK_STATE)
    plan.add(2, 2, 6, w.c2, w.tau, 1e-10, w.fit.alpha, w.fit.b)
    plan.bind()
    plan.build()
    x = torch.tensor(w.state(), device="cuda:0")
    x[0, 1, 5] = float("nan")
    before = x.clone()
    with pytest.raises(hpsexp.HxError) as e:
        plan.step([x], 1)
    assert e.value.status == hpsexp.HX_ESTATE
    torch.cuda.synchronize()
    assert torch.equal(torch.nan_to_num(x), torch.nan_to_num(before))
    plan.close()


def test_eigenmode_at_full_size_100_steps():
    """32 x 32 elements x 16^2 nodes, 101 poles, 100 steps of the pulse time
    step, constant c: a Dirichlet mode must come back as cos(n tau w) times
    itself (closed form; error <= n * fit error + discretisation error)."""
    say("full size 32x32 p=16, 101 poles, const c, 100 steps")
    rec = configs.RECIPES["wave_32x32_p16"]
    w = configs.make(rec)
    X, Y = layout.interior_nodes(w.mesh)
    k, l = 3, 2
    phi = fields.dirichlet_mode(X, Y, k, l)
    w.c2 = np.ones_like(w.c2)
    w.u0 = phi[None, :].copy()
    w.v0 = np.zeros_like(w.u0)
    n = 100
    got = gpu_run([w], n)[0]
    om = np.pi * np.hypot(k, l)
    t = n * w.tau
    assert np.abs(got[0, 0] - np.cos(om * t) * phi).max() < 1e-8
    assert np.abs(got[0, 1] + om * np.sin(om * t) * phi).max() < 1e-8 * om


# ---- many right-hand sides on the matrix cores ------------------------------------

@pytest.mark.parametrize("nex,ney,p,nrhs", [(4, 4, 10, 2), (4, 2, 8, 16), (2, 4, 12, 17),
                                            (4, 4, 10, 32), (2, 2, 16, 40), (2, 1, 18, 20),
                                            (1, 1, 7, 3), (8, 8, 6, 33)])
def test_batched_rhs_match_oracle(nex, ney, p, nrhs):
    say(f"batched {nex}x{ney} p={p} nrhs={nrhs}")
    w = make(nex, ney, p, n_rhs=nrhs)
    rng = np.random.default_rng(nrhs)
    w.v0 = 0.2 * rng.standard_normal(w.u0.shape) * w.u0      # nonzero velocities
    got = gpu_run([w], 2)[0]
    check(w, got, 2)


def test_batched_equals_unbatched():
    say("batched vs one pass per RHS, 4x4 p=10, 24 RHS")
    from paper_1402_5168_amd import hpsexp
    w = make(4, 4, 10, n_rhs=24)
    a = gpu_run([w], 3)[0]
    b = gpu_run([w], 3, flags=hpsexp.HX_FLAG_UNBATCHED)[0]
    assert rel_err(a, b) <= 1e-13


# ---- precision form: FP32 operators and sweeps + FP64 residual correction --------

TOL32 = 1e-7


@pytest.mark.parametrize("nex,ney,p,nrhs,steps", [(4, 4, 12, 1, 10), (4, 2, 8, 3, 10),
                                                  (2, 2, 10, 32, 5), (1, 1, 8, 2, 5),
                                                  (8, 4, 6, 17, 5), (2, 1, 18, 1, 3)])
def test_precision_form_matches_oracle(nex, ney, p, nrhs, steps):
    say(f"fp32+refine {nex}x{ney} p={p} nrhs={nrhs} steps={steps}")
    w = make(nex, ney, p, n_rhs=nrhs)
    rng = np.random.default_rng(3 + nrhs)
    w.v0 = 0.2 * rng.standard_normal(w.u0.shape) * w.u0
    got = gpu_run([w], steps, precision=1)[0]
    check(w, got, steps, tol=TOL32)


@pytest.fixture(scope="module")
def wave_16x16_p10():
    """16x16 elements, p = 10, 17 RHS with nonzero velocities, and the
    oracle's state after 2 steps (shared by both precisions)."""
    w = make(16, 16, 10, n_rhs=17)
    rng = np.random.default_rng(11)
    w.v0 = 0.2 * rng.standard_normal(w.u0.shape) * w.u0
    say("oracle: 16x16 p=10, 17 RHS, 2 steps")
    return w, oracle_run(w, 2)


@pytest.mark.parametrize("precision", [0, 1])
def test_batched_merges_with_several_chunks_and_row_groups(wave_16x16_p10, precision):
    """The upper merges of a 16x16 mesh (p = 10) have exteriors of 128-160
    rows and interfaces of 64-128 nodes: the matrix-core upward blocks run
    several row groups, the downward ones several row groups (128-row top
    interface) and several staged k-chunks (ext + n3 = 192 columns: two
    chunks of 128 in FP32, three of 64 in FP64), and the two-tile RHS blocks
    end ragged (17 of 32 columns)."""
    w, ref = wave_16x16_p10
    say(f"batched 16x16 p=10 nrhs=17, precision {precision}, 2 steps")
    got = gpu_run([w], 2, precision=precision)[0]
    tol = TOL if precision == 0 else TOL32
    worst = 0.0
    for r, (u, v) in enumerate(ref):
        worst = max(worst, rel_err(got[r, 0], u), rel_err(got[r, 1], v))
    say(f"max rel err {worst:.3e} (tol {tol:.0e})")
    assert worst <= tol


def test_precision_form_wave_4x4_p12_100_steps():
    say("fp32+refine wave_4x4_p12, 100 steps")
    w = configs.make(configs.scaled("wave_4x4_p12", 4, 4, n_steps=100))
    got = gpu_run([w], 100, precision=1)[0]
    check(w, got, 100, tol=TOL32)
