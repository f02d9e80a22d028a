"""GPU long runs at the full workload sizes: the precision form (FP32 sweeps
with one FP64 residual correction per step) against the FP64 form after 100
steps, on the 64x64 p=10 wave workload (131 poles, 32 RHS) and the 32x32
p=12 shallow-water workload (101 poles, 64 RHS), in the launch form the
benchmark times (autotuned plans).

The FP64 form is the reference here: the oracle cannot take 100 steps of
these sizes in a test, and the FP64 GPU path is pinned to the oracle
(<= 1e-10 on smaller meshes, closed-form modes at full size).  Error norm:
relative L-infinity over each RHS's whole state, max over the RHS; bound
1e-7 for the precision form.
"""
import numpy as np
import pytest

from workloads import configs

pytestmark = pytest.mark.gpu

TOL = 1e-7
STEPS = 100


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def run(w, precision, n_steps):
    torch = _torch()
    from paper_1402_5168_amd import hpsexp
    plan = hpsexp.Plan(device=0, precision=precision, flags=hpsexp.HX_FLAG_AUTOTUNE)
    m = w.mesh
    if isinstance(w, configs.SWInputs):
        plan.add_sw(m.nex, m.ney, m.p, w.recipe.f, w.recipe.gH, w.tau, configs.DELTA, w.fit.alpha,
                    w.fit.b, nrhs=w.state().shape[0])
    else:
        plan.add(m.nex, m.ney, m.p, w.c2, w.tau, configs.DELTA, w.fit.alpha, w.fit.b,
                 nrhs=w.state().shape[0])
    plan.bind()
    plan.build()
    state = torch.tensor(w.state(), device="cuda:0")
    stream = torch.cuda.Stream(device=0)
    with torch.cuda.stream(stream):
        plan.step([state], n_steps, stream=stream)
    stream.synchronize()
    out = state.cpu().numpy()
    plan.close()
    del state
    torch.cuda.empty_cache()
    return out


def worst_rel(got, ref):
    n = ref.shape[0]
    g, r = got.reshape(n, -1), ref.reshape(n, -1)
    return max(np.abs(g[k] - r[k]).max() / np.abs(r[k]).max() for k in range(n))


@pytest.mark.parametrize("name,maker", [("wave_64x64_p10", configs.make),
                                        ("sw_32x32_p12", configs.make_sw)])
def test_precision_form_tracks_fp64_for_100_steps(name, maker):
    say(f"{name}: precision form vs FP64 after {STEPS} steps")
    w = maker(name)
    f32 = run(w, 1, STEPS)
    f64 = run(w, 0, STEPS)
    assert np.isfinite(f64).all() and np.isfinite(f32).all()
    e = worst_rel(f32, f64)
    say(f"max over RHS of the relative L-inf difference: {e:.3e} (tol {TOL:.0e})")
    assert e <= TOL
