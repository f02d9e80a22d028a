"""C-ABI checks that need no GPU: the library loads, exports every entry
point declared in include/hpsexp.h, and its host-side validation rejects
bad input with the documented status codes before touching a device."""
import os
import re
from ctypes import POINTER, c_double

import numpy as np
import pytest

from conftest import ROOT
from paper_1402_5168_amd import hpsexp as hx
from workloads.rational import calibrated_fit

HEADER = os.path.join(ROOT, "include", "hpsexp.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:hx_status|const char\*|void)\s+(hx_\w+)\s*\(",
                                 text, flags=re.M)))


def test_library_exports_every_declared_symbol():
    lib = hx.load()
    names = declared_functions()
    assert set(names) == set(hx.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings():
    assert hx.hx_status_str(hx.HX_OK) == "HX_OK"
    assert hx.hx_status_str(hx.HX_ESINGULAR) == "HX_ESINGULAR"
    assert hx.hx_status_str(12345) == "HX_UNKNOWN"


def _add(plan, nex=4, ney=4, p=8, c2=None, tau=0.5, delta=1e-10, fit=None, nrhs=1,
         alpha=None, b=None):
    fit = fit or calibrated_fit(21)
    if c2 is None:
        c2 = np.ones(nex * ney * p * p)
    return plan.add(nex, ney, p, c2, tau, delta,
                    fit.alpha if alpha is None else alpha,
                    fit.b if b is None else b, nrhs)


def status_of(fn):
    with pytest.raises(hx.HxError) as e:
        fn()
    return e.value.status


def test_create_rejects_bad_arguments():
    assert status_of(lambda: hx.hx_plan_create(7, 0, 0)) == hx.HX_EINVAL
    hx.hx_plan_destroy(hx.hx_plan_create(hx.HX_FP32_REFINE, 0, 0))
    assert status_of(lambda: hx.hx_plan_create(hx.HX_FP64, -1, 0)) == hx.HX_EINVAL
    assert status_of(lambda: hx.hx_plan_create(hx.HX_FP64, 0, 0x100)) == hx.HX_EINVAL


def test_add_validation():
    plan = hx.Plan()
    assert status_of(lambda: _add(plan, nex=3)) == hx.HX_EINVAL          # not a power of 2
    assert status_of(lambda: _add(plan, p=3)) == hx.HX_EINVAL
    assert status_of(lambda: _add(plan, p=19)) == hx.HX_EINVAL
    bad = np.ones(4 * 4 * 64)
    bad[17] = -1.0
    assert status_of(lambda: _add(plan, c2=bad)) == hx.HX_EINVAL
    bad[17] = np.nan
    assert status_of(lambda: _add(plan, c2=bad)) == hx.HX_EINVAL
    assert status_of(lambda: _add(plan, tau=0.0)) == hx.HX_EINVAL
    assert status_of(lambda: _add(plan, nrhs=0)) == hx.HX_EINVAL
    fit = calibrated_fit(21)
    b = fit.b.copy()
    b[0] += 1e-3                                                        # breaks b_{-m} = conj(b_m)
    assert status_of(lambda: _add(plan, b=b)) == hx.HX_EINVAL
    assert status_of(lambda: _add(plan, alpha=fit.alpha[:-1], b=fit.b[:-1])) == hx.HX_EINVAL
    a = fit.alpha.copy()
    a.real[:] = 0.0                                                     # poles on the axis
    assert status_of(lambda: _add(plan, alpha=a)) == hx.HX_EINVAL
    assert "HX_EINVAL" in hx.hx_last_error()
    plan.close()


def test_add_rejects_unstable_rational_function():
    from workloads.rational import fit_exp
    fit = fit_exp(41, 6.0, 6.0, n_samples=2000)        # |R| reaches 1.09 on the real line
    plan = hx.Plan()
    assert status_of(lambda: _add(plan, fit=fit)) == hx.HX_EUNSTABLE
    plan.close()
    plan = hx.Plan(flags=hx.HX_FLAG_ALLOW_UNSTABLE)
    _add(plan, fit=fit)
    assert plan.query()["max_abs_R"] > 1.05
    plan.close()


def test_query_reports_sizes_and_fit():
    plan = hx.Plan()
    _add(plan, nex=4, ney=2, p=8, nrhs=3)
    info = plan.query()
    q = 6
    assert info["dof_state"] == 2 * 8 * q * q * 3
    assert info["dof_nodes"] == 2 * 8 * 64 * 3
    assert info["folded_poles"] == 11
    assert info["n_instances"] == 1
    assert 2.5 <= info["fit_X"] <= 3.5
    assert info["max_abs_R"] <= 1 + 1e-6
    assert info["operator_bytes"] > 0 and info["arena_bytes"] > info["operator_bytes"]
    assert info["workspace_min_bytes"] <= info["workspace_bytes"]
    # 3 right-hand sides are batched: every stored entry is read once per step
    assert info["op_bytes_per_step"] == pytest.approx(info["operator_bytes"], rel=0.01)
    plan.close()
    plan = hx.Plan(flags=hx.HX_FLAG_UNBATCHED)
    _add(plan, nex=4, ney=2, p=8, nrhs=3)
    info = plan.query()
    assert info["op_bytes_per_step"] == pytest.approx(3 * info["operator_bytes"], rel=0.01)
    plan.close()
    plan = hx.Plan(precision=hx.HX_FP32_REFINE)
    _add(plan, nex=4, ney=2, p=8, nrhs=3)
    info32 = plan.query()
    assert info32["operator_bytes"] * 2 == info["operator_bytes"]
    # two FP32 sweeps per step read as many bytes as one FP64 sweep
    assert info32["op_bytes_per_step"] == pytest.approx(info["op_bytes_per_step"] / 3, rel=0.01)
    plan.close()


def test_stage_order_is_enforced():
    plan = hx.Plan()
    assert status_of(lambda: plan.query()) == hx.HX_ESTAGE              # no instance yet
    _add(plan)
    assert status_of(lambda: hx.hx_plan_build(plan.handle, 256, 1 << 20)) == hx.HX_ESTAGE
    assert status_of(lambda: hx.hx_step(plan.handle, [256], 1)) == hx.HX_ESTAGE
    assert status_of(lambda: hx.hx_plan_bind(plan.handle, 0, 1 << 20)) == hx.HX_EINVAL
    assert status_of(lambda: hx.hx_plan_bind(plan.handle, 256 + 8, 1 << 40)) == hx.HX_EINVAL
    assert status_of(lambda: hx.hx_plan_bind(plan.handle, 256, 16)) == hx.HX_ENOMEM
    plan.close()


def test_shallow_water_add_validation_and_sizes():
    fit = calibrated_fit(21)
    plan = hx.Plan()
    sw = lambda **k: plan.add_sw(k.get("nex", 4), k.get("ney", 2), k.get("p", 8),
                                 k.get("f", 1.0), k.get("gH", 1.0), 0.5, 1e-10, fit.alpha,
                                 fit.b, nrhs=k.get("nrhs", 2))
    assert status_of(lambda: sw(gH=0.0)) == hx.HX_EINVAL
    assert status_of(lambda: sw(gH=-1.0)) == hx.HX_EINVAL
    assert status_of(lambda: sw(f=np.inf)) == hx.HX_EINVAL
    sw(f=0.0)
    info = plan.query()
    q = 6
    assert info["dof_state"] == 3 * 8 * q * q * 2
    assert info["dof_nodes"] == 3 * 8 * 64 * 2
    plan.close()
    plan = hx.Plan(precision=hx.HX_FP32_REFINE)
    sw()
    assert plan.query()["operator_bytes"] * 2 == info["operator_bytes"]
    plan.close()


def test_tile_counts_default_rule():
    plan = hx.Plan()
    a = _add(plan, nex=2, ney=2, p=6, nrhs=1)          # one pass per RHS: no tiles
    b = _add(plan, nex=2, ney=2, p=6, nrhs=3)
    c = _add(plan, nex=2, ney=2, p=6, nrhs=20)
    assert plan.tiles(a) == [0] * hx.HX_STAGES
    assert plan.tiles(b) == [1] * hx.HX_STAGES
    assert plan.tiles(c) == [2] * hx.HX_STAGES
    assert status_of(lambda: plan.tiles(3)) == hx.HX_EINVAL
    # default variants: small elements stage their sources; merges follow
    # the level rule; an unbatched instance reports none
    assert plan.variants(a) == [0] * hx.HX_STAGES
    assert plan.variants(b) == [1, 0, 0, 0, 0]
    assert plan.variants(c) == [1, 0, 0, 0, 0]
    assert status_of(lambda: plan.variants(-1)) == hx.HX_EINVAL
    plan.close()
    assert status_of(lambda: hx.hx_plan_create(hx.HX_FP64, 0, 0x40)) == hx.HX_EINVAL
    hx.hx_plan_destroy(hx.hx_plan_create(hx.HX_FP64, 0, hx.HX_FLAG_AUTOTUNE))
