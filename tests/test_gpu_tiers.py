"""Launch tiers (lb_config.fixed_bounds = 0, the default): while the bonds
are far below the caps a step runs with every launch bounded by a power of
two above the largest bond, and a step whose truncation that bound capped is
undone and run again under a larger tier.  The results must be those of
steps bounded by the caps (fixed_bounds = 1) up to rounding."""
import numpy as np
import pytest

import workload as wl

pytestmark = pytest.mark.gpu

# observables agree to this relative error: FP64 rounding differs only where a
# kernel picks its variant from the launch bound; the FP32 form carries its
# complex64 increment rounding (about 1e-7 per step) into that choice as well
RTOL = {"fp64": 1e-9, "fp32": 2e-5}


def _api():
    from paper_2605_27515_amd import api
    return api


def _observables(s):
    out = [s.observe(s.mpo([(1.0, {0: ("NUM_POW", 1)})])),
           s.observe(s.mpo([(1.0, {1: ("NUM_POW", 1)})])),
           s.observe(s.mpo([(1.0, {0: ("A_POW", 1)})]))]
    tr, pur = s.trace_purity()
    return np.array(out + [tr, pur], np.complex128)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_tiered_trajectory_matches_fixed_bounds(precision):
    """From a product state the bonds grow from 1: the first steps run under
    small tiers; every block of steps ends in the same state either way."""
    api = _api()
    m = wl.model_cat_buffer(Ra=5, Rb=4, alpha2=4.0, dt=2.5e-5)
    print(f"tiers vs fixed bounds, cat-buffer 2^5 x 2^4, chi 64, {precision}", flush=True)
    a = api.solver_from_model(m, precision=precision, chi=64, chi_mu=8)
    b = api.solver_from_model(m, precision=precision, chi=64, chi_mu=8, fixed_bounds=True)
    tiers = set()
    for blk in range(6):
        a.step(8)
        b.step(8)
        da, db = a.diagnostics(), b.diagnostics()
        tiers.add(da["tier"])
        assert db["tier"] == 0 and db["bound_redos"] == 0
        oa, ob = _observables(a), _observables(b)
        err = np.max(np.abs(oa - ob) / np.maximum(np.abs(ob), 1e-3))
        print(f"  block {blk}: tier {da['tier']} redos {da['bound_redos']} bonds {da['bonds']} "
              f"err {err:.2e}", flush=True)
        assert err < RTOL[precision], (blk, oa, ob)
        if precision == "fp64":
            assert da["bonds"] == db["bonds"]
            assert da["chi_mu"] == db["chi_mu"]
    assert any(t > 0 for t in tiers), tiers
    a.close()
    b.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_tier_overflow_is_undone(precision):
    """A random bond-8 state on 12 sites at a tight tolerance: its first step
    starts under tier 16 and keeps more than 16 values at some bond, so it is
    undone and run again; the result is that of the caps."""
    api = _api()
    m = wl.model_cat_buffer(Ra=6, Rb=6, alpha2=4.0, dt=2.5e-5)
    L = sum(m.bits)
    sites = wl.synthetic_mps(L, 4, 8, decay=1.0, seed=11)
    print(f"tier overflow, cat-buffer 2^6 x 2^6, random bond-8 state, {precision}", flush=True)
    kw = dict(precision=precision, chi=64, chi_mu=4, tol=1e-10, state="none")
    a = api.solver_from_model(m, **kw)
    b = api.solver_from_model(m, fixed_bounds=True, **kw)
    a.set_state_mps(sites)
    b.set_state_mps(sites)
    a.step(2)
    b.step(2)
    da, db = a.diagnostics(), b.diagnostics()
    print(f"  tier {da['tier']} redos {da['bound_redos']} bonds {da['bonds']} vs {db['bonds']}", flush=True)
    assert da["bound_redos"] >= 1
    assert max(db["bonds"]) > 16
    oa, ob = _observables(a), _observables(b)
    err = np.max(np.abs(oa - ob) / np.maximum(np.abs(ob), 1e-3))
    assert err < RTOL[precision], (oa, ob)
    if precision == "fp64":
        assert da["bonds"] == db["bonds"]
    # a batch step runs at the caps and continues the same trajectory
    api.step_batch([a], 1)
    b.step(1)
    assert a.diagnostics()["tier"] == 0
    oa, ob = _observables(a), _observables(b)
    assert np.max(np.abs(oa - ob) / np.maximum(np.abs(ob), 1e-3)) < RTOL[precision]
    a.close()
    b.close()
