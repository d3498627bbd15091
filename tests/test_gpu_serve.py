"""GPU tests of the request loop (include/lindblad_serve.h): every result is
the same alone and in the mix, admission respects slots and the memory
budget, and a served solve equals the same solve stepped directly."""
import numpy as np
import pytest

import workload as wl

pytestmark = pytest.mark.gpu


def _models():
    return [wl.model_coherent_loss(),
            wl.model_two_photon_cat(R=5, alpha2=2.0, dt=1e-3),
            wl.model_cat_buffer(Ra=4, Rb=3, alpha2=2.0, dt=1e-3),
            wl.model_transmon_resonator(Rt=4, Rr=3, eps=2.0, dt=2e-4),
            wl.model_two_photon_cat(R=6, alpha2=4.0, dt=1e-4),
            wl.model_cat_buffer(Ra=3, Rb=3, alpha2=3.0, dt=1e-3)]


def _obs_terms(m):
    t = [[(1.0, {0: ("NUM_POW", 1)})], [(1.0, {0: ("A_POW", 1)})]]
    if m.n_modes > 1:
        t.append([(1.0, {1: ("A_POW", 1)})])
    return t


def _requests(api, precision):
    out = []
    for m in _models():
        s = api.solver_from_model(m, precision=precision, chi=16, chi_mu=8, state="none")
        obs = [s.mpo(t) for t in _obs_terms(m)]
        out.append((m, s, obs))
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_same_alone_and_in_the_mix(precision):
    from paper_2605_27515_amd import api
    reqs = _requests(api, precision)
    steps = 25
    print(f"serve alone/mix {precision}", flush=True)
    # alone: one slot, requests one after another
    alone = api.Server(n_slots=1)
    for m, s, obs in reqs:
        alone.submit(s, m.init, steps, obs)
    alone.run()
    ref = [alone.result(i) for i in range(len(reqs))]
    assert all(r["status"] == 0 for r in ref)
    # in the mix: 4 slots, staggered arrivals, a budget that holds ~3 solves
    fp = [s.footprint() for _, s, _ in reqs]
    budget = sum(sorted(fp)[-3:])
    mix = api.Server(n_slots=4, hbm_budget=budget)
    for k, (m, s, obs) in enumerate(reqs):
        mix.submit(s, m.init, steps, obs, arrival=0.002 * k)
    mix.run()
    st = mix.stats()
    assert st["completed"] == len(reqs)
    assert st["peak_running"] <= 4
    assert st["peak_bytes"] <= budget
    assert st["peak_running"] >= 2          # solves did overlap
    for k in range(len(reqs)):
        r = mix.result(k)
        assert r["status"] == 0
        assert r["admitted"] >= r["arrival"] - 1e-6
        assert r["done"] >= r["admitted"]
        for a, b in zip(r["observables"], ref[k]["observables"]):
            assert abs(a - b) <= 1e-12 * max(1.0, abs(b)), (k, a, b)
    # a served solve equals the same solve stepped directly
    m, _, _ = reqs[2]
    d = api.solver_from_model(m, precision=precision, chi=16, chi_mu=8)
    d.step(steps)
    for t, v in zip(_obs_terms(m), ref[2]["observables"]):
        assert abs(d.observe(d.mpo(t)) - v) <= 1e-12 * max(1.0, abs(v))
    d.close()
    for _, s, _ in reqs:
        s.close()
    alone.close()
    mix.close()


def test_oversized_request_runs_alone():
    """A request larger than the whole budget is admitted only when nothing
    else runs (it cannot wait for memory that will never be free)."""
    from paper_2605_27515_amd import api
    reqs = _requests(api, "fp64")[:3]
    sv = api.Server(n_slots=3, hbm_budget=1)
    for m, s, obs in reqs:
        sv.submit(s, m.init, 5, obs)
    sv.run()
    st = sv.stats()
    assert st["completed"] == 3 and st["peak_running"] == 1
    for k in range(3):
        assert sv.result(k)["status"] == 0
    for _, s, _ in reqs:
        s.close()
    sv.close()
