#!/usr/bin/env python
"""Benchmark of the purified-MPS Kraus step on one MI355X.

Workload (the chi = 128 configuration): cat mode + lossy buffer, two modes of
2^8 Fock levels each (16 quantics sites), H = g2 (a^dag^2 b + a^2 b^dag)
+ eps_d (b + b^dag) with alpha^2 = 8, jumps sqrt(10) b and sqrt(1e-3) a
(9 Kraus operators), bond cap chi = 128, purification cap chi_mu = 16,
tol = 1e-8, dt = 2.5e-5; the state is a seeded synthetic MPS saturated at
the caps (bonds min(2^i, 2^(16-i) 16, 128), Schmidt spectra decaying
geometrically), so every step runs at the full chi = 128 cost.

One step = zip-up application of the stacked Kraus MPO, purification
truncation, right-to-left truncated-SVD sweep and trace renormalisation.
The timed form computes the MPO/MPS contractions in complex64 (FP32 MFMA,
FP32 accumulation) and every Gram matrix, factorisation, truncation weight
and trace in FP64.  A few steps of the plain FP64 form are timed beside it,
and the CPU oracle (NumPy/LAPACK) on a bounded sample of the same workload.

The serving leg runs the seeded parameter-sweep request stream (512
requests: two-photon cat, cat + buffer, driven transmon; Fock sizes 64-4096,
bond caps 32-256, 100 steps each) through the library's continuous-batching
loop (include/lindblad_serve.h): a burst (every request at t = 0) gives
solves/s, a Poisson stream at 0.7 x that rate gives the p50/p99 latency from
arrival to completion; the plain-FP64 one-at-a-time baseline runs on a seeded
subsample (its first --serve-baseline-requests requests) with the same
arrivals.  The host-side Kraus-MPO builds (once per request) are done before
the timed runs and reported separately.

The chi = 256 leg steps the driven transmon + resonator (22 sites, chi_mu =
32) from a seeded state saturated at the caps and checks that the bonds stay
at the cap.  The CPU oracle runs on all host cores and on one core.

Prints one JSON line.  --gpus above 1 is not supported (one GPU).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

# one hardware queue per serving slot (HIP's default of 4 would funnel the
# 16 slots' streams through 4 queues); read when the runtime starts
os.environ.setdefault("GPU_MAX_HW_QUEUES", "16")

# hardware queues for the overlapping solves of the serving leg (HIP reads
# this when it initialises, so it is set before torch is imported): at least
# 16, one per slot (HIP's default is 4, which serialises the slots' streams)
try:
    _hwq = int(os.environ.get("GPU_MAX_HW_QUEUES", "0"))
except ValueError:
    _hwq = 0
os.environ["GPU_MAX_HW_QUEUES"] = str(min(32, max(_hwq, 16)))

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "purified-MPS steps/s at chi=128; batched solves/s + p50/p99 vs plain FP64"
# fully timed steps (an event pair around every launch) run after the warm-up
# for the per-class breakdown; the timed steps carry events around the
# dominant kernel only
PROFILE_STEPS = 3
PEAKS = {  # MI355X published dense peaks
    ("mfma", "f32"): 157.3, ("mfma", "f64"): 78.6, ("alu", "f64"): 78.6, ("alu", "f32"): 157.3,
    ("hbm", None): 8000.0,
}
ALU_CLASSES = {"hetrd", "stebz", "stein", "ormtr", "jacobi"}
# HBM bytes per launch from the rocprofv3 FETCH_SIZE / WRITE_SIZE runs of this
# workload, scaled by a plain 256 MiB copy (profiles/step_catbuffer_chi128_fp32_kernels.md);
# hetrd is per reduction call (all instantiations a call launches, summed
# over the run, divided by the calls; the multi-workgroup form polls its
# mailboxes with agent-scope atomic loads, which go to memory).  A kernel
# absent here reports traffic null
PMC_TRAFFIC_BYTES = {"hetrd": 1.817e6}


def workload():
    import workload as wl
    m = wl.model_cat_buffer(Ra=8, Rb=8, alpha2=8.0, dt=2.5e-5)
    L, chi, chi_mu = 16, 128, 16
    raw = wl.synthetic_mps(L, chi_mu, chi)
    return m, L, chi, chi_mu, raw


def roofline_entry(prof: dict, precision: str) -> dict:
    name = max(prof, key=lambda k: prof[k]["ms"])
    p = prof[name]
    ms_per_launch = p["ms"] / max(p["launches"], 1)
    if name in ALU_CLASSES:
        bound, unit, dt = "alu", "TFLOP/s", "f64"
    else:
        bound, unit = "mfma", "TFLOP/s"
        dt = "f32" if (precision == "fp32" and name == "gemm_contract") else "f64"
    achieved = (p["flop"] / p["launches"]) / (ms_per_launch * 1e-3) / 1e12 if p["ms"] > 0 else 0.0
    peak = PEAKS[(bound, dt)]
    out = {"kernel": name, "bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
           "frac": achieved / peak, "traffic": PMC_TRAFFIC_BYTES.get(name), "avg_launch_us": ms_per_launch * 1e3,
           "launches": p["launches"], "flop_per_launch": p["flop"] / max(p["launches"], 1),
           "dtype": dt}
    if name == "hetrd":
        # CUs a launch occupies: one workgroup per matrix up to order 128,
        # then 16 (orders 129-256) or 32 (257-512) workgroups of one CU each
        out["workgroups_per_launch"] = {"n<=128": 1, "n<=256": 16, "n<=512": 32}
    return out


def contraction_roofline(prof: dict, precision: str) -> dict:
    """MFMA utilisation of the contraction GEMMs (MPO/MPS products and
    carries) and of the Gram GEMMs, the kernels the dense-contraction roofline
    applies to."""
    out = {}
    for name, dt in (("gemm_contract", "f32" if precision == "fp32" else "f64"), ("gemm_gram", "f64"),
                     ("gemm_lead_f64", "f64")):
        p = prof.get(name)
        if not p or not p["ms"]:
            continue
        achieved = p["flop"] / (p["ms"] * 1e-3) / 1e12
        peak = PEAKS[("mfma", dt)]
        out[name] = {"bound": "mfma", "dtype": dt, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "launches": p["launches"]}
    return out


def gpu_run(steps: int, warmup: int, precision: str):
    import torch
    from paper_2605_27515_amd import api
    m, L, chi, chi_mu, raw = workload()
    # autotune: the first step times the split-K count of each GEMM on its
    # operands (include/lindblad.h, lb_config.autotune); it is a warm-up step
    s = api.solver_from_model(m, precision=precision, chi=chi, chi_mu=chi_mu, state="none", device=0,
                              autotune=True)
    s.set_state_mps(raw)
    if warmup:
        s.step(warmup)
    # per-class breakdown from a few fully timed steps outside the timed
    # region (an event pair around every launch costs ~7 % of the step)
    s.profile(True)
    s.step(PROFILE_STEPS)
    breakdown = s.profile_read()
    dominant = max(breakdown, key=lambda k: breakdown[k]["ms"])
    s.profile(False)
    # the timed region: the captured step graph, replayed, no events (the
    # production path; a graph with event nodes would need a host wait per
    # replay to read them)
    s.step(1)
    s.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps, sync=False)
    s.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # the same number of steps again with live HIP events around the dominant
    # kernel class only (direct launches), for its average launch duration
    s.profile(True, classes=[dominant])
    s.step(steps)
    live = s.profile_read()
    s.profile(False)
    d = s.diagnostics()
    s.close()
    return (t1 - t0), breakdown, live, dominant, d


def copy_calibration() -> None:
    """One plain 256 MiB device copy: its counter readings scale the HBM
    counters of the other kernels."""
    import torch
    src = torch.ones(1 << 25, dtype=torch.float64, device="cuda")   # 256 MiB
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def counter_run(steps: int, precision: str) -> None:
    """The step workload's solver (as gpu_run builds it) for a few steps, a line
    after each: a short program for rocprofv3 counter passes, which serialise
    every dispatch."""
    from paper_2605_27515_amd import api
    m, L, chi, chi_mu, raw = workload()
    s = api.solver_from_model(m, precision=precision, chi=chi, chi_mu=chi_mu, state="none", device=0,
                              autotune=True)
    s.set_state_mps(raw)
    print("bench: counter run, state set", file=sys.stderr, flush=True)
    for k in range(steps):
        s.step(1)
        print(f"bench: counter run, step {k + 1} of {steps} done", file=sys.stderr, flush=True)
    s.close()


def build_requests(reqs, precision: str, threads: int = 16):
    """Solvers (generator set, no state) and observables for serving requests;
    the host builds run in parallel threads (the C calls release the GIL)."""
    from concurrent.futures import ThreadPoolExecutor
    import workload as wl
    from paper_2605_27515_amd import api

    def one(r):
        m = wl.model_from_request(r)
        s = api.solver_from_model(m, precision=precision, state="none")
        obs = [s.mpo([(1.0, {0: ("NUM_POW", 1)})]), s.mpo([(1.0, {0: ("A_POW", 1)})])]
        return m, s, obs

    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(one, reqs))


def serve_once(built, slots: int, budget: int, arrivals):
    from paper_2605_27515_amd import api
    sv = api.Server(n_slots=slots, hbm_budget=budget)
    for (m, s, obs), t in zip(built, arrivals):
        sv.submit(s, m.init, m.steps, obs, arrival=float(t))
    # the run blocks in the library (the GIL released); this thread reports
    # each further eighth of the requests as it completes
    import threading
    err = []

    def go():
        try:
            sv.run()
        except Exception as e:   # noqa: BLE001 - re-raised below
            err.append(e)

    th = threading.Thread(target=go)
    th.start()
    step = max(1, len(built) // 8)
    mark = step
    while th.is_alive():
        th.join(timeout=1.0)
        done = sv.stats()["completed"]
        if done >= mark:
            print(f"bench: serving: {done} of {len(built)} requests done", file=sys.stderr, flush=True)
            mark = (done // step + 1) * step
    if err:
        raise err[0]
    res = [sv.result(k) for k in range(len(built))]
    st = sv.stats()
    sv.close()
    bad = [r for r in res if r["status"] != 0]
    if bad:
        raise RuntimeError(f"{len(bad)} serving requests failed (status {bad[0]['status']})")
    return res, st


def serving(n_req: int, slots: int, budget_gb: float, n_base: int) -> dict:
    import numpy as np
    import workload as wl
    reqs = wl.serving_requests(512)[:n_req]
    n_base = min(n_base, n_req)
    t0 = time.perf_counter()
    fast = build_requests(reqs, "fp32")
    plain = build_requests(reqs[:n_base], "fp64")
    build_s = time.perf_counter() - t0
    print(f"bench: serving: {n_req} + {n_base} solvers built on the host in {build_s:.1f} s", file=sys.stderr,
          flush=True)
    budget = int(budget_gb * (1 << 30))
    # burst: every request at t = 0
    res, st = serve_once(fast, slots, budget, [0.0] * n_req)
    burst = n_req / st["makespan"]
    print(f"bench: serving: burst of {n_req} done in {st['makespan']:.1f} s", file=sys.stderr, flush=True)
    # Poisson stream at 0.7 x the burst rate
    rate = 0.7 * burst
    arr = wl.poisson_arrivals(n_req, rate)
    res_p, st_p = serve_once(fast, slots, budget, arr)
    lat = np.array([r["done"] - r["arrival"] for r in res_p])
    print(f"bench: serving: Poisson stream done in {st_p['makespan']:.1f} s", file=sys.stderr, flush=True)
    # the baseline subsample one at a time in plain FP64, same arrivals
    res_b, st_b = serve_once(plain, 1, 0, arr[:n_base])
    lat_b = np.array([r["done"] - r["arrival"] for r in res_b])
    print(f"bench: serving: FP64 one-at-a-time baseline done in {st_b['makespan']:.1f} s", file=sys.stderr,
          flush=True)
    svc_b = np.array([r["done"] - r["admitted"] for r in res_b])
    # observables of the two forms (FP32 contractions vs plain FP64)
    dev = max(abs(a - b) / max(1.0, abs(b)) for r1, r2 in zip(res_p[:n_base], res_b)
              for a, b in zip(r1["observables"], r2["observables"]))
    svc_f = np.array([r["done"] - r["admitted"] for r in res_p])
    for _, s, _ in fast + plain:
        s.close()
    fam = {}
    for r in reqs:
        fam[r["family"]] = fam.get(r["family"], 0) + 1
    return {
        "requests": n_req, "families": fam, "steps_per_request": reqs[0]["steps"], "slots": slots,
        "hbm_budget_gb": budget_gb, "host_build_s": build_s,
        "burst_solves_per_s": burst, "burst_peak_running": st["peak_running"],
        "burst_peak_gb": st["peak_bytes"] / (1 << 30),
        "poisson_rate_per_s": rate, "poisson_solves_per_s": n_req / st_p["makespan"],
        "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
        "service_p50_s": float(np.percentile(svc_f, 50)), "service_p99_s": float(np.percentile(svc_f, 99)),
        "baseline_fp64_one_at_a_time": {
            "requests": n_base, "sample": f"the first {n_base} requests of the stream, same arrival times",
            "solves_per_s": n_base / st_b["makespan"],
            "p50_s": float(np.percentile(lat_b, 50)), "p99_s": float(np.percentile(lat_b, 99)),
            "service_p50_s": float(np.percentile(svc_b, 50)), "service_p99_s": float(np.percentile(svc_b, 99))},
        "solves_per_s_vs_baseline": burst / (n_base / st_b["makespan"]),
        "max_rel_observable_diff_fp32_vs_fp64": dev,
    }


def cpu_baseline(budget_s: float, one_core: bool = False) -> dict:
    """The oracle as it stands, on the same workload, for a bounded sample;
    on the host's BLAS threads, or on one core (BLAS limited to one thread)."""
    import contextlib
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import mps, tt
    m, L, chi, chi_mu, raw = workload()
    ctx = threadpool_limits(limits=1) if one_core else contextlib.nullcontext()
    with ctx:
        K = tt.KrausMPO(m, m.dt)
        X, _ = mps.right_canonicalize(raw, tol=1e-14)
        X, _ = mps.k2_step(X, K.at(0.0), m.tol, chi, chi_mu)       # warm-up step
        n = 0
        t0 = time.perf_counter()
        while True:
            X, _ = mps.k2_step(X, K.at(n * m.dt), m.tol, chi, chi_mu)
            n += 1
            if time.perf_counter() - t0 > budget_s or n >= 50:
                break
        dt = time.perf_counter() - t0
        threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    return {"value": n / dt, "unit": "steps/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{n} steps of the same chi=128 cat+buffer workload (oracle NumPy/LAPACK FP64, "
                      f"{dt:.1f} s), after one warm-up step", "host_cpus": os.cpu_count()}


def trajectory_leg(steps: int, precision: str) -> dict:
    """The chi = 128 configuration from vacuum x vacuum for a short stretch:
    the small-bond regime, where a step is bound by its launches, not by
    flops (launch tiers follow the bonds)."""
    import torch
    import workload as wl
    from paper_2605_27515_amd import api
    m = wl.model_cat_buffer(Ra=8, Rb=8, alpha2=8.0, dt=2.5e-5)
    s = api.solver_from_model(m, precision=precision, chi=128, chi_mu=16, device=0)
    s.step(32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    d = s.diagnostics()
    s.close()
    return {"workload": "cat+buffer 2x256 Fock (16 sites), chi=128, chi_mu=16, tol=1e-8, dt=2.5e-5, "
                        "vacuum x vacuum start, after 32 steps", "precision": precision, "steps": steps,
            "steps_per_s": steps / el, "ms_per_step": 1e3 * el / steps, "max_bond": max(d["bonds"]),
            "chi_mu": d["chi_mu"], "tier": d["tier"]}


def chi256_leg(steps: int, precision: str) -> dict:
    """Driven transmon + resonator (charge states -512..511, resonator 4096
    levels, 22 sites), chi = 256, chi_mu = 32, from a seeded state saturated
    at the caps: steps/s, and whether the bonds stay at the cap."""
    import torch
    import workload as wl
    from paper_2605_27515_amd import api
    m = wl.model_transmon_resonator()
    L, chi, chi_mu = 22, 256, 32
    raw = wl.synthetic_mps(L, chi_mu, chi)
    s = api.solver_from_model(m, precision=precision, chi=chi, chi_mu=chi_mu, state="none", device=0,
                              autotune=True)
    s.set_state_mps(raw)
    s.step(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    d = s.diagnostics()
    s.close()
    cap = wl.saturated_bonds(L, chi_mu, chi)[1:-1]
    return {"workload": "driven transmon + resonator, 2^10 charges x 2^12 Fock (22 sites), chi=256, chi_mu=32, "
                        "tol=1e-8, dt=1.5e-7, seeded saturated MPS", "precision": precision,
            "steps": steps, "steps_per_s": steps / el, "ms_per_step": 1e3 * el / steps,
            "bonds": d["bonds"], "cap_bonds": cap, "bonds_at_cap": d["bonds"] == cap, "chi_mu": d["chi_mu"]}


def kerr_rk4_leg(n_run: int, dt: float, warmup: int) -> dict:
    """Pure-state global RK4 (paper Sec. 3.1.1) on the driven Kerr oscillator
    at the paper's parameters (Sec. 3.2: R = 8, w0 = 1, K = 1/25, alpha0 = 4,
    the two-frequency drive, tol 1e-8): steps/s of both forms and their
    distance to the dense scheme (computed after the timed region)."""
    import numpy as np
    import torch
    import workload as wl
    from oracle import dense, mps
    from paper_2605_27515_amd import api
    m = wl.model_driven_kerr(R=8, dt=dt)
    dm = dense.DenseModel(m)
    ref = dense.rk4_pure_evolve(dm, dm.psi0, m.dt, n_run)
    rr = np.outer(ref, ref.conj())
    aop = np.diag(np.sqrt(np.arange(1, 256)), 1)
    a_ref = np.vdot(ref, aop @ ref)
    out = {}
    for prec in ("fp32", "fp64"):
        s = api.solver_from_model(m, precision=prec, order=4, chi=64, chi_mu=1, device=0)
        if warmup:
            s.step(warmup)
            s.close()
            s = api.solver_from_model(m, precision=prec, order=4, chi=64, chi_mu=1, device=0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(n_run)
        s.sync()
        elapsed = time.perf_counter() - t0
        X = s.get_state_mps()
        a = s.observe(s.mpo([(1.0, {0: ("A_POW", 1)})]))
        bonds = s.diagnostics()["bonds"]
        s.close()
        psi = mps.to_dense(X, m.bits, m.site_order())[:, 0]
        err = float(np.abs(np.outer(psi, psi.conj()) - rr).max() / np.abs(rr).max())
        out[prec] = {"steps_per_s": n_run / elapsed, "rho_max_rel_error_vs_dense": err,
                     "a_abs_error_vs_dense": float(abs(a - a_ref)), "bonds": bonds}
        print(f"bench: kerr RK4 {prec}: {n_run / elapsed:.1f} steps/s, rho error {err:.2e}, bonds {bonds}",
              file=sys.stderr, flush=True)
    out["steps"] = n_run
    out["dt"] = dt
    out["a_dense"] = [a_ref.real, a_ref.imag]
    return out


def kerr_rk4_main(args) -> None:
    out = kerr_rk4_leg(args.kerr_steps, args.kerr_dt, args.warmup)
    n_run = args.kerr_steps
    forms = {k: out[k] for k in ("fp32", "fp64")}
    line = {"metric": "pure-state global RK4 steps/s, driven Kerr oscillator", "value": out[args.precision]["steps_per_s"],
            "unit": "steps/s", "n_gpus": 1, "steps": n_run, "warmup": args.warmup,
            "ms_per_step": 1e3 / out[args.precision]["steps_per_s"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32+f64" if args.precision == "fp32" else "f64", "data": "synthetic",
            "config": {"workload": f"driven Kerr oscillator, 2^8 Fock levels (8 sites), K=1/25, alpha0=4, "
                                   f"two-frequency drive, dt={args.kerr_dt}, tol=1e-8, chi=64", "precision": args.precision},
            "forms": forms, "a_dense": out["a_dense"]}
    print(json.dumps(line), flush=True)


def kerr_tdvp_leg(n_run: int, dt: float, warmup: int, cpu_seconds: float | None) -> dict:
    """One-site TDVP with the fourth-order Magnus Hamiltonian (order 5, paper
    Sec. 3.1.3) on the driven Kerr oscillator at the paper's parameters (Sec.
    3.2: R = 8, w0 = 1, K = 1/25, alpha0 = 4, the two-frequency drive), FP64,
    from the coherent state as the library compresses it: steps/s, the bonds
    the state keeps, and its distance to the dense Magnus-4 steps (the exact
    propagator up to O(h^5) per step; the rest is TDVP's projection),
    computed after the timed region; with cpu_seconds, the oracle's TDVP
    timed on a few steps."""
    import numpy as np
    import torch
    import workload as wl
    from oracle import dense, mps, tdvp, tt
    from paper_2605_27515_amd import api
    m = wl.model_driven_kerr(R=8, dt=dt)
    s = api.solver_from_model(m, order=5, chi=64, chi_mu=1, device=0)
    if warmup:
        s.step(warmup)
        s.close()
        s = api.solver_from_model(m, order=5, chi=64, chi_mu=1, device=0)
    bonds0 = s.diagnostics()["bonds"]
    print(f"bench: kerr TDVP, {n_run} steps of dt={m.dt}, bonds {bonds0}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(n_run)
    s.sync()
    elapsed = time.perf_counter() - t0
    X = s.get_state_mps()
    a = s.observe(s.mpo([(1.0, {0: ("A_POW", 1)})]))
    s.close()
    psi = mps.to_dense(X, m.bits, m.site_order())[:, 0]
    dm = dense.DenseModel(m)
    ref = tdvp.magnus4_dense_evolve(dm.H0, dm.H1, dm.f, dm.psi0, m.dt, n_run)
    err = float(np.linalg.norm(psi - ref))
    aop = np.diag(np.sqrt(np.arange(1, 256)), 1)
    a_ref = np.vdot(ref, aop @ ref)
    print(f"bench: kerr TDVP fp64: {n_run / elapsed:.1f} steps/s, state error {err:.2e}, "
          f"|<a> - dense| {abs(a - a_ref):.2e}", file=sys.stderr, flush=True)
    cpu = None
    if cpu_seconds:
        # the oracle's TDVP from its own compression of the same start, a few steps
        so = m.site_order()
        X0 = tdvp.right_orthonormal(mps.product_state(m.init, m.bits, so, tol=1e-14))
        H0m, H1m = tt.operator_mpo(m.H0, m.bits, so), tt.operator_mpo(m.H1, m.bits, so)
        n_cpu, t_cpu = 0, 0.0
        while t_cpu < cpu_seconds and n_cpu < n_run:
            c0 = time.perf_counter()
            X0 = tdvp.magnus4_tdvp_evolve(X0, H0m, H1m, dm.f, m.dt, 1, t0=n_cpu * m.dt)
            t_cpu += time.perf_counter() - c0
            n_cpu += 1
        cpu = {"value": n_cpu / t_cpu, "unit": "steps/s", "cores": torch.get_num_threads(), "kind": "oracle",
               "sample": f"the first {n_cpu} steps of the same run (oracle.tdvp, dense local exponentials)"}
    return {"steps_per_s": n_run / elapsed, "ms_per_step": 1e3 * elapsed / n_run, "steps": n_run, "dt": dt,
            "bonds": bonds0, "state_error_vs_dense_magnus4": err,
            "a_abs_error_vs_dense_magnus4": float(abs(a - a_ref)), "cpu_baseline": cpu}


def kerr_tdvp_main(args) -> None:
    out = kerr_tdvp_leg(args.kerr_steps, args.kerr_dt, args.warmup, None if args.no_cpu else args.cpu_seconds)
    line = {"metric": "Magnus-4 one-site TDVP steps/s, driven Kerr oscillator", "value": out["steps_per_s"],
            "unit": "steps/s", "n_gpus": 1, "steps": out["steps"], "warmup": args.warmup,
            "ms_per_step": out["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"driven Kerr oscillator, 2^8 Fock levels (8 sites), K=1/25, alpha0=4, "
                                   f"two-frequency drive, dt={out['dt']}, coherent start compressed at 1e-14, chi=64"},
            "bonds": out["bonds"], "state_error_vs_dense_magnus4": out["state_error_vs_dense_magnus4"],
            "a_abs_error_vs_dense_magnus4": out["a_abs_error_vs_dense_magnus4"], "cpu_baseline": out["cpu_baseline"]}
    print(json.dumps(line), flush=True)


def zgate_main(args) -> None:
    """Cat-qubit Z gate at the paper's scan point N_a = 2^8, N_b = 2^4,
    |alpha|^2 = N_a / 3 (paper Sec. 6.2): the whole gate, timed, and its
    phase-flip probability against the leading-order law pi / (40 |alpha|^3)."""
    import math
    import torch
    import workload as wl
    from paper_2605_27515_amd import api
    m, z = wl.model_cat_zgate(Ra=8, Rb=4, dt_max=args.zgate_dt, chi=args.zgate_chi, chi_mu=16)
    print(f"bench: cat Z gate, {m.steps} steps of dt={m.dt:.3e}, {args.precision}; building the Kraus MPO",
          file=sys.stderr, flush=True)
    floor = args.zgate_fp32_floor if args.precision == "fp32" else 0.0
    w = api.solver_from_model(m, precision=args.precision, device=0, fp32_tol_floor=floor)
    if args.warmup:
        w.step(args.warmup)
    w.close()
    s = api.solver_from_model(m, precision=args.precision, device=0, fp32_tol_floor=floor)
    parity = s.mpo(wl.parity_operator(0, m.dims[0]))
    n_run = m.steps if args.zgate_steps <= 0 else min(args.zgate_steps, m.steps)
    chunk = 250
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < n_run:
        n = min(chunk, n_run - done)
        s.step(n)
        done += n
        torch.cuda.synchronize()
        print(f"bench: {done}/{n_run} steps, {time.perf_counter() - t0:.1f} s, bonds {s.diagnostics()['bonds']}",
              file=sys.stderr, flush=True)
    elapsed = time.perf_counter() - t0
    p = s.observe(parity).real
    tr, pur = s.trace_purity()
    diag = s.diagnostics()
    # per-class breakdown from a few fully timed steps past the timed run, at
    # the bond dimensions the gate reached
    s.profile(True)
    s.step(PROFILE_STEPS)
    prof = s.profile_read()
    s.profile(False)
    s.close()
    whole = n_run == m.steps
    p_z = 0.5 * (1.0 + p) if whole else None
    law = math.pi / (40.0 * z.alpha2 ** 1.5)
    cpu = None
    if not args.no_cpu:
        from threadpoolctl import threadpool_info
        from oracle import mps, tt
        K = tt.KrausMPO(m, m.dt)
        X, _ = mps.right_canonicalize(mps.product_state(m.init, m.bits, m.site_order()), tol=1e-14)
        n = 0
        c0 = time.perf_counter()
        while time.perf_counter() - c0 < args.cpu_seconds and n < n_run:
            X, _ = mps.k2_step(X, K.at(n * m.dt), m.tol, m.chi, m.chi_mu)
            n += 1
        cdt = time.perf_counter() - c0
        threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
        cpu = {"value": n / cdt, "unit": "steps/s", "cores": int(threads), "kind": "oracle",
               "sample": f"the first {n} steps of the same gate from the even cat (oracle NumPy/LAPACK FP64, "
                         f"{cdt:.1f} s)", "host_cpus": os.cpu_count()}
    total_ms = sum(v["ms"] for v in prof.values())
    line = {
        "metric": "cat Z gate: purified-MPS steps/s over the whole gate; phase-flip probability",
        "value": n_run / elapsed, "unit": "steps/s", "n_gpus": 1, "steps": n_run, "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / n_run, "whole_gate": whole, "gate_steps": m.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64" if args.precision == "fp32" else "f64", "data": "synthetic",
        "config": {"workload": f"cat Z gate: memory 2^8 Fock, buffer 2^4 (12 sites), |alpha|^2={z.alpha2:.3f}, "
                               f"g2=1, kappa_b=10, eps_Z={z.eps_z}, theta=pi, T_Z={z.t_gate:.4f}, dt={m.dt:.4e}, "
                               f"4 Kraus ops, chi cap {m.chi}, chi_mu cap {m.chi_mu}, tol {m.tol}, even-cat start",
                   "precision": args.precision, "parallelism": "single solve, one GPU",
                   "fp32_tol_floor": floor},
        "gate_seconds": elapsed,
        "p_z": p_z, "p_z_law": law, "p_z_over_law": p_z / law if whole else None, "final_parity": p,
        "trace": tr, "purity": pur, "final_bonds": diag["bonds"], "final_chi_mu": diag["chi_mu"],
        "roofline_profiled_steps": roofline_entry(prof, args.precision) if total_ms else None,
        "profiled_steps_note": f"{PROFILE_STEPS} fully timed steps after the timed run",
        "kernel_ms_per_step": {k: v["ms"] / PROFILE_STEPS for k, v in prof.items() if v["launches"]},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def trajectory_main(args) -> None:
    """The chi = 128 configuration run as physics: cat + buffer from vacuum x
    vacuum, the same operators, caps and dt as the step benchmark, for
    --trajectory-steps steps; bond profile, chi_mu and <n_a> every 500 steps."""
    import torch
    import workload as wl
    from paper_2605_27515_amd import api
    m = wl.model_cat_buffer(Ra=8, Rb=8, alpha2=8.0, dt=2.5e-5)
    n_steps = args.trajectory_steps
    print(f"bench: cat+buffer trajectory from vacuum, {n_steps} steps, {args.precision}", file=sys.stderr, flush=True)
    s = api.solver_from_model(m, precision=args.precision, chi=128, chi_mu=16, device=0)
    na = s.mpo([(1.0, {0: ("NUM_POW", 1)})])
    history = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < n_steps:
        n = min(500, n_steps - done)
        s.step(n)
        done += n
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        d = s.diagnostics()
        history.append({"steps": done, "t": done * m.dt, "elapsed_s": el, "bonds": d["bonds"], "chi_mu": d["chi_mu"]})
        print(f"bench: {done}/{n_steps} steps, {el:.1f} s, bonds {d['bonds']}, chi_mu {d['chi_mu']}",
              file=sys.stderr, flush=True)
    elapsed = time.perf_counter() - t0
    n_a = s.observe(na).real
    tr, pur = s.trace_purity()
    s.close()
    line = {
        "metric": "purified-MPS steps/s of the physical chi=128 trajectory (vacuum start)",
        "value": n_steps / elapsed, "unit": "steps/s", "n_gpus": 1, "steps": n_steps, "warmup": 0,
        "ms_per_step": 1e3 * elapsed / n_steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "fp32" else "f64", "data": "synthetic",
        "config": {"workload": "cat+buffer 2x256 Fock (16 sites), alpha^2=8, 9 Kraus ops, chi=128, chi_mu=16, "
                               "tol=1e-8, dt=2.5e-5, vacuum x vacuum start",
                   "precision": args.precision, "parallelism": "single solve, one GPU"},
        "final_n_a": n_a, "trace": tr, "purity": pur, "history": history,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--fp64-steps", type=int, default=3, help="steps of the plain FP64 form timed beside")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--serve-requests", type=int, default=256,
                    help="requests of the seeded serving stream (its first N of 512; 512 runs the whole "
                         "stream, ~7 min; 0: skip the serving leg)")
    ap.add_argument("--serve-baseline-requests", type=int, default=64,
                    help="requests of the plain-FP64 one-at-a-time baseline (the stream's first ones)")
    ap.add_argument("--chi256-steps", type=int, default=3, help="steps of the chi=256 leg (0: skip)")
    ap.add_argument("--trajectory-leg-steps", type=int, default=960,
                    help="steps of the small-bond trajectory leg (0: skip)")
    ap.add_argument("--serve-slots", type=int, default=16)
    ap.add_argument("--serve-budget-gb", type=float, default=8.0)
    ap.add_argument("--kerr-steps", type=int, default=1000, help="steps of the kerr-rk4 and kerr-tdvp workloads")
    ap.add_argument("--pure-steps", type=int, default=200,
                    help="steps of the pure-state legs (RK4 and Magnus-4 TDVP on the Kerr oscillator) of the "
                         "default run (0: skip)")
    ap.add_argument("--kerr-dt", type=float, default=1e-3, help="time step of the kerr-rk4 and kerr-tdvp workloads")
    ap.add_argument("--workload", choices=["chi128", "cat-zgate", "chi128-trajectory", "kerr-rk4", "kerr-tdvp"],
                    default="chi128",
                    help="chi128: the step benchmark (default); cat-zgate: the whole cat-qubit Z gate; "
                         "chi128-trajectory: the same configuration run as physics from vacuum; "
                         "kerr-rk4: the pure-state RK4 on the driven Kerr oscillator; "
                         "kerr-tdvp: the Magnus-4 one-site TDVP on the same oscillator")
    ap.add_argument("--trajectory-steps", type=int, default=5000)
    ap.add_argument("--zgate-dt", type=float, default=2e-4, help="largest time step of the Z-gate run")
    ap.add_argument("--zgate-chi", type=int, default=128, help="bond cap of the Z-gate run")
    ap.add_argument("--zgate-fp32-floor", type=float, default=1e-7,
                    help="FP32 form of the Z-gate run: floor of the back-sweep and purification tolerance "
                         "(lb_config.fp32_tol_floor; 0: the paper's tol 1e-8, whose cuts keep the complex64 "
                         "noise of the 10628 steps until it fills the caps)")
    ap.add_argument("--zgate-steps", type=int, default=0,
                    help="time only the first N steps of the gate (0: the whole gate, with its phase-flip probability)")
    ap.add_argument("--counter-run", type=int, default=0,
                    help="only take N steps of the step workload, a line after each, and exit (for rocprofv3 "
                         "counter passes)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 256 MiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (the method's step is a "
              "sequential sweep per solve; independent solves shard across GPUs without communication)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.counter_run > 0:
        if args.copy_calibration:
            copy_calibration()
        counter_run(args.counter_run, args.precision)
        return
    if args.workload == "cat-zgate":
        zgate_main(args)
        return
    if args.workload == "chi128-trajectory":
        trajectory_main(args)
        return
    if args.workload == "kerr-rk4":
        kerr_rk4_main(args)
        return
    if args.workload == "kerr-tdvp":
        kerr_tdvp_main(args)
        return
    print(f"bench: {args.precision} steps={args.steps} warmup={args.warmup}", file=sys.stderr, flush=True)
    if args.copy_calibration:
        copy_calibration()
    elapsed, prof, live, dominant, diag = gpu_run(args.steps, args.warmup, args.precision)
    value = args.steps / elapsed
    print(f"bench: {value:.3f} steps/s, bonds {diag['bonds']}, chi_mu {diag['chi_mu']}",
          file=sys.stderr, flush=True)
    fp64 = None
    if args.fp64_steps > 0 and args.precision != "fp64":
        e64 = gpu_run(args.fp64_steps, 1, "fp64")[0]
        fp64 = args.fp64_steps / e64
        print(f"bench: plain fp64 {fp64:.3f} steps/s", file=sys.stderr, flush=True)
    traj = None
    if args.trajectory_leg_steps > 0:
        traj = trajectory_leg(args.trajectory_leg_steps, args.precision)
        print(f"bench: trajectory from vacuum {traj['steps_per_s']:.1f} steps/s (max bond {traj['max_bond']})",
              file=sys.stderr, flush=True)
    c256 = None
    if args.chi256_steps > 0:
        c256 = chi256_leg(args.chi256_steps, args.precision)
        print(f"bench: chi=256 {c256['steps_per_s']:.3f} steps/s, bonds at cap {c256['bonds_at_cap']}",
              file=sys.stderr, flush=True)
    serve = None
    if args.serve_requests > 0:
        serve = serving(args.serve_requests, args.serve_slots, args.serve_budget_gb, args.serve_baseline_requests)
        print(f"bench: serving {serve['burst_solves_per_s']:.2f} solves/s (burst), p50 {serve['p50_s']:.3f} s "
              f"p99 {serve['p99_s']:.3f} s; one-at-a-time FP64 "
              f"{serve['baseline_fp64_one_at_a_time']['solves_per_s']:.2f} solves/s", file=sys.stderr, flush=True)
    pure = None
    if args.pure_steps > 0:
        # the pure-state integrators on the paper's Kerr oscillator; a failure
        # here is reported in the line and does not cost the headline
        pure = {}
        for name, fn in (("kerr_rk4", lambda: kerr_rk4_leg(args.pure_steps, args.kerr_dt, 5)),
                         ("kerr_tdvp", lambda: kerr_tdvp_leg(args.pure_steps, args.kerr_dt, 5, None))):
            try:
                pure[name] = fn()
            except Exception as e:   # noqa: BLE001 - recorded, not hidden
                pure[name] = {"error": f"{type(e).__name__}: {e}"}
                print(f"bench: {name} leg failed: {e}", file=sys.stderr, flush=True)
    cpu = cpu1 = None
    if not args.no_cpu:
        cpu = cpu_baseline(args.cpu_seconds)
        print(f"bench: cpu oracle {cpu['value']:.4f} steps/s on {cpu['cores']} threads", file=sys.stderr,
              flush=True)
        cpu1 = cpu_baseline(args.cpu_seconds, one_core=True)
        print(f"bench: cpu oracle {cpu1['value']:.4f} steps/s on one core", file=sys.stderr, flush=True)
    total_ms = sum(p["ms"] for p in prof.values())
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": "cat+buffer 2x256 Fock (16 sites), alpha^2=8, 9 Kraus ops, chi=128, "
                               "chi_mu=16, tol=1e-8, dt=2.5e-5, seeded saturated MPS",
                   "precision": args.precision, "parallelism": "single solve, one GPU",
                   "gemm_splits": "autotuned on the warm-up step"},
        "roofline": dict(roofline_entry({dominant: live[dominant]}, args.precision),
                         timing="HIP events on the solver's stream around every launch of the class, over a "
                                "second pass of the timed steps (direct launches); the timed pass replays the "
                                "captured step graph without events"),
        "roofline_contractions": contraction_roofline(prof, args.precision),
        "cpu_baseline": cpu,
        "cpu_baseline_one_core": cpu1,
        "fp64_plain_steps_per_s": fp64,
        "chi256": c256,
        "trajectory": traj,
        "kernel_ms_per_step": {k: v["ms"] / PROFILE_STEPS for k, v in prof.items() if v["launches"]},
        "kernel_share": {k: v["ms"] / total_ms for k, v in prof.items() if v["launches"]} if total_ms else {},
        "final_bonds": diag["bonds"],
        "serving": serve,
        "pure_state": pure,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
