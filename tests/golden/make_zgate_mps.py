"""Writes zgate_mps.json: the cat-qubit Z gate (paper Sec. 6.2) run by
Oracle-M (the purified-MPS second-order Kraus step on the CPU, tol 1e-8) from
the even cat, in two records:

* "paper_prefix": the paper's scan point, memory 2^8 Fock levels, buffer
  2^4, |alpha|^2 = 256/3, dt <= 2e-4, caps chi 128 / chi_mu 16, for the first
  PREFIX steps of the gate (the whole gate, 10628 steps, takes the oracle
  hours);
* "paper_check": the same scan point over its first CHECK steps (the record
  the CPU tests recompute in seconds);
* "small_whole_gate": memory 2^5, buffer 2^2, |alpha|^2 = 32/3, dt <= 1e-3,
  caps chi 64 / chi_mu 16, over the whole gate (6012 steps).

Each stores the memory's parity, <n_a>, <a>, <n_b>, the trace before the
last renormalisation and the bond profile.  Calls only the oracle and the
workload description (a few minutes):  python tests/golden/make_zgate_mps.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workload as wl          # noqa: E402
from oracle import mps, tt     # noqa: E402

PAPER = dict(Ra=8, Rb=4, dt_max=2e-4, chi=128, chi_mu=16)
PREFIX = 300
CHECK = 12
SMALL = dict(Ra=5, Rb=2, alpha2=32.0 / 3.0, dt_max=1e-3, chi=64, chi_mu=16)


def run(case, n_steps=None):
    m, z = wl.model_cat_zgate(**case)
    n_steps = m.steps if n_steps is None else n_steps
    so = m.site_order()
    K = tt.KrausMPO(m, m.dt)
    X, _ = mps.right_canonicalize(mps.product_state(m.init, m.bits, so), tol=1e-14)

    def op(terms):
        return tt.operator_mpo(terms, m.bits, so)

    t0 = time.time()
    for n in range(n_steps):
        X, info = mps.k2_step(X, K.at(n * m.dt), m.tol, m.chi, m.chi_mu)
        if (n + 1) % 500 == 0:
            print(f"{m.bits}: {n + 1}/{n_steps} steps, {time.time() - t0:.0f} s, bonds {mps.bond_dims(X)}",
                  flush=True)
    ea = mps.expect(X, op([(1.0, {0: ("A_POW", 1)})]))
    out = dict(case)
    out.update({"alpha2": z.alpha2, "gate_steps": m.steps, "steps": n_steps, "dt": m.dt, "t_gate": z.t_gate,
                "tol": m.tol, "parity": mps.expect(X, op(wl.parity_operator(0, m.dims[0]))).real,
                "n_a": mps.expect(X, op([(1.0, {0: ("NUM_POW", 1)})])).real, "a": [ea.real, ea.imag],
                "n_b": mps.expect(X, op([(1.0, {1: ("NUM_POW", 1)})])).real, "tau": info.tau,
                "final_bonds": mps.bond_dims(X),
                "source": "oracle.mps.k2_step (Oracle-M), second-order Kraus scheme, purified MPS"})
    return out


def main():
    out = {"paper_prefix": run(PAPER, PREFIX), "paper_check": run(PAPER, CHECK), "small_whole_gate": run(SMALL)}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "zgate_mps.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
