"""Writes zgate_mps.json: the cat-qubit Z gate (paper Sec. 6.2) at the paper's
scan point memory 2^8 Fock levels, buffer 2^4, |alpha|^2 = 256/3, theta = pi,
dt <= 2e-4, run by Oracle-M (the purified-MPS second-order Kraus step on the
CPU, tol 1e-8, caps chi 128 / chi_mu 16) from the even cat for the first
PREFIX steps of the gate (the whole gate, 10628 steps, takes the oracle
hours).  Stores the memory's parity, <n_a>, <a>, <n_b>, the trace before
the last renormalisation and the bond profile.  Calls only the oracle and the
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

CASE = dict(Ra=8, Rb=4, dt_max=2e-4, chi=128, chi_mu=16)
PREFIX = 300


def main():
    m, z = wl.model_cat_zgate(**CASE)
    so = m.site_order()
    K = tt.KrausMPO(m, m.dt)
    X, _ = mps.right_canonicalize(mps.product_state(m.init, m.bits, so), tol=1e-14)
    par = tt.operator_mpo(wl.parity_operator(0, m.dims[0]), m.bits, so)
    na = tt.operator_mpo([(1.0, {0: ("NUM_POW", 1)})], m.bits, so)
    a = tt.operator_mpo([(1.0, {0: ("A_POW", 1)})], m.bits, so)
    nb = tt.operator_mpo([(1.0, {1: ("NUM_POW", 1)})], m.bits, so)
    t0 = time.time()
    max_bonds = [1] * (len(so) - 1)
    for n in range(PREFIX):
        X, info = mps.k2_step(X, K.at(n * m.dt), m.tol, m.chi, m.chi_mu)
        b = mps.bond_dims(X)
        max_bonds = [max(u, v) for u, v in zip(max_bonds, b)]
        if (n + 1) % 50 == 0:
            print(f"{n + 1}/{PREFIX} steps, {time.time() - t0:.0f} s, bonds {b}", flush=True)
    p = mps.expect(X, par).real
    out = dict(CASE)
    ea = mps.expect(X, a)
    out.update({"alpha2": z.alpha2, "gate_steps": m.steps, "steps": PREFIX, "dt": m.dt, "t_gate": z.t_gate,
                "tol": m.tol, "parity": p, "n_a": mps.expect(X, na).real, "a": [ea.real, ea.imag],
                "n_b": mps.expect(X, nb).real, "tau": info.tau,
                "final_bonds": mps.bond_dims(X), "max_bonds": max_bonds,
                "source": "oracle.mps.k2_step (Oracle-M), second-order Kraus scheme, purified MPS"})
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "zgate_mps.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
