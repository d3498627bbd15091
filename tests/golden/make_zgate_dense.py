"""Writes zgate_dense.json: the cat-qubit Z gate (paper Sec. 6.2) run on a dense
density matrix by the oracle's second-order Kraus scheme, at a size the
oracle finishes in seconds (memory 2^5 Fock levels, buffer 2^2, |alpha|^2 =
32/3, theta = pi).  The phase-flip probability is p_Z = (1 + <(-1)^n_a>)/2 at
T_Z, starting from the even cat.  Calls only the oracle and the workload
description:  python tests/golden/make_zgate_dense.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workload as wl                       # noqa: E402
from oracle import dense                    # noqa: E402
from oracle.operators import dense_operator  # noqa: E402

CASE = dict(Ra=5, Rb=2, alpha2=32.0 / 3.0, dt_max=1e-3)


def run(case=CASE, order=2):
    m, z = wl.model_cat_zgate(**case)
    dm = dense.DenseModel(m)
    rho = np.outer(dm.psi0, dm.psi0.conj())
    rho = dense.kraus_evolve(dm, rho, m.dt, m.steps, order)
    par = dense_operator(wl.parity_operator(0, m.dims[0]), m.dims)
    na = dense_operator([(1.0, {0: ("NUM_POW", 1)})], m.dims)
    return {"parity": float(np.trace(par @ rho).real), "n_a": float(np.trace(na @ rho).real),
            "p_z": float((1.0 + np.trace(par @ rho).real) / 2.0), "steps": m.steps, "dt": m.dt,
            "t_gate": z.t_gate}


if __name__ == "__main__":
    out = dict(CASE)
    out.update(run())
    out["source"] = "oracle.dense.kraus_evolve, second-order Kraus scheme (paper Sec. 5.2.2), dense rho"
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "zgate_dense.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))
