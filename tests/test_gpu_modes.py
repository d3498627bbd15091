"""Three modes on the device: the chain layout of the step (each mode a
contiguous block of quantics sites) against the comb oracle (oracle/comb.py,
paper Sec. 4.2-4.3), which reaches the same density matrix through backbone
tensors and teeth.  Without active truncation both are the Kraus map, so
their rho agree to rounding (FP64) or to the FP32 form's bound."""
import numpy as np
import pytest

import workload as wl
from oracle import comb, mps

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,tol,rtol", [("fp64", 1e-12, 1e-10), ("fp32", 1e-8, 1e-5)])
def test_three_modes_chain_step_equals_comb_oracle(precision, tol, rtol):
    """Three beam-splitter-coupled cavities of 2^3 levels (the second with a
    Kerr term, the first lossy: 4 Kraus operators), coherent start in the
    first: 6 steps of dt = 0.02 (purification rank 31 by then)."""
    from paper_2605_27515_amd import api
    m = wl.model_coupled_cavities(bits=(3, 3, 3), dt=0.02)
    m.jumps = m.jumps[:1]
    print(f"case three modes 2^3 x 2^3 x 2^3, {precision}", flush=True)
    fam = comb.kraus_ops(comb.op_terms(m.H0, m.dims), [comb.op_terms(j, m.dims) for j in m.jumps], m.dt)
    C = comb.product_comb(m.init, m.bits)
    for k in range(6):
        C, _ = comb.kraus_step(C, fam, 1e-12)
    ref = comb.rho(C)
    s = api.solver_from_model(m, precision=precision, chi=128, chi_mu=64, tol=tol)
    s.step(6)
    X = mps.to_dense(s.get_state_mps(), m.bits, m.site_order())
    d = s.diagnostics()
    s.close()
    rho = X @ X.conj().T
    err = np.abs(rho - ref).max() / np.abs(ref).max()
    print(f"  rho max-element error {err:.2e}, bonds {d['bonds']}, chi_mu {d['chi_mu']}", flush=True)
    assert err <= rtol
