"""CPU FP64 oracle for the purified-MPS Lindblad step.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.
The GPU library never calls it and shares no code with it; the only shared
module is ``workload`` (seeded inputs, no arithmetic of the method).

Three levels, each a plain NumPy/LAPACK implementation in float64/complex128:

* ``oracle.dense``  -- Oracle-D: dense density matrix, RK4 on the Lindblad
  equation (paper Eq. lindblad, RK4 stages of Sec. 3.1.1).
  Oracle-K: the dense second-order Kraus map and its purified form
  (paper Sec. 5.2, Kraus maps U, U', first/second-order schemes).
* ``oracle.tt``     -- quantics tensor trains: TT-SVD of dense vectors and
  per-mode operators, MPO algebra (sum, product, dagger, compression) and the
  stacked Kraus-family MPO (paper Sec. 2.1-2.2, Sec. 5.1 matrix addition).
* ``oracle.mps``    -- Oracle-M: the purified-MPS step (zip-up apply,
  purification truncation, truncated-SVD back-sweep, renormalisation) and
  observables by transfer matrices; the pure-state global RK4 (Sec. 3.1.1).
* ``oracle.tdvp``   -- one-site TDVP with the fourth-order Magnus Hamiltonian
  for a pure state (Sec. 3.1.3), dense local exponentials.
* ``oracle.comb``   -- the quantics comb for M modes (Sec. 4.2-4.3: backbone
  tensors with one quantics tooth per mode) and the purified Kraus step on
  it, operators as sums of products of single-mode matrices.

Pins (``tests/test_oracle_*.py``, marked ``not gpu``): closed forms for a
coherent state and a Fock state under loss, RK4 order 4 / Kraus order 2
convergence, Taylor-2 propagator for the jump-free rank-1 case, identity for
H = 0 and no jumps, the two-photon-pumped even-cat steady state, trace and
positivity invariants, exact polynomial MPO ranks (paper Table I, exact row),
and brute-force agreement of the MPS step with the dense Kraus map on small
Hilbert spaces.

The zip-up truncation inside Oracle-M, an approximation with no exact
target when it is active, is pinned by its error bound: with a cap below the
exact zip-up ranks, its product stays within the telescoped sum of the
discarded weights times the exact continuations to their right
(``tests/test_oracle_pins.py``), and without the cap it equals the exact
product; where it is inactive, the brute-force step tests pin it as well.
"""
