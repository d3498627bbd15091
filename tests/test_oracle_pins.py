"""Pins of the oracle parts that the brute-force step tests leave open.

* ``mps.expect`` against the dense definition Tr(O rho) for non-Hermitian,
  complex operators on mixed states with complex amplitudes (an exchanged pair
  of operator legs returns Tr(O^T rho), which differs here);
* ``mps.rho_distance2`` against the dense ||rho1 - rho2||_F for two
  different states (the gauge-invariant comparison of two purifications,
  Sec. 4.1), ``mps.rows`` (entries of rho one by one) against the contracted
  purification, and ``mps.sample_indices`` against the diagonal of rho;
* the zip-up with its truncation active (Sec. 3.1.1 zip-up, Sec. 5.1
  compression): its product differs from the exact MPO-MPS product by no
  more than the telescoped bound sum_i eps_i ||R_i||, eps_i the discarded
  Frobenius weight of cut i and R_i the exact continuation to the right of
  it, formed here by plain contractions.
"""
import dataclasses

import numpy as np

import workload as wl
from oracle import mps, tt
from oracle.operators import dense_operator


def _complex_mixed_state(steps=12, chi_mu=4):
    """Two modes (2^3 x 2^2) from complex coherent states, evolved with the
    cat+buffer Kraus map so that rho is mixed and has complex entries."""
    m = wl.model_cat_buffer(Ra=3, Rb=2, alpha2=2.0, dt=2e-3)
    m = dataclasses.replace(m, init=[wl.coherent_amplitudes(8, 0.9 + 0.6j),
                                     wl.coherent_amplitudes(4, -0.3 + 0.5j)])
    so = m.site_order()
    K = tt.KrausMPO(m, m.dt)
    X, _ = mps.right_canonicalize(mps.product_state(m.init, m.bits, so))
    for s in range(steps):
        X, _ = mps.k2_step(X, K.at(s * m.dt), 1e-12, 64, chi_mu)
    return m, X


def _dense_rho(X, m):
    Xd = mps.to_dense(X, m.bits, m.site_order())
    return Xd @ Xd.conj().T


def test_expect_equals_dense_trace_for_complex_operators():
    m, X = _complex_mixed_state()
    so = m.site_order()
    rho = _dense_rho(X, m)
    assert X[-1].shape[2] > 1                      # mixed: purification rank > 1
    rng = np.random.Generator(np.random.PCG64(wl.SEED + 7))
    dense0 = rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8))
    cases = [
        [(1.0, {0: ("A_POW", 1)})],
        [(1.0, {0: ("A_POW", 2)})],
        [(1.0, {0: ("ADAG_POW", 1), 1: ("A_POW", 1)})],
        [(0.3 - 0.7j, {0: ("ADAG_A", 1, 2)}), (1j, {1: ("ADAG_POW", 1)})],
        [(1.0, {0: ("SHIFT", 1)}), (-2.0, {1: ("SHIFT", -1)})],
        [(1.0, {0: ("DENSE", dense0)})],
    ]
    for terms in cases:
        O = dense_operator(terms, m.dims)
        ref = complex(np.trace(O @ rho))
        got = mps.expect(X, tt.operator_mpo(terms, m.bits, so))
        assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)), (terms, got, ref)
        # the legs matter: Tr(O^T rho) is a different number for these cases
        swapped = complex(np.trace(O.T @ rho))
        assert abs(swapped - ref) > 1e-3, (terms, swapped, ref)


def test_expect_of_a_on_a_complex_coherent_state():
    """<a> from the amplitudes themselves: sum_n conj(c_n) c_{n+1} sqrt(n+1)."""
    m = wl.Model(name="coh", bits=[5], init=[wl.coherent_amplitudes(32, 1.3 - 0.8j)])
    so = m.site_order()
    X, _ = mps.right_canonicalize(mps.product_state(m.init, m.bits, so))
    c = np.asarray(m.init[0], complex)
    c = c / np.linalg.norm(c)
    ref = complex(np.sum(np.conj(c[:-1]) * c[1:] * np.sqrt(np.arange(1, 32))))
    got = mps.expect(X, tt.operator_mpo([(1.0, {0: ("A_POW", 1)})], m.bits, so))
    assert abs(got - ref) < 1e-13
    assert abs(ref - (1.3 - 0.8j)) < 1e-6          # and that is alpha, to truncation


def test_rho_distance2_against_dense():
    m, X1 = _complex_mixed_state(steps=4)
    _, X2 = _complex_mixed_state(steps=14)
    r1, r2 = _dense_rho(X1, m), _dense_rho(X2, m)
    ref = np.linalg.norm(r1 - r2)
    n1 = np.linalg.norm(r1)
    assert ref > 1e-3 * n1
    assert abs(mps.rho_distance2(X1, X2) - ref ** 2) <= 1e-12 * n1 ** 2
    assert abs(mps.rho_distance2(X2, X1) - ref ** 2) <= 1e-12 * n1 ** 2
    assert abs(mps.rho_distance2(X1, X1)) <= 1e-14 * n1 ** 2


def _site_order_dense(X):
    t = X[0]
    for A in X[1:]:
        t = np.tensordot(t, A, axes=([t.ndim - 1], [0]))
    return t.reshape(1 << len(X), -1)               # row index: digits in site order


def test_rows_are_the_purification_rows():
    m, X = _complex_mixed_state(steps=6)
    L = len(X)
    Xd = _site_order_dense(X)
    idx = np.array([[(n >> (L - 1 - i)) & 1 for i in range(L)] for n in range(1 << L)])
    R = mps.rows(X, idx)
    assert np.abs(R - Xd).max() <= 1e-14 * np.abs(Xd).max()
    # entries of rho one by one
    rho = Xd @ Xd.conj().T
    assert np.abs(R @ R.conj().T - rho).max() <= 1e-14


def test_sample_indices_follow_the_diagonal_of_rho():
    m, X = _complex_mixed_state(steps=6)
    L = len(X)
    Xd = _site_order_dense(X)
    p = np.sum(np.abs(Xd) ** 2, axis=1)
    p = p / p.sum()
    rng = np.random.Generator(np.random.PCG64(wl.SEED + 3))
    idx = mps.sample_indices(X, 20000, rng)
    n = idx @ (1 << np.arange(L - 1, -1, -1))
    freq = np.bincount(n, minlength=1 << L) / len(n)
    assert 0.5 * np.abs(freq - p).sum() < 0.02     # total variation
    assert np.all(p[np.unique(n)] > 0.0)


def _contract_dense_product(X, W):
    """Exact MPO . MPS product as a dense array [s'_1..s'_L, mu, kappa]
    (plain contractions, no truncation)."""
    out = np.einsum('asb,uzsv->zbv', X[0], W[0])              # a = u = 1
    for A, w in zip(X[1:], W[1:]):
        out = np.tensordot(out, A, axes=([out.ndim - 2], [0]))     # [..., v, s, b]
        out = np.tensordot(out, w, axes=([out.ndim - 3, out.ndim - 2], [0, 2]))  # [..., b, z, v]
        nd = out.ndim
        out = out.transpose(list(range(nd - 3)) + [nd - 2, nd - 3, nd - 1])    # [..., z, b, v]
    return out


def _continuation(X, W, i):
    """R_i: the exact map from the bond (b_i, v_i) right of site i to the
    outputs of sites i+1..L (physical, purification, Kraus), as a matrix."""
    A, w = X[i + 1], W[i + 1]
    out = np.einsum('bsc,vzsx->bvzcx', A, w)                      # [b, v, z, c, x]
    for A, w in zip(X[i + 2:], W[i + 2:]):
        out = np.tensordot(out, A, axes=([out.ndim - 2], [0]))     # [..., x, s, c]
        out = np.tensordot(out, w, axes=([out.ndim - 3, out.ndim - 2], [0, 2]))  # [..., c, z, x]
        nd = out.ndim
        out = out.transpose(list(range(nd - 3)) + [nd - 2, nd - 3, nd - 1])
    b, v = out.shape[0], out.shape[1]
    return out.reshape(b * v, -1)


def test_zipup_with_active_truncation_is_within_its_bound():
    m, X = _complex_mixed_state(steps=10, chi_mu=4)
    W = tt.KrausMPO(m, m.dt).at(10 * m.dt)
    exact = _contract_dense_product(X, W)
    Y = exact.reshape(1 << len(X), -1)                 # rows: site order, cols (mu, kappa)
    # exact zip-up ranks first, then a cap below them
    free = mps.StepInfo()
    mps.zipup(X, W, 0.0, 10 ** 6, 0.0, 10 ** 6, free)
    cap = max(free.zip_bonds) - 3
    assert cap >= 2
    info = mps.StepInfo()
    Z = mps.zipup(X, W, 0.0, cap, 0.0, 10 ** 6, info)
    assert max(info.zip_bonds) == cap
    tails = np.sqrt(np.asarray(info.zip_tail2))
    assert tails.max() > 0.0
    bound = sum(e * np.linalg.norm(_continuation(X, W, i), 2)
                for i, e in enumerate(tails) if e > 0.0)
    t = Z[0]
    for A in Z[1:]:
        t = np.tensordot(t, A, axes=([t.ndim - 1], [0]))
    Yz = t.reshape(1 << len(X), -1)                    # V^dag of the last cut dropped
    rho, rho_z = Y @ Y.conj().T, Yz @ Yz.conj().T
    err = np.linalg.norm(rho - rho_z)
    nY, nZ = np.linalg.norm(Y), np.linalg.norm(Yz)
    assert err > 1e-10 * np.linalg.norm(rho)           # the cut is active
    assert err <= bound * (nY + nZ) * (1 + 1e-9) + 1e-13 * np.linalg.norm(rho), (err, bound)
    # without the cap the zip-up is exact
    Zf = mps.zipup(X, W, 0.0, 10 ** 6, 0.0, 10 ** 6, mps.StepInfo())
    t = Zf[0]
    for A in Zf[1:]:
        t = np.tensordot(t, A, axes=([t.ndim - 1], [0]))
    Yf = t.reshape(1 << len(X), -1)
    assert np.linalg.norm(Yf @ Yf.conj().T - rho) <= 1e-12 * np.linalg.norm(rho)
