"""CPU tests of the C-ABI library: it loads, exports every declared symbol,
and its host-side MPO construction (no device work) matches the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

import workload as wl
from oracle import dense, tt
from oracle.operators import factor_matrix

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib_or_skip():
    from paper_2605_27515_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("liblindblad.so not built")
    return _lib


def _declared_symbols():
    names = set()
    for h in ("lindblad.h", "lindblad_kernels.h", "lindblad_serve.h"):
        text = open(os.path.join(ROOT, "include", h)).read()
        names |= set(re.findall(r"^\s*(?:lb_status|void|const char\*|int64_t)\s+(lindblad_\w+)\s*\(", text, re.M))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib_mod = _lib_or_skip()
    raw = ctypes.CDLL(lib_mod.LIB_PATH)
    declared = _declared_symbols()
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(raw, name), name
    assert set(declared) == set(lib_mod.EXPORTED)


@pytest.mark.parametrize("factor", ["ID", ("A_POW", 1), ("A_POW", 2), ("ADAG_POW", 2), ("ADAG_A", 2, 1),
                                    ("ADAG_A", 1, 2), ("NUM_POW", 2), ("CHARGE_POW", 2, 8),
                                    ("SHIFT", 1), ("SHIFT", -3)])
@pytest.mark.parametrize("msb_first", [True, False])
def test_host_mpo_builder_matches_dense(factor, msb_first):
    _lib_or_skip()
    from paper_2605_27515_amd import api
    so = [(0, b) for b in (range(5) if msb_first else reversed(range(5)))]
    s = api.Solver([5], 8, 2, site_order=so)
    op = s.mpo([(1.0, {0: factor})])
    ref = factor_matrix(factor, 32)
    err = np.linalg.norm(tt.mpo_to_dense(op.sites(), [5], so) - ref)
    assert err <= 1e-13 * max(1.0, np.linalg.norm(ref))
    s.close()


def test_host_polynomial_ranks_exact():
    """(a^dag)^m a^m has exact quantics rank m + 1 (paper Table I)."""
    _lib_or_skip()
    from paper_2605_27515_amd import api
    s = api.Solver([10], 8, 2)
    for m in (1, 2, 3):
        assert max(s.mpo([(1.0, {0: ("ADAG_A", m, m)})]).bonds()) == m + 1
    s.close()


@pytest.mark.parametrize("which", ["coherent", "cat-buffer", "transmon"])
def test_host_kraus_mpo_matches_dense_family(which):
    _lib_or_skip()
    from paper_2605_27515_amd import api
    m = {"coherent": wl.model_coherent_loss(),
         "cat-buffer": wl.model_cat_buffer(Ra=3, Rb=2, alpha2=2.0, dt=1e-3),
         "transmon": wl.model_transmon_resonator(Rt=3, Rr=2, dt=1e-3)}[which]
    s = api.solver_from_model(m, state="none")
    W = s.kraus_sites()
    so = m.site_order()
    dm = dense.DenseModel(m)
    K = tt.KrausMPO(m, m.dt)
    for t in (0.0, 0.3):
        fam = dense.kraus_family(dm, t, m.dt)
        Wt = W
        if W[0].shape[0] > 1:
            f = K.f(t + 0.5 * m.dt)
            Wt = tt.contract_boundary(W, [f ** p for p in range(W[0].shape[0])])
        for j, kd in enumerate(fam):
            w = list(Wt)
            w[-1] = w[-1][:, :, :, j:j + 1]
            assert np.abs(tt.mpo_to_dense(w, m.bits, so) - kd).max() < 1e-12
    bonds, nk = s.kraus_info()
    assert nk == len(fam)
    assert bonds == K.bonds
    # canonical gauge: sites 1..L-2 right-orthonormal; at the last site the
    # leading block's rows and the increment's rows feed the same Kraus
    # indices, so each block's rows are orthonormal among themselves
    for w in W[1:-1]:
        M = w.reshape(w.shape[0], -1)
        assert np.abs(M @ M.conj().T - np.eye(w.shape[0])).max() < 1e-12
    M = W[-1].reshape(W[-1].shape[0], -1)
    if len(W) > 1:
        G = M @ M.conj().T
        r = K.lead[-1].shape[0]
        assert np.abs(G[:r, :r] - np.eye(r)).max() < 1e-12
        assert np.abs(G[r:, r:] - np.eye(G.shape[0] - r)).max() < 1e-12
    s.close()


def test_argument_errors():
    _lib_or_skip()
    from paper_2605_27515_amd import api
    from paper_2605_27515_amd._lib import LB_ERR_ARG, LB_ERR_UNSTABLE, LB_ERR_STATE
    with pytest.raises(api.LindbladError) as e:
        api.Solver([0], 8, 2)
    assert e.value.code == LB_ERR_ARG
    with pytest.raises(api.LindbladError) as e:
        api.Solver([4], 1000, 2)
    assert e.value.code == LB_ERR_ARG
    s = api.Solver([4], 8, 2)
    with pytest.raises(api.LindbladError) as e:
        s.mpo([(1.0, {3: ("A_POW", 1)})])
    assert e.value.code == LB_ERR_ARG
    with pytest.raises(api.LindbladError) as e:
        s.step(1)
    assert e.value.code == LB_ERR_STATE
    s.close()
    # the stated dt of the two-photon cat violates the explicit-scheme bound
    m = wl.model_two_photon_cat(R=8, dt=1e-3)
    with pytest.raises(api.LindbladError) as e:
        api.solver_from_model(m, state="none")
    assert e.value.code == LB_ERR_UNSTABLE
    s = api.solver_from_model(wl.model_two_photon_cat(R=8, dt=5e-5), state="none")
    s.close()


def test_footprint_host_only():
    """The device footprint is computed on the host from the caps and the
    Kraus MPO; it grows with chi and is smaller in the FP32 form."""
    _lib_or_skip()
    from paper_2605_27515_amd import api
    m = wl.model_cat_buffer(Ra=5, Rb=5, alpha2=4.0, dt=2.5e-5)
    s0 = api.Solver(m.bits, 16, 4, site_order=m.site_order())
    with pytest.raises(api.LindbladError):
        s0.footprint()                      # no generator yet
    s0.close()
    f = {}
    for prec in ("fp64", "fp32"):
        for chi in (16, 64):
            s = api.solver_from_model(m, precision=prec, chi=chi, chi_mu=8, state="none")
            f[prec, chi] = s.footprint()
            s.release()                     # nothing on the device: a no-op
            s.close()
    assert f["fp64", 16] < f["fp64", 64]
    assert f["fp32", 64] < f["fp64", 64]
    assert 1 << 20 < f["fp64", 16] < 1 << 30


def test_footprint_counts_the_tier_backup():
    """Launch tiers keep a device copy of the state to undo a run: the
    footprint with them exceeds the one with fixed bounds by that copy (every
    site at its capacity, the size table, status and discarded weights, in
    the block cache's size classes), and the other config fields change
    nothing on the device."""
    _lib_or_skip()
    from paper_2605_27515_amd import api
    m = wl.model_cat_buffer(Ra=5, Rb=5, alpha2=4.0, dt=2.5e-5)
    f = {}
    for kw in ({}, {"fixed_bounds": True}, {"autotune": True}, {"fp64_jacobi_pass": True}):
        s = api.solver_from_model(m, precision="fp64", chi=32, chi_mu=8, state="none", **kw)
        f[tuple(kw)] = s.footprint()
        s.close()
    backup = f[()] - f[("fixed_bounds",)]
    L = sum(m.bits)
    site_bytes = 32 * 2 * 32 * 16                 # the largest site at chi = 32
    # at least every site at chi = 32; a site's capacity also covers the
    # zip-up's wider bonds, and the block is rounded up to a power of two
    assert L * site_bytes <= backup <= 16 * L * site_bytes, (backup, f)
    assert f[("autotune",)] == f[()]
    assert f[("fp64_jacobi_pass",)] == f[()]


def test_server_argument_errors_host_only():
    _lib_or_skip()
    from paper_2605_27515_amd import api
    with pytest.raises(api.LindbladError):
        api.Server(n_slots=0)
    sv = api.Server(n_slots=2, hbm_budget=1 << 30)
    m = wl.model_coherent_loss()
    s = api.Solver(m.bits, 16, 4, site_order=m.site_order())
    with pytest.raises(api.LindbladError):
        sv.submit(s, m.init, 10)            # generator not set
    sv.run()                                # nothing queued: no device work
    assert sv.stats()["completed"] == 0
    with pytest.raises(api.LindbladError):
        sv.result(0)
    s.close()
    sv.close()


def test_arena_rejects_bad_arguments():
    """An arena without a size, or not 256-byte aligned, is refused at create
    (host-side validation, no device touched)."""
    _lib_or_skip()
    from paper_2605_27515_amd import api
    from paper_2605_27515_amd._lib import LB_ERR_ARG
    with pytest.raises(api.LindbladError) as e:
        api.Solver([4], 8, 2, arena=4096, arena_bytes=0)
    assert e.value.code == LB_ERR_ARG
    with pytest.raises(api.LindbladError) as e:
        api.Solver([4], 8, 2, arena=4096 + 8, arena_bytes=1 << 20)
    assert e.value.code == LB_ERR_ARG


@pytest.mark.parametrize("drive", [False, True])
def test_host_rk4_mpo_matches_dense_step(drive):
    """order = 4 (pure-state global RK4, paper Sec. 3.1.1): without a drive the
    host MPO is the dense RK4 step operator of the oracle; with one, the dense
    step operator at several t lies in the span of the 31 channels (the empty word and the 30 words) of
    site 0's boundary index plus the identity (the coefficients are the device's, checked by
    the GPU parity tests)."""
    _lib_or_skip()
    from paper_2605_27515_amd import api
    m = wl.model_driven_kerr(R=4, alpha0=1.5, drive=drive, dt=1e-2)
    s = api.solver_from_model(m, order=4, chi=16, chi_mu=1, state="none")
    W = s.kraus_sites()
    so = m.site_order()
    dm = dense.DenseModel(m)
    bonds, nk = s.kraus_info()
    assert nk == 1
    if not drive:
        assert W[0].shape[0] == 1
        P = tt.mpo_to_dense(W, m.bits, so)
        assert np.abs(P - dense.rk4_pure_operator(dm, 0.0, m.dt)).max() < 1e-12
    else:
        D = W[0].shape[0]
        assert D == 31
        chans = []
        for p in range(D):
            e = np.zeros(D)
            e[p] = 1.0
            chans.append(tt.mpo_to_dense(tt.contract_boundary(W, list(e)), m.bits, so).ravel())
        # the leading part (the identity) sits in channel 0 beside its word
        eye = np.eye(16, dtype=complex).ravel()
        chans[0] = chans[0] - eye
        A = np.array([eye] + chans).T
        for t in (0.0, 0.37, 1.9):
            P = dense.rk4_pure_operator(dm, t, m.dt).ravel()
            c, *_ = np.linalg.lstsq(A, P, rcond=None)
            assert np.abs(A @ c - P).max() < 1e-11
            assert abs(c[0] - 1.0) < 1e-9
    s.close()


def test_rk4_order_refuses_jumps_and_unstable_dt():
    _lib_or_skip()
    from paper_2605_27515_amd import api
    from paper_2605_27515_amd._lib import LB_ERR_ARG, LB_ERR_UNSTABLE
    m = wl.model_driven_kerr(R=8, dt=1e-2)
    with pytest.raises(api.LindbladError) as e:
        api.solver_from_model(m, order=4, chi=16, chi_mu=1, state="none")
    assert e.value.code == LB_ERR_UNSTABLE
    m = wl.model_coherent_loss()
    with pytest.raises(api.LindbladError) as e:
        api.solver_from_model(m, order=4, chi=16, chi_mu=1, state="none")
    assert e.value.code == LB_ERR_ARG


def test_tdvp_order_refuses_fp32_jumps_and_counts_its_work():
    """order = 5 (one-site TDVP with the Magnus-4 Hamiltonian, paper Sec.
    3.1.3): the FP32 form is refused at create, jump operators and a
    non-Hermitian H0 at set_generator (a Hermitian one with complex
    coefficients passes), and the footprint counts the dense local work (four
    512 x 512 complex matrices at least) beside the state."""
    _lib_or_skip()
    from paper_2605_27515_amd import api
    from paper_2605_27515_amd._lib import LB_ERR_ARG
    m = wl.model_driven_kerr(R=6, dt=1e-3)
    with pytest.raises(api.LindbladError) as e:
        api.solver_from_model(m, order=5, precision="fp32", chi=16, chi_mu=1, state="none")
    assert e.value.code == LB_ERR_ARG
    with pytest.raises(api.LindbladError) as e:
        api.solver_from_model(wl.model_coherent_loss(), order=5, chi=16, chi_mu=1, state="none")
    assert e.value.code == LB_ERR_ARG
    # a non-Hermitian H0 (the local problems are Hermitian eigen-decompositions)
    bad = wl.Model(name="a", bits=[3], H0=[(1.0, {0: ("A_POW", 1)})], jumps=[], init=[wl.vacuum(8)], dt=0.01)
    with pytest.raises(api.LindbladError) as e:
        api.solver_from_model(bad, order=5, chi=8, chi_mu=1, state="none")
    assert e.value.code == LB_ERR_ARG and "Hermitian" in str(e.value)
    ok = wl.Model(name="p", bits=[3], H0=[(1j, {0: ("A_POW", 1)}), (-1j, {0: ("ADAG_POW", 1)})], jumps=[],
                  init=[wl.vacuum(8)], dt=0.01)
    api.solver_from_model(ok, order=5, chi=8, chi_mu=1, state="none").close()
    s5 = api.solver_from_model(m, order=5, chi=16, chi_mu=1, state="none")
    s4 = api.solver_from_model(m, order=4, chi=16, chi_mu=1, state="none")
    assert s5.footprint() >= s4.footprint() // 4 + 4 * 512 * 512 * 16
    s5.close()
    s4.close()


@pytest.mark.parametrize("drive", [False, True, "two-modes"])
def test_host_tdvp_mpo_channels_are_h0_h1_and_their_commutator(drive):
    """order = 5: the MPO the TDVP step combines, exported, is H0 (no drive) or
    H0, H1 and [H0, H1] on the channels of site 0's left index, each equal to
    the dense operator (paper Sec. 3.1.3: the commutator formed once); also
    for two coupled modes (H0 only, bonds across the mode boundary)."""
    _lib_or_skip()
    from paper_2605_27515_amd import api
    if drive == "two-modes":
        m = wl.model_coupled_cavities(bits=(2, 3), kappa=0.0, chi_mu=1)
        m.jumps = []
        drive = False
    else:
        m = wl.model_driven_kerr(R=4, alpha0=1.5, drive=drive, dt=1e-2)
    s = api.solver_from_model(m, order=5, chi=16, chi_mu=1, state="none")
    W = s.kraus_sites()
    so = m.site_order()
    dm = dense.DenseModel(m)
    bonds, nk = s.kraus_info()
    assert nk == 1
    want = [dm.H0] if not drive else [dm.H0, dm.H1, dm.H0 @ dm.H1 - dm.H1 @ dm.H0]
    assert W[0].shape[0] == len(want)
    for p, ref in enumerate(want):
        e = np.zeros(len(want))
        e[p] = 1.0
        got = tt.mpo_to_dense(tt.contract_boundary(W, list(e)), m.bits, so)
        assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max()), p
    s.close()


def test_gemm_tune_table_round_trip(tmp_path):
    """The split-count table (lb_config.autotune) saved and loaded as JSON
    lines: entries merge, a saved file reloads to the same entries, and a
    line missing a field or with splits outside 1..64 is refused."""
    import json
    from paper_2605_27515_amd import api
    n0 = api.gemm_tune_entries()
    rows = [dict(M=256, N=256, K=11648, batch=1, pa=1, pb=1, pc=0, comp=0, herm=1, conjA=0, conjB=1, akf=1,
                 bnf=0, splits=8),
            dict(M=64, N=64, K=4093, batch=1, pa=0, pb=0, pc=0, comp=0, herm=0, conjA=1, conjB=0, akf=0,
                 bnf=1, splits=16)]
    src = tmp_path / "tune.jsonl"
    src.write_text("".join(json.dumps(r) + "\n" for r in rows) + "\n")
    api.gemm_tune_load(src)
    assert api.gemm_tune_entries() == n0 + 2
    out = tmp_path / "out.jsonl"
    api.gemm_tune_save(out)
    saved = [json.loads(line) for line in out.read_text().splitlines()]
    for r in rows:
        assert r in saved
    # a second load of the same entries adds nothing
    api.gemm_tune_load(out)
    assert api.gemm_tune_entries() == n0 + 2
    bad = tmp_path / "bad.jsonl"
    bad.write_text(json.dumps({k: v for k, v in rows[0].items() if k != "herm"}) + "\n")
    with pytest.raises(api.LindbladError):
        api.gemm_tune_load(bad)
    bad.write_text(json.dumps(dict(rows[0], splits=0)) + "\n")
    with pytest.raises(api.LindbladError):
        api.gemm_tune_load(bad)
    with pytest.raises(api.LindbladError):
        api.gemm_tune_load(tmp_path / "missing.jsonl")
    assert api.gemm_tune_entries() == n0 + 2
