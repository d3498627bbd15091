"""GPU parity of the one-site TDVP with the fourth-order Magnus Hamiltonian
(order = 5; paper Sec. 3.1.3) on the driven Kerr oscillator (Sec. 3.2)
through the C ABI, against the TDVP oracle (oracle/tdvp.py): both start from
the same MPS built by the oracle; the state vectors agree to 1e-10 (FP64).
Also the undriven K = 0 exact phase rotation at the state's own bonds, the
clock carried across calls, and the size limit of the dense local problems."""
import numpy as np
import pytest

import workload as wl
from oracle import dense, mps, tdvp, tt

pytestmark = pytest.mark.gpu


def _api():
    from paper_2605_27515_amd import api
    return api


def _oracle(m, X0, steps):
    so = m.site_order()
    H0m = tt.operator_mpo(m.H0, m.bits, so)
    if not m.H1:
        return tdvp.magnus4_tdvp_evolve(X0, H0m, None, None, m.dt, steps)
    H1m = tt.operator_mpo(m.H1, m.bits, so)
    return tdvp.magnus4_tdvp_evolve(X0, H0m, H1m, dense.DenseModel(m).f, m.dt, steps)


def _vec(sites, m):
    return mps.to_dense(sites, m.bits, m.site_order())[:, 0]


def _gpu(m, X0, blocks, chi=64):
    api = _api()
    s = api.solver_from_model(m, order=5, chi=chi, chi_mu=1, state="none")
    s.set_state_mps(X0)
    b0 = s.diagnostics()["bonds"]
    for n in blocks:
        s.step(n)
    X = s.get_state_mps()
    d = s.diagnostics()
    s.close()
    return _vec(X, m), b0, d


def test_tdvp_full_bond_random_state_against_oracle():
    """R = 5 (bonds 2, 4, 4, 2: the whole Hilbert space), a random state,
    six steps of h = 0.05 under the drive, in two calls (3 + 3)."""
    m = wl.model_driven_kerr(R=5, alpha0=1.0, dt=0.05)
    rng = np.random.Generator(np.random.PCG64(wl.SEED + 41))
    v = rng.standard_normal(32) + 1j * rng.standard_normal(32)
    v /= np.linalg.norm(v)
    X0 = tdvp.right_orthonormal(mps.product_state([v], m.bits, m.site_order(), tol=0.0))
    print("case tdvp kerr R=5 full bonds, 6 steps", flush=True)
    ref = _vec(_oracle(m, X0, 6), m)
    pg, b0, d = _gpu(m, X0, [3, 3])
    assert b0 == mps.bond_dims(X0)
    err = np.linalg.norm(pg - ref)
    print(f"  state error {err:.2e}, bonds {d['bonds']}", flush=True)
    assert err < 1e-10
    assert d["steps"] == 6
    assert abs(np.linalg.norm(pg) - 1.0) < 1e-12


def test_tdvp_full_bond_local_orders_256_against_oracle():
    """R = 8 at full bonds (2, 4, 8, 16, 8, 4, 2): the site and bond problems
    reach order 256, where the eigen-decomposition's reduction runs on several
    workgroups; two steps of dt = 1e-3 under the drive."""
    m = wl.model_driven_kerr(R=8, dt=1e-3)
    rng = np.random.Generator(np.random.PCG64(wl.SEED + 47))
    v = rng.standard_normal(256) + 1j * rng.standard_normal(256)
    v /= np.linalg.norm(v)
    X0 = tdvp.right_orthonormal(mps.product_state([v], m.bits, m.site_order(), tol=0.0))
    print(f"case tdvp kerr R=8 full bonds {mps.bond_dims(X0)}, 2 steps", flush=True)
    ref = _vec(_oracle(m, X0, 2), m)
    pg, b0, d = _gpu(m, X0, [2])
    assert b0 == mps.bond_dims(X0)
    err = np.linalg.norm(pg - ref)
    print(f"  state error {err:.2e}", flush=True)
    assert err < 1e-10


def test_tdvp_paper_kerr_coherent_start_against_oracle():
    """The paper's benchmark parameters (R = 8, w0 = 1, K = 1/25, alpha0 = 4,
    the two-frequency drive, dt = 1e-3) from the coherent state compressed by
    the oracle at the paper's tolerance 1e-8: 20 steps."""
    m = wl.model_driven_kerr(R=8, dt=1e-3)
    X0 = tdvp.right_orthonormal(mps.product_state(m.init, m.bits, m.site_order(), tol=1e-8))
    nrm = np.linalg.norm(_vec(X0, m))
    X0[0] = X0[0] / nrm
    print(f"case tdvp kerr paper size, bonds {mps.bond_dims(X0)}, 20 steps", flush=True)
    ref = _vec(_oracle(m, X0, 20), m)
    pg, b0, d = _gpu(m, X0, [20])
    assert b0 == mps.bond_dims(X0)
    err = np.linalg.norm(pg - ref)
    aop = np.diag(np.sqrt(np.arange(1, 256)), 1)
    print(f"  state error {err:.2e}, <a> {np.vdot(pg, aop @ pg):.6f}", flush=True)
    assert err < 1e-10
    assert d["bonds"] == b0


def test_tdvp_undriven_exact_phase_at_own_bonds():
    """K = 0, f = 0: psi_n(t) = psi_n(0) exp(-i w0 n t) keeps the coherent
    state's bonds, so TDVP at those bonds is exact (10 steps of h = 0.1)."""
    m = wl.model_driven_kerr(R=6, kerr=0.0, alpha0=1.2 + 0.4j, drive=False, dt=0.1)
    dm = dense.DenseModel(m)
    X0 = tdvp.right_orthonormal(mps.product_state([dm.psi0], m.bits, m.site_order(), tol=0.0))
    print(f"case tdvp undriven phase R=6, bonds {mps.bond_dims(X0)}", flush=True)
    pg, b0, d = _gpu(m, X0, [10])
    exact = dm.psi0 * np.exp(-1j * np.arange(64) * 1.0)
    err = np.linalg.norm(pg - exact)
    print(f"  error to the exact phase {err:.2e}", flush=True)
    assert err < 1e-10
    assert d["bonds"] == b0


def test_tdvp_refuses_local_problems_above_512():
    """R = 10 at full bonds has a site with 2 l r = 2 x 16 x 32 > 512: the step
    is refused on the host before any launch."""
    api = _api()
    m = wl.model_driven_kerr(R=10, dt=1e-3)
    rng = np.random.Generator(np.random.PCG64(wl.SEED + 43))
    v = rng.standard_normal(1024) + 1j * rng.standard_normal(1024)
    v /= np.linalg.norm(v)
    X0 = tdvp.right_orthonormal(mps.product_state([v], m.bits, m.site_order(), tol=0.0))
    s = api.solver_from_model(m, order=5, chi=64, chi_mu=1, state="none")
    s.set_state_mps(X0)
    with pytest.raises(api.LindbladError) as e:
        s.step(1)
    assert "512" in str(e.value)
    s.close()


class _Mem:
    """hipMalloc / hipFree of the library's runtime (test plumbing)."""

    def __init__(self):
        import ctypes as C
        from paper_2605_27515_amd import _lib
        _lib.load()
        self.C = C
        self.h = C.CDLL("libamdhip64.so.7", mode=C.RTLD_GLOBAL)
        self.h.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
        self.h.hipFree.argtypes = [C.c_void_p]
        self.h.hipSetDevice.argtypes = [C.c_int]
        assert self.h.hipSetDevice(0) == 0

    def alloc(self, nbytes):
        p = self.C.c_void_p()
        assert self.h.hipMalloc(self.C.byref(p), nbytes) == 0
        return p.value

    def free(self, p):
        self.h.hipFree(p)


def _same(Xa, Xb):
    assert len(Xa) == len(Xb)
    for a, b in zip(Xa, Xb):
        assert a.shape == b.shape
        assert np.array_equal(a, b)


def test_tdvp_resume_batch_and_arena_are_bitwise():
    """A checkpoint taken after 5 of 10 steps and restored continues bit for
    bit (the drive's clock included); two solvers stepped together by
    step_batch each equal one stepped alone; a solver whose buffers come from
    an arena of lindblad_footprint bytes gives the same state."""
    api = _api()
    m = wl.model_driven_kerr(R=6, alpha0=2.0, dt=2e-3)
    X0 = tdvp.right_orthonormal(mps.product_state(m.init, m.bits, m.site_order(), tol=1e-10))
    X0[0] = X0[0] / np.linalg.norm(_vec(X0, m))
    print(f"case tdvp resume/batch/arena R=6, bonds {mps.bond_dims(X0)}", flush=True)

    def mk(**kw):
        s = api.solver_from_model(m, order=5, chi=32, chi_mu=1, state="none", **kw)
        s.set_state_mps(X0)
        return s
    a = mk()
    a.step(10)
    Xa = a.get_state_mps()
    need = a.footprint()
    a.close()
    b = mk()
    b.step(5)
    ck = b.get_state_mps()
    b.close()
    c = api.solver_from_model(m, order=5, chi=32, chi_mu=1, state="none")
    c.restore_state(ck, 5)
    c.step(5)
    _same(c.get_state_mps(), Xa)
    assert c.diagnostics()["steps"] == 10
    c.close()
    d, e = mk(), mk()
    api.step_batch([d, e], 10)
    _same(d.get_state_mps(), Xa)
    _same(e.get_state_mps(), Xa)
    d.close()
    e.close()
    mem = _Mem()
    size = need + (8 << 20)
    arena = mem.alloc(size)
    try:
        f = mk(arena=arena, arena_bytes=size)
        f.step(10)
        _same(f.get_state_mps(), Xa)
        f.close()
    finally:
        mem.free(arena)


def test_tdvp_two_modes_undriven_and_single_site():
    """Two beam-splitter-coupled Kerr cavities (2^3 levels each, no loss, so a
    pure state; H0 only, the unstacked path) from a random full-bond state
    against the oracle, 5 steps of h = 0.02; and a chain of one site (a
    two-level mode), where each step is two exponentials of h/2 of its 2 x 2
    Hamiltonian, against the exact propagator."""
    from scipy.linalg import expm
    api = _api()
    m = wl.model_coupled_cavities(bits=(3, 3), kappa=0.0, dt=0.02, chi_mu=1)
    m.jumps = []
    rng = np.random.Generator(np.random.PCG64(wl.SEED + 59))
    v = rng.standard_normal(64) + 1j * rng.standard_normal(64)
    v /= np.linalg.norm(v)
    # the state on the model's own site order: a TT-SVD of the 64-vector, mode 0 first
    sites = tdvp.right_orthonormal(_two_mode_mps(v, m))
    print(f"case tdvp two modes 2^3 x 2^3, bonds {mps.bond_dims(sites)}", flush=True)
    ref = _vec(_oracle(m, sites, 5), m)
    pg, b0, d = _gpu(m, sites, [5])
    err = np.linalg.norm(pg - ref)
    print(f"  state error {err:.2e}", flush=True)
    assert err < 1e-10
    m1 = wl.model_driven_kerr(R=1, kerr=0.0, alpha0=0.5, dt=0.1)
    psi0 = np.array([0.6, 0.8j])
    X1 = [psi0.reshape(1, 2, 1)]
    pg1, _, _ = _gpu(m1, X1, [7])
    H = dense.DenseModel(m1).H0
    exact = expm(-1j * 0.7 * H) @ psi0
    print(f"  single site error {np.linalg.norm(pg1 - exact):.2e}", flush=True)
    assert np.linalg.norm(pg1 - exact) < 1e-12


def _two_mode_mps(v, m):
    """MPS of the 64-vector v (mode 0 the most significant index) in the
    model's site order, by the oracle's TT-SVD at tol 0."""
    so = m.site_order()
    t = v.reshape([2] * 6)             # bits of mode 0 (MSB first), then of mode 1
    perm = [b if md == 0 else 3 + b for (md, b) in so]
    cores = tt.tt_svd(t.transpose(perm).reshape(-1), 2, 6, 0.0)
    return cores
