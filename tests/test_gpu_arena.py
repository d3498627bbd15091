"""Solvers whose device buffers come from a caller-owned arena
(lb_config.arena): the same results as a solver that allocates, an
undersized arena failing with LB_ERR_OOM, and the arena reused after a
release."""
import ctypes as C

import numpy as np
import pytest

import workload as wl

pytestmark = pytest.mark.gpu


def _api():
    from paper_2605_27515_amd import api
    return api


class _Mem:
    """hipMalloc / hipFree of the library's runtime (test plumbing)."""

    def __init__(self):
        from paper_2605_27515_amd import _lib
        _lib.load()
        self.h = C.CDLL("libamdhip64.so.7", mode=C.RTLD_GLOBAL)
        self.h.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
        self.h.hipFree.argtypes = [C.c_void_p]
        self.h.hipSetDevice.argtypes = [C.c_int]
        assert self.h.hipSetDevice(0) == 0

    def alloc(self, nbytes):
        p = C.c_void_p()
        assert self.h.hipMalloc(C.byref(p), nbytes) == 0
        return p.value

    def free(self, p):
        self.h.hipFree(p)


def _solver(api, m, precision, **kw):
    return api.solver_from_model(m, precision=precision, chi=32, chi_mu=8, **kw)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_arena_solver_matches_and_reports_oom(precision):
    api = _api()
    from paper_2605_27515_amd import _lib
    m = wl.model_cat_buffer(Ra=4, Rb=3, alpha2=4.0, dt=2.5e-5)
    print(f"arena, cat-buffer 2^4 x 2^3, {precision}", flush=True)
    ref = _solver(api, m, precision)
    ref.step(20)
    Xr = ref.get_state_mps()
    n_ref = ref.observe(ref.mpo([(1.0, {0: ("NUM_POW", 1)})]))
    need = ref.footprint()
    ref.close()
    mem = _Mem()
    # the footprint plus room for the temporaries of observe
    size = need + (8 << 20)
    arena = mem.alloc(size)
    try:
        s = _solver(api, m, precision, arena=arena, arena_bytes=size)
        s.step(20)
        Xa = s.get_state_mps()
        assert len(Xa) == len(Xr)
        for a, b in zip(Xa, Xr):
            assert a.shape == b.shape
            assert np.array_equal(a, b)
        n_a = s.observe(s.mpo([(1.0, {0: ("NUM_POW", 1)})]))
        assert n_a == n_ref
        # observe's temporaries came back: a second call fits as well
        assert s.observe(s.mpo([(1.0, {1: ("NUM_POW", 1)})])).real >= 0.0
        # after a release the same arena holds the solver again
        s.release()
        s.set_state_product(m.init)
        s.step(20)
        for a, b in zip(s.get_state_mps(), Xr):
            assert np.array_equal(a, b)
        s.close()
        # an arena an eighth of the footprint: the first call that needs the
        # device fails with LB_ERR_OOM
        small = max(need // 8, 4096)
        t = _solver(api, m, precision, arena=arena, arena_bytes=small, state="none")
        with pytest.raises(api.LindbladError) as e:
            t.set_state_product(m.init)
            t.step(1)
        assert e.value.code == _lib.LB_ERR_OOM
        t.close()
    finally:
        mem.free(arena)

