"""The eigen-decomposition entry point that allocates nothing
(lindblad_kernel_heev_noalloc: caller-owned device buffers, static scratch)
against the allocating one, on two calls in a row, the second smaller.

The caller's device buffers come from the HIP runtime the library itself
uses (loaded in this process with it), so the test does not depend on a
second runtime's initialisation order."""
import ctypes as C

import numpy as np
import pytest

import workload as wl

pytestmark = pytest.mark.gpu

H2D, D2H = 1, 2


class _Hip:
    """hipMalloc / hipMemcpy / hipFree of the library's runtime (test plumbing)."""

    def __init__(self):
        from paper_2605_27515_amd import _lib
        _lib.load()                                   # the library's runtime is now loaded
        self.h = C.CDLL("libamdhip64.so.7", mode=C.RTLD_GLOBAL)
        self.h.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
        self.h.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        self.h.hipFree.argtypes = [C.c_void_p]
        self.h.hipSetDevice.argtypes = [C.c_int]
        assert self.h.hipSetDevice(0) == 0

    def alloc(self, nbytes):
        p = C.c_void_p()
        assert self.h.hipMalloc(C.byref(p), nbytes) == 0
        return p.value

    def put(self, ptr, arr):
        arr = np.ascontiguousarray(arr)
        assert self.h.hipMemcpy(ptr, arr.ctypes.data, arr.nbytes, H2D) == 0

    def get(self, ptr, shape, dtype):
        out = np.zeros(shape, dtype)
        assert self.h.hipMemcpy(out.ctypes.data, ptr, out.nbytes, D2H) == 0
        return out

    def free(self, *ptrs):
        for p in ptrs:
            self.h.hipFree(p)


def _hermitian(n, seed):
    X = wl.random_matrix(n, n + 5, seed=seed)
    return X @ X.conj().T / n


@pytest.mark.parametrize("method,sizes", [("tridiag", (200, 72)), ("jacobi", (120, 40))])
def test_heev_noalloc_matches_allocating_entry_point(method, sizes):
    from paper_2605_27515_amd import api
    hip = _Hip()
    for n in sizes:
        print(f"heev no-alloc {method} n={n}", flush=True)
        G = _hermitian(n, 40 + n)
        w_ref, U_ref, sw_ref = api.kernel_heev(G, method)
        g, w, u = hip.alloc(16 * n * n), hip.alloc(8 * n), hip.alloc(16 * n * n)
        try:
            hip.put(g, G)
            sw = api.kernel_heev_noalloc(n, g, w, u, method)
            wh = hip.get(w, (n,), np.float64)
            Uh = hip.get(u, (n, n), np.complex128)
            Gh = hip.get(g, (n, n), np.complex128)
        finally:
            hip.free(g, w, u)
        scale = np.abs(w_ref).max()
        assert np.abs(wh - w_ref).max() <= 1e-13 * scale
        assert np.abs(Uh - U_ref).max() <= 1e-12
        assert sw == sw_ref
        assert np.array_equal(Gh, G)                  # the input is only read
        assert np.abs(G @ Uh - Uh * wh).max() <= 1e-12 * scale


def test_heev_noalloc_rejects_orders_beyond_its_scratch():
    from paper_2605_27515_amd import _lib, api
    hip = _Hip()
    n = 257
    g = hip.alloc(16 * n * n)
    try:
        with pytest.raises(api.LindbladError) as e:
            api.kernel_heev_noalloc(n, g, g, g)
    finally:
        hip.free(g)
    assert e.value.code == _lib.LB_ERR_ARG and "static scratch limit" in str(e.value)
