"""Python binding of the C ABI: argument marshalling only.

Every step of the method runs in the HIP library; this module converts
NumPy arrays and operator descriptions (see ``workload``) into the C
structures of include/lindblad.h and raises on error status codes.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L


class LindbladError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where} failed with status {code}: {msg}")
        self.code = code


def _check(code: int, where: str):
    if code != L.LB_OK and code != L.LB_WARN_UNSTABLE:
        msg = L.load().lindblad_last_error().decode(errors="replace")
        raise LindbladError(code, where, msg)
    return code


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Op:
    """Handle of an MPO owned by a solver."""

    def __init__(self, handle: int, n_sites: int):
        self.handle = C.c_void_p(handle)
        self.n_sites = n_sites

    def bonds(self) -> list[int]:
        lib = L.load()
        n = C.c_int32()
        b = (C.c_int32 * max(self.n_sites, 1))()
        _check(lib.lindblad_op_info(self.handle, C.byref(n), b), "op_info")
        return [int(b[i]) for i in range(n.value - 1)]

    def sites(self) -> list[np.ndarray]:
        """Host copies of the site tensors W[l, s_out, s_in, r]."""
        return _export_sites(L.load().lindblad_op_site, self.handle, self.n_sites)


def _export_sites(fn, handle, n_sites) -> list[np.ndarray]:
    out = []
    for k in range(n_sites):
        l, r = C.c_int32(), C.c_int32()
        _check(fn(handle, k, C.byref(l), C.byref(r), None), "site export")
        w = np.zeros((l.value, 2, 2, r.value), np.complex128)
        _check(fn(handle, k, C.byref(l), C.byref(r), _dptr(w.view(np.float64))), "site export")
        out.append(w)
    return out


class Solver:
    def __init__(self, bits, chi: int, chi_mu: int, tol: float = 1e-8, order: int = 2,
                 precision: str = "fp64", chi_zip: int = 0, tol_zip: float = 0.0,
                 site_order=None, stream: int | None = None, device: int = 0,
                 allow_unstable: bool = False, fp32_tol_floor: float = 0.0, tau_warn: float = 0.0,
                 arena: int | None = None, arena_bytes: int = 0, fixed_bounds: bool = False,
                 fp64_jacobi_pass: bool = False, autotune: bool = False):
        lib = L.load()
        cfg = L.LbConfig()
        lib.lindblad_default_config(C.byref(cfg))
        cfg.n_modes = len(bits)
        for m, r in enumerate(bits):
            cfg.bits[m] = int(r)
        if site_order is not None:
            cfg.n_sites = len(site_order)
            for i, (m, b) in enumerate(site_order):
                cfg.site_order[i][0] = int(m)
                cfg.site_order[i][1] = int(b)
        cfg.chi_cap = int(chi)
        cfg.chi_mu_cap = int(chi_mu)
        cfg.chi_zip_cap = int(chi_zip)
        cfg.tol = float(tol)
        cfg.tol_zip = float(tol_zip)
        cfg.order = int(order)
        cfg.precision = L.LB_FP32_CONTRACT if precision == "fp32" else L.LB_FP64
        cfg.allow_unstable = 1 if allow_unstable else 0
        cfg.stream = stream
        cfg.device = int(device)
        cfg.fp32_tol_floor = float(fp32_tol_floor)
        cfg.tau_warn = float(tau_warn)
        cfg.arena = arena
        cfg.arena_bytes = int(arena_bytes)
        cfg.fixed_bounds = 1 if fixed_bounds else 0
        cfg.fp64_jacobi_pass = 1 if fp64_jacobi_pass else 0
        cfg.autotune = 1 if autotune else 0
        h = C.c_void_p()
        _check(lib.lindblad_create(C.byref(cfg), C.byref(h)), "create")
        self.h = h
        self.bits = list(bits)
        self.n_sites = sum(bits)
        self.precision = precision
        self._keep = []

    # ---- operators ------------------------------------------------------
    def mpo(self, terms, tol: float = 1e-14) -> Op:
        lib = L.load()
        cterms = (L.LbTerm * max(len(terms), 1))()
        keep = []
        for t, (coef, factors) in enumerate(terms):
            items = sorted(factors.items())
            fa = (L.LbFactor * max(len(items), 1))()
            for j, (mode, f) in enumerate(items):
                fa[j].mode = int(mode)
                if f == "ID":
                    fa[j].kind = 0
                    continue
                kind = f[0]
                fa[j].kind = L.FACTOR_KINDS[kind]
                if kind in ("A_POW", "ADAG_POW", "NUM_POW", "SHIFT"):
                    fa[j].p = int(f[1])
                elif kind == "ADAG_A":
                    fa[j].p, fa[j].q = int(f[1]), int(f[2])
                elif kind == "CHARGE_POW":
                    fa[j].p, fa[j].offset = int(f[1]), int(f[2])
                elif kind == "DENSE":
                    arr = np.ascontiguousarray(np.asarray(f[1], np.complex128))
                    keep.append(arr)
                    fa[j].dense = _dptr(arr.view(np.float64))
            keep.append(fa)
            c = complex(coef)
            cterms[t].re, cterms[t].im = c.real, c.imag
            cterms[t].n_factors = len(items)
            cterms[t].factors = fa
        out = C.c_void_p()
        _check(lib.lindblad_mpo_build(self.h, cterms, len(terms), tol, C.byref(out)), "mpo_build")
        return Op(out.value, self.n_sites)

    def set_generator(self, H0: Op, jumps, dt: float, H1: Op | None = None, drive=None):
        lib = L.load()
        arr = (C.c_void_p * max(len(jumps), 1))(*[j.handle.value for j in jumps])
        dptr = None
        if drive:
            c = np.array([d[0] for d in drive], float)
            w = np.array([d[1] for d in drive], float)
            p = np.array([d[2] for d in drive], float)
            self._drive = (c, w, p)
            dr = L.LbDrive(len(drive), _dptr(c), _dptr(w), _dptr(p))
            dptr = C.byref(dr)
        _check(lib.lindblad_set_generator(self.h, H0.handle, H1.handle if H1 else None, dptr, arr,
                                          len(jumps), float(dt)), "set_generator")

    def kraus_sites(self) -> list[np.ndarray]:
        """Host copies of the stacked Kraus MPO site tensors."""
        return _export_sites(L.load().lindblad_kraus_site, self.h, self.n_sites)

    def kraus_info(self):
        lib = L.load()
        b = (C.c_int32 * max(self.n_sites, 1))()
        k = C.c_int32()
        _check(lib.lindblad_kraus_info(self.h, b, C.byref(k)), "kraus_info")
        return [int(b[i]) for i in range(self.n_sites - 1)], int(k.value)

    # ---- state -------------------------------------------------------------
    def set_state_product(self, vectors):
        lib = L.load()
        arrs = [np.ascontiguousarray(np.asarray(v, np.complex128)) for v in vectors]
        ptrs = (C.POINTER(C.c_double) * len(arrs))(*[_dptr(a.view(np.float64)) for a in arrs])
        _check(lib.lindblad_set_state_product(self.h, ptrs), "set_state_product")

    def set_state_mps(self, sites):
        lib = L.load()
        arrs = [np.ascontiguousarray(np.asarray(s, np.complex128)) for s in sites]
        bonds = [1] + [a.shape[2] for a in arrs]
        b = (C.c_int32 * len(bonds))(*bonds)
        ptrs = (C.POINTER(C.c_double) * len(arrs))(*[_dptr(a.view(np.float64)) for a in arrs])
        _check(lib.lindblad_set_state_mps(self.h, b, ptrs), "set_state_mps")

    def restore_state(self, sites, steps: int):
        """Resume from a checkpoint taken with get_state_mps after `steps` steps."""
        lib = L.load()
        arrs = [np.ascontiguousarray(np.asarray(s, np.complex128)) for s in sites]
        bonds = [1] + [a.shape[2] for a in arrs]
        b = (C.c_int32 * len(bonds))(*bonds)
        ptrs = (C.POINTER(C.c_double) * len(arrs))(*[_dptr(a.view(np.float64)) for a in arrs])
        _check(lib.lindblad_restore_state(self.h, b, ptrs, int(steps)), "restore_state")

    def get_state_mps(self) -> list[np.ndarray]:
        lib = L.load()
        b = (C.c_int32 * (self.n_sites + 1))()
        _check(lib.lindblad_get_state_mps(self.h, b, None), "get_state_mps")
        bonds = [int(b[i]) for i in range(self.n_sites + 1)]
        arrs = [np.zeros((bonds[i], 2, bonds[i + 1]), np.complex128) for i in range(self.n_sites)]
        ptrs = (C.POINTER(C.c_double) * len(arrs))(*[_dptr(a.view(np.float64)) for a in arrs])
        _check(lib.lindblad_get_state_mps(self.h, b, ptrs), "get_state_mps")
        return arrs

    # ---- stepping and observation -------------------------------------------
    def step(self, n: int = 1, sync: bool = True):
        """Enqueue n steps; with sync (the default) wait for them and return
        the status of lindblad_sync (LB_OK or LB_WARN_UNSTABLE; errors raise)."""
        rc = _check(L.load().lindblad_step(self.h, int(n)), "step")
        if not sync:
            return rc
        return self.sync()

    def sync(self):
        return _check(L.load().lindblad_sync(self.h), "sync")

    def observe(self, op: Op) -> complex:
        out = (C.c_double * 2)()
        _check(L.load().lindblad_observe(self.h, op.handle, out), "observe")
        return complex(out[0], out[1])

    def trace_purity(self):
        t, p = C.c_double(), C.c_double()
        _check(L.load().lindblad_trace_purity(self.h, C.byref(t), C.byref(p)), "trace_purity")
        return t.value, p.value

    def diagnostics(self) -> dict:
        d = L.LbDiag()
        _check(L.load().lindblad_diagnostics(self.h, C.byref(d)), "diagnostics")
        n = d.n_sites
        return dict(steps=d.steps, t=d.t, tau=d.tau, max_tau_defect=d.max_tau_defect,
                    bonds=[d.bonds[i] for i in range(n - 1)], chi_mu=d.chi_mu,
                    zip_bonds=[d.zip_bonds[i] for i in range(n)],
                    discarded=[d.discarded[i] for i in range(n)], tier=d.tier,
                    bound_redos=d.bound_redos)

    def profile(self, enable: bool = True, classes=None):
        """Reset and switch live kernel timing on or off; `classes` limits it to
        the named kernel classes (names as in profile_read)."""
        if classes is None or not enable:
            _check(L.load().lindblad_profile(self.h, 1 if enable else 0), "profile")
            return
        names = list(self.profile_read())
        mask = 0
        for c in classes:
            if c not in names:
                raise ValueError(f"unknown kernel class {c!r}; classes are {names}")
            mask |= 1 << names.index(c)
        _check(L.load().lindblad_profile_mask(self.h, mask), "profile")

    def profile_read(self) -> dict:
        p = L.LbProfile()
        _check(L.load().lindblad_profile_read(self.h, C.byref(p)), "profile_read")
        return {p.name[i].value.decode(): dict(launches=int(p.launches[i]), ms=p.ms[i], flop=p.flop[i],
                                                bytes=p.bytes[i]) for i in range(p.n)}

    def footprint(self) -> int:
        b = C.c_int64()
        _check(L.load().lindblad_footprint(self.h, C.byref(b)), "footprint")
        return int(b.value)

    def release(self):
        _check(L.load().lindblad_release(self.h), "release")

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            L.load().lindblad_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gemm_tune_save(path: str) -> None:
    """Write the process-wide table of tuned GEMM split counts (lb_config.autotune)."""
    _check(L.load().lindblad_gemm_tune_save(str(path).encode()), "gemm_tune_save")


def gemm_tune_load(path: str) -> None:
    """Merge a saved split-count table into the process-wide one."""
    _check(L.load().lindblad_gemm_tune_load(str(path).encode()), "gemm_tune_load")


def gemm_tune_entries() -> int:
    return int(L.load().lindblad_gemm_tune_entries())


def step_batch(solvers, n_steps: int = 1):
    arr = (C.c_void_p * len(solvers))(*[s.h.value for s in solvers])
    return _check(L.load().lindblad_step_batch(arr, len(solvers), int(n_steps)), "step_batch")


def solver_from_model(model, precision: str = "fp64", chi: int | None = None,
                      chi_mu: int | None = None, tol: float | None = None, dt: float | None = None,
                      order: int = 2, chi_zip: int = 0, state: str = "init", **kw) -> Solver:
    """Create a solver for a ``workload.Model``: operators, generator, initial state."""
    s = Solver(model.bits, chi if chi is not None else model.chi,
               chi_mu if chi_mu is not None else model.chi_mu,
               tol=model.tol if tol is None else tol, order=order, precision=precision,
               chi_zip=chi_zip, site_order=model.site_order(), **kw)
    H0 = s.mpo(model.H0)
    H1 = s.mpo(model.H1) if model.H1 else None
    jumps = [s.mpo(j) for j in model.jumps]
    s.set_generator(H0, jumps, model.dt if dt is None else dt, H1=H1,
                    drive=model.drive if model.H1 else None)
    if state == "init":
        s.set_state_product(model.init)
    return s


# ---- request loop (include/lindblad_serve.h) --------------------------------

class Server:
    """Continuous-batching loop over independent solves (lindblad_server_*)."""

    def __init__(self, n_slots: int = 8, hbm_budget: int = 0):
        lib = L.load()
        cfg = L.LbServerConfig(int(n_slots), int(hbm_budget))
        h = C.c_void_p()
        _check(lib.lindblad_server_create(C.byref(cfg), C.byref(h)), "server_create")
        self.h = h
        self.n_obs = []

    def submit(self, solver: Solver, init, n_steps: int, observables=(), arrival: float = 0.0) -> int:
        arrs = [np.ascontiguousarray(np.asarray(v, np.complex128)) for v in init]
        ptrs = (C.POINTER(C.c_double) * len(arrs))(*[_dptr(a.view(np.float64)) for a in arrs])
        obs = (C.c_void_p * max(len(observables), 1))(*[o.handle.value for o in observables])
        req = L.LbRequest(solver.h.value, ptrs, int(n_steps), obs, len(observables), float(arrival))
        t = C.c_int32()
        _check(L.load().lindblad_server_submit(self.h, C.byref(req), C.byref(t)), "server_submit")
        self.n_obs.append(len(observables))
        return int(t.value)

    def run(self):
        _check(L.load().lindblad_server_run(self.h), "server_run")

    def result(self, ticket: int) -> dict:
        r = L.LbResult()
        n_obs = self.n_obs[ticket] if 0 <= ticket < len(self.n_obs) else 0
        out = np.zeros(2 * max(n_obs, 1))
        _check(L.load().lindblad_server_result(self.h, int(ticket), C.byref(r), _dptr(out)), "server_result")
        vals = [complex(out[2 * i], out[2 * i + 1]) for i in range(n_obs)]
        return dict(status=r.status, arrival=r.arrival, admitted=r.admitted, done=r.done, bytes=r.bytes,
                    max_tau_defect=r.max_tau_defect, chi_mu=r.chi_mu, max_bond=r.max_bond,
                    observables=vals)

    def stats(self) -> dict:
        st = L.LbServerStats()
        _check(L.load().lindblad_server_stats(self.h, C.byref(st)), "server_stats")
        return dict(makespan=st.makespan, peak_bytes=st.peak_bytes, peak_running=st.peak_running,
                    completed=st.completed)

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            L.load().lindblad_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- component entry points (include/lindblad_kernels.h) ---------------------

def kernel_zgemm(A: np.ndarray, B: np.ndarray, adj_a: bool = False, adj_b: bool = False,
                 precision: str = "fp64", splits: int = 1) -> np.ndarray:
    A = np.ascontiguousarray(A, np.complex128)
    B = np.ascontiguousarray(B, np.complex128)
    M = A.shape[1] if adj_a else A.shape[0]
    K = A.shape[0] if adj_a else A.shape[1]
    N = B.shape[0] if adj_b else B.shape[1]
    C_ = np.zeros((M, N), np.complex128)
    prec = L.LB_FP32_CONTRACT if precision == "fp32" else L.LB_FP64
    _check(L.load().lindblad_kernel_zgemm(M, N, K, _dptr(A.view(np.float64)), int(adj_a),
                                          _dptr(B.view(np.float64)), int(adj_b),
                                          _dptr(C_.view(np.float64)), prec, int(splits)), "kernel_zgemm")
    return C_


def kernel_heev(G: np.ndarray, method: str = "jacobi"):
    G = np.ascontiguousarray(G, np.complex128)
    n = G.shape[0]
    w = np.zeros(n)
    U = np.zeros((n, n), np.complex128)
    sw = C.c_int32()
    _check(L.load().lindblad_kernel_heev(n, _dptr(G.view(np.float64)), _dptr(w),
                                         _dptr(U.view(np.float64)), C.byref(sw),
                                         1 if method == "tridiag" else 0), "kernel_heev")
    return w, U, sw.value


def kernel_heev_noalloc(n: int, g_ptr: int, w_ptr: int, u_ptr: int, method: str = "tridiag",
                        stream: int = 0) -> int:
    """lindblad_kernel_heev_noalloc on caller-owned device buffers (device
    addresses, e.g. torch's data_ptr()): G (n x n complex, read), w (n
    doubles) and U (n x n complex) written.  Returns the sweep count."""
    sw = C.c_int32()
    _check(L.load().lindblad_kernel_heev_noalloc(int(n), C.c_void_p(g_ptr), C.c_void_p(w_ptr), C.c_void_p(u_ptr),
                                                 C.byref(sw), 1 if method == "tridiag" else 0,
                                                 C.c_void_p(stream) if stream else None),
           "kernel_heev_noalloc")
    return sw.value


def kernel_set_wait_limit(ticks: int):
    """Bound (100 MHz wall-clock ticks; <= 0: default 2 s) of the waits of the
    multi-workgroup Householder reduction (include/lindblad_kernels.h)."""
    _check(L.load().lindblad_kernel_set_wait_limit(int(ticks)), "kernel_set_wait_limit")


def kernel_truncate(lam: np.ndarray, tol: float, cap: int):
    lam = np.ascontiguousarray(lam, np.float64)
    k = C.c_int32()
    d = C.c_double()
    _check(L.load().lindblad_kernel_truncate(len(lam), _dptr(lam), float(tol), int(cap), C.byref(k),
                                             C.byref(d)), "kernel_truncate")
    return k.value, d.value
