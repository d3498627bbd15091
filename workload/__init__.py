"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle.

This module holds *inputs only*: physical parameters of the studied models,
operator descriptions as plain data (sums of products of named single-mode
factors), seeded random numbers and initial-state amplitudes.  It contains
none of the method's arithmetic (no MPO/MPS construction, no time stepping,
no factorisation); the oracle and the GPU library each interpret these
descriptions with their own code.

Operator description
--------------------
An operator is a list of terms ``(coef, factors)`` where ``factors`` maps a
mode index to a factor ``(kind, args)``.  Kinds (matching ``lb_factor_kind``
in ``include/lindblad.h``):

* ``"ID"``                      identity
* ``("A_POW", p)``              a^p,           <n|a^p|n'> = d(n+p,n') sqrt(n'!/n!)
* ``("ADAG_POW", p)``           (a^dagger)^p
* ``("ADAG_A", p, q)``          (a^dagger)^p a^q (normal ordered)
* ``("NUM_POW", p)``            diag(n^p), n = 0..N-1
* ``("CHARGE_POW", p, off)``    diag((n-off)^p)   (charge basis, offset binary)
* ``("SHIFT", k)``              (T_k)_{n,n'} = d(n+k, n'), open boundary
* ``("DENSE", M)``              an explicit N x N complex matrix

The quantics index of a mode with R bits is n = sum_i 2^(R-i) sigma_i with
sigma_1 the most significant bit (paper, Sec. 2.1, quantics encoding).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED = 20261203

# --------------------------------------------------------------------------
# model descriptions
# --------------------------------------------------------------------------


@dataclass
class Model:
    """A Lindblad problem: H(t) = H0 + f(t) H1, jumps L_k, initial product state."""

    name: str
    bits: list[int]                      # R per mode (N = 2^R)
    H0: list = field(default_factory=list)
    H1: list = field(default_factory=list)     # optional drive operator
    drive: list = field(default_factory=list)  # f(t) = sum c cos(w t + phi): (c, w, phi)
    jumps: list = field(default_factory=list)  # list of operator descriptions
    init: list = field(default_factory=list)   # per-mode dense amplitude vectors
    dt: float = 1e-3
    steps: int = 100
    chi: int = 16
    chi_mu: int = 4
    tol: float = 1e-8

    @property
    def n_modes(self) -> int:
        return len(self.bits)

    @property
    def dims(self) -> list[int]:
        return [1 << r for r in self.bits]

    def site_order(self) -> list[tuple[int, int]]:
        """Default site order: (mode, bit) with bit 0 = most significant digit.

        One mode: [sigma_R ... sigma_1] then the purification bond.
        Two modes: [a: sigma_R ... sigma_1][b: sigma_1 ... sigma_R], so both
        most significant digits face the inter-mode bond (paper, Sec. 4.3).
        """
        return default_site_order(self.bits)


def default_site_order(bits: list[int]) -> list[tuple[int, int]]:
    order: list[tuple[int, int]] = []
    for m, r in enumerate(bits):
        if m == 0:
            order += [(0, b) for b in reversed(range(r))]
        else:
            order += [(m, b) for b in range(r)]
    return order


def coherent_amplitudes(n_levels: int, alpha: complex) -> np.ndarray:
    """c_n = exp(-|alpha|^2/2) alpha^n / sqrt(n!), n < N, renormalised."""
    n = np.arange(n_levels)
    logmag = -0.5 * abs(alpha) ** 2 + n * math.log(abs(alpha) if alpha != 0 else 1.0) \
        - 0.5 * np.array([math.lgamma(k + 1.0) for k in n])
    c = np.exp(logmag).astype(complex)
    if alpha == 0:
        c[:] = 0.0
        c[0] = 1.0
    else:
        c *= np.exp(1j * np.angle(alpha) * n)
    return c / np.linalg.norm(c)


def fock_amplitudes(n_levels: int, m: int) -> np.ndarray:
    c = np.zeros(n_levels, complex)
    c[m] = 1.0
    return c


def vacuum(n_levels: int) -> np.ndarray:
    return fock_amplitudes(n_levels, 0)


# ---- the five workloads -----------------------------------------------------

def model_coherent_loss(R: int = 4, delta: float = 1.0, kappa: float = 1.0,
                        alpha: complex = 2.0, dt: float = 0.01, steps: int = 100,
                        chi: int = 16, chi_mu: int = 4) -> Model:
    """Single mode, H = Delta a^dag a, L = sqrt(kappa) a, coherent start."""
    return Model(
        name="coherent-loss",
        bits=[R],
        H0=[(delta, {0: ("NUM_POW", 1)})],
        jumps=[[(math.sqrt(kappa), {0: ("A_POW", 1)})]],
        init=[coherent_amplitudes(1 << R, alpha)],
        dt=dt, steps=steps, chi=chi, chi_mu=chi_mu)


def model_coupled_cavities(bits=(3, 3, 3), omega=(1.0, 1.3, 0.8), g: float = 0.4, kerr: float = 0.2,
                           kappa: float = 0.3, alpha: complex = 1.5, dt: float = 0.01, steps: int = 100,
                           chi: int = 32, chi_mu: int = 8) -> Model:
    """M lossy cavities in a row, each coupled to the next by a beam splitter,
    with a Kerr term on the second one (a multi-mode test system for the
    quantics comb of paper Sec. 4.3):
    H = sum_a w_a n_a + g sum_a (a_a^dag a_{a+1} + h.c.) + (K/2) a_1^dag^2 a_1^2,
    L_a = sqrt(kappa) a_a, coherent |alpha> in mode 0 and vacuum elsewhere."""
    M = len(bits)
    H0 = [(float(omega[a]), {a: ("NUM_POW", 1)}) for a in range(M)]
    for a in range(M - 1):
        H0.append((g, {a: ("ADAG_POW", 1), a + 1: ("A_POW", 1)}))
        H0.append((g, {a: ("A_POW", 1), a + 1: ("ADAG_POW", 1)}))
    if kerr != 0.0 and M > 1:
        H0.append((0.5 * kerr, {1: ("ADAG_A", 2, 2)}))
    jumps = [[(math.sqrt(kappa), {a: ("A_POW", 1)})] for a in range(M)]
    init = [coherent_amplitudes(1 << bits[0], alpha)] + [vacuum(1 << bits[a]) for a in range(1, M)]
    return Model(name="coupled-cavities", bits=list(bits), H0=H0, jumps=jumps, init=init,
                 dt=dt, steps=steps, chi=chi, chi_mu=chi_mu)


def model_two_photon_cat(R: int = 8, alpha2: float = 8.0, kappa2: float = 1.0,
                         kappa1: float = 1e-3, dt: float = 5e-5, steps: int = 5000,
                         chi: int = 64, chi_mu: int = 8) -> Model:
    """H = 0, L2 = sqrt(k2)(a^2 - alpha^2), L1 = sqrt(k1) a, vacuum start."""
    s2 = math.sqrt(kappa2)
    jumps = [[(s2, {0: ("A_POW", 2)}), (-s2 * alpha2, {0: "ID"})]]
    if kappa1 > 0:
        jumps.append([(math.sqrt(kappa1), {0: ("A_POW", 1)})])
    return Model(name="two-photon-cat", bits=[R], H0=[], jumps=jumps,
                 init=[vacuum(1 << R)], dt=dt, steps=steps, chi=chi, chi_mu=chi_mu)


def model_driven_kerr(R: int = 8, omega0: float = 1.0, kerr: float = 1.0 / 25.0, alpha0: complex = 4.0,
                      drive: bool = True, dt: float = 1e-3, steps: int = 1000, chi: int = 64,
                      tol: float = 1e-8) -> Model:
    """Driven Kerr oscillator of the pure-state benchmark (paper Sec. 3.2):
    H(t) = w0 a^dag a + (K/2) a^dag^2 a^2 + f(t)(a^2 + a^dag^2),
    f(t) = (2/100) cos(sqrt(2) t) + (2 pi/100) cos(sqrt(3) t), coherent start
    |alpha0>, no jumps; a pure state (purification rank 1)."""
    H0 = [(omega0, {0: ("NUM_POW", 1)})]
    if kerr != 0.0:
        H0.append((0.5 * kerr, {0: ("ADAG_A", 2, 2)}))
    H1, drv = [], []
    if drive:
        H1 = [(1.0, {0: ("A_POW", 2)}), (1.0, {0: ("ADAG_POW", 2)})]
        drv = [(2.0 / 100.0, math.sqrt(2.0), 0.0), (2.0 * math.pi / 100.0, math.sqrt(3.0), 0.0)]
    return Model(name="driven-kerr", bits=[R], H0=H0, H1=H1, drive=drv, jumps=[],
                 init=[coherent_amplitudes(1 << R, alpha0)], dt=dt, steps=steps, chi=chi, chi_mu=1, tol=tol)


def model_cat_buffer(Ra: int = 8, Rb: int = 8, alpha2: float = 8.0, g2: float = 1.0,
                     kappa_b: float = 10.0, kappa_a: float = 1e-3, dt: float = 2.5e-5,
                     steps: int = 200, chi: int = 128, chi_mu: int = 16) -> Model:
    """Cat mode a + lossy buffer b (paper Sec. 6.1, Eq. cb):
    H = g2 (a^dag^2 b + a^2 b^dag) + eps_d (b + b^dag), eps_d = -alpha^2 g2,
    L_b = sqrt(kappa_b) b, L_a = sqrt(kappa_a) a; vacuum x vacuum start."""
    eps_d = -alpha2 * g2
    H0 = [(g2, {0: ("ADAG_POW", 2), 1: ("A_POW", 1)}),
          (g2, {0: ("A_POW", 2), 1: ("ADAG_POW", 1)}),
          (eps_d, {1: ("A_POW", 1)}),
          (eps_d, {1: ("ADAG_POW", 1)})]
    jumps = [[(math.sqrt(kappa_b), {1: ("A_POW", 1)})]]
    if kappa_a > 0:
        jumps.append([(math.sqrt(kappa_a), {0: ("A_POW", 1)})])
    return Model(name="cat-buffer", bits=[Ra, Rb], H0=H0, jumps=jumps,
                 init=[vacuum(1 << Ra), vacuum(1 << Rb)], dt=dt, steps=steps,
                 chi=chi, chi_mu=chi_mu)


def even_cat_amplitudes(n_levels: int, alpha: float) -> np.ndarray:
    """(|alpha> + |-alpha>) / norm over the first n_levels Fock states."""
    c = coherent_amplitudes(n_levels, alpha) + coherent_amplitudes(n_levels, -alpha)
    return c / np.linalg.norm(c)


@dataclass
class ZGate:
    """Parameters of the cat-qubit Z gate (paper Sec. 6.2): gate angle theta,
    memory drive eps_Z, gate time T_Z = theta / (4 alpha eps_Z)."""
    alpha2: float
    g2: float
    kappa_b: float
    eps_z: float
    theta: float
    t_gate: float


def model_cat_zgate(Ra: int = 8, Rb: int = 4, alpha2: float | None = None, g2: float = 1.0,
                    kappa_b: float = 10.0, theta: float = math.pi, dt_max: float = 2e-4,
                    chi: int = 64, chi_mu: int = 16) -> tuple[Model, ZGate]:
    """Z gate on a cat qubit (paper Sec. 6.1-6.2): the cat + buffer generator
    with kappa_a = 0 plus the memory drive H_Z = eps_Z (a + a^dag),
    eps_Z = (1/10) 4 g2^2 / kappa_b, for the time T_Z that turns the even cat
    |+> into the odd cat |-> (theta = pi).  The cat size follows the paper's
    scan, |alpha|^2 = N_a / 3, unless given.  Start: even cat x buffer vacuum.
    The step count is the smallest with dt <= dt_max, so steps * dt = T_Z."""
    Na = 1 << Ra
    if alpha2 is None:
        alpha2 = Na / 3.0
    alpha = math.sqrt(alpha2)
    eps_z = 0.1 * 4.0 * g2 * g2 / kappa_b
    t_gate = theta / (4.0 * alpha * eps_z)
    steps = max(1, math.ceil(t_gate / dt_max - 1e-9))
    m = model_cat_buffer(Ra=Ra, Rb=Rb, alpha2=alpha2, g2=g2, kappa_b=kappa_b, kappa_a=0.0,
                         dt=t_gate / steps, steps=steps, chi=chi, chi_mu=chi_mu)
    m.name = "cat-zgate"
    m.H0 = m.H0 + [(eps_z, {0: ("A_POW", 1)}), (eps_z, {0: ("ADAG_POW", 1)})]
    m.init = [even_cat_amplitudes(Na, alpha), vacuum(1 << Rb)]
    return m, ZGate(alpha2=alpha2, g2=g2, kappa_b=kappa_b, eps_z=eps_z, theta=theta, t_gate=t_gate)


def parity_operator(mode: int, n_levels: int) -> list:
    """Photon-number parity (-1)^n of one mode, as an explicit diagonal factor."""
    return [(1.0, {mode: ("DENSE", np.diag((-1.0) ** np.arange(n_levels)).astype(complex))})]


def model_transmon_resonator(Rt: int = 10, Rr: int = 12, ej_over_ec: float = 50.0,
                             ng: float = 0.25, omega_r: float = 30.0, g: float = 0.5,
                             eps: float = 2.0, omega_d: float = 30.0, kappa: float = 0.05,
                             dt: float = 1.5e-7, steps: int = 200, chi: int = 256,
                             chi_mu: int = 32, init_t: np.ndarray | None = None) -> Model:
    """Transmon in the charge basis (offset binary, n = q - 2^(Rt-1)) coupled to a
    resonator (paper Sec. 7.1, Eq. transmon_cavity with the readout drive written
    as eps cos(w_d t)(a + a^dag)); E_C = 1 units.

    H0 = 4 (n - ng)^2 - E_J cos(phi) + w_r a^dag a + i g n (a^dag - a)
    H1 = eps (a + a^dag),  f(t) = cos(w_d t),  L = sqrt(kappa) a.
    cos(phi) = (T_1 + T_-1)/2 with open shifts.
    """
    off = 1 << (Rt - 1)
    ej = ej_over_ec
    H0 = [(4.0, {0: ("CHARGE_POW", 2, off)}),
          (-8.0 * ng, {0: ("CHARGE_POW", 1, off)}),
          (4.0 * ng * ng, {0: "ID"}),
          (-0.5 * ej, {0: ("SHIFT", 1)}),
          (-0.5 * ej, {0: ("SHIFT", -1)}),
          (omega_r, {1: ("NUM_POW", 1)}),
          (1j * g, {0: ("CHARGE_POW", 1, off), 1: ("ADAG_POW", 1)}),
          (-1j * g, {0: ("CHARGE_POW", 1, off), 1: ("A_POW", 1)})]
    H1 = [(eps, {1: ("A_POW", 1)}), (eps, {1: ("ADAG_POW", 1)})]
    jumps = [[(math.sqrt(kappa), {1: ("A_POW", 1)})]]
    Nt = 1 << Rt
    if init_t is None:
        init_t = np.zeros(Nt, complex)
        init_t[off] = 1.0          # charge state n = 0
    return Model(name="transmon-resonator", bits=[Rt, Rr], H0=H0, H1=H1,
                 drive=[(1.0, omega_d, 0.0)], jumps=jumps,
                 init=[init_t, vacuum(1 << Rr)], dt=dt, steps=steps, chi=chi,
                 chi_mu=chi_mu)


def transmon_ground_state(Rt: int, ej_over_ec: float = 50.0, ng: float = 0.25) -> np.ndarray:
    """Ground state of H_t = 4 (n - ng)^2 - (E_J/2)(T_1 + T_-1) on the charge
    states n = q - 2^(Rt-1) (E_C = 1), by a dense symmetric eigensolve."""
    N = 1 << Rt
    n = np.arange(N) - (N >> 1)
    H = np.diag(4.0 * (n - ng) ** 2) - 0.5 * ej_over_ec * (np.eye(N, k=1) + np.eye(N, k=-1))
    w, v = np.linalg.eigh(H)
    g = v[:, 0].astype(complex)
    return g * np.sign(g[np.argmax(np.abs(g))].real)


def transmon_eigenbasis(n_keep: int, charges: np.ndarray, ej_over_ec: float = 50.0,
                        ng: float = 0.25) -> tuple[np.ndarray, np.ndarray]:
    """Lowest n_keep eigenstates Psi_a of H_t = 4 (n - ng)^2 - (E_J/2)(T_1 + T_-1)
    on the given charge states (E_C = 1): their energies and the charge
    operator in that basis, [n]_ab = sum_n Psi_a(n) n Psi_b(n) (paper Sec. 7.2)."""
    n = np.asarray(charges, dtype=float)
    H = np.diag(4.0 * (n - ng) ** 2) - 0.5 * ej_over_ec * (np.eye(len(n), k=1) + np.eye(len(n), k=-1))
    w, v = np.linalg.eigh(H)
    V = v[:, :n_keep]
    return w[:n_keep], V.T @ (n[:, None] * V)


def model_transmon_eigen(Rt: int = 5, Rr: int = 10, n_cut: int = 500, charges: np.ndarray | None = None,
                         ej_over_ec: float = 50.0, ng: float = 0.25, omega_r: float = 30.0, g: float = 0.5,
                         eps: float = 2.0, omega_d: float = 30.0, kappa: float = 0.05, dt: float = 2e-5,
                         steps: int = 200, chi: int = 256, chi_mu: int = 32) -> Model:
    """The driven transmon + resonator of model_transmon_resonator with the
    transmon in its own eigenbasis (paper Sec. 7.2): the charge Hamiltonian is
    diagonalised on |n| <= n_cut (or the given charges), the lowest 2^Rt
    states are kept, and the transmon enters as explicit matrices: diag of the
    energies (counted from the ground state) and the charge operator in that
    basis.  Start: transmon ground state x resonator vacuum."""
    if charges is None:
        charges = np.arange(-n_cut, n_cut + 1)
    e, nmat = transmon_eigenbasis(1 << Rt, charges, ej_over_ec, ng)
    Ht = np.diag(e - e[0]).astype(complex)
    nm = nmat.astype(complex)
    H0 = [(1.0, {0: ("DENSE", Ht)}),
          (omega_r, {1: ("NUM_POW", 1)}),
          (1j * g, {0: ("DENSE", nm), 1: ("ADAG_POW", 1)}),
          (-1j * g, {0: ("DENSE", nm), 1: ("A_POW", 1)})]
    H1 = [(eps, {1: ("A_POW", 1)}), (eps, {1: ("ADAG_POW", 1)})]
    jumps = [[(math.sqrt(kappa), {1: ("A_POW", 1)})]]
    return Model(name="transmon-eigen-resonator", bits=[Rt, Rr], H0=H0, H1=H1,
                 drive=[(1.0, omega_d, 0.0)], jumps=jumps,
                 init=[fock_amplitudes(1 << Rt, 0), vacuum(1 << Rr)], dt=dt, steps=steps, chi=chi,
                 chi_mu=chi_mu)


# stable time steps of the three families (explicit-scheme bound, E_C = 1 units)
SERVING_DT = {"two-photon-cat": 5e-5, "cat-buffer": 2.5e-5, "transmon-resonator": 1.5e-7}


def model_from_request(req: dict) -> Model:
    """The model of one serving request (see serving_requests)."""
    fam = req["family"]
    if fam == "two-photon-cat":
        return model_two_photon_cat(R=req["R"], alpha2=req["alpha2"], dt=SERVING_DT[fam],
                                    steps=req["steps"], chi=req["chi"], chi_mu=req["chi_mu"])
    if fam == "cat-buffer":
        return model_cat_buffer(Ra=req["R"], Rb=req["R"], alpha2=req["alpha2"], dt=SERVING_DT[fam],
                                steps=req["steps"], chi=req["chi"], chi_mu=req["chi_mu"])
    if fam == "transmon-resonator":
        return model_transmon_resonator(Rt=req["Rt"], Rr=req["Rr"], eps=req["eps"], ng=req["ng"],
                                        dt=SERVING_DT[fam], steps=req["steps"], chi=req["chi"],
                                        chi_mu=req["chi_mu"],
                                        init_t=transmon_ground_state(req["Rt"], 50.0, req["ng"]))
    raise ValueError(f"unknown family {fam}")


def poisson_arrivals(n: int, rate: float, seed: int = SEED) -> np.ndarray:
    """Arrival times (seconds) of a Poisson stream of n requests at `rate` per second."""
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    return np.cumsum(rng.exponential(1.0 / rate, n))


# --------------------------------------------------------------------------
# synthetic saturated state (timing workloads)
# --------------------------------------------------------------------------

def saturated_bonds(n_sites: int, chi_mu: int, chi: int, d: int = 2) -> list[int]:
    """Bond dims b_0..b_L with b_i = min(d^i, d^(L-i) chi_mu, chi), b_0 = 1, b_L = chi_mu."""
    b = [min(d ** i, d ** (n_sites - i) * chi_mu, chi) for i in range(n_sites + 1)]
    b[0] = 1
    b[-1] = chi_mu
    return b


def synthetic_mps(n_sites: int, chi_mu: int, chi: int, decay: float = 0.93,
                  seed: int = SEED) -> list[np.ndarray]:
    """Raw (not canonical) random site tensors A_i[b_{i-1}, 2, b_i].

    Entries are i.i.d. complex Gaussian from PCG64(seed); the right bond
    index j of every site is scaled by decay^j so that after canonicalisation
    the Schmidt spectra decay roughly geometrically and a 1e-8 tolerance keeps
    the caps.  Canonicalisation and normalisation are the consumer's job.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    b = saturated_bonds(n_sites, chi_mu, chi)
    sites = []
    for i in range(n_sites):
        g = (rng.standard_normal((b[i], 2, b[i + 1]))
             + 1j * rng.standard_normal((b[i], 2, b[i + 1]))) / math.sqrt(2.0)
        g *= (decay ** np.arange(b[i + 1]))[None, None, :]
        sites.append(np.ascontiguousarray(g))
    return sites


def random_matrix(m: int, n: int, seed: int = SEED, spectrum: np.ndarray | None = None):
    """Seeded complex Gaussian m x n matrix; with ``spectrum`` given, the matrix
    U diag(spectrum) V^H built from seeded random unitaries (Haar via QR)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = (rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))) / math.sqrt(2.0)
    if spectrum is None:
        return g
    k = len(spectrum)
    qa, ra = np.linalg.qr((rng.standard_normal((m, k)) + 1j * rng.standard_normal((m, k))))
    qb, rb = np.linalg.qr((rng.standard_normal((n, k)) + 1j * rng.standard_normal((n, k))))
    qa = qa * (np.diag(ra) / np.abs(np.diag(ra)))[None, :]
    qb = qb * (np.diag(rb) / np.abs(np.diag(rb)))[None, :]
    return (qa * np.asarray(spectrum)[None, :]) @ qb.conj().T


def serving_requests(n: int = 512, seed: int = SEED) -> list[dict]:
    """Parameter-sweep solve requests: uniform over the three model families with
    the parameter ranges of the serving workload; arrival order is the list order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n):
        fam = int(rng.integers(0, 3))
        if fam == 0:
            out.append(dict(family="two-photon-cat", R=int(rng.integers(6, 9)),
                            alpha2=float(rng.uniform(2, 16)),
                            chi=int(rng.choice([32, 64])), chi_mu=8, steps=100))
        elif fam == 1:
            out.append(dict(family="cat-buffer", R=int(rng.integers(6, 9)),
                            alpha2=float(rng.uniform(4, 12)),
                            chi=int(rng.choice([32, 64, 128])), chi_mu=16, steps=100))
        else:
            out.append(dict(family="transmon-resonator", Rt=int(rng.integers(6, 11)),
                            Rr=int(rng.integers(6, 13)), eps=float(rng.uniform(0, 5)),
                            ng=float(rng.uniform(0, 0.5)),
                            chi=int(rng.choice([32, 64, 128, 256])), chi_mu=32, steps=100))
    return out
