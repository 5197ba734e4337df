"""Seeded synthetic Hubbard inputs shared by the HIP path and the CPU oracle.

This module only builds inputs: the lattice hopping matrix, the two hopping
exponentials, the auxiliary fields and the named workload configurations.  It
holds none of the stabilization arithmetic (chain products, decompositions,
inversions); those live in the HIP library on one side and in the oracle on
the other, and neither imports the other.

Model (paper Sec. 3, the half-filled Hubbard model with hopping t and on-site
U, decoupled in the spin channel with Hirsch's discrete field; Sec. 2 for the
slice propagators).  The workloads use a periodic L x L square lattice with
site index i = x + L*y, nearest-neighbour hopping K_ij = -t and mu = 0.  The
slice matrix is B_l = exp(-dtau K) diag(exp(alpha f_l)), with alpha =
sigma*lambda, lambda = acosh(exp(U dtau / 2)) and f_l in {+1,-1}^N for the
Ising field, or alpha = dtau*g and f_l ~ N(0,1) for a continuous field.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field as dc_field

import numpy as np

BASE_SEED = 2003052860


def site(x: int, y: int, L: int) -> int:
    return (x % L) + L * (y % L)


def hopping_matrix(L: int, t: float = 1.0) -> np.ndarray:
    """K for the periodic L x L square lattice, K_ij = -t per bond (mu = 0).

    For L = 2 the two neighbours in one direction coincide, so the bond is
    counted twice (K_ij = -2t), the literal periodic sum.
    """
    n = L * L
    K = np.zeros((n, n))
    for y in range(L):
        for x in range(L):
            i = site(x, y, L)
            for dx, dy in ((1, 0), (0, 1)):
                j = site(x + dx, y + dy, L)
                K[i, j] -= t
                K[j, i] -= t
    return K


def chain_hopping_matrix(n: int, t: float = 1.0) -> np.ndarray:
    """K for the periodic 1-D chain of the paper's Sec. 3 model."""
    K = np.zeros((n, n))
    for i in range(n):
        j = (i + 1) % n
        K[i, j] -= t
        K[j, i] -= t
    return K


def expk_pair(K: np.ndarray, dtau: float) -> tuple[np.ndarray, np.ndarray]:
    """exp(-dtau K) and exp(+dtau K) of a symmetric K, via its eigenbasis."""
    w, V = np.linalg.eigh(K)
    e = (V * np.exp(-dtau * w)) @ V.T
    ei = (V * np.exp(dtau * w)) @ V.T
    # symmetrize: both are exactly symmetric in exact arithmetic
    return 0.5 * (e + e.T), 0.5 * (ei + ei.T)


def hirsch_lambda(U: float, dtau: float) -> float:
    return math.acosh(math.exp(U * dtau / 2.0))


def rng_streams(seed: int, count: int) -> list[np.random.Generator]:
    ss = np.random.SeedSequence(seed)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(count)]


def ising_field(rng: np.random.Generator, m: int, n: int) -> np.ndarray:
    return 2.0 * rng.integers(0, 2, size=(m, n)).astype(np.float64) - 1.0


def normal_field(rng: np.random.Generator, m: int, n: int) -> np.ndarray:
    return rng.standard_normal((m, n))


@dataclass
class Instance:
    """One chain: B_l = expk diag(exp(alpha * field[l-1])) for l = 1..m."""
    L: int
    m: int
    k: int
    alpha: float
    field: np.ndarray  # (m, n) float64
    expk: np.ndarray   # (n, n)
    expk_inv: np.ndarray
    dtau: float = 0.1
    label: str = ""

    @property
    def n(self) -> int:
        return self.expk.shape[0]


@dataclass
class Workload:
    name: str
    instances: list = dc_field(default_factory=list)
    l_list: list = dc_field(default_factory=list)  # time-displaced slices, if any
    notes: str = ""


_EXPK_CACHE: dict = {}


def expk_for(L: int, dtau: float, t: float = 1.0):
    key = (L, dtau, t)
    if key not in _EXPK_CACHE:
        _EXPK_CACHE[key] = expk_pair(hopping_matrix(L, t), dtau)
    return _EXPK_CACHE[key]


def hubbard_ising(L: int, beta: float, chains: int, flavours: int = 1,
                  U: float = 4.0, dtau: float = 0.1, k: int = 10,
                  seed: int = BASE_SEED) -> list[Instance]:
    """chains x flavours instances; both flavours of a chain share its field."""
    m = int(round(beta / dtau))
    n = L * L
    lam = hirsch_lambda(U, dtau)
    e, ei = expk_for(L, dtau)
    out = []
    for c, rng in enumerate(rng_streams(seed, chains)):
        s = ising_field(rng, m, n)
        for f in range(flavours):
            sigma = 1.0 if f == 0 else -1.0
            out.append(Instance(L, m, k, sigma * lam, s, e, ei, dtau,
                                f"L{L}_b{beta:g}_c{c}_s{int(sigma):+d}"))
    return out


def hubbard_continuous(L: int, beta: float, chains: int, g: float = 1.0,
                       dtau: float = 0.1, k: int = 10,
                       seed: int = BASE_SEED) -> list[Instance]:
    m = int(round(beta / dtau))
    n = L * L
    e, ei = expk_for(L, dtau)
    return [Instance(L, m, k, dtau * g, normal_field(rng, m, n), e, ei, dtau,
                     f"L{L}_b{beta:g}_phi_c{c}")
            for c, rng in enumerate(rng_streams(seed, chains))]


def uneven_batch(count: int = 512, Ls=(6, 8, 10, 12), betas=(10, 20, 40),
                 U: float = 4.0, dtau: float = 0.1, k: int = 10,
                 seed: int = BASE_SEED + 2) -> list[Instance]:
    base = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    Lsel = base.choice(np.array(Ls), size=count)
    bsel = base.choice(np.array(betas, dtype=float), size=count)
    lam = hirsch_lambda(U, dtau)
    out = []
    for c, rng in enumerate(rng_streams(seed + 1, count)):
        L, beta = int(Lsel[c]), float(bsel[c])
        m = int(round(beta / dtau))
        e, ei = expk_for(L, dtau)
        out.append(Instance(L, m, k, lam, ising_field(rng, m, L * L), e, ei,
                            dtau, f"L{L}_b{beta:g}_c{c}"))
    return out


def complex_batch(count: int, n: int, seed: int = BASE_SEED + 8, decades: float = 30.0) -> np.ndarray:
    """Seeded complex n x n matrices shaped like the products a stabilized
    chain factorizes: X diag(s) with X complex Gaussian and column scales s
    spanning `decades` orders of magnitude, the columns in random order
    (so the pivoting has work to do).  [count, n, n] complex128."""
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(count, n, n)) + 1j * rng.normal(size=(count, n, n))
    s = 10.0 ** (-np.linspace(0.0, decades, n))
    for b in range(count):
        X[b] *= s[rng.permutation(n)][None, :]
    return X


def complex_hubbard(L: int, beta: float, chains: int, phase_amp: float = 0.3, U: float = 4.0,
                    dtau: float = 0.1, seed: int = BASE_SEED + 10):
    """Inputs of chains of complex slices B_l = E diag(exp(lambda s_l + i phi_l)):
    a Hubbard chain whose auxiliary field carries a seeded phase phi ~
    U(-phase_amp, phase_amp) per site and slice (the paper's complex model of
    App. B has parameters the paper does not give; these slices have its
    shape: complex, dense after the product with E).  Returns (E, lambda,
    s [chains, m, n], phi [chains, m, n]); the slices themselves are formed by
    the caller (on the device for the benchmark)."""
    m = int(round(beta / dtau))
    n = L * L
    e, _ = expk_for(L, dtau)
    lam = hirsch_lambda(U, dtau)
    s, phi = [], []
    for rng in rng_streams(seed, chains):
        s.append(ising_field(rng, m, n))
        phi.append(rng.uniform(-phase_amp, phase_amp, (m, n)))
    return e, lam, np.stack(s), np.stack(phi)


def workload(name: str, scale: float = 1.0) -> Workload:
    """Named workloads.  `scale` < 1 shrinks the batch (never the shapes)."""
    def nb(x):
        return max(1, int(round(x * scale)))
    if name == "hubbard_L4_b10_single":
        return Workload(name, hubbard_ising(4, 10.0, 1, 1, seed=BASE_SEED + 0),
                        notes="L=4 (N=16), beta=10, M=100, k=10, one chain, sigma=+1")
    if name == "hubbard_L8_b40_batch512":
        ws = Workload(name, hubbard_ising(8, 40.0, nb(256), 2, seed=BASE_SEED + 1),
                      l_list=list(range(10, 401, 10)),
                      notes="L=8 (N=64), beta=40, M=400, k=10, 256 chains x 2 flavours; "
                            "G and G(tau_l,0) for l = 10, 20, ..., 400")
        return ws
    if name == "hubbard_L8_b40_metropolis256":
        return Workload(name, hubbard_ising(8, 40.0, nb(256), 2, seed=BASE_SEED + 5),
                        notes="L=8 (N=64), beta=40, M=400, k=10, 256 chains x 2 flavours sharing "
                              "their field; global Metropolis steps flipping one time slice")
    if name == "hubbard_L8_b40_local256":
        return Workload(name, hubbard_ising(8, 40.0, nb(256), 2, seed=BASE_SEED + 6),
                        notes="L=8 (N=64), beta=40, M=400, k=10, 256 chains x 2 flavours sharing "
                              "their field; one sweep of single-site flips per step")
    if name == "hubbard_uneven_batch512":
        return Workload(name, uneven_batch(nb(512)),
                        notes="L in {6,8,10,12}, beta in {10,20,40}, k=10, U=4")
    if name == "hubbard_L8_b20_phi_batch128":
        return Workload(name, hubbard_continuous(8, 20.0, nb(128), seed=BASE_SEED + 3),
                        notes="L=8, beta=20, M=200, continuous phi ~ N(0,1), g=1, k=10")
    if name == "hubbard_L8_b20_phi_langevin128":
        return Workload(name, hubbard_continuous(8, 20.0, nb(128), seed=BASE_SEED + 3),
                        notes="L=8, beta=20, M=200, continuous phi ~ N(0,1) at the start, g=1, k=10; "
                              "one Langevin step of every chain per step")
    if name == "hubbard_L8_b20_phi_hmc128":
        return Workload(name, hubbard_continuous(8, 20.0, nb(128), seed=BASE_SEED + 3),
                        notes="L=8, beta=20, M=200, continuous phi ~ N(0,1) at the start, g=1, k=10; "
                              "one hybrid Monte Carlo trajectory (10 leapfrog steps of 0.05) per chain "
                              "per step")
    if name == "hubbard_L8_b40_dense128":
        return Workload(name, hubbard_ising(8, 40.0, nb(128), 1, seed=BASE_SEED + 7),
                        l_list=list(range(10, 401, 10)),
                        notes="L=8 (N=64), beta=40, M=400, k=10, 128 chains whose slices "
                              "E diag(exp(lambda s_l)) are handed over as dense matrices; "
                              "G and G(tau,0) at every 10th slice")
    if name == "hubbard_L32_b40_single":
        return Workload(name, hubbard_ising(32, 40.0, 1, 1, seed=BASE_SEED + 9),
                        l_list=list(range(1, 401)),
                        notes="L=32 (N=1024), beta=40, M=400, k=10, one chain, sigma=+1; "
                              "G and G(tau_l,0) for l = 1..400")
    if name == "hubbard_L16_b40_batch128":
        return Workload(name, hubbard_ising(16, 40.0, nb(64), 2, seed=BASE_SEED + 4),
                        l_list=list(range(1, 401)),
                        notes="L=16 (N=256), beta=40, M=400, k=10, 64 chains x 2")
    raise KeyError(name)
