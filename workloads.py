"""Seeded, synthetic inputs shared by the oracle, the tests and the benchmark.

This module only *describes problems*: bond lists of spin-1/2 Heisenberg
Hamiltonians H = sum_b J_b s_i . s_j (the models of the paper's Sec. III:
ladder, ring, sawtooth chain, plus J1-J2 chains and random regular graphs),
the S^z >= 0 sectors of a cluster (Sec. II, remark after the susceptibility
formula), and temperature grids.  It holds none of the method's arithmetic
(no basis ranking, no matrix elements, no moments, no thermodynamics), so the
oracle and the HIP path can both take their inputs from here without sharing
any computation.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Cluster:
    """A spin-1/2 cluster: N sites and a bond list (i, j, J_ij)."""

    n_sites: int
    bond_i: np.ndarray
    bond_j: np.ndarray
    J: np.ndarray
    name: str = ""

    def __post_init__(self):
        self.bond_i = np.ascontiguousarray(self.bond_i, dtype=np.int32)
        self.bond_j = np.ascontiguousarray(self.bond_j, dtype=np.int32)
        self.J = np.ascontiguousarray(self.J, dtype=np.float64)

    @property
    def n_bonds(self) -> int:
        return int(self.J.shape[0])

    def with_J(self, J) -> "Cluster":
        return Cluster(self.n_sites, self.bond_i.copy(), self.bond_j.copy(),
                       np.asarray(J, dtype=np.float64).copy(), self.name)


@dataclass
class Sector:
    """One (cluster, S^z) problem: n_up spins up out of N; S^z = n_up - N/2."""

    cluster: Cluster
    n_up: int
    cluster_id: int = 0
    e_lo: float = float("nan")
    e_hi: float = float("nan")

    @property
    def dim(self) -> int:
        return math.comb(self.cluster.n_sites, self.n_up)

    @property
    def sz(self) -> float:
        return self.n_up - 0.5 * self.cluster.n_sites

    @property
    def weight(self) -> int:
        """Multiplicity of the S^z >= 0 sector: the S^z < 0 mirror is degenerate."""
        return 1 if 2 * self.n_up == self.cluster.n_sites else 2


@dataclass
class SpinSector:
    """One (cluster, S^z) problem of spin-s sites (two_s = 2s): the site digits
    d = s + m sum to n, S^z = n - N s.  `n_up` is that sum (the name of the
    field in the C problem record)."""

    cluster: Cluster
    two_s: int
    n: int
    cluster_id: int = 0
    e_lo: float = float("nan")
    e_hi: float = float("nan")

    @property
    def n_up(self) -> int:
        return self.n

    @property
    def dim(self) -> int:
        """Number of digit strings (digits 0..2s) of length N with sum n."""
        ways = [1]
        for _ in range(self.cluster.n_sites):
            nxt = [0] * (len(ways) + self.two_s)
            for r, w in enumerate(ways):
                for d in range(self.two_s + 1):
                    nxt[r + d] += w
            ways = nxt
        return ways[self.n] if 0 <= self.n < len(ways) else 0

    @property
    def sz(self) -> float:
        return self.n - 0.5 * self.two_s * self.cluster.n_sites

    @property
    def weight(self) -> int:
        return 1 if 2 * self.n == self.two_s * self.cluster.n_sites else 2


def spin_sectors(cluster: Cluster, two_s: int, cluster_id: int = 0, only_sz0: bool = False):
    """The S^z >= 0 sectors of a spin-s cluster (S^z = 0 or 1/2 first)."""
    N = cluster.n_sites
    lo = (two_s * N + 1) // 2
    hi = lo if only_sz0 else two_s * N
    return [SpinSector(cluster, two_s, n, cluster_id) for n in range(lo, hi + 1)]


def fe10(J: float = 1.0) -> Cluster:
    """The ferric wheel Fe10 of Sec. III.B as a model: ten spin-5/2 sites on a
    ring with one antiferromagnetic nearest-neighbour coupling J (in units of
    the exchange; use with two_s = 5)."""
    c = ring(10, J)
    c.name = "fe10"
    return c


def ring(n: int, J: float = 1.0) -> Cluster:
    """Periodic nearest-neighbour chain (Sec. III.B)."""
    i = np.arange(n)
    return Cluster(n, i, (i + 1) % n, np.full(n, J), name=f"ring{n}")


def j1j2_chain(n: int, J1: float = 1.0, J2: float = 0.5) -> Cluster:
    """Periodic chain with nearest (J1) and next-nearest (J2) bonds: 2n bonds."""
    i = np.arange(n)
    bi = np.concatenate([i, i])
    bj = np.concatenate([(i + 1) % n, (i + 2) % n])
    J = np.concatenate([np.full(n, J1), np.full(n, J2)])
    return Cluster(n, bi, bj, J, name=f"j1j2_{n}")


def ladder(n: int, J1: float = 1.0, J2: float = 1.0) -> Cluster:
    """Periodic two-leg ladder of n sites (Sec. III.A): rung i holds sites 2i, 2i+1.

    J1 couples the two sites of a rung, J2 couples neighbouring rungs along a leg.
    """
    assert n % 2 == 0
    L = n // 2
    bi, bj, J = [], [], []
    for r in range(L):
        bi.append(2 * r); bj.append(2 * r + 1); J.append(J1)
    for r in range(L):
        for leg in range(2):
            bi.append(2 * r + leg); bj.append(2 * ((r + 1) % L) + leg); J.append(J2)
    return Cluster(n, np.array(bi), np.array(bj), np.array(J), name=f"ladder{n}")


def sawtooth(n: int, J1: float = -1.0, J2: float = 0.45) -> Cluster:
    """Periodic sawtooth (delta) chain (Sec. III.C): J1 between neighbours, J2
    between consecutive odd (1-based) sites, i.e. even 0-based sites 2k, 2k+2."""
    assert n % 2 == 0
    i = np.arange(n)
    k = np.arange(n // 2)
    bi = np.concatenate([i, 2 * k])
    bj = np.concatenate([(i + 1) % n, (2 * k + 2) % n])
    J = np.concatenate([np.full(n, J1), np.full(n // 2, J2)])
    return Cluster(n, bi, bj, J, name=f"sawtooth{n}")


def dimer(J: float = 1.0) -> Cluster:
    return Cluster(2, np.array([0]), np.array([1]), np.array([J]), name="dimer")


def random_regular(n: int, degree: int, rng: np.random.Generator,
                   max_tries: int = 100000) -> tuple[np.ndarray, np.ndarray]:
    """Simple graph with every vertex of the given degree (configuration model,
    rejecting self-loops and repeated edges).  When n*degree is odd, one vertex
    gets degree-1 (a near-regular graph)."""
    stubs_per = np.full(n, degree)
    if (n * degree) % 2:
        stubs_per[n - 1] -= 1
    stubs = np.repeat(np.arange(n), stubs_per)
    for _ in range(max_tries):
        perm = rng.permutation(stubs)
        a, b = perm[0::2], perm[1::2]
        if np.any(a == b):
            continue
        lo, hi = np.minimum(a, b), np.maximum(a, b)
        key = lo * n + hi
        if np.unique(key).size != key.size:
            continue
        order = np.argsort(key, kind="stable")
        return lo[order].astype(np.int32), hi[order].astype(np.int32)
    raise RuntimeError("random_regular: no simple graph found")


def random_regular_cluster(n: int, degree: int, seed, J=1.0, J_range=None) -> Cluster:
    rng = np.random.default_rng(seed)
    bi, bj = random_regular(n, degree, rng)
    if J_range is not None:
        Jv = rng.uniform(J_range[0], J_range[1], size=bi.size)
    else:
        Jv = np.full(bi.size, float(J))
    return Cluster(n, bi, bj, Jv, name=f"rr{degree}_{n}")


def sectors(cluster: Cluster, cluster_id: int = 0, only_sz0: bool = False) -> list[Sector]:
    """The S^z >= 0 sectors of a cluster, largest first."""
    N = cluster.n_sites
    lo = (N + 1) // 2
    ups = [lo] if only_sz0 else list(range(lo, N + 1))
    return [Sector(cluster, k, cluster_id) for k in ups]


def log_temperatures(n: int, t_lo: float, t_hi: float) -> np.ndarray:
    return np.logspace(math.log10(t_lo), math.log10(t_hi), n)


# ---------------------------------------------------------------------------
# The named workloads.  Each returns the problem list and the run parameters.
# ---------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    problems: list
    M: int
    R: int
    vec_kind: str            # "rademacher" | "complex_gaussian" | "gaussian" | "basis"
    eps: float = 0.025
    precision: str = "fp64"  # "fp64" | "fp32"
    seed: int = 0
    kernel: str = "jackson"
    temperatures: np.ndarray = field(default_factory=lambda: log_temperatures(200, 0.01, 10.0))


def ring12_full() -> Workload:
    """Heisenberg ring N=12, J=1, all seven S^z >= 0 sectors (2^12 states
    counting multiplicity), M=256, R=20 Rademacher vectors, eps=0.025,
    Jackson kernel, 200 log-spaced T in [0.01, 10]."""
    c = ring(12)
    return Workload("ring12_full", sectors(c), M=256, R=20, vec_kind="rademacher",
                    eps=0.025, precision="fp64", seed=0, kernel="jackson")


def ring24(only_sz0: bool = True, precision: str = "fp32", M: int = 2000) -> Workload:
    """Heisenberg ring N=24, J=1 (S^z=0 sector: 2,704,156 states), 10 complex
    Gaussian vectors (20 real columns), M=2000, eps=0.025."""
    c = ring(24)
    return Workload("ring24_sz0" if only_sz0 else "ring24_all", sectors(c, only_sz0=only_sz0),
                    M=M, R=10, vec_kind="complex_gaussian", eps=0.025,
                    precision=precision, seed=0)


def batched_clusters(n_clusters: int = 64, n_lo: int = 16, n_hi: int = 22, seed: int = 0):
    """Clusters for the batched form: N ~ U{n_lo..n_hi}, seeded random 3-regular
    bond graphs (near-regular for odd N) with J ~ U[0.5, 1.5]."""
    rng = np.random.default_rng(seed)
    Ns = rng.integers(n_lo, n_hi + 1, size=n_clusters)
    out = []
    for c, n in enumerate(Ns):
        out.append(random_regular_cluster(int(n), 3, [seed, c], J_range=(0.5, 1.5)))
    return out


def batched_workload(n_clusters: int = 64, M: int = 1024, R: int = 32) -> Workload:
    probs = []
    for cid, cl in enumerate(batched_clusters(n_clusters)):
        probs.extend(sectors(cl, cluster_id=cid))
    return Workload("batched_rr3", probs, M=M, R=R, vec_kind="rademacher",
                    eps=0.025, precision="fp32", seed=0)


def j1j2_grad_workload(n: int = 20, M: int = 1000, R: int = 16) -> Workload:
    c = j1j2_chain(n, 1.0, 0.5)
    return Workload("j1j2_%d_sz0" % n, sectors(c, only_sz0=True), M=M, R=R,
                    vec_kind="rademacher", eps=0.025, precision="fp64", seed=0,
                    kernel="none", temperatures=log_temperatures(64, 0.05, 5.0))


def rr4_30_workload(precision: str = "fp32", M: int = 500) -> Workload:
    c = random_regular_cluster(30, 4, 0)
    return Workload("rr4_30_sz0", sectors(c, only_sz0=True), M=M, R=4,
                    vec_kind="rademacher", eps=0.025, precision=precision, seed=0)


def fe10_workload(precision: str = "fp32", M: int = 200, R: int = 100) -> Workload:
    """The ferric wheel Fe10 of Sec. III.B: ten spin-5/2 sites on a J = 1 ring,
    all 26 S^z >= 0 sectors (32,430,816 states; S^z = 0: 4,395,456), R = 100
    random vectors and N_deg = 200 as in the paper's best estimate, no kernel."""
    return Workload("fe10_all", spin_sectors(fe10(), 5), M=M, R=R, vec_kind="rademacher",
                    eps=0.025, precision=precision, seed=0, kernel="none",
                    temperatures=log_temperatures(200, 0.05, 50.0))
