"""Seeded synthetic inputs for the parallel-tempering QMC sampler.

This module produces problem instances only: graphs, couplings, fields, a proper
colouring with colour-contiguous vertex labels, and temperature ladders expressed as
the per-rung pair (b_r, K_r).  It holds none of the sampler's own arithmetic (no
Metropolis step, no random draws of the chain, no energies), so both the CPU oracle
and the HIP library consume exactly the same inputs.

Model conventions (Section 2 of the paper names the method; the Suzuki-Trotter
mapping is its reference [14], "128 copies of the classical system", Section 6):

* classical energy of one Trotter slice  E(s) = sum_edges J_ij s_i s_j + sum_i h_i s_i
* quantum Hamiltonian  H = E(sigma^z) - Gamma * sum_i sigma^x_i
* a replica at rung r with M slices has action  S_r = b_r * E_cl - K_r * C, where
  b_r = beta_r / M and K_r = -1/2 ln tanh(beta_r Gamma / M)   (M >= 2),
  E_cl = sum_k E(s^k) and C = sum_k sum_i s_i^k s_i^{k+1 mod M}.
  For M == 1 the model is classical and K is unused (set to 0).

The instance recipes follow the workload shapes of the paper (Table 1: many Trotter
copies of a small Ising problem per chain, tens of chains) at the five sizes used by
the tests and the benchmark; see ``config1`` .. ``config5``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence

import numpy as np

SEED_BASE = 10040023
SAMPLER_SEED_BASE = 0x10040023_00000000


@dataclasses.dataclass
class Instance:
    """One Ising problem plus its replica ladder.

    Vertex labels are colour-contiguous: ``color`` is non-decreasing, so the sites of
    colour g form one label range.  Edges are listed once with ``i < j``.
    """

    N: int
    M: int
    R: int
    edges: np.ndarray  # int32 [E, 2], i < j
    J: np.ndarray  # int8 [E]
    h: np.ndarray  # int8 [N]
    color: np.ndarray  # uint8 [N]
    n_colors: int
    b: np.ndarray  # float64 [R], rung 0 coldest
    K: np.ndarray  # float64 [R]
    T: np.ndarray  # float64 [R] temperatures (metadata)
    Gamma: float
    name: str = ""

    @property
    def n_edges(self) -> int:
        return int(self.edges.shape[0])

    @property
    def spins_per_replica(self) -> int:
        return self.N * self.M

    @property
    def flips_per_sweep(self) -> int:
        return self.N * self.M * self.R

    def F(self) -> int:
        """max_i (|h_i| + sum_j |J_ij|): bound on the local field."""
        acc = np.abs(self.h.astype(np.int64)).copy()
        if self.n_edges:
            np.add.at(acc, self.edges[:, 0], np.abs(self.J.astype(np.int64)))
            np.add.at(acc, self.edges[:, 1], np.abs(self.J.astype(np.int64)))
        return int(acc.max()) if self.N else 0

    def with_ladder(self, b: np.ndarray, K: np.ndarray, T=None) -> "Instance":
        b = np.ascontiguousarray(b, dtype=np.float64)
        K = np.ascontiguousarray(K, dtype=np.float64)
        return dataclasses.replace(self, R=int(b.shape[0]), b=b, K=K,
                                   T=np.asarray(T if T is not None else np.full(b.shape, np.nan)))


# ----------------------------------------------------------------------------- graphs

def random_regular_graph(n: int, d: int, rng: np.random.Generator) -> np.ndarray:
    """Uniform-ish simple d-regular graph on n vertices by stub pairing with local
    rejection and restart (Steger-Wormald style).  Returns int32 [n*d/2, 2], i < j."""
    if (n * d) % 2:
        raise ValueError("n*d must be even")
    if d >= n:
        raise ValueError("need d < n")
    for _attempt in range(1000):
        stubs = np.repeat(np.arange(n, dtype=np.int64), d)
        rng.shuffle(stubs)
        stubs = list(stubs)
        adj = [set() for _ in range(n)]
        edges = []
        ok = True
        while stubs:
            placed = False
            for _try in range(64):
                a = int(rng.integers(len(stubs)))
                b = int(rng.integers(len(stubs)))
                if a == b:
                    continue
                u, v = stubs[a], stubs[b]
                if u == v or v in adj[u]:
                    continue
                adj[u].add(v)
                adj[v].add(u)
                edges.append((min(u, v), max(u, v)))
                for idx in sorted((a, b), reverse=True):
                    stubs[idx] = stubs[-1]
                    stubs.pop()
                placed = True
                break
            if not placed:
                # check whether any valid pair exists at all
                rem = stubs
                found = False
                for x in range(len(rem)):
                    for y in range(x + 1, len(rem)):
                        if rem[x] != rem[y] and rem[y] not in adj[rem[x]]:
                            found = True
                            break
                    if found:
                        break
                if not found:
                    ok = False
                    break
        if ok:
            e = np.array(sorted(edges), dtype=np.int32)
            return e
    raise RuntimeError("failed to draw a simple regular graph")


def cubic_lattice(Lx: int, Ly: int, Lz: int) -> np.ndarray:
    """Periodic simple-cubic lattice, site i = x + Lx*y + Lx*Ly*z; int32 [3N, 2], i<j."""
    if min(Lx, Ly, Lz) < 3:
        raise ValueError("periodic lattice needs every side >= 3 (no double bonds)")
    edges = set()
    for z in range(Lz):
        for y in range(Ly):
            for x in range(Lx):
                i = x + Lx * y + Lx * Ly * z
                for (dx, dy, dz) in ((1, 0, 0), (0, 1, 0), (0, 0, 1)):
                    j = ((x + dx) % Lx) + Lx * ((y + dy) % Ly) + Lx * Ly * ((z + dz) % Lz)
                    edges.add((min(i, j), max(i, j)))
    return np.array(sorted(edges), dtype=np.int32)


def greedy_colouring(n: int, edges: np.ndarray) -> np.ndarray:
    """Deterministic proper colouring by DSatur (Brelaz): repeatedly colour the uncoloured
    vertex with the most distinct neighbour colours (ties: higher degree, then lower
    label) with the smallest free colour.  Fewer colours mean fewer update classes per
    sweep.  The next vertex comes from a max-heap on that key with stale entries skipped,
    O((n + edges) log n).  Returns uint8 [n]."""
    import heapq
    adj = [[] for _ in range(n)]
    for a, b in edges:
        adj[int(a)].append(int(b))
        adj[int(b)].append(int(a))
    col = np.full(n, -1, dtype=np.int64)
    sat = [set() for _ in range(n)]
    heap = [(0, -len(adj[u]), u) for u in range(n)]
    heapq.heapify(heap)
    while heap:
        neg_sat, _, v = heapq.heappop(heap)
        if col[v] >= 0 or -neg_sat != len(sat[v]):
            continue  # coloured already, or an entry from before v's saturation grew
        c = 0
        while c in sat[v]:
            c += 1
        col[v] = c
        for u in adj[v]:
            if col[u] < 0 and c not in sat[u]:
                sat[u].add(c)
                heapq.heappush(heap, (-len(sat[u]), -len(adj[u]), u))
    if n and col.max() > 255:
        raise ValueError("more than 256 colours")
    return col.astype(np.uint8)


def relabel_by_colour(n: int, edges: np.ndarray, h: np.ndarray, J: np.ndarray,
                      color: np.ndarray):
    """Relabel vertices so that colour classes are contiguous label ranges (stable in
    the old label).  Returns (edges, J, h, color) in the new labelling, edges sorted."""
    order = np.lexsort((np.arange(n), color))  # new label -> old label
    new_of_old = np.empty(n, dtype=np.int64)
    new_of_old[order] = np.arange(n)
    if edges.shape[0]:
        a = new_of_old[edges[:, 0]]
        b = new_of_old[edges[:, 1]]
        lo = np.minimum(a, b)
        hi = np.maximum(a, b)
        perm = np.lexsort((hi, lo))
        new_edges = np.stack([lo[perm], hi[perm]], axis=1).astype(np.int32)
        new_J = J[perm].astype(np.int8)
    else:
        new_edges = edges.astype(np.int32).reshape(0, 2)
        new_J = J.astype(np.int8)
    return new_edges, new_J, h[order].astype(np.int8), color[order].astype(np.uint8)


# ----------------------------------------------------------------------------- ladders

def geometric_temperatures(t_min: float, t_max: float, R: int) -> np.ndarray:
    """T_r = t_min * (t_max/t_min)^(r/(R-1)); rung 0 is the coldest."""
    if R < 2:
        return np.array([t_min], dtype=np.float64)
    r = np.arange(R, dtype=np.float64)
    return t_min * (t_max / t_min) ** (r / (R - 1))


def st_rungs(T: Sequence[float], Gamma: float, M: int):
    """Per-rung (b_r, K_r) of the Suzuki-Trotter action for temperatures T at fixed
    transverse field Gamma with M slices: b = beta/M, K = -1/2 ln tanh(beta*Gamma/M)."""
    T = np.asarray(T, dtype=np.float64)
    beta = 1.0 / T
    b = beta / M
    if M == 1:
        K = np.zeros_like(b)
    else:
        K = -0.5 * np.log(np.tanh(beta * Gamma / M))
    return b.astype(np.float64), K.astype(np.float64)


# ----------------------------------------------------------------------------- builders

def make_instance(N: int, edges: np.ndarray, J: np.ndarray, h: np.ndarray, M: int,
                  T: Sequence[float], Gamma: float, name: str = "",
                  relabel: bool = True) -> Instance:
    edges = np.asarray(edges, dtype=np.int32).reshape(-1, 2)
    J = np.asarray(J, dtype=np.int8)
    h = np.asarray(h, dtype=np.int8)
    color = greedy_colouring(N, edges)
    if relabel:
        edges, J, h, color = relabel_by_colour(N, edges, h, J, color)
    b, K = st_rungs(T, Gamma, M)
    n_colors = int(color.max()) + 1 if N else 1
    return Instance(N=N, M=M, R=len(b), edges=np.ascontiguousarray(edges),
                    J=np.ascontiguousarray(J), h=np.ascontiguousarray(h),
                    color=np.ascontiguousarray(color), n_colors=n_colors,
                    b=b, K=K, T=np.asarray(T, dtype=np.float64), Gamma=float(Gamma), name=name)


def config1() -> Instance:
    """N=8 spins on a random 3-regular graph, J in {-1,+1}, h in {-1,0,+1}, M=16,
    R=8 on a geometric ladder T in [0.1, 2.0], Gamma = 1."""
    rng = np.random.default_rng([SEED_BASE, 1, 0])
    N, d = 8, 3
    edges = random_regular_graph(N, d, rng)
    J = rng.choice(np.array([-1, 1], dtype=np.int8), size=edges.shape[0])
    h = rng.choice(np.array([-1, 0, 1], dtype=np.int8), size=N)
    T = geometric_temperatures(0.1, 2.0, 8)
    return make_instance(N, edges, J, h, 16, T, 1.0, name="c1")


def config2() -> Instance:
    """N=128 on a random 6-regular graph, J uniform in [-3,3] without 0, h=0, M=64,
    R=32 on a geometric ladder T in [0.05, 3.0], Gamma = 1."""
    rng = np.random.default_rng([SEED_BASE, 2, 0])
    N, d = 128, 6
    edges = random_regular_graph(N, d, rng)
    J = rng.choice(np.array([-3, -2, -1, 1, 2, 3], dtype=np.int8), size=edges.shape[0])
    h = np.zeros(N, dtype=np.int8)
    T = geometric_temperatures(0.05, 3.0, 32)
    return make_instance(N, edges, J, h, 64, T, 1.0, name="c2")


def config3_instance(idx: int, config: int = 3) -> Instance:
    """One instance of the batched workload: N ~ U[32,512], d ~ U{4..8} d-regular
    (N+1 when N*d is odd), J in {-1,+1}, h in {-1,0,+1}, M in {32,64,128},
    R in {16,32,64}, geometric T in [0.1, 3.0], Gamma = 1."""
    rng = np.random.default_rng([SEED_BASE, config, idx])
    N = int(rng.integers(32, 513))
    d = int(rng.integers(4, 9))
    if (N * d) % 2:
        N += 1
    M = int(rng.choice([32, 64, 128]))
    R = int(rng.choice([16, 32, 64]))
    edges = random_regular_graph(N, d, rng)
    J = rng.choice(np.array([-1, 1], dtype=np.int8), size=edges.shape[0])
    h = rng.choice(np.array([-1, 0, 1], dtype=np.int8), size=N)
    T = geometric_temperatures(0.1, 3.0, R)
    return make_instance(N, edges, J, h, M, T, 1.0, name=f"c{config}_{idx}")


def config3(n_instances: int = 512, start: int = 0) -> List[Instance]:
    return [config3_instance(i) for i in range(start, start + n_instances)]


def config4() -> Instance:
    """8x8x16 periodic cubic lattice (N=1024), J = +-1 with p = 0.5, h = 0, M=256,
    R=64, Gamma=1.5, geometric T in [0.2, 2.0]."""
    rng = np.random.default_rng([SEED_BASE, 4, 0])
    edges = cubic_lattice(8, 8, 16)
    N = 8 * 8 * 16
    J = rng.choice(np.array([-1, 1], dtype=np.int8), size=edges.shape[0])
    h = np.zeros(N, dtype=np.int8)
    T = geometric_temperatures(0.2, 2.0, 64)
    return make_instance(N, edges, J, h, 256, T, 1.5, name="c4")


def sweeps_per_exchange(config: int) -> int:
    return {1: 1, 2: 10, 3: 10, 4: 10, 5: 10}[config]


def total_sweeps(config: int) -> int:
    return {1: 10_000, 2: 100_000, 3: 20_000, 4: 100_000, 5: 20_000}[config]


def sampler_seed(config: int) -> int:
    return SAMPLER_SEED_BASE + config


def random_small_instance(rng: np.random.Generator, N: int, M: int, R: int,
                          d: int = 3, jmax: int = 1, hmax: int = 1,
                          t_min: float = 0.3, t_max: float = 3.0, Gamma: float = 1.0,
                          relabel: bool = True, name: str = "small") -> Instance:
    """Small random instance for edge-case tests: d-regular when possible, otherwise
    a ring; J uniform in [-jmax, jmax] without 0, h uniform in [-hmax, hmax]."""
    if N >= d + 1 and (N * d) % 2 == 0 and d > 0:
        edges = random_regular_graph(N, d, rng)
    elif N >= 3:
        edges = np.array([(min(i, (i + 1) % N), max(i, (i + 1) % N)) for i in range(N)],
                         dtype=np.int32)
        edges = np.unique(edges, axis=0)
    elif N == 2:
        edges = np.array([[0, 1]], dtype=np.int32)
    else:
        edges = np.zeros((0, 2), dtype=np.int32)
    jv = np.array([v for v in range(-jmax, jmax + 1) if v != 0], dtype=np.int8)
    J = rng.choice(jv, size=edges.shape[0]) if edges.shape[0] else np.zeros(0, np.int8)
    h = rng.integers(-hmax, hmax + 1, size=N).astype(np.int8)
    T = geometric_temperatures(t_min, t_max, R)
    return make_instance(N, edges, J, h, M, T, Gamma, name=name, relabel=relabel)
