"""Problem presets and seeded random inputs.

A workload is the Stokes Poiseuille problem on the unit cube (Section 4 of the
paper): an ``n x n x n`` hexahedral mesh with Q2 velocity and Q1 pressure, a
parabolic inflow ``u_x = c*y*(1-y)*z*(1-z)`` on ``x = 0``, no-slip walls on
``y, z in {0, 1}`` and a do-nothing outflow on ``x = 1``.  The decomposition
is ``m x m x m`` cubic subdomains with ``overlap`` element layers.

Nothing here computes any part of the method.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Dict, List, Tuple

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    n: int                    # elements per axis
    m: int                    # subdomains per axis
    overlap: int = 1          # element layers of algebraic overlap
    levels: int = 2           # 2 or 3
    group: int = 2            # three-level: subdomains per subregion per axis
    viscosity: float = 1.0
    inflow: float = 16.0      # c in u_x = c*y(1-y)z(1-z)
    manufactured: int = 0     # 1: body force that makes the quadratic profile exact
    rtol: float = 1e-8
    restart: int = 100
    max_it: int = 1000
    precision: str = "fp64"   # local factor storage: fp64 | fp32 | bf16
    nrhs: int = 1
    local_algebraic: int = 0  # 1: algebraic overlap instead of Dirichlet u, p on the artificial boundary
    level2_layer: int = 0     # 1: level-2 local sets get one more A_0-graph layer
    pressure: str = "q1"      # q1 | p1disc (the paper's pair)
    coarse: str = "gdsw"      # gdsw | gdsw* (vertices grouped with adjacent edges)
    note: str = ""

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


WORKLOADS: Dict[str, Workload] = {
    # 4^3 mesh, 2^3 subdomains: the small case the CPU checker finishes in seconds.
    "C1": Workload("C1", n=4, m=2),
    # 16^3 mesh, 4^3 subdomains of 4^3 elements, FP64 dense local LU.
    "C2": Workload("C2", n=16, m=4),
    # the 16^3 workload with the algebraic overlap reading of the local problems
    "C2alg": Workload("C2alg", n=16, m=4, local_algebraic=1),
    # 24^3 mesh, 6^3 subdomains; 32 right-hand sides with amplitudes ~U[0.5, 2].
    "C3": Workload("C3", n=24, m=6, nrhs=32, precision="fp32"),
    # 32^3 mesh, 8^3 subdomains, three levels with 2^3 grouping, FP32 level-1 factors.
    "C4": Workload("C4", n=32, m=8, levels=3, group=2, precision="fp32"),
    # the paper's own variant: Q2/P1disc, GDSW* coarse space, algebraic overlap
    "P16": Workload("P16", n=16, m=4, local_algebraic=1, pressure="p1disc", coarse="gdsw*"),
    # Table 1, first row: 32^3 hexahedra (954,947 DOFs), 8^3 subdomains, 5,573 coarse DOFs
    "P32": Workload("P32", n=32, m=8, local_algebraic=1, pressure="p1disc", coarse="gdsw*"),
    # a long unrestarted three-level run: 12^3 mesh, 6^3 subdomains in 3^3 subregions of 2^3, the
    # algebraic readings on both levels (about 170 iterations)
    "L3long": Workload("L3long", n=12, m=6, levels=3, group=2, viscosity=0.5, inflow=2.0, restart=200,
                       local_algebraic=1, level2_layer=1),
}


def workload(name: str) -> Workload:
    return WORKLOADS[name]


def random_vector(n: int, seed: int = 1, ncols: int = 1) -> np.ndarray:
    """Standard normal vector(s) on the free DOFs, ``numpy.random.default_rng(seed)``.

    Returns shape ``(n,)`` for one column, else ``(n, ncols)`` (column-major use).
    """
    rng = np.random.default_rng(seed)
    if ncols == 1:
        return rng.standard_normal(n)
    return rng.standard_normal((ncols, n)).T.copy(order="F")


def c3_inflow_amplitudes(k: int = 32, seed: int = 3) -> np.ndarray:
    """Inflow amplitudes c_k ~ U[0.5, 2] for the multi-right-hand-side workload."""
    return np.random.default_rng(seed).uniform(0.5, 2.0, size=k)


def c5_batch_draws(count: int = 16, seed: int = 5) -> List[Tuple[int, float, float]]:
    """Uneven batch: n ~ U{8, 12, 16, 20}, viscosity 10^U[-1, 1], amplitude ~U[0.5, 2].

    Returns ``(n, viscosity, amplitude)`` per problem; subdomains are 4^3 elements.
    """
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.array([8, 12, 16, 20]), size=count)
    mus = 10.0 ** rng.uniform(-1.0, 1.0, size=count)
    cs = rng.uniform(0.5, 2.0, size=count)
    return [(int(a), float(b), float(c)) for a, b, c in zip(ns, mus, cs)]


def paper_variant_cases() -> List[Workload]:
    """Small Q2/P1disc problems (the paper's element pair and coarse spaces)."""
    return [
        Workload("p4m2s", n=4, m=2, local_algebraic=1, pressure="p1disc", coarse="gdsw*"),
        Workload("p6m3s", n=6, m=3, local_algebraic=1, pressure="p1disc", coarse="gdsw*", viscosity=0.6,
                 inflow=2.0),
        Workload("p8m4s", n=8, m=4, local_algebraic=1, pressure="p1disc", coarse="gdsw*"),
        Workload("p6m3f", n=6, m=3, local_algebraic=1, pressure="p1disc", coarse="gdsw"),
        Workload("q6m3s", n=6, m=3, coarse="gdsw*"),
    ]


def small_parity_cases() -> List[Workload]:
    """Problems small enough for the CPU checker that still span several TRSV
    tiles, uneven local sizes and ragged tails."""
    return [
        WORKLOADS["C1"],
        Workload("n6m3", n=6, m=3),
        Workload("n8m2", n=8, m=2),
        Workload("n8m4", n=8, m=4),
        Workload("n9m3", n=9, m=3, viscosity=0.37, inflow=1.3),
        Workload("n8m4alg", n=8, m=4, local_algebraic=1),
        Workload("n9m3alg", n=9, m=3, viscosity=0.37, inflow=1.3, local_algebraic=1),
    ]


def voronoi_partition(n: int, parts: int, seed: int = 11) -> np.ndarray:
    """An unstructured partition of the n^3 hexahedra: each element goes to
    the nearest of `parts` seeded random points (element centres in the unit
    cube, ties to the lower index).  Returns the part of each element,
    elements numbered x fastest.  Only describes the decomposition."""
    rng = np.random.default_rng(seed)
    pts = rng.random((parts, 3))
    e = np.arange(n ** 3)
    c = (np.stack([e % n, (e // n) % n, e // (n * n)], 1) + 0.5) / n
    d2 = ((c[:, None, :] - pts[None, :, :]) ** 2).sum(-1)
    part = np.argmin(d2, axis=1)
    # renumber parts in order of first appearance so every index is used
    _, first = np.unique(part, return_index=True)
    order = np.argsort(first)
    rank = np.empty(parts, dtype=np.int64)
    rank[np.unique(part)[order]] = np.arange(order.size)
    return rank[part]
