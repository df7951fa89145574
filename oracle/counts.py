"""Enumerated interface entities and coarse-space dimensions (CPU, integers).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

These counts tie the entity classification to numbers the paper prints:

* Table 1 (two-level, GDSW* second level, Q2 velocity / P1-discontinuous
  pressure): 5,573 / 48,781 / 407,837 coarse DOFs for 8^3 / 16^3 / 32^3
  subdomains.  GDSW* groups each vertex with its adjacent edges (Section 4);
  the discontinuous pressure has one constant per subdomain (Section 3).
* Table 2 (three-level): 65 / 901 / 4,213 third-level DOFs for 8 / 64 / 256
  subregions, from full GDSW velocity entities on the subregion grid plus one
  pressure constant per subregion.

The classification is the same as in ``decomposition``: velocity nodes are
classed by their set of closed subdomain boxes, nodes on the Dirichlet faces
(x = 0, y and z walls) carry no DOF, and boundary nodes of the outflow face
fall into the class of the same subdomain set.
"""
from __future__ import annotations

import numpy as np

from .decomposition import box_range_1d


def velocity_interface_classes(m, s=2):
    """Classes of free Q2 velocity interface nodes on an (s m)^3 mesh.

    Returns an int array (n_classes, 6): per axis the closed-box index range
    [lo, hi] (lo_x, lo_y, lo_z, hi_x, hi_y, hi_z).
    """
    n = s * m
    coords = np.arange(2 * n + 1)
    lo1, hi1 = box_range_1d(coords, s, m)
    # free velocity nodes: a != 0, b and c not on the walls
    fa = coords != 0
    fbc = (coords != 0) & (coords != 2 * n)
    keys = set()
    xa = np.nonzero(fa)[0]
    yb = np.nonzero(fbc)[0]
    zc = np.nonzero(fbc)[0]
    LX, HX = lo1[xa], hi1[xa]
    LY, HY = lo1[yb], hi1[yb]
    LZ, HZ = lo1[zc], hi1[zc]
    # distinct per-axis ranges, combined (the classification is a product)
    rx = np.unique(np.stack([LX, HX], 1), axis=0)
    ry = np.unique(np.stack([LY, HY], 1), axis=0)
    rz = np.unique(np.stack([LZ, HZ], 1), axis=0)
    for (lx, hx) in rx:
        for (ly, hy) in ry:
            for (lz, hz) in rz:
                if (hx - lx + 1) * (hy - ly + 1) * (hz - lz + 1) >= 2:
                    keys.add((lx, ly, lz, hx, hy, hz))
    return np.array(sorted(keys), dtype=np.int64)


def full_gdsw_count(m):
    return len(velocity_interface_classes(m))


def full_gdsw_closed_form(m):
    """Faces + edges + vertices of an m^3 box grid: 3(m-1)m^2 + 3m(m-1)^2 + (m-1)^3."""
    return 3 * (m - 1) * m * m + 3 * m * (m - 1) ** 2 + (m - 1) ** 3


def _subdomain_set(key):
    lo, hi = key[:3], key[3:]
    return {(I, J, K) for I in range(lo[0], hi[0] + 1)
            for J in range(lo[1], hi[1] + 1) for K in range(lo[2], hi[2] + 1)}


def gdsw_star_entities(m, s=2):
    """GDSW* velocity entities: every vertex class absorbs the edge classes
    whose subdomain set it contains; faces stay.  Returns a list of subdomain
    sets (one per entity)."""
    cls = [tuple(int(v) for v in k) for k in velocity_interface_classes(m, s)]
    index = {k: i for i, k in enumerate(cls)}
    width = [tuple(k[3 + d] - k[d] for d in range(3)) for k in cls]
    members = {}
    claimed = set()
    for i, k in enumerate(cls):
        if sum(width[i]) == 3:                       # vertex: 8 subdomains
            members[i] = [i]
    for i, k in enumerate(cls):
        if sum(width[i]) != 2:                       # edges only: 4 subdomains
            continue
        d = width[i].index(0)                        # the axis along the edge
        for lo in (k[d] - 1, k[d]):                  # vertex ranges containing k[d]
            v = list(k)
            v[d], v[3 + d] = lo, lo + 1
            j = index.get(tuple(v))
            if j is not None and j in members:
                members[j].append(i)
                claimed.add(i)
    ents = [set().union(*(_subdomain_set(cls[c]) for c in mem))
            for mem in members.values()]
    ents += [_subdomain_set(cls[i]) for i in range(len(cls))
             if sum(width[i]) == 2 and i not in claimed]
    ents += [_subdomain_set(cls[i]) for i in range(len(cls)) if sum(width[i]) == 1]
    return ents


def paper_two_level_coarse_dim(m):
    """3 * #GDSW* velocity entities + m^3 pressure constants (Table 1)."""
    return 3 * len(gdsw_star_entities(m)) + m ** 3


def paper_three_level_coarse_dim(m, grid):
    """Third-level dimension on a grid = (a, b, c) of subregions (Table 2):
    the second-level GDSW* velocity entities are classed by their set of
    subregions; classes with two or more subregions are the level-3 full GDSW
    entities (3 translations each), plus one pressure constant per subregion."""
    a, b, c = grid
    gx, gy, gz = m // a, m // b, m // c
    classes = set()
    for ent in gdsw_star_entities(m):
        regions = frozenset((I // gx, J // gy, K // gz) for (I, J, K) in ent)
        if len(regions) >= 2:
            classes.add(regions)
    return 3 * len(classes) + a * b * c
