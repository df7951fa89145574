"""Subdomains, overlap and interface entities (CPU).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Section 2.1 of the paper: Omega is split into N non-overlapping subdomains
Omega_i; Omega_i' adds k layers of overlap.  The interface Gamma is split into
vertices, edges and faces, and each such entity carries the null space of the
operator (three velocity translations and the pressure constant).

Readings (pinned by ``tests/test_oracle_decomposition.py``):

* Subdomain (I, J, K) is the closed element box [I s, (I+1) s] x ... with
  s = n / m, numbered I + m (J + m K).
* Overlap delta = element layers around the closed box, clipped to the cube.
  Default (``local_dirichlet``): S_i holds the free DOFs of the grown box
  except the nodes on its faces inside the cube, for velocity and pressure
  alike, so the local problem carries homogeneous Dirichlet conditions for
  both fields on its artificial boundary, which is how Section 2.1 explains
  why the local problems are invertible.  Alternative (``local_dirichlet=
  False``): every node of the grown box, i.e. one layer of matrix-graph
  neighbours of the closed box for delta = 1 (algebraic overlap).
* Gamma holds the free DOFs whose node lies in at least two closed boxes
  (nodes on the outer boundary that belong to one box are not interface).
* An entity is a class of Gamma nodes with the same set of subdomains; a
  face has 2, an edge 4 and a vertex 8 subdomains.  Boundary nodes fall into
  the class of the same subdomain set, which is how faces absorb the
  outflow edges and edges absorb the outflow vertices.
* Coarse DOF order: entities sorted by the smallest Q2 node id of a node that
  carries a free DOF of the entity, then fields u_x, u_y, u_z, p.
* I_i: free DOFs of closed box i that are not in Gamma.

The paper's own coarse space and element pair (Sections 3 and 4):

* ``coarse="gdsw*"``: each vertex class is grouped with its adjacent edge
  classes (an edge whose subdomain set lies inside the vertex's) into one
  entity.  The paper does not say what happens to an edge between two
  vertices; reading: it joins the adjacent vertex that comes first in the
  entity order (the smallest node id), so entities stay disjoint and Phi_Gamma
  stays a 0/1 partition of unity.  Faces stay entities of their own.  Every
  entity of the grouped space is then ordered by the smallest node id of its
  merged class.
* Discontinuous pressure (``pressure="p1disc"``): pressure DOFs sit at element
  centres, so none lies on Gamma; the coarse space gets one pressure column
  per subdomain instead (constant over the subdomain), after the interface
  columns, in subdomain order.  Its local problems need the algebraic overlap:
  with Dirichlet velocity on the whole artificial boundary the constant
  pressure of an interior local problem is a null vector.
"""
from __future__ import annotations

import numpy as np


def box_range_1d(coord, s, m):
    """Indices of the closed boxes that contain a node with the given
    coordinate (half-element units) along one axis: [lo, hi]."""
    coord = np.asarray(coord)
    two_s = 2 * s
    lo = np.where(coord % two_s == 0, np.maximum(coord // two_s - 1, 0), coord // two_s)
    hi = np.minimum(coord // two_s, m - 1)
    return lo, hi


class Decomposition:
    """Structured m^3 decomposition of a ``StokesProblem``."""

    def __init__(self, prob, m, overlap=1, local_dirichlet=True, coarse="gdsw"):
        n = prob.n
        if n % m != 0:
            raise ValueError("n must be a multiple of m")
        if overlap < 1:
            raise ValueError("overlap must be >= 1")
        if coarse not in ("gdsw", "gdsw*"):
            raise ValueError("coarse must be 'gdsw' or 'gdsw*'")
        disc = getattr(prob, "pressure", "q1") == "p1disc"
        if disc and local_dirichlet:
            raise ValueError("discontinuous pressure needs the algebraic overlap (local_dirichlet=False)")
        self.coarse = coarse
        self.m = m
        self.s = n // m
        self.overlap = overlap
        self.n_sub = m ** 3
        s = self.s
        abc = prob.dof_node           # (n_free, 3) half-element units
        field = prob.dof_field
        self.dof_field = field
        self.dof_null = getattr(prob, "dof_null", np.ones(field.size))

        # per-axis closed-box index ranges and the subdomain set of each free DOF
        lo = np.zeros_like(abc)
        hi = np.zeros_like(abc)
        for d in range(3):
            lo[:, d], hi[:, d] = box_range_1d(abc[:, d], s, m)
        self.lo, self.hi = lo, hi
        mult = np.prod(hi - lo + 1, axis=1)
        self.multiplicity = mult
        self.is_gamma = mult >= 2

        # closed box and overlapping box membership
        self.S = []          # overlapping index sets (sorted free DOF indices)
        self.box = []        # closed-box DOFs
        self.I = []          # interior DOFs (closed box, not Gamma)
        for K in range(m):
            for J in range(m):
                for I in range(m):
                    ijk = np.array([I, J, K])
                    inside_closed = np.all((abc >= 2 * s * ijk) & (abc <= 2 * s * (ijk + 1)), axis=1)
                    lo_o = 2 * (s * ijk - overlap)
                    hi_o = 2 * (s * (ijk + 1) + overlap)
                    if local_dirichlet:
                        lo_o = np.where(lo_o > 0, lo_o + 1, lo_o)
                        hi_o = np.where(hi_o < 2 * n, hi_o - 1, hi_o)
                    inside_ovl = np.all((abc >= lo_o) & (abc <= hi_o), axis=1)
                    self.S.append(np.nonzero(inside_ovl)[0])
                    self.box.append(np.nonzero(inside_closed)[0])
                    self.I.append(np.nonzero(inside_closed & ~self.is_gamma)[0])

        # entities: classes of Gamma DOFs by subdomain set (lo, hi per axis)
        g = np.nonzero(self.is_gamma)[0]
        key = np.concatenate([lo[g], hi[g]], axis=1)
        uniq, inv = np.unique(key, axis=0, return_inverse=True)
        inv = inv.ravel()
        # sort classes by smallest Q2 node id
        q2id = prob.dof_q2id[g]
        minid = np.full(len(uniq), np.iinfo(np.int64).max)
        np.minimum.at(minid, inv, q2id)
        order = np.argsort(minid, kind="stable")
        rank = np.empty_like(order)
        rank[order] = np.arange(order.size)
        keys = uniq[order]
        ent = rank[inv]
        if coarse == "gdsw*":
            ent, keys = self._group_vertices_and_edges(ent, keys, q2id)
        self.n_ent = len(keys)
        self.entity_key = keys                       # (lo0..2, hi0..2)
        self.gamma = g
        self.gamma_entity = ent                      # entity of each Gamma DOF
        self.gamma_field = field[g]

        # coarse columns (e, f) that carry at least one DOF
        has = np.zeros((self.n_ent, 4), dtype=bool)
        has[self.gamma_entity, self.gamma_field] = True
        col = -np.ones((self.n_ent, 4), dtype=np.int64)
        col[has] = np.arange(has.sum())
        self.coarse_col = col
        self.n_coarse = int(has.sum())
        self.coarse_entity = np.repeat(np.arange(self.n_ent), 4).reshape(self.n_ent, 4)[has]
        self.coarse_field = np.tile(np.arange(4), (self.n_ent, 1))[has]
        # discontinuous pressure: one constant pressure column per subdomain
        self.sub_pressure_col = None
        if disc:
            self.sub_pressure_col = self.n_coarse + np.arange(self.n_sub)
            self.coarse_entity = np.concatenate([self.coarse_entity, self.n_ent + np.arange(self.n_sub)])
            self.coarse_field = np.concatenate([self.coarse_field, np.full(self.n_sub, 3)])
            self.n_coarse += self.n_sub

    @staticmethod
    def _kind_size(key):
        return int(np.prod(key[3:] - key[:3] + 1))

    def _group_vertices_and_edges(self, ent, keys, q2id):
        """GDSW*: merge each edge class (4 subdomains) into the first adjacent
        vertex class (8 subdomains, set containing the edge's) in entity
        order; faces and unmatched classes stay.  Returns the new entity of
        every Gamma DOF and the keys, re-ordered by smallest node id."""
        size = np.array([self._kind_size(k) for k in keys])
        target = np.arange(len(keys))
        verts = np.nonzero(size == 8)[0]
        for e in np.nonzero(size == 4)[0]:
            lo, hi = keys[e, :3], keys[e, 3:]
            for v in verts:  # ascending entity order: the first match wins
                if np.all(keys[v, :3] <= lo) and np.all(hi <= keys[v, 3:]):
                    target[e] = v
                    break
        groups = np.unique(target)
        new = np.searchsorted(groups, target)[ent]
        minid = np.full(groups.size, np.iinfo(np.int64).max)
        np.minimum.at(minid, new, q2id)
        order = np.argsort(minid, kind="stable")
        rank = np.empty_like(order)
        rank[order] = np.arange(order.size)
        return rank[new], keys[groups][order]

    # --- entity bookkeeping -------------------------------------------------
    def entity_subdomains(self, e):
        """Sorted subdomain indices of entity e (e >= n_ent: the pressure
        column of subdomain e - n_ent)."""
        if e >= self.n_ent:
            return [int(e - self.n_ent)]
        lo, hi = self.entity_key[e, :3], self.entity_key[e, 3:]
        out = []
        for K in range(lo[2], hi[2] + 1):
            for J in range(lo[1], hi[1] + 1):
                for I in range(lo[0], hi[0] + 1):
                    out.append(I + self.m * (J + self.m * K))
        return sorted(out)

    def entity_kind(self, e):
        """'face', 'edge' or 'vertex' by the number of subdomains (2, 4, 8)."""
        k = int(np.prod(self.entity_key[e, 3:] - self.entity_key[e, :3] + 1))
        return {2: "face", 4: "edge", 8: "vertex"}[k]

    def local_sizes(self):
        return np.array([len(S) for S in self.S])


class AlgebraicDecomposition:
    """Decomposition from the distribution of the DOFs alone (Section 3: the
    implementation needs only which subdomains hold each velocity and
    pressure DOF), for any matrix and any partition.

    Inputs: the free-DOF matrix A (its graph gives the overlap), the field of
    each DOF (0-2 velocity components, 3 pressure), the value of its field's
    null-space vector (1 for translations and a continuous constant
    pressure), and for every DOF the sorted subdomains that hold it (the
    closures of the non-overlapping subdomains: an interface DOF is held by
    several).  Definitions, as for the structured cube:

    * D_i = DOFs held by subdomain i; Gamma = DOFs held by at least two;
      I_i = D_i minus Gamma.
    * Entities: classes of Gamma DOFs with the same subdomain set, ordered by
      their smallest DOF index; coarse columns (entity, field) in that order.
    * S_i = D_i grown by `overlap` layers of the matrix graph.
    * A field with DOFs but none on Gamma (a discontinuous pressure) gets one
      column per subdomain instead, its null-space values on the subdomain's
      DOFs of that field, after the interface columns.
    """

    def __init__(self, A, field, dof_subs, null=None, overlap=1):
        A = A.tocsr()
        n = A.shape[0]
        field = np.asarray(field)
        self.dof_field = field
        self.dof_null = np.ones(n) if null is None else np.asarray(null, dtype=np.float64)
        subs = [tuple(int(v) for v in s) for s in dof_subs]
        self.n_sub = 1 + max(max(s) for s in subs if s)
        self.overlap = overlap
        self.box = [[] for _ in range(self.n_sub)]
        for d, s in enumerate(subs):
            for i in s:
                self.box[i].append(d)
        self.box = [np.array(b, dtype=np.int64) for b in self.box]
        mult = np.array([len(s) for s in subs])
        self.multiplicity = mult
        self.is_gamma = mult >= 2
        self.I = [b[~self.is_gamma[b]] for b in self.box]
        self.S = []
        for b in self.box:
            mark = np.zeros(n, dtype=bool)
            mark[b] = True
            for _ in range(overlap):
                rows = np.nonzero(mark)[0]
                mark[A[rows].indices] = True
            self.S.append(np.nonzero(mark)[0])
        g = np.nonzero(self.is_gamma)[0]
        cls = {}
        ent = np.empty(g.size, dtype=np.int64)
        for k, d in enumerate(g):           # ascending d: classes appear in order of their smallest DOF
            ent[k] = cls.setdefault(subs[d], len(cls))
        self.entity_sets = list(cls.keys())
        self.n_ent = len(cls)
        self.gamma = g
        self.gamma_entity = ent
        self.gamma_field = field[g]
        has = np.zeros((self.n_ent, 4), dtype=bool)
        has[self.gamma_entity, self.gamma_field] = True
        col = -np.ones((self.n_ent, 4), dtype=np.int64)
        col[has] = np.arange(has.sum())
        self.coarse_col = col
        self.n_coarse = int(has.sum())
        self.coarse_entity = np.repeat(np.arange(self.n_ent), 4).reshape(self.n_ent, 4)[has]
        self.coarse_field = np.tile(np.arange(4), (self.n_ent, 1))[has]
        self.sub_pressure_col = None
        if np.any(field == 3) and not np.any(self.gamma_field == 3) and self.n_sub > 1:
            self.sub_pressure_col = self.n_coarse + np.arange(self.n_sub)
            self.coarse_entity = np.concatenate([self.coarse_entity, self.n_ent + np.arange(self.n_sub)])
            self.coarse_field = np.concatenate([self.coarse_field, np.full(self.n_sub, 3)])
            self.n_coarse += self.n_sub

    def entity_subdomains(self, e):
        if e >= self.n_ent:
            return [int(e - self.n_ent)]
        return list(self.entity_sets[e])

    def local_sizes(self):
        return np.array([len(S) for S in self.S])
