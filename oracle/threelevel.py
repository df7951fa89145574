"""Three-level monolithic GDSW preconditioner (CPU, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

eq. (2.5): the two-level method is applied recursively to A_0, whose inverse
is replaced by

    Phi^(3) A_0^(3)^{-1} Phi^(3)^T + sum_j R_j^(2)^T A_j^(2)^{-1} R_j^(2)

on the N^(2) subregions; the first level is unchanged.

Readings (the paper defers the details to its references; all stated here and
pinned by ``tests/test_oracle_threelevel.py``):

* Subregion j is a group^3 block of subdomains (j = X + M (Y + M Z), M = m /
  group).  A level-2 coarse DOF belongs to every subregion that holds a
  subdomain of its entity.
* Level-2 local set of subregion j (default): the coarse DOFs of the
  subregion, i.e. of every entity that touches one of its subdomains;
  neighbouring subregions share their interface entities.  Alternative
  (``level2_layer``): plus one layer of the A_0 graph, every coarse DOF
  whose entity shares a subdomain with an entity of the subregion.
* Level-3 interface: coarse DOFs that belong to at least two subregions,
  classed by their subregion set; the level-3 null space is the indicator of
  one field (u_x, u_y, u_z or p) on a class.  Level-3 entities are ordered by
  their smallest coarse index.
* Phi^(3) is eq. (2.4) applied to A_0, and A_0^(3) = Phi^(3)^T A_0 Phi^(3).
* Apply order: level-1 local sum (ascending i); inside the coarse term, the
  level-2 local sum (ascending j) and then the level-3 correction.
* Level-2 local matrices, the subregion interior blocks of the level-3
  extension and A_0^(3) are factored like A_0: LU with partial pivoting.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .gdsw import TwoLevelGDSW


class ThreeLevelGDSW(TwoLevelGDSW):
    def __init__(self, A, dec, group, factor_local=True, level2_layer=False):
        super().__init__(A, dec, factor_local=factor_local)
        m = dec.m
        if m % group != 0:
            raise ValueError("m must be a multiple of group")
        self.group = group
        Ms = m // group
        self.n_subregions = Ms ** 3
        Nc = dec.n_coarse
        ent_sub = [dec.entity_subdomains(e) for e in range(dec.n_ent)]

        def subregion(i):
            I, J, K = i % m, (i // m) % m, i // (m * m)
            return I // group + Ms * (J // group + Ms * (K // group))

        c_ent = dec.coarse_entity
        c_field = dec.coarse_field
        c_subs = [set(ent_sub[c_ent[c]]) for c in range(Nc)]
        c_regions = [tuple(sorted({subregion(i) for i in s})) for s in c_subs]
        self.coarse_regions = c_regions

        # level-2 local sets with one layer of A_0-graph overlap
        self.S2 = []
        self.I2 = []
        for j in range(self.n_subregions):
            Cj = [c for c in range(Nc) if j in c_regions[c]]
            Tj = set()
            for c in Cj:
                Tj |= c_subs[c]
            Sj = [c for c in range(Nc) if c_subs[c] & Tj] if level2_layer else Cj
            self.S2.append(np.array(sorted(Sj), dtype=np.int64))
            self.I2.append(np.array([c for c in range(Nc) if c_regions[c] == (j,)],
                                    dtype=np.int64))

        # level-3 interface classes
        gam = [c for c in range(Nc) if len(c_regions[c]) >= 2]
        classes = {}
        for c in gam:
            classes.setdefault(c_regions[c], []).append(c)
        order = sorted(classes.values(), key=lambda cs: min(cs))
        col3 = {}
        rows_g, cols_g = [], []
        for E, cs in enumerate(order):
            for f in range(4):
                members = [c for c in cs if c_field[c] == f]
                if members:
                    col3[(E, f)] = len(col3)
                    rows_g += members
                    cols_g += [col3[(E, f)]] * len(members)
        self.n_coarse3 = len(col3)
        self.n_ent3 = len(order)
        Phi3 = np.zeros((Nc, self.n_coarse3))
        Phi3[rows_g, cols_g] = 1.0
        PhiG3 = Phi3.copy()
        A0 = self.A0
        for j in range(self.n_subregions):
            Ij = self.I2[j]
            if Ij.size == 0 or self.n_coarse3 == 0:
                continue
            rhs = A0[np.ix_(Ij, np.arange(Nc))] @ PhiG3
            fac = sla.lu_factor(A0[np.ix_(Ij, Ij)], check_finite=False)
            Phi3[Ij, :] = -sla.lu_solve(fac, rhs, check_finite=False)
        self.Phi3 = Phi3
        self.A03 = Phi3.T @ A0 @ Phi3
        f3 = np.zeros(self.n_coarse3, dtype=int)
        for (E, f), k in col3.items():
            f3[k] = f
        self.coarse3_field = f3
        self.A03_lu = sla.lu_factor(self.A03, check_finite=False) if self.n_coarse3 > 0 else None
        self.lu2 = []
        for S in self.S2:
            Aj = A0[np.ix_(S, S)]
            self.lu2.append(sla.lu_factor(Aj, check_finite=False))

    def coarse_solve(self, r0):
        """Replaces A_0^{-1}: level-2 local sum then the level-3 correction."""
        y = np.zeros_like(r0)
        for j, S in enumerate(self.S2):
            y[S] += sla.lu_solve(self.lu2[j], r0[S], check_finite=False)
        if self.A03_lu is not None:
            y += self.Phi3 @ sla.lu_solve(self.A03_lu, self.Phi3.T @ r0, check_finite=False)
        return y
