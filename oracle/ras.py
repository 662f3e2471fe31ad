"""Oracle step O7: the RAS-PML preconditioner.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Section 2, discrete RAS: each local correction solves the local operator
A_j (the form a restricted to the PML-extended subdomain Omega_j, with the
local stretch) against the global residual restricted to the local unknowns
(eq. (local-ras-discrete)); the corrections are summed with the partition of
unity chi_j (eq. (update1)).  As a preconditioner this is

    B^{-1} v = sum_j  R~_j^T  A_j^{-1}  R_j v

with R_j the Boolean restriction to the local unknowns of subdomain j and
R~_j^T the extension by zero weighted by chi_j.
"""
from __future__ import annotations

import numpy as np

from . import band, fem, geometry
from .geometry import Problem


class ZeroPivot(RuntimeError):
    pass


class RasPml:
    """Assembled global operator, every local factorisation, and B^{-1}.

    ``subset`` restricts the local factorisations to the listed subdomain
    ids (used to sample very large problems); ``apply`` then sums only those
    subdomains' contributions, and ``local_solve`` works for them alone.
    """

    def __init__(self, pb: Problem, subset=None, with_global: bool = True,
                 tol_rel: float = 1e-14):
        self.pb = pb
        if with_global:
            self.A, self.M1 = fem.assemble_global(pb)
        self.sds_all = geometry.subdomains(pb)
        ids = range(len(self.sds_all)) if subset is None else list(subset)
        self.ids = list(ids)
        self.sds = [self.sds_all[j] for j in self.ids]
        self.wx, self.wy = geometry.pou_2d(pb)
        self.local = [fem.assemble_local(pb, sd) for sd in self.sds]
        self.batch = band.BandBatch(self.local, [sd.band for sd in self.sds], tol_rel)
        bad = np.nonzero(self.batch.status)[0]
        if len(bad):
            m = int(bad[0])
            raise ZeroPivot("zero pivot in subdomain %d at column %d"
                            % (self.ids[m], self.batch.status[m] - 1))
        self.gidx = np.concatenate([geometry.global_index(pb, sd.nodes_i, sd.nodes_j)
                                    for sd in self.sds])
        self.chi = np.concatenate([self.wx[sd.px.p][sd.nodes_i] * self.wy[sd.py.p][sd.nodes_j]
                                   for sd in self.sds])

    def restrict(self, v):
        """R_j v for every subdomain, back to back."""
        return np.asarray(v, dtype=np.complex128)[self.gidx]

    def local_solve(self, v):
        """A_j^{-1} R_j v for every subdomain, back to back."""
        return self.batch.solve_all(self.restrict(v))

    def local_part(self, vec, m):
        o = self.batch.voff[m]
        return vec[o:o + self.batch.n[m]]

    def apply(self, v, weighted: bool = True):
        """z = sum_j R~_j^T A_j^{-1} R_j v.  With ``weighted=False`` the plain
        extension R_j^T replaces R~_j^T (the additive Schwarz operator)."""
        x = self.local_solve(v)
        z = np.zeros(self.pb.ndof, dtype=np.complex128)
        np.add.at(z, self.gidx, (self.chi * x) if weighted else x)
        return z
