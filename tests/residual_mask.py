"""Where one fixed-point step annihilates the residual (Section 3 (i)).

After u <- u + B^{-1}(b - A u), the residual vanishes at every unknown whose
stencil lies inside the region where a single subdomain's PoU weight is 1
and the rows of its local operator coincide with those of A: there the new
iterate is the old one plus that subdomain's correction, which solves the
local equations exactly.  The set is computed from the PoU and the matrices
alone, independently of any solve."""
import numpy as np

from oracle import geometry


def annihilation_set(R, check_rows=True):
    pb = R.pb
    A = R.A.tocsr()
    n = pb.ndof
    out = np.zeros(n, bool)
    for m, sd in enumerate(R.sds):
        g = geometry.global_index(pb, sd.nodes_i, sd.nodes_j)
        chi = R.wx[sd.px.p][sd.nodes_i] * R.wy[sd.py.p][sd.nodes_j]
        one = np.zeros(n, bool)
        one[g[chi == 1.0]] = True
        loc = -np.ones(n, np.int64)
        loc[g] = np.arange(len(g))
        Am = R.local[m].tocsr()
        for r in np.nonzero(chi == 1.0)[0]:
            gg = g[r]
            cols = A.indices[A.indptr[gg]:A.indptr[gg + 1]]
            if not one[cols].all():
                continue
            if check_rows:
                vals = A.data[A.indptr[gg]:A.indptr[gg + 1]]
                lc = Am.indices[Am.indptr[r]:Am.indptr[r + 1]]
                lv = Am.data[Am.indptr[r]:Am.indptr[r + 1]]
                a = {c: v for c, v in zip(loc[cols].tolist(), vals.tolist()) if v != 0}
                b = {c: v for c, v in zip(lc.tolist(), lv.tolist()) if v != 0}
                if a.keys() != b.keys() or any(abs(a[c] - b[c]) > 1e-13 * abs(a[c]) for c in a):
                    continue
            out[gg] = True
    return out
