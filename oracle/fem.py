"""Oracle steps O2-O5: PML stretch, P1 assembly of A and A_j, RHS.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Paper passages followed:

* Section 1: g(x) = g'(x) = 0 for x <= 0, g' > 0 beyond; per-axis profile
  g_i is g(x - b) above the interior box and -g(a - x) below it; the stretch
  is gamma_i = 1 + i g_i'.  Section 4 fixes g(x) = 10 k x^3; we keep the
  coefficient sigma in g(x) = sigma x^3 as a parameter, so
  gamma = 1 + 3 i sigma d^2 with d the distance into the PML on that axis.
* Section 2, local scaling function: inside (a_j, b_j) the local profile is
  the global one; beyond b_j (resp. below a_j) it is g(x - b_j)
  (resp. -g(a_j - x)) on sides that carry an added PML.
* Section 1 eq. (pml)/(weak): the PML operator sum_i (gamma_i^{-1} d_i)^2.
  We use its complex-symmetric weak form, obtained by multiplying the PDE by
  gamma_1 gamma_2 (same PDE, since gamma_i depends on x^i only):
      a(u,v) = int (g2/g1) u_x v_x + (g1/g2) u_y v_y - k^2 g1 g2 u v.
  (The non-symmetric form printed in the paper equals this form tested with
  gamma_1 gamma_2 v; the two agree outside the PML.)
* Section 4 uses a uniform mesh; we use P1 elements on right triangles,
  every square cell cut along its SW-NE diagonal, coefficients evaluated at
  the triangle centroid, exact P1 element matrices for those constants.
* Section 3 (ii) eq. (impedance): d_nu u - i k u = 0 on the subdomain
  boundary as a natural condition.  In stretched coordinates the boundary
  term of the symmetric form is -i k int_Gamma gamma_t u v ds, with gamma_t
  the stretch tangential to the edge, evaluated at the edge midpoint.  It is
  imposed on Gamma_j = boundary(Omega_j) minus boundary(Omega) only.
* Right-hand side int f v with f replaced by its nodal interpolant: b = M f
  with the unweighted P1 mass matrix (f is negligible in every PML).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .geometry import Problem, Subdomain, Chunk1D, global_index


# ---------------------------------------------------------------- stretch
def gamma_global(pb: Problem, x):
    """gamma(x) = 1 + i g'(x), g' = 3 sigma d^2, d = distance to [0, 1]."""
    x = np.asarray(x, dtype=np.float64)
    d = np.maximum(0.0, np.maximum(-x, x - 1.0))
    return 1.0 + 1j * 3.0 * pb.sigma * d * d


def gamma_local(pb: Problem, ch: Chunk1D, x):
    """Local stretch gamma^{(j)} along one axis (Section 2)."""
    x = np.asarray(x, dtype=np.float64)
    a = pb.node_x(ch.int_lo)
    b = pb.node_x(ch.int_hi)
    g = gamma_global(pb, x)
    if ch.pml_hi > 0:
        d = x - b
        g = np.where(x >= b, 1.0 + 1j * 3.0 * pb.sigma * d * d, g)
    if ch.pml_lo > 0:
        d = a - x
        g = np.where(x <= a, 1.0 + 1j * 3.0 * pb.sigma * d * d, g)
    return g


# ---------------------------------------------------------------- elements
def _triangles(pb: Problem, ci, cj):
    """The two P1 triangles of every cell (ci, cj): vertex node indices
    (ntri, 3, 2) and vertex coordinates (ntri, 3, 2)."""
    ci = np.asarray(ci).ravel()
    cj = np.asarray(cj).ravel()
    # lower-right triangle: SW, SE, NE ; upper-left triangle: SW, NE, NW
    lo = np.stack([np.stack([ci, cj], -1), np.stack([ci + 1, cj], -1),
                   np.stack([ci + 1, cj + 1], -1)], axis=1)
    up = np.stack([np.stack([ci, cj], -1), np.stack([ci + 1, cj + 1], -1),
                   np.stack([ci, cj + 1], -1)], axis=1)
    nodes = np.concatenate([lo, up], axis=0)
    xy = pb.node_x(nodes)
    return nodes, xy


def _p1_element_matrices(xy, cx, cy, cm, k):
    """Element matrices of a(u,v) for P1 on triangles with constant
    coefficients: K = |T|(cx gx gx^T + cy gy gy^T), M = cm |T|/12 [2 1 1;...]."""
    x1, y1 = xy[:, 0, 0], xy[:, 0, 1]
    x2, y2 = xy[:, 1, 0], xy[:, 1, 1]
    x3, y3 = xy[:, 2, 0], xy[:, 2, 1]
    det = (x2 - x1) * (y3 - y1) - (x3 - x1) * (y2 - y1)
    area = 0.5 * np.abs(det)
    # gradients of the barycentric basis functions
    gx = np.stack([y2 - y3, y3 - y1, y1 - y2], axis=1) / det[:, None]
    gy = np.stack([x3 - x2, x1 - x3, x2 - x1], axis=1) / det[:, None]
    K = area[:, None, None] * (cx[:, None, None] * gx[:, :, None] * gx[:, None, :]
                               + cy[:, None, None] * gy[:, :, None] * gy[:, None, :])
    mref = (np.ones((3, 3)) + np.eye(3)) / 12.0
    M = (cm * area)[:, None, None] * mref[None]
    return K - (k * k) * M, M


def _coefficients(g1, g2):
    """Coefficients of the symmetric PML form at a point: g2/g1, g1/g2, g1 g2."""
    return g2 / g1, g1 / g2, g1 * g2


def _scatter(nodes, Ae, index_of, n):
    """Assemble element matrices; nodes without an index (-1) are Dirichlet."""
    idx = index_of(nodes[..., 0], nodes[..., 1])          # (ntri, 3)
    rows = np.repeat(idx[:, :, None], 3, axis=2)
    cols = np.repeat(idx[:, None, :], 3, axis=1)
    keep = (rows >= 0) & (cols >= 0)
    A = sp.coo_matrix((Ae[keep], (rows[keep], cols[keep])), shape=(n, n))
    return A.tocsr()


def _global_index_of(pb: Problem):
    Nc = pb.Nc

    def f(i, j):
        inside = (i >= 1) & (i <= Nc - 1) & (j >= 1) & (j <= Nc - 1)
        return np.where(inside, global_index(pb, i, j), -1)
    return f


def assemble_global(pb: Problem):
    """Global A = K - k^2 M (complex symmetric), and the unweighted mass M1,
    both restricted to the unknowns (Dirichlet on the boundary of Omega)."""
    Nc = pb.Nc
    ci, cj = np.meshgrid(np.arange(Nc), np.arange(Nc), indexing="ij")
    nodes, xy = _triangles(pb, ci, cj)
    cen = xy.mean(axis=1)
    g1 = gamma_global(pb, cen[:, 0])
    g2 = gamma_global(pb, cen[:, 1])
    cx, cy, cm = _coefficients(g1, g2)
    Ae, _ = _p1_element_matrices(xy, cx, cy, cm, pb.k)
    ones = np.ones(len(cen), dtype=np.complex128)
    _, M1e = _p1_element_matrices(xy, ones, ones, ones, 0.0)
    idx = _global_index_of(pb)
    A = _scatter(nodes, Ae, idx, pb.ndof)
    M1 = _scatter(nodes, M1e, idx, pb.ndof)
    return A, M1


def assemble_local(pb: Problem, sd: Subdomain):
    """Local operator A_j of the PML-truncated subdomain problem, in the
    local ordering (shorter side fastest), as a CSR matrix."""
    px, py = sd.px, sd.py
    ci, cj = np.meshgrid(np.arange(px.box_lo, px.box_hi),
                         np.arange(py.box_lo, py.box_hi), indexing="ij")
    nodes, xy = _triangles(pb, ci, cj)
    cen = xy.mean(axis=1)
    g1 = gamma_local(pb, px, cen[:, 0])
    g2 = gamma_local(pb, py, cen[:, 1])
    cx, cy, cm = _coefficients(g1, g2)
    Ae, _ = _p1_element_matrices(xy, cx, cy, cm, pb.k)

    def idx(i, j):
        inside = (i >= px.u_lo) & (i <= px.u_hi) & (j >= py.u_lo) & (j <= py.u_hi)
        return np.where(inside, sd.local_index(i, j), -1)

    A = _scatter(nodes, Ae, idx, sd.n)
    return (A + impedance_local(pb, sd, idx)).tocsr()


def impedance_local(pb: Problem, sd: Subdomain, idx):
    """-i k int_{Gamma_j} gamma_t u v ds with P1 edge mass h/6 [2 1; 1 2]."""
    px, py = sd.px, sd.py
    h = pb.h
    emass = np.array([[2.0, 1.0], [1.0, 2.0]]) * h / 6.0
    edges = []   # list of (node_a (m,2), node_b (m,2), gamma_t (m,))
    # vertical sides x = const: edges (X, m)-(X, m+1), tangential stretch in y
    ms = np.arange(py.box_lo, py.box_hi)
    ymid = pb.node_x(ms) + 0.5 * h
    for on, X in ((px.imp_lo, px.box_lo), (px.imp_hi, px.box_hi)):
        if on:
            a = np.stack([np.full_like(ms, X), ms], -1)
            b = np.stack([np.full_like(ms, X), ms + 1], -1)
            edges.append((a, b, gamma_local(pb, py, ymid)))
    ms = np.arange(px.box_lo, px.box_hi)
    xmid = pb.node_x(ms) + 0.5 * h
    for on, Y in ((py.imp_lo, py.box_lo), (py.imp_hi, py.box_hi)):
        if on:
            a = np.stack([ms, np.full_like(ms, Y)], -1)
            b = np.stack([ms + 1, np.full_like(ms, Y)], -1)
            edges.append((a, b, gamma_local(pb, px, xmid)))
    n = sd.n
    B = sp.csr_matrix((n, n), dtype=np.complex128)
    for a, b, gt in edges:
        ia = idx(a[:, 0], a[:, 1])
        ib = idx(b[:, 0], b[:, 1])
        E = (-1j * pb.k * gt)[:, None, None] * emass[None]
        nodes = np.stack([np.stack([ia, ib], -1)], 0)[0]
        rows = np.repeat(nodes[:, :, None], 2, axis=2)
        cols = np.repeat(nodes[:, None, :], 2, axis=1)
        keep = (rows >= 0) & (cols >= 0)
        B = B + sp.coo_matrix((E[keep], (rows[keep], cols[keep])), shape=(n, n)).tocsr()
    return B


def rhs(M1, f_dof):
    """b = M f_I (unweighted consistent mass times the nodal source)."""
    return M1 @ np.asarray(f_dof, dtype=np.complex128)
