"""Oracle step O1: mesh, Cartesian covering, subdomain PML extension, PoU.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Paper passages followed:

* Section 1, definition of the extended domain Omega: the interior box
  Omega_int = (0,1)^2 is surrounded by a Cartesian PML of thickness kappa_g.
  On a uniform mesh of width h this is N_c = n_int + 2G cells per side with
  node coordinates x_i = (i - G) h, i = 0..N_c.  Unknowns are the interior
  nodes 1..N_c-1 (u in H^1_0(Omega)).
* Section 2, "Cartesian covering": a non-overlapping Cartesian partition is
  extended by the overlap delta to give Omega_{j,int}; every side of
  Omega_{j,int} that does not lie on the boundary of Omega is extended by a
  PML layer of thickness kappa, giving Omega_j.
* Section 2, partition of unity: sum_j chi_j = 1, supp chi_j inside
  Omega_{j,int}, chi_j = 1 on the non-overlapped part.  Section 4 says the
  experiments use tensor products of 1D functions that vary linearly across
  the overlaps.

Readings where the paper is silent (all in cell units):

* cuts c_p = floor(p N_c / P);
* Omega_{p,int} = [max(0, c_p - delta), min(N_c, c_{p+1} + delta)];
* the PML of thickness kappa is added on a side iff that side of
  Omega_{p,int} is not on the boundary of Omega, and Omega_p is clipped to
  [0, N_c];
* 1D PoU weight: product of a left ramp (0 at c_p - delta, 1 at c_p + delta)
  and a right ramp (1 at c_{p+1} - delta, 0 at c_{p+1} + delta), no ramp on a
  side at the boundary of Omega, normalised so the weights sum to one;
  the Boolean variant gives node i to the chunk with c_p <= i < c_{p+1};
* with the impedance condition the nodes on the interior boundary
  Gamma_j = boundary(Omega_j) minus boundary(Omega) are unknowns; with the
  Dirichlet condition they are not; nodes on the boundary of Omega are never
  unknowns;
* the local unknowns are numbered with the shorter side fastest, which gives
  the half-bandwidth b = n_fast + 1 (the P1 diagonal couples r and
  r + n_fast + 1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BC_IMP = 0
BC_DRCH = 1
POU_LINEAR = 0
POU_BOOLEAN = 1


@dataclass
class Problem:
    """Parameters of one RAS-PML problem (all widths in mesh cells)."""

    k: float
    n_int: int               # cells of Omega_int per side (h = 1/n_int)
    G: int                   # global PML cells
    Px: int
    Py: int
    delta: int               # overlap cells
    kappa: int               # subdomain PML cells
    sigma: float             # g(x) = sigma x^3
    bc: int = BC_IMP
    pou: int = POU_LINEAR

    @property
    def h(self) -> float:
        return 1.0 / self.n_int

    @property
    def Nc(self) -> int:
        return self.n_int + 2 * self.G

    @property
    def ndof_side(self) -> int:
        return self.Nc - 1

    @property
    def ndof(self) -> int:
        return (self.Nc - 1) ** 2

    def node_x(self, i):
        """Coordinate of node index i (Section 1: Omega = (-kappa_g, 1+kappa_g))."""
        return (np.asarray(i, dtype=np.float64) - self.G) * self.h


def paper_width_cells(k: float, h: float, C: float, k0: float = 150.0) -> int:
    """Section 3 (iii): a width of C l(k) wavelengths, l(k) = k/(k - k0) log2(k/k0)
    (its limit 1/ln 2 at k = k0), in mesh cells of width h (rounded down)."""
    lk = 1.0 / math.log(2.0) if k == k0 else k / (k - k0) * math.log2(k / k0)
    return int(math.floor(C * lk * (2.0 * math.pi / k) / h + 1e-9))


def log_width(k: float, h: float) -> int:
    """Overlap / PML width ceil(ln k / (k h)) in mesh layers (natural log)."""
    return int(math.ceil(math.log(k) / (k * h) - 1e-12))


@dataclass
class Chunk1D:
    p: int
    c_lo: int
    c_hi: int
    int_lo: int
    int_hi: int
    pml_lo: int
    pml_hi: int
    box_lo: int
    box_hi: int
    u_lo: int        # first local unknown node
    u_hi: int        # last local unknown node (inclusive)
    imp_lo: bool     # lower side of Omega_j lies on Gamma_j
    imp_hi: bool

    @property
    def n(self) -> int:
        return self.u_hi - self.u_lo + 1


def chunks_1d(Nc: int, P: int, delta: int, kappa: int, bc: int) -> list[Chunk1D]:
    """Section 2 covering along one axis."""
    out = []
    for p in range(P):
        c_lo = (p * Nc) // P
        c_hi = ((p + 1) * Nc) // P
        int_lo = max(0, c_lo - delta)
        int_hi = min(Nc, c_hi + delta)
        pml_lo = kappa if int_lo > 0 else 0
        pml_hi = kappa if int_hi < Nc else 0
        box_lo = max(0, int_lo - pml_lo)
        box_hi = min(Nc, int_hi + pml_hi)
        imp_lo = box_lo > 0
        imp_hi = box_hi < Nc
        if bc == BC_IMP:
            u_lo = max(box_lo, 1)
            u_hi = min(box_hi, Nc - 1)
        else:
            u_lo = box_lo + 1
            u_hi = box_hi - 1
        out.append(Chunk1D(p, c_lo, c_hi, int_lo, int_hi, pml_lo, pml_hi,
                           box_lo, box_hi, u_lo, u_hi, imp_lo and bc == BC_IMP,
                           imp_hi and bc == BC_IMP))
    return out


def pou_1d(Nc: int, chunks: list[Chunk1D], delta: int, kind: int) -> np.ndarray:
    """1D partition of unity, shape (P, Nc+1) over node indices 0..Nc."""
    i = np.arange(Nc + 1, dtype=np.float64)
    P = len(chunks)
    w = np.zeros((P, Nc + 1))
    for ch in chunks:
        if kind == POU_BOOLEAN:
            w[ch.p] = ((i >= ch.c_lo) & (i < ch.c_hi)).astype(np.float64)
            if ch.p == P - 1:
                w[ch.p, Nc] = 1.0
            continue
        if ch.int_lo > 0:
            if delta > 0:
                left = np.clip((i - (ch.c_lo - delta)) / (2.0 * delta), 0.0, 1.0)
            else:
                left = (i >= ch.c_lo).astype(np.float64)
        else:
            left = np.ones_like(i)
        if ch.int_hi < Nc:
            if delta > 0:
                right = np.clip(((ch.c_hi + delta) - i) / (2.0 * delta), 0.0, 1.0)
            else:
                right = (i <= ch.c_hi).astype(np.float64)
        else:
            right = np.ones_like(i)
        w[ch.p] = left * right
    s = w.sum(axis=0)
    return w / s[None, :]


@dataclass
class Subdomain:
    j: int
    px: Chunk1D
    py: Chunk1D
    nx: int
    ny: int
    x_fast: bool
    nodes_i: np.ndarray = field(repr=False)   # global node i of local unknown r
    nodes_j: np.ndarray = field(repr=False)

    @property
    def n(self) -> int:
        return self.nx * self.ny

    @property
    def n_fast(self) -> int:
        return self.nx if self.x_fast else self.ny

    @property
    def band(self) -> int:
        """Half-bandwidth of A_j in the local ordering."""
        return self.n_fast + 1

    def local_index(self, i, j):
        i = np.asarray(i)
        j = np.asarray(j)
        if self.x_fast:
            return (j - self.py.u_lo) * self.nx + (i - self.px.u_lo)
        return (i - self.px.u_lo) * self.ny + (j - self.py.u_lo)


def subdomains(pb: Problem) -> list[Subdomain]:
    cx = chunks_1d(pb.Nc, pb.Px, pb.delta, pb.kappa, pb.bc)
    cy = chunks_1d(pb.Nc, pb.Py, pb.delta, pb.kappa, pb.bc)
    out = []
    for q in range(pb.Py):
        for p in range(pb.Px):
            a, b = cx[p], cy[q]
            nx, ny = a.n, b.n
            x_fast = nx <= ny
            ii = np.arange(a.u_lo, a.u_hi + 1)
            jj = np.arange(b.u_lo, b.u_hi + 1)
            if x_fast:
                J, I = np.meshgrid(jj, ii, indexing="ij")
            else:
                I, J = np.meshgrid(ii, jj, indexing="ij")
            out.append(Subdomain(q * pb.Px + p, a, b, nx, ny, x_fast,
                                 I.ravel(), J.ravel()))
    return out


def global_index(pb: Problem, i, j):
    """Global unknown index of node (i, j): x fastest, interior nodes only."""
    return (np.asarray(j) - 1) * (pb.Nc - 1) + (np.asarray(i) - 1)


def pou_2d(pb: Problem):
    """Per-subdomain chi_j evaluated at the local unknowns (tensor product)."""
    cx = chunks_1d(pb.Nc, pb.Px, pb.delta, pb.kappa, pb.bc)
    cy = chunks_1d(pb.Nc, pb.Py, pb.delta, pb.kappa, pb.bc)
    wx = pou_1d(pb.Nc, cx, pb.delta, pb.pou)
    wy = pou_1d(pb.Nc, cy, pb.delta, pb.pou)
    return wx, wy


def config_problem(name: str, sigma_literal: bool = False) -> Problem:
    """The workload families used by the tests and the benchmark.

    ``sigma_literal`` selects g(x) = 10 x^3 instead of the paper's 10 k x^3.
    """
    def mk(k, n_int, P, G=None):
        L = log_width(k, 1.0 / n_int)
        g = L if G is None else G
        sig = 10.0 if sigma_literal else 10.0 * k
        return Problem(k=k, n_int=n_int, G=g, Px=P, Py=P, delta=L, kappa=L, sigma=sig)

    if name == "k20":
        return mk(20.0, 40, 2, G=4)
    if name == "k160":
        return mk(160.0, 320, 16)
    if name == "k640":
        return mk(640.0, 1280, 32)
    raise ValueError(name)
