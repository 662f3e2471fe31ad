"""Oracle step O8: restarted GMRES(m), right preconditioned.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Section 4.1 uses the RAS-PML iteration as a preconditioner for GMRES and
stops on the relative residual.  This is textbook right-preconditioned
GMRES: the Arnoldi process runs on A B^{-1} with modified Gram-Schmidt,
the least-squares problem is reduced by complex Givens rotations, a cycle
ends when the rotated residual estimate |g_{j+1}| reaches rtol ||b||, and the
iterate is x = x0 + B^{-1} V y.  The true residual ||b - A x|| is recomputed
at the end of every cycle; the run stops when it is <= rtol ||b|| or after
``maxit`` Arnoldi steps in total.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class GmresResult:
    x: np.ndarray
    iters: int
    relres: float
    converged: bool
    history: list = field(default_factory=list)    # estimate after each step
    true_history: list = field(default_factory=list)


def givens(a: complex, b: float):
    """Rotation [[c, s], [-conj(s), c]] (c real) with G [a; b] = [r; 0]."""
    if b == 0.0:
        return 1.0, 0.0 + 0.0j
    if a == 0:
        return 0.0, 1.0 + 0.0j
    rho = np.hypot(abs(a), b)
    c = abs(a) / rho
    s = (a / abs(a)) * b / rho
    return c, s


def gmres(matvec, precond, b, x0=None, rtol=1e-6, restart=50, maxit=500):
    b = np.asarray(b, dtype=np.complex128)
    n = b.shape[0]
    x = np.zeros(n, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return GmresResult(np.zeros(n, dtype=np.complex128), 0, 0.0, True)
    hist, true_hist = [], []
    total = 0
    r = b - matvec(x)
    beta = np.linalg.norm(r)
    true_hist.append(beta / bnorm)
    while True:
        if beta <= rtol * bnorm:
            return GmresResult(x, total, beta / bnorm, True, hist, true_hist)
        if total >= maxit:
            return GmresResult(x, total, beta / bnorm, False, hist, true_hist)
        m = min(restart, maxit - total)
        V = np.zeros((m + 1, n), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            w = matvec(precond(V[j]))
            for i in range(j + 1):                       # modified Gram-Schmidt
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            hn = np.linalg.norm(w)
            H[j + 1, j] = hn
            for i in range(j):                           # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            cs[j], sn[j] = givens(H[j, j], H[j + 1, j].real)
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            total += 1
            k = j + 1
            hist.append(abs(g[j + 1]) / bnorm)
            breakdown = hn <= 1e-14 * np.linalg.norm(H[: j + 2, j])
            if abs(g[j + 1]) <= rtol * bnorm or breakdown:
                break
            V[j + 1] = w / hn
        y = np.zeros(k, dtype=np.complex128)
        for i in range(k - 1, -1, -1):                   # R y = g
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + precond(V[:k].T @ y)
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        true_hist.append(beta / bnorm)
