"""Oracle: the RAS-PML fixed-point iteration (Algorithm 1, discrete form).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Section 2: from the current iterate, every subdomain solves its local
problem with the global residual restricted to it as data, and the new
iterate adds the partition-of-unity weighted sum of the local corrections:
    u^(n+1) = u^(n) + B^{-1} (b - A u^(n)),   B^{-1} = sum_j R~_j^T A_j^{-1} R_j.
Section 4 stops on the relative residual ||b - A u|| / ||b|| (rtol, at most
``maxit`` iterations).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class RichardsonResult:
    x: np.ndarray
    iters: int
    relres: float
    converged: bool
    history: list = field(default_factory=list)   # ||b - A u^(n)|| / ||b||, n = 0, 1, ...


def ras_richardson(matvec, apply_binv, b, x0=None, rtol=1e-6, maxit=500) -> RichardsonResult:
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return RichardsonResult(np.zeros_like(b), 0, 0.0, True, [0.0])
    r = b - matvec(x)
    hist = [np.linalg.norm(r) / bnorm]
    n = 0
    while hist[-1] > rtol and n < maxit:
        x = x + apply_binv(r)          # local solves, weighted sum (update1)
        r = b - matvec(x)
        hist.append(np.linalg.norm(r) / bnorm)
        n += 1
    return RichardsonResult(x, n, hist[-1], hist[-1] <= rtol, hist)
