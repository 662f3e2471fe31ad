"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no arithmetic of the solver: it only evaluates source
functions at mesh nodes and draws random vectors.  Nodes are
x_i = (i - G) h for i = 1..Nc-1 (x fastest), the unknowns of the Dirichlet
problem on the PML-extended square.

Sources:

* ``gaussian`` -- sum of a_s exp(-|x - c_s|^2 / w^2) (fixed-width Gaussians);
* ``paper``    -- the smoothed delta of the paper's experiments (Section 4):
  (16 k^2 / pi^3) exp(-16 k^2 |x - x_c|^2 / pi^2) at x_c = (0.5, 0.5);
* ``batch_draw`` -- a seeded multi-source problem: k from {40, 80, 160},
  1-4 Gaussians of width 0.03 with centres uniform in (0.2, 0.8)^2 and complex
  amplitudes |a| ~ U(0.5, 1) with uniform phase.
"""
from __future__ import annotations

import numpy as np


def node_coords(n_int: int, G: int):
    Nc = n_int + 2 * G
    h = 1.0 / n_int
    x = (np.arange(1, Nc, dtype=np.float64) - G) * h
    return x


def gaussian(n_int: int, G: int, centers, amps, width: float) -> np.ndarray:
    x = node_coords(n_int, G)
    X, Y = np.meshgrid(x, x, indexing="xy")     # row = y, column = x (x fastest)
    f = np.zeros(X.shape, dtype=np.complex128)
    for (cx, cy), a in zip(np.atleast_2d(centers), np.atleast_1d(amps)):
        f += a * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (width * width))
    return f.ravel()


def centre_gaussian(n_int: int, G: int, width: float = 0.05) -> np.ndarray:
    return gaussian(n_int, G, [(0.5, 0.5)], [1.0], width)


def paper(k: float, n_int: int, G: int) -> np.ndarray:
    x = node_coords(n_int, G)
    X, Y = np.meshgrid(x, x, indexing="xy")
    r2 = (X - 0.5) ** 2 + (Y - 0.5) ** 2
    f = (16.0 * k * k / np.pi ** 3) * np.exp(-16.0 * k * k * r2 / np.pi ** 2)
    return f.ravel().astype(np.complex128)


def batch_draw(seed: int):
    """Draw order: k, number of sources, centres, |a|, phase."""
    rng = np.random.default_rng(seed)
    k = float(rng.choice([40, 80, 160]))
    ns = int(rng.integers(1, 5))
    centres = rng.uniform(0.2, 0.8, (ns, 2))
    mag = rng.uniform(0.5, 1.0, ns)
    phase = rng.uniform(0.0, 2.0 * np.pi, ns)
    return {"k": k, "centres": centres, "amps": mag * np.exp(1j * phase), "width": 0.03}


def random_vector(n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def batch_source(n_int: int, G: int, draw) -> np.ndarray:
    """Nodal values of a ``batch_draw`` source on the given mesh."""
    return gaussian(n_int, G, draw["centres"], draw["amps"], draw["width"])


def warm_draw(seed: int, k: float = 320.0, width: float = 0.03):
    """A seeded source for the learned warm start: fixed k, then the draws of
    ``batch_draw`` after k (number of sources, centres, |a|, phase)."""
    rng = np.random.default_rng(seed)
    ns = int(rng.integers(1, 5))
    centres = rng.uniform(0.2, 0.8, (ns, 2))
    mag = rng.uniform(0.5, 1.0, ns)
    phase = rng.uniform(0.0, 2.0 * np.pi, ns)
    return {"k": float(k), "centres": centres, "amps": mag * np.exp(1j * phase), "width": width}


def warm_draw_narrow(seed: int, k: float = 320.0):
    """``warm_draw`` with the paper's smoothed point source (Section 4) in
    place of each Gaussian: width pi / (4 k) and peak 16 k^2 / pi^3 times the
    drawn amplitude."""
    d = warm_draw(seed, k, width=np.pi / (4.0 * k))
    d["amps"] = d["amps"] * (16.0 * k * k / np.pi ** 3)
    return d


def ws_init_weights(shapes, seed: int, gain: float = 1.0) -> np.ndarray:
    """Seeded He-normal weights for a list of (cin, cout) 3 x 3 convolutions,
    each W[ky][kx][cin][cout], concatenated as float32."""
    rng = np.random.default_rng(seed)
    parts = [rng.standard_normal(9 * ci * co) * gain * np.sqrt(2.0 / (9 * ci)) for ci, co in shapes]
    return np.concatenate(parts).astype(np.float32)
