"""Seeded synthetic inputs shared by the oracle, the HIP path, the tests and the benchmark.

This module holds no arithmetic of the multigrid method: it only draws random
numbers and evaluates the analytic data functions at grid vertices.  Vertex
(i, j) of a level with n = 2^k cells per side sits at (i/n, j/n) and has the
index j*(n+1)+i.

The paper fixes no data (its experiments use a zero right-hand side and a
random initial guess, section 3), so every workload is synthetic:

* desired state y_D = sum of 8 products sin(k pi x) sin(l pi y), the 8 mode
  pairs drawn without replacement from {1..8}^2, coefficients N(0,1);
* random vectors i.i.d. uniform on [-1, 1];
* batches of instances with side 2^k+1, k in {8, 9, 10} and alpha
  log-uniform in [1e-8, 1];
* Stokes desired velocity v_D = (d psi/dy, -d psi/dx) for a stream function
  psi of the same sine-mode form (divergence-free by construction).
"""
from __future__ import annotations

import numpy as np


def grid_coords(level: int):
    n = 1 << level
    t = np.arange(n + 1, dtype=np.float64) / n
    X, Y = np.meshgrid(t, t, indexing="xy")  # X[j, i] = i/n, Y[j, i] = j/n
    return X.ravel(), Y.ravel()


def sine_modes(seed: int, count: int = 8, kmax: int = 8):
    rng = np.random.default_rng(seed)
    idx = rng.choice(kmax * kmax, count, replace=False)
    kk = 1 + idx // kmax
    ll = 1 + idx % kmax
    c = rng.standard_normal(count)
    return kk, ll, c


def desired_state(level: int, seed: int) -> np.ndarray:
    """Nodal values of y_D on level `level` (length (2^level+1)^2)."""
    X, Y = grid_coords(level)
    kk, ll, c = sine_modes(seed)
    yd = np.zeros_like(X)
    for k, l, a in zip(kk, ll, c):
        yd += a * np.sin(k * np.pi * X) * np.sin(l * np.pi * Y)
    return yd


def uniform(n: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n)


def batch_instances(count: int = 64, seed: int = 3, levels=(8, 9, 10), log_alpha=(-8.0, 0.0)):
    """List of (level, alpha, y_D seed) for a batch of independent instances."""
    rng = np.random.default_rng(seed)
    lv = rng.choice(np.asarray(levels), count)
    al = 10.0 ** rng.uniform(log_alpha[0], log_alpha[1], count)
    return [(int(lv[b]), float(al[b]), 3000 + b) for b in range(count)]


def stream_function_velocity(X: np.ndarray, Y: np.ndarray, seed: int):
    """(v1, v2) = (d psi/dy, -d psi/dx) at the points (X, Y), psi of sine-mode form."""
    kk, ll, c = sine_modes(seed)
    v1 = np.zeros_like(X)
    v2 = np.zeros_like(X)
    for k, l, a in zip(kk, ll, c):
        v1 += a * l * np.pi * np.sin(k * np.pi * X) * np.cos(l * np.pi * Y)
        v2 -= a * k * np.pi * np.cos(k * np.pi * X) * np.sin(l * np.pi * Y)
    return v1, v2


def p2_interior_coords(level: int):
    """Points of the interior nodes of the half-step lattice of a level with
    n = 2^level cells per side: (a/(2n), b/(2n)) for 1 <= a, b <= 2n-1, in the
    order (b-1)(2n-1) + (a-1) (the velocity unknowns of the Stokes problem)."""
    n = 1 << level
    t = np.arange(1, 2 * n, dtype=np.float64) / (2 * n)
    X, Y = np.meshgrid(t, t, indexing="xy")
    return X.ravel(), Y.ravel()


def desired_velocity(level: int, seed: int) -> np.ndarray:
    """[v1 | v2] of the divergence-free desired velocity at the interior P2 nodes."""
    v1, v2 = stream_function_velocity(*p2_interior_coords(level), seed)
    return np.concatenate([v1, v2])
