"""Seeded synthetic inputs for the range-space Schur solve.

This module only generates input data (targets ybar, boundary data y_c and
random vectors).  It holds none of the solver's arithmetic and imports nothing
else from this package, so the CPU oracle's tests and the GPU path can both be
fed the very same arrays.

Node numbering convention (documented in include/sfdp.h):
* free node (i, j[, k]) with 1 <= i, j, k <= N-1 has index
  (i-1) + (N-1)(j-1) [+ (N-1)^2 (k-1)], x fastest;
* boundary nodes are the full-grid nodes (0 <= i, j, k <= N) on the boundary,
  in increasing full id i + (N+1) j [+ (N+1)^2 k].

Recipes
-------
``modes_for(kind, seed)``: sine-mode targets of the paper's thermal workload
family on the unit square/cube (Sec. 6.1 uses a smooth target on [0,1]^2;
these synthetic targets are sums of sin(k pi x) sin(l pi y) [sin(q pi z)]
with N(0,1) coefficients):
* "four2d":    4 distinct (k, l) drawn without replacement from {1..4}^2;
* "sixteen2d": all 16 (k, l) in {1..4}^2;
* "eight3d":   all 8 (k, l, q) in {1,2}^3.
``thermal_target(N)``: the target of Sec. 6.1 with y_c equal to it on the
boundary.
"""
from __future__ import annotations

import itertools

import numpy as np


def free_coords(dim: int, N: int) -> np.ndarray:
    """(dim, (N-1)^dim) physical coordinates of the free nodes, x fastest."""
    g = np.arange(1, N) / N
    mesh = np.meshgrid(*([g] * dim), indexing="ij")  # mesh[d] varies along axis d
    # flatten with x fastest: transpose so the x axis is last in C order
    return np.stack([m.transpose(tuple(range(dim))[::-1]).ravel() for m in mesh])


def bdry_coords(dim: int, N: int) -> np.ndarray:
    """(dim, m) physical coordinates of the boundary nodes in full-id order."""
    g = np.arange(0, N + 1)
    mesh = np.meshgrid(*([g] * dim), indexing="ij")
    c = np.stack([m.transpose(tuple(range(dim))[::-1]).ravel() for m in mesh])
    on = np.any((c == 0) | (c == N), axis=0)
    return c[:, on] / N


def modes_for(kind: str, seed: int):
    """Mode list and N(0,1) coefficients for a seeded sine-mode target."""
    rng = np.random.default_rng(seed)
    if kind == "four2d":
        allm = list(itertools.product(range(1, 5), repeat=2))
        pick = rng.choice(len(allm), size=4, replace=False)
        modes = [allm[i] for i in pick]
    elif kind == "sixteen2d":
        modes = list(itertools.product(range(1, 5), repeat=2))
    elif kind == "eight3d":
        modes = list(itertools.product(range(1, 3), repeat=3))
    else:
        raise ValueError(kind)
    coefs = rng.standard_normal(len(modes))
    return modes, coefs


def sine_target(dim: int, N: int, modes, coefs):
    """Nodal ybar at the free nodes, and y_c = 0 at the boundary nodes."""
    xyz = free_coords(dim, N)
    y = np.zeros(xyz.shape[1])
    for kvec, a in zip(modes, coefs):
        s = np.full(xyz.shape[1], float(a))
        for d, k in enumerate(kvec):
            s *= np.sin(k * np.pi * xyz[d])
        y += s
    nb = (N + 1) ** dim - (N - 1) ** dim
    return y, np.zeros(nb)


def thermal_target(N: int):
    """Sec. 6.1 target: (2x-1)^2 (2y-1)^2 on [0,1/2]^2, else 0; y_c = ybar on the boundary."""
    def f(c):
        x, y = c[0], c[1]
        inside = (x <= 0.5) & (y <= 0.5)
        return np.where(inside, (2 * x - 1) ** 2 * (2 * y - 1) ** 2, 0.0)
    return f(free_coords(2, N)), f(bdry_coords(2, N))


def random_vector(n: int, seed: int, complex_: bool = False) -> np.ndarray:
    """Seeded N(0,1) vector (complex if asked), for operator parity tests."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(n)
    if complex_:
        v = v + 1j * rng.standard_normal(n)
    return v


def c4_instances(count: int, seed: int, sub_elem: int = 32):
    """Batched workload: N_j = sub_elem * round(exp(U[ln 64, ln 256]) / sub_elem),
    beta_j = 10^U[-6,-1], targets of 16 sine modes seeded by (seed, j)."""
    rng = np.random.default_rng(seed)
    out = []
    for j in range(count):
        N = int(sub_elem * round(np.exp(rng.uniform(np.log(64), np.log(256))) / sub_elem))
        beta = float(10.0 ** rng.uniform(-6, -1))
        out.append({"N": max(N, 2 * sub_elem), "beta": beta, "seed": seed * 100003 + j})
    return out


def c5_requests(count: int, seed: int, mean_gap_ms: float = 5.0, sub_elem: int = 32):
    """Served request stream: exponential inter-arrival gaps (mean mean_gap_ms);
    each request is 2D with probability 0.75, N = sub_elem round(exp(U[ln 128,
    ln 1024]) / sub_elem) with subdomains of sub_elem^2, else 3D, N = 8
    round(exp(U[ln 32, ln 64]) / 8) with subdomains of 8^3; with probability
    0.25 it asks for the full-space method; beta = 10^U[-6,-1], nrhs uniform in
    1..8, targets of 16 (2D) or 8 (3D) sine modes seeded by (seed, request)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for j in range(count):
        t += float(rng.exponential(mean_gap_ms))
        dim = 2 if rng.uniform() < 0.75 else 3
        if dim == 2:
            N = int(sub_elem * round(np.exp(rng.uniform(np.log(128), np.log(1024))) / sub_elem))
            N, m = max(N, 2 * sub_elem), sub_elem
        else:
            N, m = int(8 * round(np.exp(rng.uniform(np.log(32), np.log(64))) / 8)), 8
        full_space = bool(rng.uniform() < 0.25)
        beta = float(10.0 ** rng.uniform(-6, -1))
        nrhs = int(rng.integers(1, 9))
        out.append({"arrival_ms": t, "dim": dim, "N": N, "m": m, "full_space": full_space, "beta": beta,
                    "nrhs": nrhs, "seed": seed * 100003 + j})
    return out


def cantilever_target(n: int, length: int = 3, seed: int = 0, young: float = 20.7e6, pressure: float = 1e5,
                      noise: float = 0.0):
    """Target displacement of the Sec. 6.2 cantilever shape, without any solve:
    at every free node (dof 3 f + c, free nodes x fastest over i = 1..length n,
    j, k = 0..n, h = 1 / n) the z component is the Euler-Bernoulli deflection of a
    clamped beam of length L, unit square section (I = 1/12) under the line load
    q = pressure x 1 m,
        w(x) = -q x^2 (6 L^2 - 4 L x + x^2) / (24 E I),
    (0.59 m at the tip for the paper's rubber and 100 kPa), x and y components
    zero, plus `noise` times max |w| times seeded N(0, 1) values on every dof."""
    L = float(length)
    nx = length * n
    i = np.arange(1, nx + 1)
    x = i / n
    w = -pressure * x ** 2 * (6 * L * L - 4 * L * x + x * x) / (24.0 * young / 12.0)
    nodes = (n + 1) * (n + 1) * nx
    y = np.zeros((nodes, 3))
    y[:, 2] = np.tile(w, (n + 1) * (n + 1))  # x fastest: i varies first
    y = y.ravel()
    if noise:
        y = y + noise * np.abs(w).max() * np.random.default_rng(seed).standard_normal(y.size)
    return y
