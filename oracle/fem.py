"""Q1 finite elements on the unit square / cube, assembled into sparse matrices.

Follows Sec. 2 of the paper (discrete QP): the stiffness matrix K and the
"volume" (consistent mass) matrix V over the n unconstrained dofs, and the
constrained stiffness K_c coupling those dofs to the m Dirichlet dofs.  The
paper defers the element details to its companion reference; the reading taken
here is the standard one for a unit-conductivity Poisson problem: bilinear
(2D) or trilinear (3D) elements on a uniform grid of N^d cells of side h = 1/N,
integrated exactly, with Dirichlet conditions on all of the boundary.

Numbering (shared with the C ABI documentation, it is a convention, not code):
* full-grid node (i, j[, k]), 0 <= i, j, k <= N, has full id
  i + (N+1) j [+ (N+1)^2 k]  (x fastest);
* free (unconstrained) nodes are those with 1 <= i, j, k <= N-1, numbered
  (i-1) + (N-1)(j-1) [+ (N-1)^2 (k-1)];
* boundary nodes are the remaining full-grid nodes, numbered in increasing
  full id.

Element matrices are built by Gauss quadrature of the Q1 shape functions (two
points per direction, exact for these polynomial integrands), not from a
closed-form table, so that tests can pin them against textbook values.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp


def _gauss2():
    """Two-point Gauss-Legendre rule on [0, 1] (exact to degree 3)."""
    g = 0.5 / np.sqrt(3.0)
    return np.array([0.5 - g, 0.5 + g]), np.array([0.5, 0.5])


def _shape_1d(t):
    """Linear shape functions on [0,1] at t: values and d/dt, local nodes 0, 1."""
    return np.array([1.0 - t, t]), np.array([-1.0, 1.0])


def element_matrices(dim: int, h: float):
    """Q1 element stiffness K_e and mass M_e of a cube cell of side h.

    Local node index is a + 2 b (+ 4 c) for the vertex at offset (a, b[, c]),
    x fastest.  K_e[p, q] = integral of grad(phi_p) . grad(phi_q),
    M_e[p, q] = integral of phi_p phi_q (Sec. 2, discrete QP: K and V).
    """
    if dim not in (2, 3):
        raise ValueError("dim must be 2 or 3")
    pts, wts = _gauss2()
    nloc = 2 ** dim
    # vertex l sits at offset ((l >> 0) & 1, (l >> 1) & 1[, (l >> 2) & 1]): x fastest
    offs = [tuple((l >> d) & 1 for d in range(dim)) for l in range(nloc)]
    Ke = np.zeros((nloc, nloc))
    Me = np.zeros((nloc, nloc))
    for qp in itertools.product(range(2), repeat=dim):
        w = np.prod([wts[q] for q in qp]) * h ** dim
        vals = []
        grads = []
        for o in offs:
            v = 1.0
            g = np.ones(dim)
            for d in range(dim):
                sv, sd = _shape_1d(pts[qp[d]])
                v *= sv[o[d]]
                for e in range(dim):
                    g[e] *= (sd[o[d]] / h) if e == d else sv[o[d]]
            vals.append(v)
            grads.append(g)
        vals = np.array(vals)
        grads = np.array(grads)
        Ke += w * grads @ grads.T
        Me += w * np.outer(vals, vals)
    return Ke, Me


class Mesh:
    """Uniform Q1 mesh of [0,1]^dim with N cells per direction (Sec. 2)."""

    def __init__(self, dim: int, N: int):
        if dim not in (2, 3) or N < 2:
            raise ValueError("need dim in (2,3) and N >= 2")
        self.dim = dim
        self.N = N
        self.h = 1.0 / N
        n1 = N + 1
        self.n_full = n1 ** dim
        idx = np.indices((n1,) * dim).reshape(dim, -1)  # idx[0] slowest
        # full id with x fastest: coordinate along axis d is idx[dim-1-d]
        coords = np.stack([idx[dim - 1 - d] for d in range(dim)])  # coords[0] = i (x)
        full = sum(coords[d] * n1 ** d for d in range(dim))
        orderv = np.argsort(full)
        self.coords = coords[:, orderv]  # coords of full ids 0..n_full-1
        on_bdry = np.any((self.coords == 0) | (self.coords == N), axis=0)
        self.free_full = np.nonzero(~on_bdry)[0]
        self.bdry_full = np.nonzero(on_bdry)[0]
        self.n = self.free_full.size
        self.m = self.bdry_full.size
        self.full_to_free = -np.ones(self.n_full, dtype=np.int64)
        self.full_to_free[self.free_full] = np.arange(self.n)
        self.full_to_bdry = -np.ones(self.n_full, dtype=np.int64)
        self.full_to_bdry[self.bdry_full] = np.arange(self.m)

    def node_xyz(self, which: str = "free") -> np.ndarray:
        """Physical coordinates (dim x count) of the free or boundary nodes."""
        ids = self.free_full if which == "free" else self.bdry_full
        return self.coords[:, ids] * self.h

    def element_nodes(self) -> np.ndarray:
        """(n_elem, 2^dim) full ids of each cell's vertices in local order."""
        N, dim, n1 = self.N, self.dim, self.N + 1
        e = np.indices((N,) * dim).reshape(dim, -1)
        ecoord = np.stack([e[dim - 1 - d] for d in range(dim)])  # ecoord[0] = x index
        base = sum(ecoord[d] * n1 ** d for d in range(dim))
        loc = []
        for l in range(2 ** dim):
            off = sum(((l >> d) & 1) * n1 ** d for d in range(dim))
            loc.append(base + off)
        return np.stack(loc, axis=1)


def assemble(mesh: Mesh):
    """Assemble K, V(=M) over free dofs and K_c (free x boundary), Sec. 2.

    Returns a dict with CSR matrices ``K``, ``M``, ``Kc`` and the full
    (boundary-inclusive) matrices ``K_full``, ``M_full``.
    """
    Ke, Me = element_matrices(mesh.dim, mesh.h)
    en = mesh.element_nodes()
    nl = en.shape[1]
    rows = np.repeat(en, nl, axis=1).ravel()
    cols = np.tile(en, (1, nl)).ravel()
    kv = np.tile(Ke.ravel(), en.shape[0])
    mv = np.tile(Me.ravel(), en.shape[0])
    nf = mesh.n_full
    K_full = sp.csr_matrix((kv, (rows, cols)), shape=(nf, nf))
    M_full = sp.csr_matrix((mv, (rows, cols)), shape=(nf, nf))
    F, B = mesh.free_full, mesh.bdry_full
    K = K_full[F][:, F].tocsr()
    M = M_full[F][:, F].tocsr()
    Kc = K_full[F][:, B].tocsr()
    return {"K": K, "M": M, "Kc": Kc, "K_full": K_full, "M_full": M_full}
