"""Trilinear (Q1) linear-elasticity elements on a uniform box mesh: the solid
cantilever control problem of Sec. 6.2 (test infrastructure; only tests/,
__graft_entry__.smoke() and bench.py's cpu_baseline use the oracle).

The state equation of Sec. 2 becomes the elastostatic one: K is the stiffness
of an isotropic linear-elastic solid (Young's modulus E, Poisson's ratio nu,
Lame constants lambda = E nu / ((1 + nu)(1 - 2 nu)), mu = E / (2 (1 + nu))), V
the consistent vector mass matrix (the control is a body force, Sec. 6.2), and
the dofs are the three displacement components of every node.  The paper's
cantilever is the box [0, 3] x [0, 1] x [0, 1] (m), clamped on the face x = 0
and free elsewhere; its target is the displacement under a uniform downward
pressure on the bottom face z = 0 (Sec. 6.2 and its figure).  Elements are
integrated with the 2 x 2 x 2 Gauss rule (exact for the trilinear products).

Numbering (a convention of this module and the library's documentation):
* grid node (i, j, k), 0 <= i <= nx, 0 <= j <= ny, 0 <= k <= nz, with
  nx = L n, ny = nz = n cells of side h = 1 / n;
* free nodes are those not clamped, numbered x fastest over (i, j, k) in the
  box minus the clamped face; free dof 3 f + c carries displacement component
  c (0: x, 1: y, 2: z) of free node f;
* "cantilever": clamped face i = 0; "cube": all six faces clamped (L = 1),
  for manufactured-solution tests.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp

from . import fem

# rubber of Sec. 6.2
YOUNG = 20.7e6
POISSON = 0.45


def lame(E: float, nu: float):
    """Lame constants (lambda, mu) of an isotropic solid."""
    return E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu)), E / (2.0 * (1.0 + nu))


def elasticity_element(h: float, E: float = YOUNG, nu: float = POISSON):
    """24 x 24 stiffness of a cube cell of side h: integral of eps(phi_p) : sigma(phi_q).

    Local dof 3 l + c, vertex l = a + 2 b + 4 c at offset (a, b, c) (x fastest).
    Strains in Voigt order (xx, yy, zz, yz, xz, xy) with engineering shears."""
    lam, mu = lame(E, nu)
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[np.arange(3), np.arange(3)] += 2.0 * mu
    D[np.arange(3, 6), np.arange(3, 6)] = mu
    pts, wts = fem._gauss2()
    offs = [((l >> 0) & 1, (l >> 1) & 1, (l >> 2) & 1) for l in range(8)]
    Ke = np.zeros((24, 24))
    for qp in itertools.product(range(2), repeat=3):
        w = wts[qp[0]] * wts[qp[1]] * wts[qp[2]] * h ** 3
        B = np.zeros((6, 24))
        for l, o in enumerate(offs):
            g = np.ones(3)
            for d in range(3):
                sv, sd = fem._shape_1d(pts[qp[d]])
                for e in range(3):
                    g[e] *= (sd[o[d]] / h) if e == d else sv[o[d]]
            gx, gy, gz = g
            c = 3 * l
            B[0, c] = gx
            B[1, c + 1] = gy
            B[2, c + 2] = gz
            B[3, c + 1], B[3, c + 2] = gz, gy
            B[4, c], B[4, c + 2] = gz, gx
            B[5, c], B[5, c + 1] = gy, gx
        Ke += w * B.T @ D @ B
    return Ke


def mass_element(h: float):
    """24 x 24 consistent vector mass of a cube cell: the scalar Q1 mass times I_3."""
    _, Me = fem.element_matrices(3, h)
    return np.kron(Me, np.eye(3))


class Box:
    """Uniform hexahedral mesh of [0, L] x [0, 1] x [0, 1], n cells per unit length."""

    def __init__(self, n: int, length: int = 3, clamp: str = "cantilever"):
        if clamp not in ("cantilever", "cube"):
            raise ValueError("clamp must be 'cantilever' or 'cube'")
        if clamp == "cube":
            length = 1
        self.n, self.length, self.clamp = n, length, clamp
        self.nx, self.ny, self.nz = length * n, n, n
        self.h = 1.0 / n
        i, j, k = np.meshgrid(np.arange(self.nx + 1), np.arange(self.ny + 1), np.arange(self.nz + 1),
                              indexing="ij")
        i, j, k = (a.transpose(2, 1, 0).ravel() for a in (i, j, k))  # x fastest
        self.ijk = np.stack([i, j, k], axis=1)
        if clamp == "cantilever":
            fixed = i == 0
        else:
            fixed = (i == 0) | (i == self.nx) | (j == 0) | (j == self.ny) | (k == 0) | (k == self.nz)
        self.fixed = fixed
        self.free_of_node = -np.ones(i.size, dtype=np.int64)
        self.free_of_node[~fixed] = np.arange(int((~fixed).sum()))
        self.nfree_nodes = int((~fixed).sum())
        self.n_dof = 3 * self.nfree_nodes

    def node(self, i, j, k):
        return i + (self.nx + 1) * (j + (self.ny + 1) * k)

    def coords(self):
        """Coordinates of the free nodes (in free-node order)."""
        return self.ijk[~self.fixed] * self.h


def assemble(box: Box, E: float = YOUNG, nu: float = POISSON):
    """Stiffness K and vector mass V over the free dofs (Sec. 2 with the elastostatic
    constraint of Sec. 6.2); K_c has no columns (homogeneous clamp)."""
    Ke = elasticity_element(box.h, E, nu)
    Me = mass_element(box.h)
    rows, cols, kv, mv = [], [], [], []
    for ez in range(box.nz):
        for ey in range(box.ny):
            for ex in range(box.nx):
                nodes = [box.node(ex + a, ey + b, ez + c) for c in (0, 1) for b in (0, 1) for a in (0, 1)]
                fr = box.free_of_node[nodes]
                dofs = np.array([3 * f + c if f >= 0 else -1 for f in fr for c in range(3)])
                ok = dofs >= 0
                d = dofs[ok]
                rows.append(np.repeat(d, d.size))
                cols.append(np.tile(d, d.size))
                kv.append(Ke[np.ix_(ok, ok)].ravel())
                mv.append(Me[np.ix_(ok, ok)].ravel())
    r, c = np.concatenate(rows), np.concatenate(cols)
    n = box.n_dof
    K = sp.csr_matrix((np.concatenate(kv), (r, c)), shape=(n, n))
    M = sp.csr_matrix((np.concatenate(mv), (r, c)), shape=(n, n))
    K.sum_duplicates()
    M.sum_duplicates()
    return {"K": K, "M": M, "Kc": sp.csr_matrix((n, 0))}


def body_load(box: Box, f_nodes: np.ndarray):
    """Load vector of a body force given at every grid node (shape (nodes, 3)): the
    integral of its Q1 interpolant against each free dof's shape function, cell by
    cell with the consistent mass (clamped nodes' values included)."""
    Me = mass_element(box.h)
    b = np.zeros(box.n_dof)
    for ez in range(box.nz):
        for ey in range(box.ny):
            for ex in range(box.nx):
                nodes = [box.node(ex + a, ey + bb, ez + c) for c in (0, 1) for bb in (0, 1) for a in (0, 1)]
                be = Me @ f_nodes[nodes].ravel()
                for l, nd in enumerate(nodes):
                    fr = box.free_of_node[nd]
                    if fr >= 0:
                        b[3 * fr:3 * fr + 3] += be[3 * l:3 * l + 3]
    return b


def pressure_load(box: Box, pressure: float):
    """Consistent nodal forces of a uniform pressure on the bottom face z = 0, pushing
    in -z: each bottom face cell gives its four vertices -pressure h^2 / 4 (the bilinear
    shape functions integrate to a quarter of the face each)."""
    f = np.zeros(box.n_dof)
    q = -pressure * box.h * box.h / 4.0
    for ey in range(box.ny):
        for ex in range(box.nx):
            for a in (0, 1):
                for b in (0, 1):
                    fr = box.free_of_node[box.node(ex + a, ey + b, 0)]
                    if fr >= 0:
                        f[3 * fr + 2] += q
    return f


def reactions(box: Box, u_free: np.ndarray, E: float = YOUNG, nu: float = POISSON):
    """Sum over the clamped nodes of the elastic forces K_full u (per component):
    the support reaction, which balances the applied load."""
    Ke = elasticity_element(box.h, E, nu)
    tot = np.zeros(3)
    for ez in range(box.nz):
        for ey in range(box.ny):
            for ex in range(box.nx):
                nodes = [box.node(ex + a, ey + b, ez + c) for c in (0, 1) for b in (0, 1) for a in (0, 1)]
                ue = np.zeros(24)
                for l, nd in enumerate(nodes):
                    fr = box.free_of_node[nd]
                    if fr >= 0:
                        ue[3 * l:3 * l + 3] = u_free[3 * fr:3 * fr + 3]
                fe = Ke @ ue
                for l, nd in enumerate(nodes):
                    if box.fixed[nd]:
                        tot += fe[3 * l:3 * l + 3]
    return tot
