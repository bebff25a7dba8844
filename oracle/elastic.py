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

Decomposition cuts the cantilever into cubic subdomains for FETI-DP (Sec. 5)
and exposes it on dofs to the dense routines of oracle.feti, so the same
definitions of F_DP, d, K_cc*, S_bb and the recovery serve the elastic case.
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


class _Dofs:
    """Dof view of a Box for the generic FETI-DP routines of oracle.feti: full dof
    3 node + c over all grid nodes, free dofs in the free numbering above."""

    def __init__(self, box: Box):
        node_of_free = np.nonzero(~box.fixed)[0]
        self.n_full = 3 * box.ijk.shape[0]
        self.free_full = (3 * node_of_free[:, None] + np.arange(3)[None, :]).ravel()
        self.n = self.free_full.size


class Decomposition:
    """FETI-DP partition of a cantilever Box into Px x Py x Pz cubes of m^3 cells
    (Sec. 5 applied to the Sec. 6.2 state equation), with the attributes the
    dense routines of oracle.feti read (subs[s]: full, r, c, delta_loc, Br, Bc;
    nmu, nC, mults, mult, corner_full, mesh; local_matrices, split_rhs), on dofs.

    Readings (the paper names FETI-DPH without its primal set for this problem):
    * corners: the three dofs of every subdomain vertex that is not clamped;
    * Delta dofs: the other unclamped dofs of nodes shared by two or more
      subdomains; fully redundant multipliers, one per pair (s_a < s_b) of the
      subdomains sharing the node, per component, signed +1 on s_a, ordered by
      the full dof (node, then component), then by pair;
    * the remaining unclamped dofs (subdomain interior and free surface) are
      local to their subdomain;
    * local dof 3 l + c of local node l = a + (m+1) b + (m+1)^2 c (x fastest);
      r and c sets in increasing local dof; subdomain s = sx + Px (sy + Py sz);
      corners in increasing full dof.
    """

    def __init__(self, box: Box, m: int, E: float = YOUNG, nu: float = POISSON):
        if box.clamp != "cantilever":
            raise ValueError("the partition is written for the cantilever")
        if box.n % m != 0 or m < 2:
            raise ValueError("need n % m == 0 and m >= 2")
        self.box, self.m, self.E, self.nu = box, m, E, nu
        self.mesh = _Dofs(box)
        self.Px, self.Py, self.Pz = box.nx // m, box.ny // m, box.nz // m
        self.nsub = self.Px * self.Py * self.Pz
        ml = m + 1
        lc, lb, la = np.indices((ml, ml, ml)).reshape(3, -1)  # local node a + ml b + ml^2 c
        vert = ((la == 0) | (la == m)) & ((lb == 0) | (lb == m)) & ((lc == 0) | (lc == m))
        nodes = []
        count = np.zeros(box.ijk.shape[0], dtype=np.int64)
        for s in range(self.nsub):
            sx, sy, sz = s % self.Px, (s // self.Px) % self.Py, s // (self.Px * self.Py)
            nd = box.node(la + sx * m, lb + sy * m, lc + sz * m)
            nodes.append(nd)
            count[nd] += 1
        self.mult = np.repeat(count, 3)  # per full dof
        self.subs = []
        for s in range(self.nsub):
            nd = nodes[s]
            clamped = box.fixed[nd]
            corner_n = vert & ~clamped
            delta_n = ~vert & ~clamped & (count[nd] >= 2)
            local_n = ~vert & ~clamped & (count[nd] == 1)
            rep = lambda mask: np.repeat(mask, 3)
            full = (3 * nd[:, None] + np.arange(3)[None, :]).ravel()
            self.subs.append({"nodes": nd, "full": full, "corner": rep(corner_n), "delta": rep(delta_n),
                              "inter": rep(local_n)})
        cset = np.unique(np.concatenate([sd["full"][sd["corner"]] for sd in self.subs]))
        self.corner_full = cset
        self.corner_id = {int(f): i for i, f in enumerate(cset)}
        self.nC = cset.size
        owners = {}
        for s, sd in enumerate(self.subs):
            for f in sd["full"][sd["delta"]]:
                owners.setdefault(int(f), []).append(s)
        self.mults = []
        for f in sorted(owners):
            ss = sorted(owners[f])
            for a in range(len(ss)):
                for b in range(a + 1, len(ss)):
                    self.mults.append((f, ss[a], ss[b]))
        self.nmu = len(self.mults)
        for s, sd in enumerate(self.subs):
            r = np.nonzero(sd["inter"] | sd["delta"])[0]
            c = np.nonzero(sd["corner"])[0]
            sd["r"], sd["c"], sd["delta_loc"] = r, c, np.nonzero(sd["delta"])[0]
            pos = {int(l): i for i, l in enumerate(r)}
            where = {int(f): i for i, f in enumerate(sd["full"])}
            Br = np.zeros((self.nmu, r.size))
            for k, (f, sa, sb) in enumerate(self.mults):
                if s == sa or s == sb:
                    Br[k, pos[where[f]]] = 1.0 if s == sa else -1.0
            sd["Br"] = Br
            Bc = np.zeros((c.size, self.nC))
            for i, l in enumerate(c):
                Bc[i, self.corner_id[int(sd["full"][l])]] = 1.0
            sd["Bc"] = Bc

    def local_matrices(self, alpha: float, shift: str = "imag"):
        """Z^s = K^s + i alpha M^s (shift "imag") or K^s + alpha M^s ("real") of the
        subdomain's elements over its local dofs, as dense rr, rc, cc blocks."""
        m, ml = self.m, self.m + 1
        Ke = elasticity_element(self.box.h, self.E, self.nu)
        Me = mass_element(self.box.h)
        Ze = Ke + (1j * alpha if shift == "imag" else alpha) * Me
        Zloc = np.zeros((3 * ml ** 3, 3 * ml ** 3), dtype=np.complex128)
        for ec in range(m):
            for eb in range(m):
                for ea in range(m):
                    ln = [(ea + a) + ml * (eb + b) + ml * ml * (ec + c)
                          for c in (0, 1) for b in (0, 1) for a in (0, 1)]
                    dofs = np.array([3 * l + k for l in ln for k in range(3)])
                    Zloc[np.ix_(dofs, dofs)] += Ze
        out = []
        for sd in self.subs:
            r, c = sd["r"], sd["c"]
            out.append({"rr": Zloc[np.ix_(r, r)], "rc": Zloc[np.ix_(r, c)], "cc": Zloc[np.ix_(c, c)]})
        return out

    def split_rhs(self, f_free: np.ndarray):
        """Per-subdomain remainder loads f_r^s = f / multiplicity, and global f_c."""
        ffull = np.zeros(self.mesh.n_full, dtype=np.complex128)
        ffull[self.mesh.free_full] = f_free
        fr = []
        for sd in self.subs:
            fl = sd["full"][sd["r"]]
            fr.append(ffull[fl] / self.mult[fl])
        return fr, ffull[self.corner_full]
