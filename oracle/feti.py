"""FETI-DP written out from its definitions, dense, for small meshes (test oracle).

Sec. 5 of the paper: the domain is cut into non-overlapping subdomains; each
subdomain s minimises its local energy with its own copy y^s of the interface
unknowns, and continuity is imposed by sum_s B^s y^s = 0 with signed Boolean
matrices B^s.  Stationarity of the Lagrangian gives Z^s y^s = f^s - B^sT mu
(this module writes mu for the interface multipliers to keep lambda for the
adjoint of the control problem).  FETI-DP (Sec. 5) keeps the subdomain
vertices ("corners") as global unknowns, so every remainder block Z_rr^s is
nonsingular, and the corner unknowns form a coarse problem.  With
F = sum B K^+ B^T and d = sum B K^+ f (Sec. 5, definition of F, d) written for
the remainder blocks, eliminating the subdomain and corner unknowns gives

    F_rr   = sum_s B_r Z_rr^-1 B_r^T
    F_rc   = sum_s B_r Z_rr^-1 Z_rc B_c
    K_cc*  = sum_s B_c^T (Z_cc - Z_cr Z_rr^-1 Z_rc) B_c
    f_c*   = f_c - sum_s B_c^T Z_cr Z_rr^-1 f_r
    d      = sum_s B_r Z_rr^-1 f_r - F_rc K_cc*^-1 f_c*
    F_DP   = F_rr + F_rc K_cc*^-1 F_rc^T,     F_DP mu = d,

and the solution is recovered as u_c = K_cc*^-1 (f_c* + F_rc^T mu),
u_r^s = Z_rr^-1 (f_r - Z_rc B_c u_c - B_r^T mu).  The Dirichlet preconditioner
of Sec. 5 is P^-1 = W (sum_s B_r [0 0; 0 S_bb] B_r^T) W with W = (sum B B^T)^+
and S_bb the Schur complement of Z_rr on its interface (Delta) dofs.

Readings where the paper is silent (they do not change the solution):
* corners are the subdomain vertices that are not Dirichlet nodes;
* Delta nodes are the other non-Dirichlet nodes on subdomain boundaries;
  a node shared by subdomains s_1 < ... < s_k gets one multiplier per pair
  (s_a, s_b), a < b (fully redundant), signed +1 on s_a and -1 on s_b; in 2D
  and on 3D faces k = 2, so this is one multiplier per node;
* multipliers are ordered by the node's full id, then by pair;
* the local load on a shared node is f / (number of subdomains sharing it);
* the primal solution on a Delta node is the average of the subdomain copies.

Local numbering: subdomain (sx, sy[, sz]) has id sx + P sy [+ P^2 sz] with P =
N / m subdomains per direction; its node at local offset (a, b[, c]),
0 <= a, b, c <= m, has local index a + (m+1) b [+ (m+1)^2 c].  Delta and
corner nodes of a subdomain are listed in increasing local index; global
corners in increasing full id.
"""
from __future__ import annotations

import numpy as np

from .fem import Mesh, element_matrices


class Decomposition:
    """Subdomains of a uniform mesh into P^dim boxes of m^dim cells (Sec. 5, Fig. 1)."""

    def __init__(self, mesh: Mesh, m: int):
        N, dim = mesh.N, mesh.dim
        if N % m != 0 or m < 2:
            raise ValueError("need N % m == 0 and m >= 2")
        self.mesh, self.m, self.dim = mesh, m, dim
        self.P = N // m
        n1, ml = N + 1, m + 1
        self.nsub = self.P ** dim
        loc = np.indices((ml,) * dim).reshape(dim, -1)
        loc = np.stack([loc[dim - 1 - d] for d in range(dim)])  # loc[0] = a (x), x fastest
        self.loc_coords = loc
        self.subs = []
        count = np.zeros(mesh.n_full, dtype=np.int64)
        for s in range(self.nsub):
            sc = [(s // self.P ** d) % self.P for d in range(dim)]
            g = np.stack([loc[d] + sc[d] * m for d in range(dim)])
            full = sum(g[d] * n1 ** d for d in range(dim))
            dirich = np.any((g == 0) | (g == N), axis=0)
            vert = np.all((loc == 0) | (loc == m), axis=0)
            inter = np.all((loc > 0) & (loc < m), axis=0)
            corner = vert & ~dirich
            delta = ~vert & ~inter & ~dirich
            self.subs.append({"coord": sc, "full": full, "dirich": dirich, "corner": corner,
                              "delta": delta, "inter": inter})
            count[full] += 1
        self.mult = count
        # global corners
        cset = np.unique(np.concatenate([sd["full"][sd["corner"]] for sd in self.subs]))
        self.corner_full = cset
        self.corner_id = {int(f): i for i, f in enumerate(cset)}
        self.nC = cset.size
        # multipliers: fully redundant pairs over sharing subdomains
        owners = {}
        for s, sd in enumerate(self.subs):
            for f in sd["full"][sd["delta"]]:
                owners.setdefault(int(f), []).append(s)
        mults = []
        for f in sorted(owners):
            ss = sorted(owners[f])
            for a in range(len(ss)):
                for b in range(a + 1, len(ss)):
                    mults.append((f, ss[a], ss[b]))
        self.mults = mults
        self.nmu = len(mults)
        # per subdomain: r set (interior + delta, increasing local index), corners
        for s, sd in enumerate(self.subs):
            r = np.nonzero(sd["inter"] | sd["delta"])[0]
            c = np.nonzero(sd["corner"])[0]
            sd["r"], sd["c"] = r, c
            sd["delta_loc"] = np.nonzero(sd["delta"])[0]
            pos = {int(l): i for i, l in enumerate(r)}
            Br = np.zeros((self.nmu, r.size))
            for k, (f, sa, sb) in enumerate(mults):
                if s == sa or s == sb:
                    l = int(np.nonzero(sd["full"] == f)[0][0])
                    Br[k, pos[l]] = 1.0 if s == sa else -1.0
            sd["Br"] = Br
            Bc = np.zeros((c.size, self.nC))
            for i, l in enumerate(c):
                Bc[i, self.corner_id[int(sd["full"][l])]] = 1.0
            sd["Bc"] = Bc

    def local_matrices(self, alpha: float):
        """Local Neumann matrices Z^s = K^s + i alpha M^s (subdomain elements only).

        Returned over the subdomain's non-Dirichlet local nodes as dense blocks
        rr, rc, cc in the r / c orders documented in the module docstring.
        """
        dim, m = self.dim, self.m
        Ke, Me = element_matrices(dim, self.mesh.h)
        Ze = Ke + 1j * alpha * Me
        ml = m + 1
        nl = ml ** dim
        Zloc = np.zeros((nl, nl), dtype=np.complex128)
        e = np.indices((m,) * dim).reshape(dim, -1)
        e = np.stack([e[dim - 1 - d] for d in range(dim)])
        base = sum(e[d] * ml ** d for d in range(dim))
        ids = np.stack([base + sum(((l >> d) & 1) * ml ** d for d in range(dim))
                        for l in range(2 ** dim)], axis=1)
        for el in ids:
            Zloc[np.ix_(el, el)] += Ze
        out = []
        for sd in self.subs:
            r, c = sd["r"], sd["c"]
            out.append({"rr": Zloc[np.ix_(r, r)], "rc": Zloc[np.ix_(r, c)],
                        "cc": Zloc[np.ix_(c, c)]})
        return out

    def split_rhs(self, f_free: np.ndarray):
        """Per-subdomain remainder loads f_r^s = f / multiplicity, and global f_c."""
        mesh = self.mesh
        ffull = np.zeros(mesh.n_full, dtype=np.complex128)
        ffull[mesh.free_full] = f_free
        fr = []
        for sd in self.subs:
            fl = sd["full"][sd["r"]]
            fr.append(ffull[fl] / self.mult[fl])
        fc = ffull[self.corner_full]
        return fr, fc


def fetidp_operators(dec: Decomposition, alpha: float):
    """Dense FETI-DP operators (module docstring) and per-subdomain pieces.

    Returns F_rr, F_rc, K_cc*, per-subdomain Z_rr^-1, the Delta Schur
    complements S_bb and the local condensed corner blocks Phi = Z_rr^-1 Z_rc.
    """
    loc = dec.local_matrices(alpha)
    nmu, nC = dec.nmu, dec.nC
    Frr = np.zeros((nmu, nmu), dtype=np.complex128)
    Frc = np.zeros((nmu, nC), dtype=np.complex128)
    Kcc = np.zeros((nC, nC), dtype=np.complex128)
    pieces = []
    for sd, L in zip(dec.subs, loc):
        X = np.linalg.inv(L["rr"])
        Br, Bc = sd["Br"], sd["Bc"]
        Phi = X @ L["rc"]
        Frr += Br @ X @ Br.T
        Frc += Br @ Phi @ Bc
        Kcc += Bc.T @ (L["cc"] - L["rc"].T @ Phi) @ Bc
        # Schur complement of Z_rr on its Delta dofs (interior eliminated)
        r = sd["r"]
        isd = np.isin(r, sd["delta_loc"])
        A = L["rr"]
        Aii, Aib = A[np.ix_(~isd, ~isd)], A[np.ix_(~isd, isd)]
        Sbb = A[np.ix_(isd, isd)] - Aib.T @ np.linalg.solve(Aii, Aib)
        pieces.append({"Zrr_inv": X, "Phi": Phi, "Sbb": Sbb, "is_delta": isd,
                       "Zrc": L["rc"], "Zcc": L["cc"], "Zrr": L["rr"]})
    return {"Frr": Frr, "Frc": Frc, "Kcc": Kcc, "pieces": pieces}


def fetidp_rhs(dec: Decomposition, ops, f_free):
    """d and f_c* of the FETI-DP interface problem (module docstring)."""
    fr, fc = dec.split_rhs(f_free)
    dr = np.zeros(dec.nmu, dtype=np.complex128)
    fcs = fc.astype(np.complex128).copy()
    for sd, pc, f in zip(dec.subs, ops["pieces"], fr):
        x = pc["Zrr_inv"] @ f
        dr += sd["Br"] @ x
        fcs -= sd["Bc"].T @ (pc["Zrc"].T @ x)
    d = dr - ops["Frc"] @ np.linalg.solve(ops["Kcc"], fcs)
    return d, fcs, fr


def fetidp_apply(ops, mu):
    """F_DP mu = F_rr mu + F_rc K_cc*^-1 F_rc^T mu (plain transpose: complex symmetric)."""
    return ops["Frr"] @ mu + ops["Frc"] @ np.linalg.solve(ops["Kcc"], ops["Frc"].T @ mu)


def dirichlet_preconditioner(dec: Decomposition, ops):
    """Dense P^-1 = W (sum_s B_r diag(0, S_bb) B_r^T) W, W = (sum_s B_r B_r^T)^+ (Sec. 5)."""
    nmu = dec.nmu
    BB = np.zeros((nmu, nmu))
    acc = np.zeros((nmu, nmu), dtype=np.complex128)
    for sd, pc in zip(dec.subs, ops["pieces"]):
        Br = sd["Br"]
        BB += Br @ Br.T
        nr = Br.shape[1]
        Sfull = np.zeros((nr, nr), dtype=np.complex128)
        isd = pc["is_delta"]
        Sfull[np.ix_(isd, isd)] = pc["Sbb"]
        acc += Br @ Sfull @ Br.T
    W = np.linalg.pinv(BB)
    return W @ acc @ W


def fetidp_solve_dense(dec: Decomposition, alpha: float, f_free):
    """Solve Z x = f by FETI-DP with a dense solve of F_DP mu = d; returns x on free nodes."""
    ops = fetidp_operators(dec, alpha)
    d, fcs, fr = fetidp_rhs(dec, ops, f_free)
    F = ops["Frr"] + ops["Frc"] @ np.linalg.solve(ops["Kcc"], ops["Frc"].T)
    # fully redundant multipliers (3D edges) make F_DP singular but consistent:
    # least squares returns one of the equivalent multiplier sets
    mu = np.linalg.lstsq(F, d, rcond=None)[0]
    uc = np.linalg.solve(ops["Kcc"], fcs + ops["Frc"].T @ mu)
    mesh = dec.mesh
    acc = np.zeros(mesh.n_full, dtype=np.complex128)
    for sd, pc, f in zip(dec.subs, ops["pieces"], fr):
        ur = pc["Zrr_inv"] @ (f - pc["Zrc"] @ (sd["Bc"] @ uc) - sd["Br"].T @ mu)
        acc[sd["full"][sd["r"]]] += ur
    cnt = dec.mult.astype(np.float64)
    x_full = acc / np.maximum(cnt, 1)
    x_full[dec.corner_full] = uc
    return x_full[mesh.free_full], {"mu": mu, "d": d, "F": F, "ops": ops}


# ---------------------------------------------------------------------------
# Edge augmentation of the coarse problem (Sec. 5, the FETI-DPH augmentation
# compared in Table 1).  For a scalar problem the edge modes are averages:
# Q has one column per pair of subdomains that share multipliers (an interface
# edge in 2D), with ones on those multipliers.  The constraint Q^T B_r u_r = 0
# is enforced exactly at every iterate through extra coarse unknowns nu (one per
# column of Q), eliminated with the corners.  From the subdomain equations
#   Z_rr u_r + Z_rc B_c u_c + B_r^T (mu + Q nu) = f_r
# and the corner and augmentation equations one gets, with
#   G  = [F_rc, F_rr Q],
#   Kt = [[K_cc*, -F_rc^T Q], [-Q^T F_rc, -Q^T F_rr Q]],
#   c0 = [f_c*; -Q^T d_r],  d_r = sum_s B_r Z_rr^-1 f_r,
# the interface problem  F_aug mu = d_aug  with
#   F_aug = F_rr + G Kt^-1 G^T,   d_aug = d_r - G Kt^-1 c0,
# the coarse solution (u_c; nu) = Kt^-1 (c0 + G^T mu), and the subdomain
# solution u_r = Z_rr^-1 (f_r - Z_rc B_c u_c - B_r^T (mu + Q nu)).

def edge_space(dec: Decomposition):
    """Q: one column per pair (s_a, s_b) of subdomains sharing multipliers, in
    increasing pair order, with ones on the pair's multipliers."""
    pairs = {}
    for k, (_, sa, sb) in enumerate(dec.mults):
        pairs.setdefault((sa, sb), []).append(k)
    keys = sorted(pairs)
    Q = np.zeros((dec.nmu, len(keys)))
    for e, key in enumerate(keys):
        Q[pairs[key], e] = 1.0
    return Q, keys


def fetidp_aug_operators(ops, Q):
    """G and the augmented coarse matrix Kt (definitions above)."""
    Frr, Frc, Kcc = ops["Frr"], ops["Frc"], ops["Kcc"]
    G = np.hstack([Frc, Frr @ Q])
    Kt = np.block([[Kcc, -Frc.T @ Q], [-Q.T @ Frc, -Q.T @ Frr @ Q]])
    return {"G": G, "Kt": Kt, "Q": Q}


def fetidp_aug_apply(ops, aug, mu):
    """F_aug mu = F_rr mu + G Kt^-1 G^T mu (plain transposes: complex symmetric)."""
    G = aug["G"]
    return ops["Frr"] @ mu + G @ np.linalg.solve(aug["Kt"], G.T @ mu)


def fetidp_aug_rhs(dec: Decomposition, ops, aug, f_free):
    """d_aug and c0 of the augmented interface problem."""
    fr, fc = dec.split_rhs(f_free)
    dr = np.zeros(dec.nmu, dtype=np.complex128)
    fcs = fc.astype(np.complex128).copy()
    for sd, pc, f in zip(dec.subs, ops["pieces"], fr):
        x = pc["Zrr_inv"] @ f
        dr += sd["Br"] @ x
        fcs -= sd["Bc"].T @ (pc["Zrc"].T @ x)
    c0 = np.concatenate([fcs, -aug["Q"].T @ dr])
    d = dr - aug["G"] @ np.linalg.solve(aug["Kt"], c0)
    return d, c0, fr


def fetidp_aug_solve_dense(dec: Decomposition, alpha: float, f_free):
    """Solve Z x = f by edge-augmented FETI-DP with a dense solve of F_aug mu = d_aug."""
    ops = fetidp_operators(dec, alpha)
    Q, _ = edge_space(dec)
    aug = fetidp_aug_operators(ops, Q)
    d, c0, fr = fetidp_aug_rhs(dec, ops, aug, f_free)
    F = ops["Frr"] + aug["G"] @ np.linalg.solve(aug["Kt"], aug["G"].T)
    mu = np.linalg.lstsq(F, d, rcond=None)[0]
    co = np.linalg.solve(aug["Kt"], c0 + aug["G"].T @ mu)
    uc, nu = co[:dec.nC], co[dec.nC:]
    lam = mu + Q @ nu
    mesh = dec.mesh
    acc = np.zeros(mesh.n_full, dtype=np.complex128)
    for sd, pc, f in zip(dec.subs, ops["pieces"], fr):
        ur = pc["Zrr_inv"] @ (f - pc["Zrc"] @ (sd["Bc"] @ uc) - sd["Br"].T @ lam)
        acc[sd["full"][sd["r"]]] += ur
    cnt = dec.mult.astype(np.float64)
    x_full = acc / np.maximum(cnt, 1)
    x_full[dec.corner_full] = uc
    return x_full[mesh.free_full], {"mu": mu, "d": d, "F": F, "ops": ops, "aug": aug, "nu": nu}


def gmres_iterations(A, Pinv, b, tol, kmax=300):
    """Iterations of right-preconditioned GMRES (zero start, Gram-Schmidt twice)
    until the residual estimate ||b - A x|| / ||b|| <= tol (dense, small cases)."""
    n = b.size
    beta = np.linalg.norm(b)
    Qb = np.zeros((n, kmax + 1), dtype=np.complex128)
    H = np.zeros((kmax + 1, kmax), dtype=np.complex128)
    Qb[:, 0] = b / beta
    g = np.zeros(kmax + 1, dtype=np.complex128)
    g[0] = beta
    cs, sn = [], []
    for j in range(kmax):
        w = A @ (Pinv @ Qb[:, j])
        for _ in range(2):
            h = Qb[:, :j + 1].conj().T @ w
            w = w - Qb[:, :j + 1] @ h
            H[:j + 1, j] += h
        H[j + 1, j] = np.linalg.norm(w)
        Qb[:, j + 1] = w / H[j + 1, j]
        for i in range(j):
            t0 = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
            H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + np.conj(cs[i]) * H[i + 1, j]
            H[i, j] = t0
        den = np.hypot(abs(H[j, j]), abs(H[j + 1, j]))
        c, s = np.conj(H[j, j] / den), np.conj(H[j + 1, j] / den)
        cs.append(c)
        sn.append(s)
        H[j, j] = c * H[j, j] + s * H[j + 1, j]
        H[j + 1, j] = 0
        g[j + 1] = -np.conj(s) * g[j]
        g[j] = c * g[j]
        if abs(g[j + 1]) / beta <= tol:
            return j + 1
    return kmax
