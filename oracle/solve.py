"""Direct FP64 solvers for the KKT system of Sec. 2 (test oracle).

O1  ``range_space_two_factor``: the paper's range-space method (Sec. 3.1, Schur
    system and primal recovery) with S applied through its complex
    factorization (Sec. 4): both complex factors are solved with one sparse LU
    of Z = K + i alpha M, alpha = beta^(-1/2); the second factor Zbar is solved
    by conjugation of the same LU.
O1' ``range_space_one_solve``: the same LU used once, reading (y, lam) off the
    complex solution (see ``range_space_one_solve``).
O2  ``reduced_saddle``: the 2n real saddle system left after eliminating u
    exactly (KKT rows 1 and 3), sparse LU; independent of the factorization.
O3  ``dense_kkt``: numpy.linalg.solve of the full 3n system (tiny meshes).
O4  ``closed_form_sines``: exact discrete solution for targets made of
    discrete sine modes, which are common eigenvectors of K and M.
O5  ``full_space_minres``: the full-space method (Sec. 3.2): MINRES on the
    KKT system with the block-diagonal preconditioner P_mgw = blkdiag(V,
    phi V, S) of Murphy, Golub and Wathen, S^-1 by the two complex factors,
    or with S replaced by the approximation S_p of Pearson and Wathen.
O6  ``pearson_wathen_inverse``: S_p^-1 r, S_p = F V^-1 F with the real
    factor F = K + phi^(-1/2) V (Sec. 3.2, the equation of S_p).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import kkt as _kkt


def schur_rhs(K, Kc, ybar, yc):
    """b = K_c y_c + K ybar, right-hand side of the Schur system (Sec. 3.1)."""
    b = K @ ybar
    if yc is not None:
        b = b + Kc @ yc
    return b


def complex_factor(K, M, beta: float):
    """Z = K + i beta^(-1/2) M, the factor of S (Sec. 4, complex factorization).

    The paper writes S_c = (K + V/(i sqrt(phi))) V^-1 (K - V/(i sqrt(phi))).
    Since 1/i = -i the left factor is K - i alpha M = conj(Z) and the right one
    is Z; S = conj(Z) M^-1 Z = Z M^-1 conj(Z) because the cross terms
    +-i alpha K cancel in either order.
    """
    alpha = beta ** -0.5
    return (K.astype(np.complex128) + 1j * alpha * M).tocsc()


def range_space_two_factor(K, M, Kc, beta, ybar, yc=None, lu=None, paper_y=True):
    """O1: range-space solve with the two complex factors (Sec. 3.1 + Sec. 4).

    lam = S^-1 b = conj(Z)^-1 M Z^-1 b: factor one w1 = Z^-1 b, the middle
    factor v = M w1, factor two lam_hat = conj(Z)^-1 v computed as
    conj(Z^-1 conj(v)) with the same LU.  u = lam / beta (Sec. 3.1, primal
    recovery).  y is read off factor one as y = ybar - Re(w1): with
    z = M^-1 K lam one has w1 = z - i alpha lam exactly, so Re(w1) is the
    paper's M^-1 K lam without a mass solve.  The paper's own formula
    y = ybar - M^-1 K lam is returned as ``y_paper`` for comparison (it needs
    an extra mass-matrix LU; ``paper_y=False`` skips this diagnostic).
    """
    if lu is None:
        lu = spla.splu(complex_factor(K, M, beta))
    b = schur_rhs(K, Kc, ybar, yc).astype(np.complex128)
    w1 = lu.solve(b)
    v = M @ w1
    lam_hat = np.conj(lu.solve(np.conj(v)))
    lam = lam_hat.real.copy()
    u = lam / beta
    y = ybar - w1.real
    y_paper = ybar - spla.splu(M.tocsc()).solve(K @ lam) if paper_y else None
    imag_ratio = float(np.linalg.norm(lam_hat.imag) / max(np.linalg.norm(lam), 1e-300))
    return {"y": y, "u": u, "lam": lam, "w1": w1, "lam_hat": lam_hat,
            "y_paper": y_paper, "imag_ratio": imag_ratio}


def range_space_one_solve(K, M, Kc, beta, ybar, yc=None, lu=None):
    """O1': one solve with Z gives the KKT solution.

    With w = Z^-1 b and lam the solution of the Schur system, w = M^-1 K lam -
    i alpha lam (multiply out Z w = K M^-1 K lam + alpha^2 M lam = S lam = b).
    Hence lam = -Im(w) / alpha, u = lam / beta, y = ybar - Re(w).
    """
    if lu is None:
        lu = spla.splu(complex_factor(K, M, beta))
    alpha = beta ** -0.5
    w = lu.solve(schur_rhs(K, Kc, ybar, yc).astype(np.complex128))
    lam = -w.imag / alpha
    return {"y": ybar - w.real, "u": lam / beta, "lam": lam, "w": w}


def reduced_saddle(K, M, Kc, beta, ybar, yc=None):
    """O2: eliminate u = lam / beta from KKT row 2 and solve rows 1 and 3.

        [ M   K       ] [y  ]   [ M ybar   ]
        [ K  -M/beta  ] [lam] = [ -K_c y_c ]
    """
    n = K.shape[0]
    A2 = sp.bmat([[M, K], [K, -M / beta]], format="csc")
    rhs = np.concatenate([M @ ybar, -(Kc @ yc) if yc is not None else np.zeros(n)])
    x = spla.splu(A2).solve(rhs)
    y, lam = x[:n], x[n:]
    return {"y": y, "u": lam / beta, "lam": lam}


def dense_kkt(K, M, Kc, beta, ybar, yc=None):
    """O3: dense brute-force solve of the 3n KKT system (tiny meshes only)."""
    n = K.shape[0]
    if n > 1500:
        raise ValueError("dense_kkt is for tiny meshes")
    A = _kkt.kkt_matrix(K, M, beta).toarray()
    x = np.linalg.solve(A, _kkt.kkt_rhs(M, Kc, ybar, yc))
    return {"y": x[:n], "u": x[n:2 * n], "lam": x[2 * n:]}


def dense_schur(K, M, beta):
    """S = K M^-1 K + M / beta as a dense matrix (Sec. 3.1), tiny meshes."""
    Kd, Md = K.toarray(), M.toarray()
    return Kd @ np.linalg.solve(Md, Kd) + Md / beta


def sine_mode_eigs(N: int, kvec):
    """Eigenvalues of K and M for the discrete sine mode with wave numbers kvec.

    1D interior rows of the P1 stiffness (1/h)(-1, 2, -1) and mass
    (h/6)(1, 4, 1) act on s(i) = sin(k pi i h) as multiplication by
    kappa_k = (4/h) sin^2(k pi h / 2) and m_k = (h/3)(2 + cos(k pi h)).  The Q1
    matrices are Kronecker sums/products of these (Sec. 2 discretisation on a
    uniform grid), so in d dimensions
        mu_M = prod_d m_kd,  mu_K = sum_d kappa_kd prod_{e != d} m_ke.
    """
    h = 1.0 / N
    kap = [(4.0 / h) * np.sin(k * np.pi * h / 2) ** 2 for k in kvec]
    ms = [(h / 3.0) * (2.0 + np.cos(k * np.pi * h)) for k in kvec]
    muM = float(np.prod(ms))
    muK = 0.0
    for d in range(len(kvec)):
        t = kap[d]
        for e in range(len(kvec)):
            if e != d:
                t *= ms[e]
        muK += t
    return muK, muM


def closed_form_sines(mesh, beta: float, modes, coefs):
    """O4: exact discrete KKT solution for ybar = sum_j a_j s_{k_j} (y_c = 0).

    Each discrete sine s_k (nodal sin(k1 pi x) sin(k2 pi y) [sin(k3 pi z)]) is
    an eigenvector of K and M (``sine_mode_eigs``).  Per mode the KKT system
    of Sec. 2 reduces to 2x2 scalar equations
        mu_M y + mu_K lam = mu_M a,   mu_K y - mu_M lam / beta = 0,
    whose solution is lam = a mu_K mu_M / (mu_K^2 + mu_M^2 / beta),
    y = a (mu_M^2 / beta) / (mu_K^2 + mu_M^2 / beta), u = lam / beta.
    Also returns w = Z^-1 b = sum a mu_K / (mu_K + i alpha mu_M) s_k.
    """
    xyz = mesh.node_xyz("free")
    n = xyz.shape[1]
    y = np.zeros(n)
    lam = np.zeros(n)
    w = np.zeros(n, dtype=np.complex128)
    alpha = beta ** -0.5
    for kvec, a in zip(modes, coefs):
        s = np.ones(n)
        for d, k in enumerate(kvec):
            s = s * np.sin(k * np.pi * xyz[d])
        muK, muM = sine_mode_eigs(mesh.N, kvec)
        den = muK ** 2 + muM ** 2 / beta
        lam += a * muK * muM / den * s
        y += a * (muM ** 2 / beta) / den * s
        w += a * muK / (muK + 1j * alpha * muM) * s
    return {"y": y, "u": lam / beta, "lam": lam, "w": w}


def schur_inverse_two_factor(lu, M, r):
    """S^-1 r for real r by the complex factorization (Sec. 4): with
    S = Z M^-1 conj(Z), S^-1 = conj(Z)^-1 M Z^-1, and for real r the result
    is real: conj(Z^-1 conj(M Z^-1 r)) taken with the LU of Z."""
    w = lu.solve(np.asarray(r, dtype=np.complex128))
    v = M @ w
    return np.conj(lu.solve(np.conj(v))).real


def pearson_wathen_factor(K, M, beta: float):
    """F = K + beta^(-1/2) M: the outer factor of the approximation
    S_p = F M^-1 F of Pearson and Wathen (Sec. 3.2; phi is beta, V is M).
    Real and symmetric positive definite, unlike the complex factor Z."""
    return (K + beta ** -0.5 * M).tocsc()


def pearson_wathen_inverse(lu_p, M, r):
    """O6: S_p^-1 r = F^-1 M F^-1 r, with lu_p the LU of F
    (``pearson_wathen_factor``).  S_p = S + 2 beta^(-1/2) K (the second form of
    the same equation), so S_p^-1 S has its eigenvalues in [1/2, 1]."""
    return lu_p.solve(M @ lu_p.solve(np.asarray(r, dtype=np.float64)))


def full_space_minres(K, M, Kc, beta, ybar, yc=None, tol=1e-12, maxit=50, lu=None, schur="exact"):
    """O5: preconditioned MINRES (C. C. Paige and M. A. Saunders, "Solution of sparse
    indefinite systems of linear equations", SIAM J. Numer. Anal. 12 (1975) 617-629: the
    Lanczos recurrence in the preconditioner's inner product with a Givens QR of the
    tridiagonal matrix and the usual names of its scalars) on A x = b, the KKT system
    of Sec. 2, with P = blkdiag(M, beta M, S) (Sec. 3.2, the preconditioner of
    Murphy, Golub and Wathen, under which A has at most three distinct
    eigenvalues).  schur = "exact" applies S^-1 by the two complex factors;
    "pearson_wathen" puts S_p in place of S (Sec. 3.2, compared with the
    complex factorization in Table 7).  Starts from x = 0; stops when the
    preconditioned residual estimate falls below tol times its initial value.
    Returns (y, u, lam) and the iteration count."""
    n = K.shape[0]
    A = _kkt.kkt_matrix(K, M, beta)
    b = _kkt.kkt_rhs(M, Kc, ybar, yc)
    mlu = spla.splu(M.tocsc())
    if schur == "exact":
        if lu is None:
            lu = spla.splu(complex_factor(K, M, beta))

        def s_inv(r):
            return schur_inverse_two_factor(lu, M, r)
    elif schur == "pearson_wathen":
        lu_p = spla.splu(pearson_wathen_factor(K, M, beta))

        def s_inv(r):
            return pearson_wathen_inverse(lu_p, M, r)
    else:
        raise ValueError(schur)

    def pinv(r):
        return np.concatenate([mlu.solve(r[:n]), mlu.solve(r[n:2 * n]) / beta, s_inv(r[2 * n:])])

    x = np.zeros(3 * n)
    r1 = b.copy()
    y = pinv(r1)
    beta1 = np.sqrt(r1 @ y)
    # Lanczos on P^-1 A in the P-inner product, QR of the tridiagonal matrix
    # by Givens rotations, and the update of x by the search directions w.
    bet, oldb = beta1, 0.0
    dbar = epsln = 0.0
    phibar = beta1
    cs, sn = -1.0, 0.0
    w = np.zeros(3 * n)
    w2 = np.zeros(3 * n)
    r2 = r1.copy()
    its = 0
    for its in range(1, maxit + 1):
        v = y / bet
        y = A @ v
        if its >= 2:
            y = y - (bet / oldb) * r1
        alfa = v @ y
        y = y - (alfa / bet) * r2
        r1, r2 = r2, y
        y = pinv(r2)
        oldb, bet = bet, np.sqrt(r2 @ y)
        oldeps = epsln
        delta = cs * dbar + sn * alfa
        gbar = sn * dbar - cs * alfa
        epsln = sn * bet
        dbar = -cs * bet
        gamma = max(np.hypot(gbar, bet), np.finfo(float).tiny)
        cs, sn = gbar / gamma, bet / gamma
        phi = cs * phibar
        phibar = sn * phibar
        w1, w2 = w2, w
        w = (v - oldeps * w1 - delta * w2) / gamma
        x = x + phi * w
        if phibar <= tol * beta1:
            break
    return x[:n], x[n:2 * n], x[2 * n:], its
