"""The KKT saddle-point system of the discrete control problem and its metrics.

Sec. 2, discrete QP and its Lagrangian: minimise
    1/2 ||y - ybar||_V^2 + beta/2 ||u||_V^2   s.t.   K y + K_c y_c = V u,
with L = ... + lam^T (K y + K_c y_c - V u).  The first-order conditions are the
3n x 3n symmetric indefinite system (Sec. 2, KKT system)

    [ V    0     K ] [y  ]   [ V ybar    ]
    [ 0  beta V -V ] [u  ] = [ 0         ]
    [ K   -V     0 ] [lam]   [ -K_c y_c  ].

The paper's regularisation phi is called beta here, and its volume matrix V
is the consistent mass matrix M.

Metrics
-------
rel_kkt           ||b - A x||_2 / ||b||_2, the relative KKT residual.
constraint_viol   ||K y + K_c y_c - V u||_2 / ||K y||_2 (Sec. 6.2, relative
                  constraint violation).
eta_blk           max over the three block rows i of
                  ||r_i|| / (sum_j || |A_ij| |x_j| || + ||b_i||), a blockwise
                  backward error.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def kkt_matrix(K, M, beta: float):
    """Assemble A of the KKT system (Sec. 2) as a sparse CSR matrix."""
    n = K.shape[0]
    Z = sp.csr_matrix((n, n))
    return sp.bmat([[M, Z, K], [Z, beta * M, -M], [K, -M, Z]], format="csr")


def kkt_rhs(M, Kc, ybar, yc):
    """Right-hand side (V ybar, 0, -K_c y_c) of the KKT system (Sec. 2)."""
    ybar = np.asarray(ybar, dtype=np.float64)
    n = ybar.shape[0]
    yc = np.zeros(Kc.shape[1]) if yc is None else np.asarray(yc, dtype=np.float64)
    return np.concatenate([M @ ybar, np.zeros(n), -(Kc @ yc)])


def kkt_residual_blocks(K, M, Kc, beta, ybar, yc, y, u, lam):
    """Block rows (r1, r2, r3) of b - A x for x = (y, u, lam)."""
    yc = np.zeros(Kc.shape[1]) if yc is None else yc
    r1 = M @ ybar - (M @ y + K @ lam)
    r2 = -(beta * (M @ u) - M @ lam)
    r3 = -(Kc @ yc) - (K @ y - M @ u)
    return r1, r2, r3


def rel_kkt(K, M, Kc, beta, ybar, yc, y, u, lam) -> float:
    """Relative KKT residual ||b - A x|| / ||b|| in the paper's scaling."""
    r1, r2, r3 = kkt_residual_blocks(K, M, Kc, beta, ybar, yc, y, u, lam)
    b = kkt_rhs(M, Kc, ybar, yc)
    return float(np.sqrt(r1 @ r1 + r2 @ r2 + r3 @ r3) / np.linalg.norm(b))


def constraint_violation(K, M, Kc, yc, y, u) -> float:
    """Relative constraint violation of Sec. 6.2."""
    yc = np.zeros(Kc.shape[1]) if yc is None else yc
    c = K @ y + Kc @ yc - M @ u
    return float(np.linalg.norm(c) / np.linalg.norm(K @ y))


def eta_blk(K, M, Kc, beta, ybar, yc, y, u, lam) -> float:
    """Blockwise normwise backward error of x = (y, u, lam) for the KKT system."""
    yc = np.zeros(Kc.shape[1]) if yc is None else yc
    aK, aM, aKc = abs(K), abs(M), abs(Kc)
    r1, r2, r3 = kkt_residual_blocks(K, M, Kc, beta, ybar, yc, y, u, lam)
    b1, b3 = M @ ybar, -(Kc @ yc)
    ay, au, al = np.abs(y), np.abs(u), np.abs(lam)
    d1 = np.linalg.norm(aM @ ay) + np.linalg.norm(aK @ al) + np.linalg.norm(b1)
    d2 = beta * np.linalg.norm(aM @ au) + np.linalg.norm(aM @ al)
    d3 = np.linalg.norm(aK @ ay) + np.linalg.norm(aM @ au) + np.linalg.norm(aKc @ np.abs(yc))
    out = 0.0
    for r, d in ((r1, d1), (r2, d2), (r3, d3)):
        nr = np.linalg.norm(r)
        if nr > 0:
            out = max(out, nr / d)
    return float(out)
