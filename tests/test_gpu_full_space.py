"""Full-space method (Sec. 3.2): MINRES on the KKT system with the
block-diagonal preconditioner blkdiag(V, phi V, S) of Murphy, Golub and
Wathen, S^-1 by the complex factorization through FETI-DP, inside FP64
refinement on the KKT residual.  The result is the KKT solution, the same
the range-space method gives: parity against the oracle's direct solve and
its KKT gate; the iteration count reflects the three eigenvalues of the
preconditioned matrix (a few more with inexact S^-1).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import fem, kkt, solve  # noqa: E402
from paper_1312_5653_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def sf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1312_5653_amd import sfdp
    ctx = sfdp.Context(0)
    yield sfdp, ctx
    ctx.close()


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), device=DEV)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("dim,N,m,prec", [(2, 64, 8, 0), (2, 64, 8, 1), (3, 12, 4, 0), (3, 12, 4, 1)])
def test_full_space_matches_kkt_solution(sf, dim, N, m, prec):
    sfdp, ctx = sf
    beta = 1e-4
    A = fem.assemble(fem.Mesh(dim, N))
    if dim == 2:
        y0, c0 = W.thermal_target(N)
        y1, c1 = W.sine_target(2, N, *W.modes_for("sixteen2d", 3))
    else:
        y0, c0 = W.sine_target(3, N, *W.modes_for("eight3d", 0))
        y1, c1 = W.sine_target(3, N, *W.modes_for("eight3d", 1))
    ybar, yc = np.stack([y0, y1]), np.stack([c0, c1])
    prob = sfdp.Problem(ctx, dim, N, m, prec)
    prob.set_beta(beta)
    tol = 1e-10 if prec == 0 else 1e-8
    y, u, lam, info, st = prob.solve_full_space(_t(ybar), _t(yc), tol_kkt=tol)
    assert st == 0, info
    y, u, lam = (v.cpu().numpy() for v in (y, u, lam))
    for q in range(2):
        rho = kkt.rel_kkt(A["K"], A["M"], A["Kc"], beta, ybar[q], yc[q], y[q], u[q], lam[q])
        ref = solve.range_space_two_factor(A["K"], A["M"], A["Kc"], beta, ybar[q], yc[q], paper_y=False)
        rho_ref = kkt.rel_kkt(A["K"], A["M"], A["Kc"], beta, ybar[q], yc[q], ref["y"], ref["u"], ref["lam"])
        assert rho <= max(tol, 2 * rho_ref), (q, rho, info[q])
        assert _rel(lam[q], ref["lam"]) < (1e-8 if prec == 0 else 1e-6), q
        # P_mgw: three eigenvalues, so few MINRES iterations per refinement step
        assert info[q]["minres_its"] <= 6 * info[q]["outer_steps"], info[q]
        assert info[q]["n_feti"] == 2 * (info[q]["minres_its"] + info[q]["outer_steps"]), info[q]
        print(f"dim={dim} N={N} prec={prec} q={q}: rho={rho:.2e} {info[q]}")
    prob.close()


@pytest.mark.parametrize("dim,N", [(2, 48), (2, 1024), (3, 20)])
def test_mass_inverse(sf, dim, N):
    """The V block of P_mgw: M^-1 x by tridiagonal solves along each axis (M is
    the Kronecker product of the 1D free-node mass matrices), against a sparse
    direct solve."""
    import scipy.sparse.linalg as spla
    sfdp, ctx = sf
    prob = sfdp.Problem(ctx, dim, N, 4 if dim == 3 else 16)
    x = np.stack([W.random_vector((N - 1) ** dim, 3 + r) for r in range(2)])
    z = prob.apply_operator("I", _t(x)).cpu().numpy()
    M = fem.assemble(fem.Mesh(dim, N))["M"].tocsc()
    lu = spla.splu(M)
    for r in range(2):
        assert _rel(z[r], lu.solve(x[r])) < 1e-12, r
    prob.close()
