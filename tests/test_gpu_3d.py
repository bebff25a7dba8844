"""3D instances: Q1 trilinear elements on the unit cube, P^3 subdomains of m^3
cells, FETI-DP with the subdomain vertices as corners and fully redundant
multipliers (Sec. 5), in the range-space refinement of Sec. 3.1 / 4.

Parity with the oracle on the same inputs: the local operators (Z_rr^-1 on
Delta, the Delta Schur complement S_bb, Phi = Z_rr^-1 Z_rc), the coarse
matrix and its inverse, the interface products F_DP, the Dirichlet
preconditioner and the right-hand side d; FETI-DP solves against a sparse
direct solve; range-space solves against the KKT gate of the assembled
system (FP64 and mixed), up to the shape of the 64^3 configuration's
subdomains (8^3 cells, 721 remainder nodes, 378 on the interface).
Complex64 storage (mixed) bounds the operator parity at ~1e-6 relative.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

torch = pytest.importorskip("torch")

from oracle import feti, fem, kkt, solve  # noqa: E402
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


def _target(N, seed):
    return W.sine_target(3, N, *W.modes_for("eight3d", seed))


@pytest.mark.parametrize("N,m", [(4, 2), (6, 2), (12, 4)])
@pytest.mark.parametrize("prec", [0, 1])
def test_local_and_coarse_operators_3d(sf, N, m, prec):
    sfdp, ctx = sf
    beta = 1e-3
    dec = feti.Decomposition(fem.Mesh(3, N), m)
    ops = feti.fetidp_operators(dec, beta ** -0.5)
    prob = sfdp.Problem(ctx, 3, N, m, prec)
    assert prob.sizes["n_mult"] == dec.nmu and prob.sizes["n_corner"] == dec.nC
    prob.set_beta(beta)
    tol = 1e-11 if prec == 0 else 2e-6
    for s in sorted({0, dec.nsub // 2, dec.nsub - 1}):
        pc = ops["pieces"][s]
        isd = pc["is_delta"]
        got = prob.inspect(sfdp.Q_SINV, s).cpu().numpy()
        ref = pc["Zrr_inv"][np.ix_(isd, isd)]
        assert _rel(got, ref) < tol, ("Sinv", s)
        got = prob.inspect(sfdp.Q_SBB, s).cpu().numpy()
        assert _rel(got, pc["Sbb"]) < tol, ("Sbb", s)
        got = prob.inspect(sfdp.Q_PHI, s).cpu().numpy()
        assert _rel(got, pc["Phi"][isd]) < tol, ("Phi", s)
    k = prob.inspect(sfdp.Q_COARSE).cpu().numpy()
    assert _rel(k, ops["Kcc"]) < 1e-12  # FP64 on both paths
    kinv = prob.inspect(sfdp.Q_COARSE_INV).cpu().numpy()
    assert np.abs(kinv @ k - np.eye(dec.nC)).max() < 1e-10
    prob.close()


@pytest.mark.parametrize("N,m", [(6, 2), (12, 4)])
def test_interface_operators_3d(sf, N, m):
    sfdp, ctx = sf
    beta = 1e-3
    mesh = fem.Mesh(3, N)
    dec = feti.Decomposition(mesh, m)
    ops = feti.fetidp_operators(dec, beta ** -0.5)
    prob = sfdp.Problem(ctx, 3, N, m)
    prob.set_beta(beta)
    mu = W.random_vector(dec.nmu, 5, complex_=True)
    F = prob.interface_apply("F", _t(mu)).cpu().numpy()
    assert _rel(F, feti.fetidp_apply(ops, mu)) < 1e-12
    P = prob.interface_apply("P", _t(mu)).cpu().numpy()
    assert _rel(P, feti.dirichlet_preconditioner(dec, ops) @ mu) < 1e-12
    f = W.random_vector(mesh.n, 6, complex_=True)
    d = prob.interface_apply("D", _t(f)).cpu().numpy()
    dref, _, _ = feti.fetidp_rhs(dec, ops, f)
    assert _rel(d, dref) < 1e-12
    prob.close()


@pytest.mark.parametrize("conj_z", [0, 1])
@pytest.mark.parametrize("prec", [0, 1])
def test_feti_solve_3d_matches_direct(sf, conj_z, prec):
    sfdp, ctx = sf
    N, m, beta = 12, 4, 1e-4
    mesh = fem.Mesh(3, N)
    A = fem.assemble(mesh)
    Z = solve.complex_factor(A["K"], A["M"], beta)
    if conj_z:
        Z = Z.conj()
    f = np.stack([W.random_vector(mesh.n, 60 + r, complex_=True) for r in range(2)])
    prob = sfdp.Problem(ctx, 3, N, m, prec)
    prob.set_beta(beta)
    tin = 1e-12 if prec == 0 else 1e-6
    x, its = prob.feti_solve(_t(f), conj_z=bool(conj_z), tol_inner=tin)
    x = x.cpu().numpy()
    lu = spla.splu(Z.tocsc())
    for r in range(len(f)):
        ref = lu.solve(f[r])
        assert _rel(x[r], ref) < (1e-9 if prec == 0 else 1e-5), (r, its)
    print(f"3D FETI-DP N={N} m={m} prec={prec}: GMRES iterations {its}")
    prob.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_range_space_3d_against_oracle(sf, prec):
    sfdp, ctx = sf
    N, m, beta = 12, 4, 1e-4
    A = fem.assemble(fem.Mesh(3, N))
    targets = [_target(N, s) for s in range(2)]
    ybar = np.stack([t[0] for t in targets])
    yc = np.stack([t[1] for t in targets])
    prob = sfdp.Problem(ctx, 3, N, m, prec)
    prob.set_beta(beta)
    tol = 1e-10 if prec == 0 else 1e-8
    y, u, lam, info, st = prob.solve_range_space(_t(ybar), _t(yc), tol_kkt=tol)
    assert st == 0, info
    y, u, lam = (v.cpu().numpy() for v in (y, u, lam))
    for q in range(2):
        rho = kkt.rel_kkt(A["K"], A["M"], A["Kc"], beta, ybar[q], yc[q], y[q], u[q], lam[q])
        ref = solve.range_space_two_factor(A["K"], A["M"], A["Kc"], beta, ybar[q], yc[q], paper_y=False)
        rho_ref = kkt.rel_kkt(A["K"], A["M"], A["Kc"], beta, ybar[q], yc[q], ref["y"], ref["u"], ref["lam"])
        assert rho <= max(tol, 2 * rho_ref), (q, rho, rho_ref, info[q])
        if prec == 0:
            assert _rel(lam[q], ref["lam"]) < 1e-8 and _rel(y[q], ref["y"]) < 1e-8
    # one solve per refinement step (the first factor alone) gives the same solution
    y1, u1, l1, info1, st1 = prob.solve_range_space(_t(ybar), _t(yc), tol_kkt=tol, factors=1)
    assert st1 == 0 and all(i["n_feti"] == i["outer_steps"] for i in info1)
    for q in range(2):
        rho = kkt.rel_kkt(A["K"], A["M"], A["Kc"], beta, ybar[q], yc[q], *(v[q].cpu().numpy() for v in (y1, u1, l1)))
        assert rho <= max(tol, 1e-9), (q, rho)
    prob.close()


def test_range_space_3d_subdomains_of_the_64_cube_shape(sf):
    """32^3 cells in 4^3 subdomains of 8^3 (the subdomain shape of the 64^3
    configuration: 721 remainder nodes, 378 on the interface), mixed precision,
    against the KKT gate of the assembled system."""
    sfdp, ctx = sf
    N, m, beta = 32, 8, 1e-4
    A = fem.assemble(fem.Mesh(3, N))
    ybar, yc = _target(N, 0)
    prob = sfdp.Problem(ctx, 3, N, m, sfdp.SFDP_MIXED)
    prob.set_beta(beta)
    y, u, lam, info, st = prob.solve_range_space(_t(ybar[None]), None, tol_kkt=1e-8)
    assert st == 0, info
    z = np.zeros(A["Kc"].shape[1])
    rho = kkt.rel_kkt(A["K"], A["M"], A["Kc"], beta, ybar, z, *(v[0].cpu().numpy() for v in (y, u, lam)))
    print(f"3D 32^3 / 8^3 mixed: rho={rho:.2e} info={info[0]}")
    assert rho <= 1e-8
    prob.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_range_space_3d_grouping_invariance(sf, prec):
    """Three targets solved one per group and all in one group (every operator
    read once for the group; each right-hand side keeps its own Krylov basis,
    Hessenberg matrix and stopping test): the same iterates, to 1e-12."""
    sfdp, ctx = sf
    N, m, beta = 12, 4, 1e-4
    ybar = np.stack([_target(N, 10 + s)[0] for s in range(3)])
    ybar[1] *= 1e3
    prob = sfdp.Problem(ctx, 3, N, m, prec)
    prob.set_beta(beta)
    tol = 1e-10 if prec == 0 else 1e-8
    runs = {}
    for batch in (1, 4):
        y, u, lam, info, st = prob.solve_range_space(_t(ybar), None, tol_kkt=tol, batch=batch)
        assert st == 0, (batch, info)
        runs[batch] = [v.cpu().numpy() for v in (y, u, lam)], info
    (y1, u1, l1), i1 = runs[1]
    (y4, u4, l4), i4 = runs[4]
    for q in range(3):
        for a, b in ((y4[q], y1[q]), (u4[q], u1[q]), (l4[q], l1[q])):
            assert _rel(a, b) < 1e-12, q
        assert i4[q]["krylov_its"] == i1[q]["krylov_its"], q
    prob.close()


def test_range_space_3d_full_configuration(sf):
    """The 3D bench configuration itself: 64^3 cells, 8^3 subdomains of 8^3,
    beta = 1e-4, four 8-mode targets in one group, mixed precision; every
    result against the KKT gate of the oracle's assembled system."""
    sfdp, ctx = sf
    N, m, beta = 64, 8, 1e-4
    A = fem.assemble(fem.Mesh(3, N))
    ybar = np.stack([_target(N, s)[0] for s in range(4)])
    prob = sfdp.Problem(ctx, 3, N, m, sfdp.SFDP_MIXED)
    prob.set_beta(beta)
    y, u, lam, info, st = prob.solve_range_space(_t(ybar), None, tol_kkt=1e-8)
    assert st == 0, info
    z = np.zeros(A["Kc"].shape[1])
    for q in range(4):
        rho = kkt.rel_kkt(A["K"], A["M"], A["Kc"], beta, ybar[q], z, *(v[q].cpu().numpy() for v in (y, u, lam)))
        assert rho <= 1e-8, (q, rho, info[q])
        assert info[q]["rel_kkt"] <= 1e-8, info[q]
    prob.close()
