"""Complex64 set-up arithmetic (sfdp_set_setup_arithmetic(32): the line
factorization and line solves on the FP32 matrix cores) against the dense
definitions and the FP64 set-up, through the C ABI."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fem, feti, kkt, solve
from paper_1312_5653_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def sf():
    from paper_1312_5653_amd import sfdp
    ctx = sfdp.Context(0)
    yield sfdp, ctx
    sfdp.set_setup_arithmetic(64)
    ctx.close()


@pytest.mark.parametrize("N,m,beta", [(32, 8, 1e-4), (64, 32, 1e-3), (40, 20, 1e-6)])
def test_local_operators_within_complex64_rounding(sf, N, m, beta):
    """Z_rr^-1|Delta and the coarse basis from the complex64 set-up match the dense FP64
    definitions to complex64 accuracy (relative 1e-5 of the largest entry), and differ from
    the FP64 set-up's by more than its rounding (so the FP32 path really ran)."""
    sfdp, ctx = sf
    dec = feti.Decomposition(fem.Mesh(2, N), m)
    ops = feti.fetidp_operators(dec, beta ** -0.5)
    out = {}
    for bits in (64, 32):
        sfdp.set_setup_arithmetic(bits)
        p = sfdp.Problem(ctx, 2, N, m, sfdp.SFDP_MIXED)
        try:
            p.set_coarse_space(False)
            p.set_beta(beta)
            out[bits] = [(p.inspect(sfdp.Q_SINV, s).cpu().numpy(), p.inspect(sfdp.Q_PHI, s).cpu().numpy())
                         for s in range(dec.nsub)]
        finally:
            p.close()
    sfdp.set_setup_arithmetic(64)
    dmax = 0.0
    for s, pc in enumerate(ops["pieces"]):
        isd = pc["is_delta"]
        ref_sinv, ref_phi = pc["Zrr_inv"][np.ix_(isd, isd)], pc["Phi"][isd]
        for bits, tol in ((64, 1e-7), (32, 1e-5)):
            sinv, phi = out[bits][s]
            assert np.abs(sinv - ref_sinv).max() / np.abs(ref_sinv).max() < tol, (bits, s)
            assert np.abs(phi - ref_phi).max() / np.abs(ref_phi).max() < tol, (bits, s)
        dmax = max(dmax, np.abs(out[32][s][0] - out[64][s][0]).max() / np.abs(ref_sinv).max())
    assert dmax > 1e-9, dmax


@pytest.mark.parametrize("N,m,beta", [(64, 8, 1e-4), (512, 32, 1e-4)])
def test_range_space_with_complex64_setup(sf, N, m, beta):
    """The range-space solve on factors from the complex64 set-up meets the KKT gate of the
    mixed path (1e-8) through the FP64 outer refinement, and its solution matches O1."""
    sfdp, ctx = sf
    A = fem.assemble(fem.Mesh(2, N))
    ybar = np.stack([W.sine_target(2, N, *W.modes_for("sixteen2d", s))[0] for s in range(2)])
    sfdp.set_setup_arithmetic(32)
    p = sfdp.Problem(ctx, 2, N, m, sfdp.SFDP_MIXED)
    try:
        p.set_beta(beta)
        y, u, lam, info, st = p.solve_range_space(torch.tensor(ybar, device=DEV), None, tol_kkt=1e-8)
        assert st == 0, info
        y, u, lam = (t.cpu().numpy() for t in (y, u, lam))
    finally:
        p.close()
        sfdp.set_setup_arithmetic(64)
    lu = spla.splu(solve.complex_factor(A["K"], A["M"], beta))
    z = np.zeros(A["Kc"].shape[1])
    for q in range(2):
        rho = kkt.rel_kkt(A["K"], A["M"], A["Kc"], beta, ybar[q], z, y[q], u[q], lam[q])
        assert rho <= 1e-8, (q, rho, info[q])
        ref = solve.range_space_two_factor(A["K"], A["M"], A["Kc"], beta, ybar[q], None, lu=lu, paper_y=False)
        assert np.linalg.norm(lam[q] - ref["lam"]) <= 1e-6 * np.linalg.norm(ref["lam"])
        assert np.linalg.norm(y[q] - ref["y"]) <= 1e-7 * np.linalg.norm(ref["y"])
