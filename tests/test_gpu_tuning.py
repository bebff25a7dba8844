"""Launch-variant autotuning: the variants it chooses between compute the same
results, so a solve with tuning switched on (its first call times every
candidate on the real operands) equals one with the fixed defaults, to the
rounding of multiply-add contraction, with the same iteration counts."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

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
    sfdp.set_tuning(True)
    ctx.close()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("dim,N,m,prec", [(2, 64, 8, 1), (2, 64, 8, 0), (3, 12, 4, 1), (3, 12, 4, 0)])
def test_tuned_and_default_variants_agree(sf, dim, N, m, prec):
    sfdp, ctx = sf
    kind = "sixteen2d" if dim == 2 else "eight3d"
    ybar = np.stack([W.sine_target(dim, N, *W.modes_for(kind, 70 + r))[0] for r in range(3)])
    yt = torch.tensor(ybar, device=DEV)
    tol = 1e-10 if prec == 0 else 1e-8
    out = {}
    for tuned in (False, True):
        sfdp.set_tuning(tuned)
        p = sfdp.Problem(ctx, dim, N, m, prec)
        p.set_beta(1e-4)
        y, u, lam, info, st = p.solve_range_space(yt, None, tol_kkt=tol)
        assert st == 0, info
        out[tuned] = ([v.cpu().numpy() for v in (y, u, lam)], info)
        p.close()
    (a, ia), (b, ib) = out[False], out[True]
    for q in range(3):
        for x0, x1 in zip(a, b):
            assert _rel(x1[q], x0[q]) < 1e-12, q
        assert ia[q]["krylov_its"] == ib[q]["krylov_its"], q


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("N,m", [(64, 8), (96, 32), (40, 20)])
def test_local_solve_variants_agree(sf, prec, N, m):
    """The four launch forms of the 2D subdomain solve (one workgroup for every
    right-hand side, one per right-hand side, one wavefront per right-hand side, one
    workgroup with a wavefront per right-hand side and the line factors staged once)
    give the same FETI-DP solves and iteration counts, for one and for three
    right-hand sides, including subdomains of 32 x 32 cells (33-node lines, one per lane
    of a wavefront and no padding) and of 20 x 20.  The forms sum the line products in
    different orders; that rounding, carried through a GMRES solve to a relative
    interface residual of 1e-10 on an interface operator of condition ~1e4, has been
    seen at 2e-12 and 1.2e-11 (complex64 factors, 20 x 20 subdomains), so the solves are
    compared at the inner tolerance itself, 1e-10: below it the two results are equally
    good solutions."""
    sfdp, ctx = sf
    n = (N - 1) ** 2
    f = torch.tensor(np.stack([W.random_vector(n, 80 + r, complex_=True) for r in range(3)]), device=DEV)
    out = {}
    try:
        for c in (0, 1, 2, 3):
            sfdp.force_variant(c)
            p = sfdp.Problem(ctx, 2, N, m, prec)
            p.set_beta(1e-4)
            x3, its3 = p.feti_solve(f, tol_inner=1e-10)
            x1, its1 = p.feti_solve(f[:1].contiguous(), conj_z=True, tol_inner=1e-10)
            out[c] = (x3.cpu().numpy(), its3, x1.cpu().numpy(), its1)
            p.close()
    finally:
        sfdp.set_tuning(True)
    for c in (0, 1, 3):
        assert out[c][1] == out[2][1] and out[c][3] == out[2][3], c
        for q in range(3):
            assert _rel(out[c][0][q], out[2][0][q]) < 1e-10, (c, q)
        assert _rel(out[c][2][0], out[2][2][0]) < 1e-10, c
