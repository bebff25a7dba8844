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
