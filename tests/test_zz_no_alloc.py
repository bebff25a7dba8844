"""The allocation-free KKT residual (sfdp_kkt_residual_noalloc) against the
allocating sfdp_kkt_residual, through the C ABI: two calls in a row, the second
with a smaller input, on 2D and 3D problems; its size limit."""
import numpy as np
import pytest

from paper_1312_5653_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def sf():
    from paper_1312_5653_amd import sfdp
    ctx = sfdp.Context(0)
    yield sfdp, ctx
    ctx.close()


def _iterate(n, nb, nrhs, seed, bdry):
    """Arbitrary (ybar, yc, y, u, lam): random fields, so every residual block is non-zero."""
    f = lambda k, m: np.stack([W.random_vector(m, seed + 10 * k + r) for r in range(nrhs)])
    t = lambda a: torch.tensor(a, device=DEV)
    yc = t(f(1, nb)) if bdry else None
    return t(f(0, n)), yc, t(f(2, n)), t(f(3, n)), t(f(4, n))


def _both(p, nrhs, seed, bdry):
    yb, yc, y, u, lam = _iterate(p.n_free, p.n_bdry, nrhs, seed, bdry)
    ref = np.array(p.kkt_residual(yb, yc, y, u, lam))
    rel = torch.full((nrhs,), -1.0, dtype=torch.float64, device=DEV)
    p.kkt_residual_noalloc(yb, yc, y, u, lam, rel)
    torch.cuda.synchronize()
    return rel.cpu().numpy(), ref


@pytest.mark.parametrize("dim,big,small", [(2, (256, 32), (64, 8)), (3, (24, 8), (12, 4))])
def test_noalloc_residual_equals_the_allocating_one(sf, dim, big, small):
    sfdp, ctx = sf
    pb = sfdp.Problem(ctx, dim, big[0], big[1], sfdp.SFDP_FP64)
    pb.set_beta(1e-4)
    ps = sfdp.Problem(ctx, dim, small[0], small[1], sfdp.SFDP_FP64)
    ps.set_beta(1e-2)
    # first call: the larger mesh, six right-hand sides (two passes over the scratch)
    got, ref = _both(pb, 6, 100, True)
    assert np.all(ref > 0)
    assert np.all(np.abs(got - ref) <= 1e-14 * ref), (got, ref)
    # second call right after: a smaller mesh and fewer right-hand sides, so stale
    # partial sums of the first call sit past the end of what this one writes
    got, ref = _both(ps, 2, 200, False)
    assert np.all(np.abs(got - ref) <= 1e-14 * ref), (got, ref)
    pb.close()
    ps.close()


def test_noalloc_residual_refuses_a_mesh_over_its_limit(sf):
    sfdp, ctx = sf
    p = sfdp.Problem(ctx, 2, 1472, 32, sfdp.SFDP_FP64)   # 1471^2 > 2,096,640 free nodes
    z = torch.zeros(p.n_free, dtype=torch.float64, device=DEV)
    rel = torch.zeros(1, dtype=torch.float64, device=DEV)
    with pytest.raises(sfdp.SfdpError) as e:
        p.kkt_residual_noalloc(z, None, z, z, z, rel)
    assert e.value.status == -1 and "scratch" in str(e.value)
    p.close()
