"""Host arrays (sfdp_opts.host_ptrs): the calls that take sfdp_opts stage host
inputs into a device buffer of the problem and copy the outputs back.  The
kernels and their inputs are the same as with device arrays, so the results
are bitwise equal; the staging buffer is reused across calls and grows for a
larger call.
"""
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
    ctx.close()


def _same(a, b):
    return np.array_equal(a.cpu().numpy(), b.cpu().numpy())


@pytest.mark.parametrize("prec", [0, 1])
def test_poisson_calls_with_host_arrays(sf, prec):
    sfdp, ctx = sf
    N, m = 64, 8
    print(f"\n[host arrays] 2D {N}^2 m={m} prec={prec}", flush=True)
    p = sfdp.Problem(ctx, 2, N, m, prec)
    try:
        _poisson(p, N)
    finally:
        p.close()


def _poisson(p, N):
    p.set_beta(1e-4)
    yb = np.stack([W.sine_target(2, N, *W.modes_for("four2d", s))[0] for s in range(3)])
    yd, yh = torch.tensor(yb, device=DEV), torch.tensor(yb)
    rd = p.solve_range_space(yd, tol_kkt=1e-10)
    rh = p.solve_range_space(yh, tol_kkt=1e-10)
    assert rh[0].device.type == "cpu" and rh[4] == rd[4] == 0
    for a, b in zip(rd[:3], rh[:3]):
        assert _same(a, b)
    # a call with fewer right-hand sides reuses the staging buffer
    r1d = p.solve_range_space(yd[:1].contiguous(), tol_kkt=1e-10)
    r1h = p.solve_range_space(yh[:1].contiguous(), tol_kkt=1e-10)
    assert _same(r1d[0], r1h[0]) and _same(r1d[2], r1h[2])
    zd, _ = p.apply_schur_inv(yd)
    zh, _ = p.apply_schur_inv(yh)
    assert _same(zd, zh)
    n = yb.shape[1]
    f = np.stack([W.random_vector(n, 40 + r, complex_=True) for r in range(2)])
    xd, itd = p.feti_solve(torch.tensor(f, device=DEV), tol_inner=1e-10)
    xh, ith = p.feti_solve(torch.tensor(f), tol_inner=1e-10)
    assert itd == ith and _same(xd, xh)
    fd = p.solve_full_space(yd[:1].contiguous(), tol_kkt=1e-9)
    fh = p.solve_full_space(yh[:1].contiguous(), tol_kkt=1e-9)
    for a, b in zip(fd[:3], fh[:3]):
        assert _same(a, b)


def test_elastic_forward_with_host_arrays(sf):
    sfdp, ctx = sf
    print("\n[host arrays] elasticity n=4 m=2", flush=True)
    p = sfdp.ElasticProblem(ctx, 4, 2)
    try:
        fd = p.pressure_load(1e5)
        ud, itd = p.forward(fd)
        uh, ith = p.forward(fd.cpu())
        assert uh.device.type == "cpu" and itd == ith and _same(ud, uh)
    finally:
        p.close()


def test_host_ptrs_must_be_zero_or_one(sf):
    sfdp, ctx = sf
    p = sfdp.Problem(ctx, 2, 32, 8, 0)
    try:
        p.set_beta(1e-4)
        y = torch.zeros(31 * 31, dtype=torch.float64)
        with pytest.raises(sfdp.SfdpError):
            p.solve_range_space(y, host_ptrs=2)
    finally:
        p.close()
