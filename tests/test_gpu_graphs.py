"""Graph replay of the refinement steps (sfdp_set_graphs) against eager steps,
through the C ABI: every replay bitwise equal to the eager result, with eager
work and other solves between the replays; captured steps dropped after a new
beta; the mixed 512^2 group of four targets."""
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
    sfdp.set_graphs(False)
    ctx.close()


def _targets(N, nt, seed=0):
    return torch.tensor(np.stack([W.sine_target(2, N, *W.modes_for("sixteen2d", seed + s))[0]
                                  for s in range(nt)]), device=DEV)


def _solve(p, yb, **kw):
    y, u, lam = (torch.empty_like(yb) for _ in range(3))
    _, _, _, info, st = p.solve_range_space(yb, None, y, u, lam, **kw)
    assert st == 0, info
    torch.cuda.synchronize()
    return [t.cpu().numpy().copy() for t in (y, u, lam)], [i["krylov_its"] for i in info], (y, u, lam)


@pytest.mark.parametrize("prec,N,m", [(1, 128, 32), (0, 64, 8), (1, 512, 32)])
def test_graph_replays_equal_eager_steps(sf, prec, N, m):
    sfdp, ctx = sf
    p = sfdp.Problem(ctx, 2, N, m, prec)
    try:
        _replays(sfdp, p, N)
    finally:
        p.close()
        sfdp.set_graphs(False)


def _replays(sfdp, p, N):
    p.set_beta(1e-4)
    yb = _targets(N, 4)
    yb1 = _targets(N, 1, seed=7)
    sfdp.set_graphs(False)
    ref, ref_its, _ = _solve(p, yb)
    ref1, ref1_its, _ = _solve(p, yb1)
    sfdp.set_graphs(True)
    # the same caller arrays every call, so the second call captures and later ones replay
    y, u, lam = (torch.empty_like(yb) for _ in range(3))
    y1, u1, lam1 = (torch.empty_like(yb1) for _ in range(3))
    for call in range(5):
        for t in (y, u, lam):
            t.fill_(float("nan"))  # a replay must write every output
        _, _, _, info, st = p.solve_range_space(yb, None, y, u, lam)
        assert st == 0, info
        torch.cuda.synchronize()
        got = [t.cpu().numpy() for t in (y, u, lam)]
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), (call, float(np.max(np.abs(a - b))))
        assert [i["krylov_its"] for i in info] == ref_its, call
        # eager work of the program and another group's steps between replays
        z = torch.randn(1 << 20, device=DEV)
        torch.cuda.synchronize()
        assert float((z * 0).sum()) == 0.0
        _, _, _, info1, st1 = p.solve_range_space(yb1, None, y1, u1, lam1)
        assert st1 == 0
        torch.cuda.synchronize()
        for a, b in zip((y1, u1, lam1), ref1):
            assert np.array_equal(a.cpu().numpy(), b), call
        assert [i["krylov_its"] for i in info1] == ref1_its


def test_captured_steps_follow_a_new_beta(sf):
    sfdp, ctx = sf
    N, m = 64, 8
    p = sfdp.Problem(ctx, 2, N, m, sfdp.SFDP_MIXED)
    yb = _targets(N, 2)
    out = {}
    try:
        _beta_runs(sfdp, p, yb, out)
    finally:
        p.close()
        sfdp.set_graphs(False)
    for (a, ia), (b, ib) in zip(out[False], out[True]):
        assert ia == ib
        for x, z in zip(a, b):
            assert np.array_equal(x, z)


def _beta_runs(sfdp, p, yb, out):
    for graphs in (False, True):
        sfdp.set_graphs(graphs)
        res = []
        for beta in (1e-2, 1e-5):
            p.set_beta(beta)
            for _ in range(3):  # eager, captured, replayed
                got, its, _ = _solve(p, yb)
            res.append((got, its))
        out[graphs] = res
