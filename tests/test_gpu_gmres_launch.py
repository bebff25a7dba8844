"""GMRES launch forms of the range-space solve (sfdp_set_gmres_launch), through
the C ABI: cooperative launches, plain launches that check their grid's
co-residency, and plain launches whose check is made to fail (no wait), which
leave the refinement step's iterate unchanged and run the step again
cooperatively.  Every form gives the same y, u, lam bit for bit, with the same
iteration counts, with and without graph replay of the steps."""
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
    sfdp.set_gmres_launch(1)
    sfdp.set_graphs(False)
    ctx.close()


def _run(sfdp, ctx, mode, prec, N, m, graphs, calls):
    sfdp.set_gmres_launch(mode)
    sfdp.set_graphs(graphs)
    try:
        p = sfdp.Problem(ctx, 2, N, m, prec)
        p.set_beta(1e-4)
        yb = torch.tensor(np.stack([W.sine_target(2, N, *W.modes_for("sixteen2d", 40 + s))[0] for s in range(3)]),
                          device=DEV)
        out = []
        for _ in range(calls):
            y, u, lam = (torch.empty_like(yb) for _ in range(3))
            _, _, _, info, st = p.solve_range_space(yb, None, y, u, lam)
            assert st == 0, info
            torch.cuda.synchronize()
            out.append(([t.cpu().numpy().copy() for t in (y, u, lam)],
                        [(i["krylov_total"], i["outer_steps"], i["n_feti"]) for i in info]))
        p.close()
        return out
    finally:
        sfdp.set_gmres_launch(1)
        sfdp.set_graphs(False)


@pytest.mark.parametrize("prec,N,m", [(1, 64, 8), (0, 64, 16), (1, 128, 32)])
@pytest.mark.parametrize("graphs", [False, True])
def test_launch_forms_give_the_same_solves(sf, prec, N, m, graphs):
    sfdp, ctx = sf
    calls = 3 if graphs else 2  # with graphs: the second call captures, the third replays
    ref = _run(sfdp, ctx, 0, prec, N, m, graphs, calls)
    for mode in (1, 2):
        got = _run(sfdp, ctx, mode, prec, N, m, graphs, calls)
        for (xa, ia), (xb, ib) in zip(ref, got):
            assert ia == ib, (mode, ia, ib)
            for a, b in zip(xa, xb):
                assert np.array_equal(a, b), mode


def test_timing_modes_record_the_kernels_they_name(sf):
    """sfdp_timing_enable: 1 times the GMRES and subdomain-solve launches, 2 the
    GMRES launches only; the solves are the same either way."""
    sfdp, ctx = sf
    p = sfdp.Problem(ctx, 2, 64, 8, 1)
    p.set_beta(1e-4)
    yb = torch.tensor(np.stack([W.sine_target(2, 64, *W.modes_for("sixteen2d", 50 + s))[0] for s in range(2)]),
                      device=DEV)
    res = {}
    for mode in (1, 2):
        p.timing_enable(mode)
        y, u, lam = (torch.empty_like(yb) for _ in range(3))
        _, _, _, info, st = p.solve_range_space(yb, None, y, u, lam)
        assert st == 0, info
        res[mode] = (p.kernel_times(), y.cpu().numpy())
        p.timing_enable(0)
    (k1, y1), (k2, y2) = res[1], res[2]
    assert k1["gmres_launches"] > 0 and k1["local_launches"] > 0 and k1["local_ms"] > 0
    assert k2["gmres_launches"] == k1["gmres_launches"] and k2["gmres_ms"] > 0
    assert k2["local_launches"] == 0 and k2["local_ms"] == 0
    assert np.array_equal(y1, y2)
    p.close()
