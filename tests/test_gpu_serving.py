"""Serving: continuous batching of range-space requests.

Requests of different meshes, betas and target counts run through one server
worker: each tick gives every occupied slot of every resident instance one
KKT residual and one refinement step in shared launches, and waiting targets
take slots as others finish.  A request's result must not depend on what else
is in flight: alone and in a mix (submitted together and staggered) the
results agree to 1e-12 relative (the one- and four-wide kernels may contract
multiply-adds differently) with identical iteration counts, and every result
meets the KKT gate against the oracle.  Memory admission: a budget that holds
only a few instances forces idle instances out and requests to wait; a
request that can never fit is refused.
"""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import fem, kkt  # noqa: E402
from paper_1312_5653_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def sfdp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1312_5653_amd import sfdp as mod
    return mod


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), device=DEV)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _targets(N, seed, nrhs, with_bc=False):
    ys, ycs = [], []
    for r in range(nrhs):
        if with_bc and r == 0:
            y, yc = W.thermal_target(N)
        else:
            y, yc = W.sine_target(2, N, *W.modes_for("four2d", seed * 11 + r))
        ys.append(y)
        ycs.append(yc)
    return np.stack(ys), np.stack(ycs)


REQUESTS = [  # (n_elem, sub_elem, beta, nrhs, with boundary data)
    (64, 8, 1e-4, 2, False),
    (32, 8, 1e-2, 1, True),
    (96, 8, 3e-6, 3, False),
    (64, 8, 1e-4, 1, False),   # same instance as the first
    (48, 8, 1e-3, 4, True),
    (128, 16, 1e-5, 5, False),  # more targets than slots
]


def test_requests_alone_and_in_mix(sfdp):
    ctx = sfdp.Context(0)
    srv = sfdp.Server(ctx, sfdp.SFDP_MIXED, tol_kkt=1e-8)
    data = [_targets(N, i, k, bc) for i, (N, m, b, k, bc) in enumerate(REQUESTS)]
    alone = []
    for i, (N, m, b, k, bc) in enumerate(REQUESTS):
        tk = srv.submit(N, m, b, _t(data[i][0]), _t(data[i][1]))
        y, u, lam, info, lat, st = srv.poll(tk)
        assert st == 0, info
        alone.append(([t.cpu().numpy() for t in (y, u, lam)], info))
    # the mix: half at once, the rest while the first half is running
    tickets = []
    for i in (0, 2, 4):
        N, m, b, k, bc = REQUESTS[i]
        tickets.append((i, srv.submit(N, m, b, _t(data[i][0]), _t(data[i][1]))))
    time.sleep(0.005)
    for i in (1, 3, 5):
        N, m, b, k, bc = REQUESTS[i]
        tickets.append((i, srv.submit(N, m, b, _t(data[i][0]), _t(data[i][1]))))
    for i, tk in tickets:
        y, u, lam, info, lat, st = srv.poll(tk)
        assert st == 0, info
        (ya, ua, la), infoa = alone[i]
        N, m, b, k, bc = REQUESTS[i]
        ybar, yc = data[i]
        A = fem.assemble(fem.Mesh(2, N))
        for r in range(k):
            for got, ref in ((y[r].cpu().numpy(), ya[r]), (u[r].cpu().numpy(), ua[r]), (lam[r].cpu().numpy(), la[r])):
                assert _rel(got, ref) < 1e-12, (i, r)
            assert info[r]["krylov_its"] == infoa[r]["krylov_its"], (i, r)
            rho = kkt.rel_kkt(A["K"], A["M"], A["Kc"], b, ybar[r], yc[r], ya[r], ua[r], la[r])
            assert rho <= 1e-8, (i, r, rho)
    st = srv.stats()
    assert st["completed"] == 2 * len(REQUESTS) and st["failed"] == 0
    assert st["setups"] == 5  # the repeated (mesh, beta) reuses its resident factors
    srv.close()
    ctx.close()


def test_memory_admission(sfdp):
    # size one 128^2 instance (16 x 16 cells per subdomain) on a context of its own
    probe = sfdp.Context(0)
    p = sfdp.Problem(probe, 2, 128, 16, sfdp.SFDP_MIXED)
    p.set_beta(1e-3)
    p.solve_range_space(_t(_targets(128, 0, 1)[0]))
    one = p.refresh_sizes()["resident_bytes"]
    p.close()
    probe.close()
    # a budget for about two instances and their set-up scratch
    ctx = sfdp.Context(0, mem_budget=int(3.2 * one))
    srv = sfdp.Server(ctx, sfdp.SFDP_MIXED, tol_kkt=1e-8)
    betas = [1e-2, 1e-3, 1e-4, 1e-5, 1e-6]
    data = [_targets(128, 20 + i, 1) for i in range(len(betas))]
    print(f"one instance: {one} B, budget {int(3.2 * one)} B")
    tickets = [srv.submit(128, 16, b, _t(d[0])) for b, d in zip(betas, data)]
    A = fem.assemble(fem.Mesh(2, 128))
    for b, d, tk in zip(betas, data, tickets):
        y, u, lam, info, lat, st = srv.poll(tk)
        assert st == 0
        rho = kkt.rel_kkt(A["K"], A["M"], A["Kc"], b, d[0][0], d[1][0], y[0].cpu().numpy(), u[0].cpu().numpy(),
                          lam[0].cpu().numpy())
        assert rho <= 1e-8, (b, rho)
    s = srv.stats()
    assert s["completed"] == len(betas) and s["evictions"] >= 1, s
    assert s["device_bytes"] <= int(3.2 * one), s
    # a request that can never fit the budget is refused
    tk = srv.submit(512, 32, 1e-4, _t(_targets(512, 1, 1)[0]))
    with pytest.raises(sfdp.SfdpError) as e:
        srv.poll(tk)
    assert e.value.status == -6
    srv.close()
    ctx.close()


def test_large_instances_share_launches(sfdp):
    """A 1024^2 mesh (32 x 32 subdomains, 61504 multipliers) in the same ticks as
    smaller ones: every instance takes no more GMRES blocks than one launch can
    hold at once, and the shared launches narrow their width when the largest
    instance needs it."""
    ctx = sfdp.Context(0)
    srv = sfdp.Server(ctx, sfdp.SFDP_MIXED, tol_kkt=1e-8)
    reqs = [(1024, 32, 1e-4, 2), (768, 32, 1e-6, 1), (128, 32, 1e-2, 3)]
    data = [_targets(N, 40 + i, k) for i, (N, m, b, k) in enumerate(reqs)]
    tickets = [srv.submit(N, m, b, _t(d[0])) for (N, m, b, k), d in zip(reqs, data)]
    for (N, m, b, k), d, tk in zip(reqs, data, tickets):
        y, u, lam, info, lat, st = srv.poll(tk)
        assert st == 0, (N, info)
        A = fem.assemble(fem.Mesh(2, N))
        z = np.zeros(A["Kc"].shape[1])
        for r in range(k):
            rho = kkt.rel_kkt(A["K"], A["M"], A["Kc"], b, d[0][r], z, y[r].cpu().numpy(), u[r].cpu().numpy(),
                              lam[r].cpu().numpy())
            assert rho <= 1e-8, (N, r, rho, info[r])
    s = srv.stats()
    assert s["completed"] == 3 and s["failed"] == 0, s
    srv.close()
    ctx.close()


def test_solo_lane_3d_and_full_space(sfdp):
    """3D requests and full-space requests (MINRES with the factored Schur
    complement) join the same stream as 2D range-space requests: each advances
    one refinement step or MINRES iteration per worker tick, several in flight
    together.  Every result meets the KKT gate; the 3D and full-space results
    equal those of lone problems solved with the same options (1e-12, the same
    iteration counts), although they ran interleaved."""
    ctx = sfdp.Context(0)
    srv = sfdp.Server(ctx, sfdp.SFDP_MIXED, tol_kkt=1e-8)
    reqs = [  # dim, n_elem, sub_elem, beta, nrhs, full space
        (2, 64, 8, 1e-4, 2, False),
        (3, 12, 4, 1e-3, 2, False),
        (2, 48, 8, 1e-3, 1, True),
        (3, 12, 4, 1e-3, 1, True),
        (2, 64, 8, 1e-4, 1, False),
        (3, 16, 4, 1e-5, 3, False),
    ]
    data = []
    for i, (dim, N, m, b, k, fs) in enumerate(reqs):
        kind = "four2d" if dim == 2 else "eight3d"
        ys = np.stack([W.sine_target(dim, N, *W.modes_for(kind, 30 + 5 * i + r))[0] for r in range(k)])
        data.append(ys)
    tickets = [srv.submit(N, m, b, _t(data[i]), dim=dim, full_space=fs)
               for i, (dim, N, m, b, k, fs) in enumerate(reqs)]
    out = []
    for (dim, N, m, b, k, fs), ys, tk in zip(reqs, data, tickets):
        y, u, lam, info, lat, st = srv.poll(tk)
        assert st == 0, (dim, N, fs, info)
        A = fem.assemble(fem.Mesh(dim, N))
        z = np.zeros(A["Kc"].shape[1])
        for r in range(k):
            rho = kkt.rel_kkt(A["K"], A["M"], A["Kc"], b, ys[r], z, y[r].cpu().numpy(), u[r].cpu().numpy(),
                              lam[r].cpu().numpy())
            assert rho <= 1e-8, (dim, N, fs, r, rho, info[r])
            if fs:
                assert info[r]["minres_its"] > 0, info[r]
        out.append((y.cpu().numpy(), info))
    s = srv.stats()
    assert s["completed"] == len(reqs) and s["failed"] == 0, s
    # the four solo requests (two meshes and betas in 3D, two full-space) were in flight together
    assert s["solo_in_flight_max"] >= 3, s
    srv.close()
    # every solo request against a lone problem with the same options
    for i, (dim, N, m, b, k, fs) in enumerate(reqs):
        if dim == 2 and not fs:
            continue
        p = sfdp.Problem(ctx, dim, N, m, sfdp.SFDP_MIXED)
        try:
            p.set_beta(b)
            solve = p.solve_full_space if fs else p.solve_range_space
            y1, _, _, info1, st1 = solve(_t(data[i]), None, tol_kkt=1e-8)
            assert st1 == 0
            for r in range(k):
                assert np.linalg.norm(y1[r].cpu().numpy() - out[i][0][r]) <= 1e-12 * np.linalg.norm(out[i][0][r]), \
                    (i, r)
                assert info1[r]["krylov_its"] == out[i][1][r]["krylov_its"], (i, r)
                assert info1[r]["minres_its"] == out[i][1][r]["minres_its"], (i, r)
        finally:
            p.close()
    ctx.close()
