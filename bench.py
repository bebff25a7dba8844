#!/usr/bin/env python
"""Benchmark: range-space Schur solves per second on one MI355X.

Workload (the paper's thermal problem family, Sec. 6.1, at the 512^2 size):
2D unit square, Q1 Poisson, 512 x 512 cells (261,121 free dofs), 16 x 16
subdomains of 32 x 32 cells, beta = 1e-4, target ybar = 16 sine modes
sin(k pi x) sin(l pi y), k, l in 1..4, N(0,1) coefficients (seed 0), y_c = 0.
One step = one call that solves a batch of B targets (16-mode sine targets,
seeds 0..B-1), each a range-space Schur solve (two-factor complex
factorization, FETI-DP per factor, FP64 refinement) to relative KKT residual
<= 1e-8, with the subdomain factors resident (sfdp_set_beta is done once,
outside the timed region, and reported as setup_ms).  The B targets of a step
share every launch (opts.batch = B).  The headline is mixed precision at
B = 4; single-target latency (B = 1) and the FP64 path are measured beside it.

Prints one JSON line.  --gpus > 1 is not supported (one process, one GPU).
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "k_gmres_traffic_512x512.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1312_5653_amd", "csrc", "solve.hip")


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter record
    (rocprofv3 FETCH_SIZE and WRITE_SIZE, scaled by the same counters on a
    plain copy of known size), or None when the record is missing or was taken
    on a different version of the kernel source."""
    import hashlib
    try:
        rec = json.load(open(TRAFFIC_RECORD))
        src = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != src or kernel not in rec.get("kernels", {}):
        return None
    return rec["kernels"][kernel]["bytes_per_launch"]


def gmres_operator_bytes(N, m, ncoarse, edges, elem_bytes):
    """Operator bytes one GMRES loop trip must pass over, shared by all the
    right-hand sides of the launch: per subdomain the packed symmetric
    interface Schur complement (complex64) and the packed Z_rr^-1|Delta
    (storage precision), n_d (n_d + 1) / 2 entries each, and the coarse basis
    (n_d x (corners + edges when edge-augmented), storage precision); the
    coarse inverse once (n_K^2 FP64 complex)."""
    P = N // m
    tot = 0
    for sy in range(P):
        for sx in range(P):
            sides = sum(1 for side in (sx > 0, sx < P - 1, sy > 0, sy < P - 1) if side)
            nd = (m - 1) * sides
            nc = sum(1 for cx in (sx, sx + 1) for cy in (sy, sy + 1) if 0 < cx < P and 0 < cy < P)
            nq = nc + (sides if edges else 0)
            tot += nd * (nd + 1) // 2 * (8 + elem_bytes) + nd * nq * elem_bytes
    return tot + ncoarse * ncoarse * 16


def gmres_vector_bytes(nmu, mean_its):
    """Vector bytes of one GMRES iteration of one right-hand side (FP64
    complex): the Krylov basis read twice for classical Gram-Schmidt run twice
    (4 (j + 1) vectors at step j, j averaged over the solve) and six further
    vector reads or writes."""
    jmean = (mean_its - 1) / 2.0
    return (4 * (jmean + 1) + 6) * nmu * 16


def local_solve_bytes(N, m, elem_bytes, nrhs):
    """Bytes one subdomain-solve launch must move for nrhs right-hand sides: the
    line factors of every subdomain (m + 1 lines of (m + 1)^2 entries) once in
    the forward and once in the backward sweep, shared by all right-hand sides,
    plus each right-hand side's load vector and result (FP64 complex)."""
    P = N // m
    ml = m + 1
    return P * P * ml * ml * ml * elem_bytes * 2 + nrhs * 2 * (N - 1) ** 2 * 16


def _kernel_key(name):
    """'void sfdp::k_gmres<sfdp::C<float>, 4>(sfdp::Geo2, ...)' -> 'k_gmres<C<float>, 4>'."""
    name = name.replace("void ", "").replace("sfdp::", "")
    depth = 0
    for i, ch in enumerate(name):
        depth += ch == "<"
        depth -= ch == ">"
        if ch == "(" and depth == 0:
            return name[:i]
    return name


def write_traffic_record(fetch_dir, write_dir, copy_mib):
    """Turn two rocprofv3 --pmc runs of this script (FETCH_SIZE, then
    WRITE_SIZE, both with --copy-check copy_mib) into the traffic record: every
    kernel's mean counter value per dispatch, divided by the factor the same
    counter reads on the plain copy (copy_mib MiB read, copy_mib MiB written)."""
    import collections
    import csv
    import glob
    import hashlib

    def per_kernel(d, counter):
        vals = collections.defaultdict(list)
        for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(path)):
                if r.get("Counter_Name") == counter:
                    vals[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        return vals

    fet, wri = per_kernel(fetch_dir, "FETCH_SIZE"), per_kernel(write_dir, "WRITE_SIZE")
    copy = [k for k in fet if "Mul" in k]
    if len(copy) != 1:
        raise SystemExit(f"expected one calibration copy kernel, found {copy}")
    kib = copy_mib * 1024.0
    f_fac = statistics.mean(fet[copy[0]]) / kib
    w_fac = statistics.mean(wri[copy[0]]) / kib
    kernels = {}
    for k in fet:
        key = _kernel_key(k)
        if not key.startswith("k_") or k not in wri:
            continue
        fb = statistics.mean(fet[k]) / f_fac * 1024.0
        wb = statistics.mean(wri[k]) / w_fac * 1024.0
        kernels[key] = {"fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
                        "bytes_per_launch": fb + wb, "dispatches": len(fet[k])}
    rec = {"source_sha256": hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest(),
           "copy_mib": copy_mib, "fetch_factor": f_fac, "write_factor": w_fac, "kernels": kernels}
    with open(TRAFFIC_RECORD, "w") as fh:
        json.dump(rec, fh, indent=1, sort_keys=True)
    print(json.dumps({"fetch_factor": f_fac, "write_factor": w_fac,
                      "k_gmres": {k: v["bytes_per_launch"] for k, v in kernels.items() if "gmres" in k}}))


# ---- cpu_baseline leg: the CPU oracle on the same workloads --------------------------------
# The only code in this script that imports or runs oracle/: it times the oracle (cpu_baseline)
# and provides the oracle's solutions of the very inputs the GPU lines solve, against which
# each line's forward error is stated.


def cpu_model():
    """The host CPU's model name (/proc/cpuinfo) and the cores this process may use."""
    name = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                name = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"model": name, "os_cpu_count": os.cpu_count(), "usable_cores": usable}


class OracleLeg:
    """Oracle references of the GPU lines' inputs: O1 (SuperLU of Z, the paper's two-factor
    solve, FP64; one factorization per (dim, N, beta), kept) and, for sine-mode targets, the
    closed form of the exact discrete solution."""

    def __init__(self):
        self.lu = {}
        self.mats = {}

    def _mats(self, dim, N):
        from oracle import fem
        if (dim, N) not in self.mats:
            self.mats[(dim, N)] = fem.assemble(fem.Mesh(dim, N))
        return self.mats[(dim, N)]

    def o1(self, dim, N, beta, ybars):
        import scipy.sparse.linalg as spla
        from oracle import solve
        A = self._mats(dim, N)
        key = (dim, N, beta)
        if key not in self.lu:
            self.lu = {key: spla.splu(solve.complex_factor(A["K"], A["M"], beta))}  # keep one factor
        return [solve.range_space_two_factor(A["K"], A["M"], A["Kc"], beta, yb, None, lu=self.lu[key],
                                             paper_y=False) for yb in ybars]

    @staticmethod
    def closed(dim, N, beta, modes_coefs):
        from oracle import fem, solve
        mesh = fem.Mesh(dim, N)
        return [solve.closed_form_sines(mesh, beta, m, c) for m, c in modes_coefs]


def fwd_err(outs, refs):
    """Max over targets and over y, u, lam of the relative 2-norm error of the GPU result."""
    if refs is None:
        return None
    worst = 0.0
    for (y, u, lam), r in zip(outs, refs):
        for a, b in ((y, r["y"]), (u, r["u"]), (lam, r["lam"])):
            worst = max(worst, float(((a - b) ** 2).sum() ** 0.5 / max((b ** 2).sum() ** 0.5, 1e-300)))
    return worst


def cpu_baseline(N, m, beta, ybar, budget_s=15.0):
    """The CPU oracle (SciPy SuperLU of Z, two-factor solve) on the same workload."""
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    import scipy.sparse.linalg as spla
    from oracle import fem, solve
    A = fem.assemble(fem.Mesh(2, N))
    t0 = time.perf_counter()
    lu = spla.splu(solve.complex_factor(A["K"], A["M"], beta))
    t_factor = time.perf_counter() - t0
    times = []
    t_start = time.perf_counter()
    while time.perf_counter() - t_start < budget_s or len(times) < 2:
        t0 = time.perf_counter()
        solve.range_space_two_factor(A["K"], A["M"], A["Kc"], beta, ybar, None, lu=lu, paper_y=False)
        times.append(time.perf_counter() - t0)
        if len(times) >= 50:
            break
    t_solve = statistics.median(times)
    return {"value": 1.0 / t_solve, "unit": "Schur solves/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(times)} two-factor solves with one resident SuperLU factor of Z at 512^2 "
                      f"(median {t_solve:.3f} s each); the factorization itself took {t_factor:.2f} s",
            "factor_s": t_factor, "solve_s": t_solve, "cpu": cpu_model()}


_ONE_THREAD = {"OMP_NUM_THREADS": "1", "OPENBLAS_NUM_THREADS": "1", "MKL_NUM_THREADS": "1"}


def _c4_oracle_one(d):
    """One batched instance on the oracle: assembly, SuperLU factor of Z, two-factor solve."""
    import scipy.sparse.linalg as spla
    from oracle import fem, solve
    from paper_1312_5653_amd import workloads
    A = fem.assemble(fem.Mesh(2, d["N"]))
    ybar = workloads.sine_target(2, d["N"], *workloads.modes_for("sixteen2d", d["seed"]))[0]
    lu = spla.splu(solve.complex_factor(A["K"], A["M"], d["beta"]))
    r = solve.range_space_two_factor(A["K"], A["M"], A["Kc"], d["beta"], ybar, None, lu=lu, paper_y=False)
    return d["j"], r["y"], r["u"], r["lam"]


def _c4_worker_init(barrier):
    """Worker start-up outside the timed part: one BLAS thread, the oracle's imports, then
    wait until every worker (and the parent) is ready."""
    os.environ.update(_ONE_THREAD)
    import scipy.sparse.linalg  # noqa: F401
    from oracle import fem, solve  # noqa: F401
    barrier.wait()


def cpu_instances(count, seed, budget_s=15.0):
    """The oracle on the batched-instance workload, one single-threaded process per usable
    host core (at most 16) over independent instances in order, for about budget_s seconds:
    end-to-end solves/s = instances finished / wall time.  Returns the figure and the oracle
    solutions it produced."""
    import multiprocessing as mp
    from paper_1312_5653_amd import workloads
    inst = workloads.c4_instances(count, seed)
    for j, d in enumerate(inst):
        d["j"] = j
    info = cpu_model()
    cores = max(1, min(16, info["usable_cores"] or 1))
    sols = {}
    mctx = mp.get_context("spawn")
    barrier = mctx.Barrier(cores + 1)
    saved = {k: os.environ.get(k) for k in _ONE_THREAD}
    os.environ.update(_ONE_THREAD)  # inherited by the spawned workers before numpy loads
    try:
        with mctx.Pool(cores, initializer=_c4_worker_init, initargs=(barrier,)) as pool:
            barrier.wait(timeout=300)
            t_start = time.perf_counter()
            for j, y, u, lam in pool.imap_unordered(_c4_oracle_one, inst):
                sols[j] = (y, u, lam)
                if time.perf_counter() - t_start > budget_s:
                    break
            el = time.perf_counter() - t_start
            pool.terminate()
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    Ns = sorted(inst[j]["N"] for j in sols)
    return {"value": len(sols) / el, "unit": "end-to-end solves/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(sols)} of the {count} instances (N {Ns[0]}..{Ns[-1]}; assembly, SuperLU "
                      f"factor of Z and the two-factor solve each) on {cores} single-threaded processes, "
                      f"{el:.1f} s", "cpu": info}, sols


def run_instances(sfdp, torch, ctx, count, seed, tol_kkt, setup_bits=64):
    """Batched instances: `count` independent 2D instances, N_j in 64..256 (log-uniform,
    multiple of 32), subdomains of 32x32 cells, beta_j = 10^U[-6,-1], one 16-mode sine target
    each; every instance has a new beta, so a pass is set-up + solve (end to end)."""
    from paper_1312_5653_amd import workloads
    inst = workloads.c4_instances(count, seed)
    Ns = [d["N"] for d in inst]
    betas = [d["beta"] for d in inst]
    ybars = [torch.tensor(workloads.sine_target(2, d["N"], *workloads.modes_for("sixteen2d", d["seed"]))[0],
                          device="cuda:0") for d in inst]
    b = sfdp.Batch(ctx, Ns, 32, sfdp.SFDP_MIXED)
    sfdp.set_setup_arithmetic(setup_bits)
    try:
        b.set_beta(betas)
        b.solve_range_space(ybars, None, tol_kkt=tol_kkt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.set_beta(betas)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    except BaseException:
        b.close()
        raise
    finally:
        sfdp.set_setup_arithmetic(64)
    try:
        ys, us, ls, infos, st = b.solve_range_space(ybars, None, tol_kkt=tol_kkt)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
    finally:
        b.close()
    if st != 0:
        raise RuntimeError("batched instances did not converge")
    outs = [(y.cpu().numpy(), u.cpu().numpy(), l.cpu().numpy()) for y, u, l in zip(ys, us, ls)]
    rho = max(i[0]["rel_kkt"] for i in infos)
    return {"instances": count, "seed": seed, "subdomains": sum((N // 32) ** 2 for N in Ns),
            "dofs": sum((N - 1) ** 2 for N in Ns), "setup_ms": (t1 - t0) * 1e3, "solve_ms": (t2 - t1) * 1e3,
            "solves_per_s_end_to_end": count / (t2 - t0), "solves_per_s_solve_phase": count / (t2 - t1),
            "max_rel_kkt": rho, "max_constr_viol": max(i[0]["constr_viol"] for i in infos),
            "max_eta_blk": max(i[0]["eta_blk"] for i in infos),
            "krylov_its_per_solve": statistics.mean(i[0]["krylov_total"] for i in infos),
            "refinement_steps": statistics.mean(i[0]["outer_steps"] for i in infos),
            "setup_arithmetic": "complex64 (FP32 matrix cores)" if setup_bits == 32 else "FP64",
            "precision": "mixed"}, outs


def run_serving(sfdp, torch, count, seed, tol_kkt, budget_gb, mean_gap_ms=5.0, warmup_s=0.0):
    """Served request stream (see workloads.c5_requests): requests are submitted at their
    arrival times to one server (mixed precision, memory budget budget_gb) and polled at the
    end; latency is submit-to-result per request, throughput counts targets solved.  Requests
    arriving in the first warmup_s seconds are served but left out of the latency figures."""
    import numpy as np
    from paper_1312_5653_amd import workloads
    reqs = workloads.c5_requests(count, seed, mean_gap_ms)
    cache = {}  # targets per (dim, N, nrhs, seed mod 8): long streams reuse them
    inputs = []
    for r in reqs:
        kind = "sixteen2d" if r["dim"] == 2 else "eight3d"
        key = (r["dim"], r["N"], r["nrhs"], r["seed"] % 8)
        if key not in cache:
            ys = [workloads.sine_target(r["dim"], r["N"], *workloads.modes_for(kind, (r["seed"] % 8) * 8 + k))[0]
                  for k in range(r["nrhs"])]
            cache[key] = torch.tensor(np.stack(ys), device="cuda:0")
        inputs.append(cache[key])
    torch.cuda.synchronize()
    ctx = sfdp.Context(0, mem_budget=int(budget_gb * (1 << 30)))
    srv = sfdp.Server(ctx, sfdp.SFDP_MIXED, tol_kkt=tol_kkt)
    t0 = time.perf_counter()
    tickets = []
    for r, x in zip(reqs, inputs):
        delay = r["arrival_ms"] / 1e3 - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        tickets.append(srv.submit(r["N"], r["m"], r["beta"], x, dim=r["dim"], full_space=r["full_space"]))
    lat, rho, fails, errors = [], [], 0, {}
    by_kind = {}
    for r, tk in zip(reqs, tickets):
        try:
            _, _, _, info, l, st = srv.poll(tk)
            rho.extend(i["rel_kkt"] for i in info)
            if r["arrival_ms"] >= warmup_s * 1e3:
                lat.append(l)
                kind = f"{r['dim']}d_{'full' if r['full_space'] else 'range'}"
                by_kind.setdefault(kind, []).append(l)
        except sfdp.SfdpError as e:
            fails += 1
            errors[str(e)] = errors.get(str(e), 0) + 1
    wall = time.perf_counter() - t0
    stats = srv.stats()
    srv.close()
    ctx.close()
    if not lat:
        raise RuntimeError(f"every served request failed: {errors}")
    lat.sort()
    q = lambda f: lat[min(len(lat) - 1, int(round(f * (len(lat) - 1))))]
    solved = sum(r["nrhs"] for r in reqs)
    kinds = {k: {"requests": len(v), "p50_ms": sorted(v)[len(v) // 2],
                 "p99_ms": sorted(v)[min(len(v) - 1, int(round(0.99 * (len(v) - 1))))]}
             for k, v in sorted(by_kind.items())}
    return {"requests": count, "seed": seed, "targets": solved, "mean_gap_ms": mean_gap_ms,
            "offered_rps": 1e3 / mean_gap_ms, "warmup_s": warmup_s, "measured_requests": len(lat),
            "meshes": "2D N in 128..1024 (m = 32) with probability 0.75, else 3D N in 32..64 (m = 8); "
                      "a quarter of the requests use the full-space method",
            "kinds": kinds,
            "wall_s": wall, "solves_per_s": solved / wall, "requests_per_s": count / wall,
            "p50_ms": q(0.5), "p99_ms": q(0.99), "max_rel_kkt": max(rho), "failed": fails, "errors": errors,
            "setups": stats["setups"], "evictions": stats["evictions"], "ticks": stats["ticks"],
            "solo_in_flight_max": stats["solo_in_flight_max"],
            "budget_gb": budget_gb, "precision": "mixed"}


def run_serving_loads(sfdp, torch, capacity_rps, fractions, window_s, warmup_s, seed, tol_kkt, budget_gb):
    """The served stream below saturation: for each fraction f of the measured capacity
    (requests/s of the saturated stream), Poisson arrivals at f * capacity for
    warmup_s + window_s seconds; latency over the requests after the warm-up."""
    out = []
    for f in fractions:
        rate = f * capacity_rps
        count = max(1, int(round(rate * (warmup_s + window_s))))
        r = run_serving(sfdp, torch, count, seed + 1, tol_kkt, budget_gb, mean_gap_ms=1e3 / rate,
                        warmup_s=warmup_s)
        r["load_fraction"] = f
        out.append(r)
        print(f"serving load {f:.2f} of {capacity_rps:.2f} req/s: {count} requests, p50 {r['p50_ms']:.0f} ms, "
              f"p99 {r['p99_ms']:.0f} ms", file=sys.stderr, flush=True)
    return out


def run_precision(sfdp, torch, ctx, precision, N, m, beta, ybar_t, steps, warmup, tol_kkt, tol_inner,
                  batch, max_krylov=0, factors=0, edges=None, dim=2, full_space=False, schur_block=0,
                  setup_bits=64):
    p = sfdp.Problem(ctx, dim, N, m, precision)
    try:
        return _run_precision(sfdp, torch, p, beta, ybar_t, steps, warmup, tol_kkt, tol_inner, batch,
                              max_krylov, factors, edges, full_space, schur_block, setup_bits)
    finally:
        p.close()


def _run_precision(sfdp, torch, p, beta, ybar_t, steps, warmup, tol_kkt, tol_inner, batch, max_krylov,
                   factors, edges, full_space, schur_block, setup_bits=64):
    if edges is not None:
        p.set_coarse_space(edges)
    torch.cuda.synchronize()
    sfdp.set_setup_arithmetic(setup_bits)
    try:
        t0 = time.perf_counter()
        p.set_beta(beta)
        torch.cuda.synchronize()
        setup_ms = (time.perf_counter() - t0) * 1e3
    finally:
        sfdp.set_setup_arithmetic(64)
    y = torch.empty_like(ybar_t)
    u = torch.empty_like(ybar_t)
    lam = torch.empty_like(ybar_t)
    nb = ybar_t.shape[0]
    solve = p.solve_full_space if full_space else p.solve_range_space
    sb = {"schur_block": schur_block} if schur_block else {}  # S_p factors: built in the first warmup call
    kw = dict(tol_kkt=tol_kkt, tol_inner=tol_inner, batch=batch, max_krylov=max_krylov, factors=factors, **sb)
    for _ in range(warmup):
        solve(ybar_t, None, y, u, lam, **kw)
    # HIP events around the GMRES launches (the roofline's kernel) during the timed
    # calls; the subdomain solve's events (each record idles the device ~6 us) are
    # taken in a short pass of their own after the timed region
    p.timing_enable(2)
    lat, rhos, its, feti, minres, cvs, etas, steps_seen = [], [], [], [], [], [], [], []
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for _ in range(steps):
        t0 = time.perf_counter()
        _, _, _, info, st = solve(ybar_t, None, y, u, lam, **kw)
        lat.append(time.perf_counter() - t0)
        rhos.extend(i["rel_kkt"] for i in info)
        its.extend(i["krylov_total"] for i in info)
        feti.extend(i["n_feti"] for i in info)
        minres.extend(i["minres_its"] for i in info)
        cvs.extend(i["constr_viol"] for i in info)
        etas.extend(i["eta_blk"] for i in info)
        steps_seen.extend(i["outer_steps"] for i in info)
        if st != 0:
            raise RuntimeError(f"solve did not converge: {info}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_all
    kt = p.kernel_times()
    lsteps = max(2, min(steps, 5))
    p.timing_enable(1)
    for _ in range(lsteps):
        solve(ybar_t, None, y, u, lam, **kw)
    kt_local = p.kernel_times()
    p.timing_enable(False)
    kt["local_ms"], kt["local_launches"] = kt_local["local_ms"], kt_local["local_launches"]
    # the subdomain solve's share of a timed step: its time per call over the step time
    kt["local_share"] = kt_local["local_ms"] / lsteps / (elapsed * 1e3 / steps)
    # the same calls with their refinement steps replayed as captured HIP graphs
    # (the first call runs eagerly, the second captures), for the comparison
    ksteps = max(3, min(steps, 10))
    sfdp.set_graphs(True)
    try:
        for _ in range(2):
            solve(ybar_t, None, y, u, lam, **kw)
        torch.cuda.synchronize()
        t_e = time.perf_counter()
        for _ in range(ksteps):
            solve(ybar_t, None, y, u, lam, **kw)
        torch.cuda.synchronize()
        graph_ms = (time.perf_counter() - t_e) * 1e3 / ksteps
    finally:
        sfdp.set_graphs(False)
    sizes = p.refresh_sizes()
    outs = [(y[r].cpu().numpy(), u[r].cpu().numpy(), lam[r].cpu().numpy()) for r in range(nb)]
    lat_ms = sorted(x * 1e3 for x in lat)
    q = lambda f: lat_ms[min(len(lat_ms) - 1, int(round(f * (len(lat_ms) - 1))))]
    return {"solves_per_s": nb * steps / elapsed, "ms_per_step": elapsed * 1e3 / steps, "batch": nb,
            "graph_ms_per_step": graph_ms,
            "p50_ms": q(0.5), "p99_ms": q(0.99), "setup_ms": setup_ms,
            "max_rel_kkt": max(rhos), "max_constr_viol": max(cvs), "max_eta_blk": max(etas),
            "refinement_steps": statistics.mean(i for i in steps_seen) if steps_seen else None,
            "krylov_per_solve": statistics.mean(its),
            "feti_per_solve": statistics.mean(feti), "minres_per_solve": statistics.mean(minres),
            "kernel_times": kt, "sizes": sizes, "outs": outs, "beta": beta}


def run_schur_blocks(sfdp, torch, ctx, precision, N, m, betas, ybar_t, tol_kkt, tol_inner):
    """The comparison of Table 7 on this path: for each beta, the full-space
    method with the exact S (complex factorization) and with S_p (Pearson and
    Wathen) as the S block: set-up time of the factors (B), time of one S-block
    application (S), MINRES iterations (NI; the paper's NI counts outer Krylov
    iterations), FETI-DP solves and the time of one full-space solve (T)."""
    rows = []
    y0 = ybar_t[:1].contiguous()
    for beta in betas:
        p = sfdp.Problem(ctx, 2, N, m, precision)
        try:
            rows.append(_schur_block_row(p, torch, beta, y0, tol_kkt, tol_inner))
        finally:
            p.close()
    return {"workload": f"{N}x{N} Q1, {(N // m) ** 2} subdomains of {m}x{m}, one target, "
                        f"{'mixed' if precision == sfdp.SFDP_MIXED else 'fp64'}",
            "rows": rows}


def _schur_block_row(p, torch, beta, y0, tol_kkt, tol_inner):
    if True:
        sync = torch.cuda.synchronize
        sync()
        t0 = time.perf_counter()
        p.set_beta(beta)
        sync()
        row = {"beta": beta, "exact": {"B_ms": (time.perf_counter() - t0) * 1e3},
               "pearson_wathen": {}}
        # the first S_p application also factors F = K + beta^-1/2 M (the twin)
        t0 = time.perf_counter()
        p.apply_schur_inv(y0, schur_block=1, tol_inner=tol_inner)
        sync()
        first = time.perf_counter() - t0
        for key, sb in (("exact", 0), ("pearson_wathen", 1)):
            t0 = time.perf_counter()
            p.apply_schur_inv(y0, schur_block=sb, tol_inner=tol_inner)
            sync()
            row[key]["S_ms"] = (time.perf_counter() - t0) * 1e3
        row["pearson_wathen"]["B_ms"] = first * 1e3 - row["pearson_wathen"]["S_ms"]
        for key, sb in (("exact", 0), ("pearson_wathen", 1)):
            t0 = time.perf_counter()
            _, _, _, info, st = p.solve_full_space(y0, None, tol_kkt=tol_kkt, tol_inner=tol_inner, schur_block=sb)
            sync()
            row[key].update({"T_ms": (time.perf_counter() - t0) * 1e3, "NI": info[0]["minres_its"],
                             "refinement_steps": info[0]["outer_steps"], "feti_solves": info[0]["n_feti"],
                             "rel_kkt": info[0]["rel_kkt"], "status": st})
        return row


def run_c3(sfdp, torch, ctx, N, beta, steps, tol_kkt, oracle=None, m=8, B=4):
    """The 3D configuration: Q1 trilinear Poisson control on N^3 cells in
    (N/m)^3 subdomains of m^3, B eight-mode product-of-sines targets per step,
    mixed precision (complex64 local operators, FP64 coarse problem, Krylov and
    refinement)."""
    import numpy as np
    from paper_1312_5653_amd import workloads
    mc = [workloads.modes_for("eight3d", s) for s in range(B)]
    ybar = np.stack([workloads.sine_target(3, N, *x)[0] for x in mc])
    yt = torch.tensor(ybar, device="cuda:0")
    r = run_precision(sfdp, torch, ctx, sfdp.SFDP_MIXED, N, m, beta, yt, steps, 1, tol_kkt, 3e-7, B, dim=3)
    sz = r["sizes"]
    # the 3D sparse LU of the oracle runs for minutes at this size: the closed form of the
    # exact discrete solution (sine targets) is the oracle reference here
    fe = {"closed_form": fwd_err(r["outs"], OracleLeg.closed(3, N, beta, mc))} if oracle else None
    return {"workload": f"3D Q1 Poisson control {N}^3 cells, {N // m}^3 subdomains of {m}^3, beta={beta:g}, "
                        f"8-mode product-of-sines targets (seeds 0..{B - 1}), {B} targets per step",
            "precision": "mixed", "solves_per_s": r["solves_per_s"], "ms_per_step": r["ms_per_step"],
            "p50_ms": r["p50_ms"], "p99_ms": r["p99_ms"], "setup_ms": r["setup_ms"],
            "max_rel_kkt": r["max_rel_kkt"], "max_constr_viol": r["max_constr_viol"],
            "max_eta_blk": r["max_eta_blk"], "fwd_err_vs_oracle": fe,
            "krylov_its_per_solve": r["krylov_per_solve"], "dofs": (N - 1) ** 3, "n_mult": sz["n_mult"], "n_corner": sz["n_corner"],
            "resident_bytes": sz["resident_bytes"]}


def run_elastic(sfdp, torch, ctx, n, m, beta, steps, precision, B=4, length=3):
    """The Sec. 6.2 solid cantilever: rubber (E = 20.7 MPa, nu = 0.45) on [0, 3] x [0, 1]^2,
    h = 1/n, (3n/m) x (n/m)^2 cubic subdomains of m^3 cells, beta = 1e-16 (Table 5's phi).
    Targets: the beam-theory deflection under 100 kPa scaled by 1, 3/4, 1/2, 1/4 with seeded
    1e-3 noise on all but the first.  Also timed: the GPU forward solve of the pressure load
    (the paper's way of making its target) and the set-up."""
    import numpy as np
    from paper_1312_5653_amd import workloads
    p = sfdp.ElasticProblem(ctx, n, m, length=length, precision=precision)
    try:
        nf = p.n_free
        f = p.pressure_load(1e5)
        p.forward(f)  # builds the forward factors
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ub, fwd_its = p.forward(f)
        torch.cuda.synchronize()
        fwd_ms = (time.perf_counter() - t0) * 1e3
        ybar = np.stack([c * workloads.cantilever_target(n, length, seed=j, noise=1e-3 if j else 0.0)
                         for j, c in enumerate((1.0, 0.75, 0.5, 0.25)[:B])])
        ybar_t = torch.tensor(ybar, device="cuda:0")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p.set_beta(beta)
        torch.cuda.synchronize()
        setup_ms = (time.perf_counter() - t0) * 1e3
        y, u, lam = (torch.empty_like(ybar_t) for _ in range(3))
        p.solve_range_space(ybar_t, None, y, u, lam)
        lat, infos = [], []
        torch.cuda.synchronize()
        t_all = time.perf_counter()
        for _ in range(steps):
            t0 = time.perf_counter()
            _, _, _, info, st = p.solve_range_space(ybar_t, None, y, u, lam)
            lat.append((time.perf_counter() - t0) * 1e3)
            infos.extend(info)
            if st != 0:
                raise RuntimeError(f"elastic solve did not converge: {info}")
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_all
        sz = p.refresh_sizes()
        outs = [(y[r].cpu().numpy(), u[r].cpu().numpy(), lam[r].cpu().numpy()) for r in range(B)]
        its = [i["krylov_its"][k] for i in infos for k in range(min(i["n_feti"], 16))]
        lat.sort()
        return {"workload": f"Sec. 6.2 rubber cantilever [0,{length}]x[0,1]^2, h=1/{n}, "
                            f"{sz['n_sub']} subdomains of {m}^3 cells, beta={beta:g}, {B} beam-deflection "
                            f"targets per step",
                "precision": "fp64" if precision == sfdp.SFDP_FP64 else "mixed",
                "dofs": nf, "n_sub": sz["n_sub"], "n_mult": sz["n_mult"], "n_corner": sz["n_corner"],
                "resident_bytes": sz["resident_bytes"],
                "solves_per_s": B * steps / elapsed, "ms_per_step": elapsed * 1e3 / steps,
                "p50_ms": lat[len(lat) // 2], "setup_ms": setup_ms,
                "forward_ms": fwd_ms, "forward_krylov_its": fwd_its[0],
                "refinement_steps": statistics.mean(i["outer_steps"] for i in infos),
                "krylov_its_per_factor_solve": statistics.mean(its), "krylov_its_max": max(its),
                "max_eta_blk": max(i["eta_blk"] for i in infos),
                "max_constr_viol": max(i["constr_viol"] for i in infos),
                "max_rel_kkt": max(i["rel_kkt"] for i in infos),
                "outs": outs, "ybar": ybar, "n": n, "m": m, "beta": beta, "length": length}
    finally:
        p.close()


def run_elastic_betas(sfdp, torch, ctx, n, m, betas, tol_inner=1e-9, length=3):
    """Table 4's experiment on this path: the FETI-DP iterations of the two factors
    K - V/(i sqrt(phi)) = K + i alpha V (the paper's "-", the first solve of a step) and
    K + V/(i sqrt(phi)) (its "+", the second, by conjugation) over phi = beta, for the
    first refinement step of one range-space solve of the beam-deflection target,
    FP64, inner tolerance 1e-9 (the paper's threshold); corners only (no RAUG)."""
    import numpy as np
    from paper_1312_5653_amd import workloads
    p = sfdp.ElasticProblem(ctx, n, m, length=length, precision=sfdp.SFDP_FP64)
    rows = []
    try:
        yb = torch.tensor(workloads.cantilever_target(n, length)[None, :], device="cuda:0")
        for beta in betas:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            p.set_beta(beta)
            torch.cuda.synchronize()
            setup_ms = (time.perf_counter() - t0) * 1e3
            t0 = time.perf_counter()
            _, _, _, info, st = p.solve_range_space(yb, tol_inner=tol_inner)
            torch.cuda.synchronize()
            i = info[0]
            rows.append({"phi": beta, "minus_its": i["krylov_its"][0], "plus_its": i["krylov_its"][1],
                         "refinement_steps": i["outer_steps"], "solve_ms": (time.perf_counter() - t0) * 1e3,
                         "setup_ms": setup_ms, "eta_blk": i["eta_blk"], "status": st})
    finally:
        p.close()
    return {"workload": f"Sec. 6.2 rubber cantilever h=1/{n}, {(3 * n // m) * (n // m) ** 2} subdomains of {m}^3 "
                        f"cells, FP64, inner tolerance {tol_inner:g}, first refinement step's two solves",
            "rows": rows}


def elastic_oracle(r, o1_max_dofs=6000, budget_s=10.0):
    """Oracle leg of an elasticity line: the oracle's blockwise backward error of the GPU
    results (its own K and M), the forward error against O1 where the oracle's sparse LU
    is quick (h = 1/8), and the O1 timing there."""
    import scipy.sparse.linalg as spla
    from oracle import elastic as el
    from oracle import kkt, solve
    box = el.Box(r["n"], r["length"])
    A = el.assemble(box)
    K, M, Kc = A["K"], A["M"], A["Kc"]
    etas = [kkt.eta_blk(K, M, Kc, r["beta"], yb, None, *o) for yb, o in zip(r["ybar"], r["outs"])]
    res = {"oracle_eta_blk_max": max(etas)}
    if box.n_dof <= o1_max_dofs:
        t0 = time.perf_counter()
        lu = spla.splu(solve.complex_factor(K, M, r["beta"]))
        t_factor = time.perf_counter() - t0
        refs, times = [], []
        for yb in r["ybar"]:
            t0 = time.perf_counter()
            refs.append(solve.range_space_two_factor(K, M, Kc, r["beta"], yb, None, lu=lu, paper_y=False))
            times.append(time.perf_counter() - t0)
        res["fwd_err_vs_oracle"] = {"O1": fwd_err(r["outs"], refs)}
        # the conditioning floor: O1 against the real saddle-point solve O2
        o2 = solve.reduced_saddle(K, M, Kc, r["beta"], r["ybar"][0], None)
        res["o1_vs_o2"] = fwd_err([(o2["y"], o2["u"], o2["lam"])], refs[:1])
        t_solve = statistics.median(times)
        res["cpu_baseline"] = {"value": 1.0 / t_solve, "unit": "Schur solves/s", "cores": 1, "kind": "oracle",
                               "sample": f"{len(times)} two-factor solves with one resident SuperLU factor of Z "
                                         f"({box.n_dof} dofs); the factorization took {t_factor:.2f} s",
                               "factor_s": t_factor, "solve_s": t_solve}
    else:
        res["fwd_err_vs_oracle"] = None
        res["note"] = ("the oracle's SuperLU factor of Z takes about 2 minutes at 41,616 dofs and grows "
                       "quickly beyond: the result is checked by the oracle's backward error only")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--beta", type=float, default=1e-4)
    ap.add_argument("--N", type=int, default=512)
    ap.add_argument("--m", type=int, default=32)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--fp64-only", action="store_true")
    ap.add_argument("--batch", type=int, default=4, help="targets per step (1..4)")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the headline configuration (for counter runs)")
    ap.add_argument("--copy-check", type=int, default=0, metavar="MIB",
                    help="first copy a MIB-MiB device buffer once (a plain copy of known size that "
                         "calibrates the HBM byte counters of a profiler run)")
    ap.add_argument("--instances", type=int, default=256,
                    help="batched-instance workload size (0 skips it)")
    ap.add_argument("--requests", type=int, default=100,
                    help="served request stream length (0 skips it)")
    ap.add_argument("--serve-budget-gb", type=float, default=48.0)
    ap.add_argument("--serve-loads", type=str, default="0.5",
                    help="fractions of the measured serving capacity offered as Poisson streams ('' for none)")
    ap.add_argument("--serve-window", type=float, default=20.0,
                    help="seconds of arrivals per load point after a 5 s warm-up")
    ap.add_argument("--max-krylov", type=int, default=0,
                    help="GMRES iteration cap per FETI-DP solve (0: library default)")
    ap.add_argument("--c3", type=int, default=64, metavar="N",
                    help="3D configuration: N^3 cells in subdomains of 8^3 (0 skips it)")
    ap.add_argument("--c3-only", action="store_true", help="only the 3D configuration (for profiles)")
    ap.add_argument("--instances-only", action="store_true",
                    help="only the batched instances (set-up and solve; for profiles)")
    ap.add_argument("--side-stream", action="store_true",
                    help="run the library on a torch stream of its own instead of the default stream")
    ap.add_argument("--serving-only", action="store_true",
                    help="only the served stream and its load points")
    ap.add_argument("--c3-steps", type=int, default=5)
    ap.add_argument("--elastic", type=str, default="8,16", metavar="N,...",
                    help="cantilever meshes (cells per metre) of the Sec. 6.2 lines; empty to skip")
    ap.add_argument("--elastic-m6", type=int, default=24, metavar="N",
                    help="cantilever mesh of the line with 6^3-cell subdomains (0 to skip)")
    ap.add_argument("--elastic-only", action="store_true", help="only the elasticity lines")
    ap.add_argument("--elastic-betas", type=str, default="1e-7,1e-8,1e-9,1e-10,1e-11,1e-12,1e-13,1e-14,1e-15,1e-16,1e-17,1e-18",
                    help="phi values of the Table 4 analogue (cantilever at h = 1/16); empty to skip")
    ap.add_argument("--schur-betas", type=str, default="1e-2,1e-4,1e-6,1e-8,1e-10",
                    help="betas of the S versus S_p full-space comparison ('' to skip)")
    ap.add_argument("--traffic-record", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_MIB"),
                    help="write the traffic record from two rocprofv3 --pmc output folders and exit")
    args = ap.parse_args()
    if args.traffic_record:
        write_traffic_record(args.traffic_record[0], args.traffic_record[1], int(args.traffic_record[2]))
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world > 1:
        print("bench.py runs on one GPU only: the FETI-DP subdomains of an instance are a batch "
              "on a single MI355X; --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_1312_5653_amd import sfdp, workloads

    N, m, beta, B = args.N, args.m, args.beta, args.batch
    if not 1 <= B <= 4:
        print("--batch must be in 1..4", file=sys.stderr)
        sys.exit(2)
    ybar = np.stack([workloads.sine_target(2, N, *workloads.modes_for("sixteen2d", s))[0]
                     for s in range(B)])
    ybar_t = torch.tensor(ybar, device="cuda:0")
    ybar1_t = ybar_t[:1].contiguous()
    if args.copy_check > 0:
        src_buf = torch.ones(args.copy_check << 18, dtype=torch.float32, device="cuda:0")
        dst_buf = torch.empty_like(src_buf)
        torch.mul(src_buf, 1.0, out=dst_buf)  # reads and writes MIB MiB once
        torch.cuda.synchronize()
        del src_buf, dst_buf
    if args.side_stream:
        side = torch.cuda.Stream()
        torch.cuda.set_stream(side)
    ctx = sfdp.Context(0)
    tol_kkt = 1e-8
    if args.c3_only:
        print(json.dumps({"c3_3d": run_c3(sfdp, torch, ctx, args.c3, beta, args.c3_steps, tol_kkt)}), flush=True)
        ctx.close()
        return
    if args.elastic_only:
        out = {}
        for ne in [int(x) for x in args.elastic.split(",") if x]:
            for pn, pv in (("mixed", sfdp.SFDP_MIXED), ("fp64", sfdp.SFDP_FP64)):
                r = run_elastic(sfdp, torch, ctx, ne, 4, 1e-16, 5, pv)
                if not args.no_cpu:
                    r.update(elastic_oracle(r))
                out[f"elastic_h{ne}_{pn}"] = {k: v for k, v in r.items() if k not in ("outs", "ybar")}
                print(json.dumps(out[f"elastic_h{ne}_{pn}"]), file=sys.stderr, flush=True)
        if args.elastic_m6:
            r = run_elastic(sfdp, torch, ctx, args.elastic_m6, 6, 1e-16, 5, sfdp.SFDP_MIXED)
            if not args.no_cpu:
                r.update(elastic_oracle(r))
            out[f"elastic_h{args.elastic_m6}_m6_mixed"] = {k: v for k, v in r.items() if k not in ("outs", "ybar")}
        if args.elastic_betas:
            out["elastic_phi_dependence"] = run_elastic_betas(sfdp, torch, ctx, 16, 4,
                                                              [float(b) for b in args.elastic_betas.split(",")])
        print(json.dumps(out), flush=True)
        ctx.close()
        return
    if args.serving_only:
        ctx.close()
        r = {"serving": run_serving(sfdp, torch, args.requests, 0, tol_kkt, args.serve_budget_gb)}
        print(json.dumps(r), file=sys.stderr, flush=True)
        if args.serve_loads:
            fr = [float(x) for x in args.serve_loads.split(",")]
            r["serving_loads"] = run_serving_loads(sfdp, torch, r["serving"]["requests_per_s"], fr,
                                                   args.serve_window, 5.0, 0, tol_kkt, args.serve_budget_gb)
        print(json.dumps(r), flush=True)
        return
    if args.instances_only:
        r, _ = run_instances(sfdp, torch, ctx, args.instances, 0, tol_kkt)
        print(json.dumps({"instances_batch": r}), flush=True)
        ctx.close()
        return
    res = {}
    precs = [("fp64", sfdp.SFDP_FP64, 1e-13)]
    if not args.fp64_only:
        precs.insert(0, ("mixed", sfdp.SFDP_MIXED, 3e-7))
    if args.headline_only:
        precs = precs[:1]
    for name, prec, tin in precs:
        res[name] = run_precision(sfdp, torch, ctx, prec, N, m, beta, ybar_t, args.steps, args.warmup,
                                  tol_kkt, tin, B, args.max_krylov)
        if B > 1 and not args.headline_only:
            res[name + "_b1"] = run_precision(sfdp, torch, ctx, prec, N, m, beta, ybar1_t, args.steps,
                                              args.warmup, tol_kkt, tin, 1, args.max_krylov)
    head = precs[0][0]
    hp, htin = precs[0][1], precs[0][2]
    if not args.headline_only:
        # the same configuration at the other two betas of the 512^2 workload (Table 1's phi range)
        for ob in (1e-2, 1e-6):
            if ob != beta:
                res[f"{head}_beta{ob:g}"] = run_precision(sfdp, torch, ctx, hp, N, m, ob, ybar_t, args.steps,
                                                         args.warmup, tol_kkt, htin, B, args.max_krylov)
        # the complex64 set-up (line factorization and line solves on the FP32
        # matrix cores) against the FP64 one: refinement steps and solves/s
        if hp == sfdp.SFDP_MIXED:
            res[head + "_setup32"] = run_precision(sfdp, torch, ctx, hp, N, m, beta, ybar_t, args.steps,
                                                   args.warmup, tol_kkt, htin, B, args.max_krylov, setup_bits=32)
        # the one-solve range-space form (same result, half the FETI-DP solves):
        # measured beside the two-factor form, never in its place
        res[head + "_single_solve"] = run_precision(sfdp, torch, ctx, hp, N, m, beta, ybar_t, args.steps,
                                                    args.warmup, tol_kkt, htin, B, args.max_krylov, factors=1)
        # the same with the arrays in host memory (sfdp_opts.host_ptrs, which the
        # binding sets for CPU tensors): the rate including the PCIe copies of the
        # targets in and of y, u, lam out; never the headline value
        res[head + "_host_arrays"] = run_precision(sfdp, torch, ctx, hp, N, m, beta, ybar_t.cpu(), args.steps,
                                                   args.warmup, tol_kkt, htin, B, args.max_krylov)
        # the corner-only coarse space, for the effect of the edge augmentation
        res[head + "_corners_only"] = run_precision(sfdp, torch, ctx, hp, N, m, beta, ybar_t, args.steps,
                                                    args.warmup, tol_kkt, htin, B, args.max_krylov, edges=False)
        # the full-space method with the same S^-1 as its preconditioner block
        # (Sec. 3.2; targets one after another)
        res[head + "_full_space"] = run_precision(sfdp, torch, ctx, hp, N, m, beta, ybar_t,
                                                  max(2, args.steps // 5), 1, tol_kkt, htin, B, args.max_krylov,
                                                  full_space=True)
        # the same with the approximation S_p of Pearson and Wathen as the S
        # block (Sec. 3.2, the comparison of Table 7)
        res[head + "_full_space_pw"] = run_precision(sfdp, torch, ctx, hp, N, m, beta, ybar_t,
                                                     max(2, args.steps // 5), 1, tol_kkt, htin, B, args.max_krylov,
                                                     full_space=True, schur_block=1)
    r = res[head]
    kt = r["kernel_times"]
    sz = r["sizes"]
    trips = kt["gmres_iters"] / max(kt["gmres_launches"], 1)          # loop trips per launch
    rhs_its = kt["gmres_rhs_iters"] / max(kt["gmres_launches"], 1)    # RHS iterations per launch
    ebytes = 8 if head == "mixed" else 16
    op_bytes = gmres_operator_bytes(N, m, sz["n_coarse"], sz["n_coarse"] > sz["n_corner"], ebytes)
    vec_bytes = gmres_vector_bytes(sz["n_mult"], rhs_its / B)
    launch_bytes = trips * op_bytes + rhs_its * vec_bytes
    launch_ms = kt["gmres_ms"] / max(kt["gmres_launches"], 1)
    achieved = launch_bytes / (launch_ms * 1e-3) / 1e9
    local_ms = kt["local_ms"] / max(kt["local_launches"], 1)
    local_gbs = local_solve_bytes(N, m, ebytes, B) / (local_ms * 1e-3) / 1e9
    out = {
        "metric": "Schur solves/sec at rel. KKT residual 1e-8 (512² Q1); p50/p99 solve latency",
        "value": r["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": f"2D Q1 Poisson control {N}x{N} cells, {N // m}x{N // m} subdomains of "
                               f"{m}x{m}, beta={beta:g}, 16-mode sine targets (seeds 0..{B - 1}), "
                               f"{B} targets per step sharing every launch",
                   "precision": head, "tol_kkt": tol_kkt, "batch": B,
                   "coarse_space": "corners + interface-edge averages"
                   if sz["n_coarse"] > sz["n_corner"] else "corners",
                   "storage": "c64 factors and interface operators, FP64 arithmetic"
                   if head == "mixed" else "c128",
                   "max_krylov": args.max_krylov or 64,
                   "parallelism": "1 GPU, subdomains as a batch"},
        # latency of one Schur solve: a step with a single target
        "p50_ms": res.get(head + "_b1", r)["p50_ms"],
        "p99_ms": res.get(head + "_b1", r)["p99_ms"],
        "step_p50_ms": r["p50_ms"],
        # the same calls with their refinement steps replayed as captured HIP graphs
        "graph_ms_per_step": r["graph_ms_per_step"],
        "step_p99_ms": r["p99_ms"],
        "setup_ms": r["setup_ms"],
        "refinement_steps": r["refinement_steps"],
        "max_rel_kkt": r["max_rel_kkt"],
        "max_constr_viol": r["max_constr_viol"],
        "max_eta_blk": r["max_eta_blk"],
        "fwd_err_vs_oracle": None,
        "krylov_its_per_solve": r["krylov_per_solve"],
        "roofline": {"bound": "hbm", "kernel": "k_gmres (interface Krylov solve, persistent)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(f"k_gmres<{'C<float>' if head == 'mixed' else 'C<double>'}, {kt['gmres_width']}, One>"),
                     "bytes_per_launch": launch_bytes, "operator_bytes_per_trip": op_bytes,
                     "vector_bytes_per_rhs_iteration": vec_bytes, "trips_per_launch": trips,
                     "rhs_iterations_per_launch": rhs_its, "launch_ms": launch_ms,
                     "kernel_width": kt["gmres_width"], "lds_resident": bool(kt["gmres_resident"]),
                     "time_share": kt["gmres_ms"] / (r["ms_per_step"] * args.steps)},
        "subdomain_solve_kernel": {"kernel": "k_local_solve", "launch_ms": local_ms,
                                   "launches": kt["local_launches"], "rhs_per_launch": B,
                                   "achieved_gbs": local_gbs, "frac": local_gbs / HBM_PEAK_GBS,
                                   "time_share": kt["local_share"],
                                   "timed": "HIP events in a pass of their own after the timed region"},
    }
    other = [k for k in res if k != head]
    for k in other:
        o = res[k]
        out[k] = {"batch": o["batch"], "beta": o["beta"], "solves_per_s": o["solves_per_s"],
                  "ms_per_step": o["ms_per_step"], "graph_ms_per_step": o["graph_ms_per_step"], "factors": 1 if k.endswith("_single_solve") else 2,
                  "p50_ms": o["p50_ms"], "p99_ms": o["p99_ms"], "max_rel_kkt": o["max_rel_kkt"],
                  "max_constr_viol": o["max_constr_viol"], "max_eta_blk": o["max_eta_blk"],
                  "fwd_err_vs_oracle": None,
                  "krylov_its_per_solve": o["krylov_per_solve"], "feti_solves_per_solve": o["feti_per_solve"],
                  "refinement_steps": o["refinement_steps"],
                  "setup_ms": o["setup_ms"]}
        if k.endswith("_host_arrays"):
            out[k]["arrays"] = "host memory: staged by the library, PCIe copies in the timed calls"
        if k.endswith("_full_space"):
            out[k]["method"] = "full-space MINRES, P_mgw with S^-1 by the complex factorization"
            out[k]["minres_its_per_solve"] = o["minres_per_solve"]
        if k.endswith("_full_space_pw"):
            out[k]["method"] = "full-space MINRES, P_mgw with S_p (Pearson-Wathen) in place of S"
            out[k]["minres_its_per_solve"] = o["minres_per_solve"]
    oracle = None if args.no_cpu else OracleLeg()
    inst_outs = None
    if args.instances > 0 and not args.headline_only:
        out["instances_batch"], inst_outs = run_instances(sfdp, torch, ctx, args.instances, 0, tol_kkt)
        out["instances_batch_setup32"], _ = run_instances(sfdp, torch, ctx, args.instances, 0, tol_kkt,
                                                          setup_bits=32)
    if args.requests > 0 and not args.headline_only:
        out["serving"] = run_serving(sfdp, torch, args.requests, 0, tol_kkt, args.serve_budget_gb)
        if args.serve_loads:
            fr = [float(x) for x in args.serve_loads.split(",")]
            out["serving_loads"] = run_serving_loads(sfdp, torch, out["serving"]["requests_per_s"], fr,
                                                     args.serve_window, 5.0, 0, tol_kkt, args.serve_budget_gb)
    if args.c3 > 0 and not args.headline_only:
        out["c3_3d"] = run_c3(sfdp, torch, ctx, args.c3, beta, args.c3_steps, tol_kkt, oracle)
    el_lines = {}
    if args.elastic and not args.headline_only:
        for ne in [int(x) for x in args.elastic.split(",") if x]:
            for pn, pv in (("mixed", sfdp.SFDP_MIXED), ("fp64", sfdp.SFDP_FP64)):
                el_lines[f"elastic_h{ne}_{pn}"] = run_elastic(sfdp, torch, ctx, ne, 4, 1e-16, 5, pv)
        if args.elastic_m6:
            el_lines[f"elastic_h{args.elastic_m6}_m6_mixed"] = run_elastic(sfdp, torch, ctx, args.elastic_m6, 6,
                                                                          1e-16, 5, sfdp.SFDP_MIXED)
        if args.elastic_betas:
            out["elastic_phi_dependence"] = run_elastic_betas(sfdp, torch, ctx, 16, 4,
                                                              [float(b) for b in args.elastic_betas.split(",")])
    if args.schur_betas and not args.headline_only:
        betas = [float(b) for b in args.schur_betas.split(",")]
        out["schur_block_comparison"] = run_schur_blocks(sfdp, torch, ctx, precs[0][1], N, m, betas, ybar_t,
                                                         tol_kkt, precs[0][2])
    ctx.close()
    if oracle is not None:
        # the oracle leg: solutions of every line's inputs (forward error of each line) and the
        # timed baselines
        mc = [workloads.modes_for("sixteen2d", s) for s in range(B)]
        for k in sorted(res, key=lambda k: res[k]["beta"]):
            o = res[k]
            refs = oracle.o1(2, N, o["beta"], [ybar[j] for j in range(o["batch"])])
            fe = {"O1": fwd_err(o["outs"], refs),
                  "closed_form": fwd_err(o["outs"], OracleLeg.closed(2, N, o["beta"], mc[:o["batch"]]))}
            (out if k == head else out[k])["fwd_err_vs_oracle"] = fe
        out["cpu_baseline"] = cpu_baseline(N, m, beta, ybar[0])
        if inst_outs is not None:
            base, sols = cpu_instances(args.instances, 0)
            out["instances_batch"]["cpu_baseline"] = base
            out["instances_batch"]["fwd_err_vs_oracle"] = {
                "O1": fwd_err([inst_outs[j] for j in sorted(sols)], [dict(zip(("y", "u", "lam"), sols[j]))
                                                                    for j in sorted(sols)]),
                "instances_compared": len(sols)}
    for k, r in el_lines.items():
        if oracle is not None:
            r.update(elastic_oracle(r))
        out[k] = {kk: v for kk, v in r.items() if kk not in ("outs", "ybar")}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
