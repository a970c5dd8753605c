"""Throughput benchmark.  The default run prints exactly one JSON line: the
multi-RHS CG workload, with the small, rsvd, learn and batch workloads'
results (each with its roofline and CPU oracle baseline) nested under
"workloads".  --workload names others, one line each.

Workloads (synthetic, seeded; see synth/):
  multi_rhs  (default) G2 hypergraph N=50,000, E=40,000 (power-law sizes in
             [2,200], Zipf(1.1) popularity), Dirichlet(1) weights, lambda=0.5,
             Y = 50,000 x 200 binary at 2%; FP32 CG with FP64 inner products
             and residual replacement to relres 1e-6/(1+1/lambda) (forward
             error <= 1e-6).  A step = one full solve; value = solved RHS/s.
  small      G1, N=2000, E=1500, w=1/E, lambda=1, Y 2000 x 50 at 5%, FP64 CG
             to relres 1e-10.
  rsvd       50 diagonal blocks of U[500,1500] rows (N ~ 50,000, G1,
             E = 0.75 N, lambda=1), k=64, p=10, q=2, BF16 sketch; a step =
             Algorithm 1 on all blocks; value = blocks/s.  The refined solve
             (block inverse + PCG, Y N x 50 at 5%) is timed beside it.
  rsvd_power the rsvd workload with the power-scheme sketch of eq. 10 in
             place of Algorithm 1's steps 2-3; also reports the kept
             singular values' deviation from Algorithm 1 on the same sketch.
  single     the paper's query shape: G2 (alpha 2.1, sizes [2,200], Zipf
             1.1) at N=5867, E=4694, lambda=0.5, one RHS per test image
             (1292); value = latency of one query (us, lower is better)
             through the one-workgroup solver; the 1292 queries in one call
             and the multi-kernel solver are reported beside it.
  batch_small 64 G2 graphs of N_g ~ U[2000,6000] (the batch recipe at the
             one-workgroup solver's sizes), 100 RHS each: every (graph,
             column) one workgroup; the multi-kernel batched solver beside it.
  learn      G1, N=100,000, E=80,000, Y 100,000 x 500 at 5%, lambda=1,
             mu=0.01; a step = one outer projected-gradient step (forward CG,
             adjoint gradient, projection, re-weighting); value = steps/s.
  batch      64 G2 hypergraphs, N_g ~ U[2000,30000], E_g = 0.8 N_g, 100 RHS
             each at 3%, lambda=0.5, FP32 to relres 1e-6/(1+1/lambda);
             value = solved RHS/s over the batch.

Every value counts only results that met their tolerance (checked by the
library's FP64-recomputed residuals).  The roofline object is the dominant
kernel of the step with its duration measured by HIP events that the library
records around every launch during the timed steps.  The CPU baseline is the
FP64 oracle timed on a bounded sample of the same workload on one thread,
with an "all_cores" figure beside it: the same oracle on every core of the
host (worker processes, each on its share of the independent columns,
graphs or blocks).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
NESTED = ("small", "rsvd", "learn", "batch")  # nested in the default line
BF16_PEAK_TFLOPS = 2500.0
FP32_MFMA_PEAK_TFLOPS = 157.3


def gather_bytes(N, E, nnz, k, elem=4, covered=None, hubs=0, decoupled=0):
    """Algorithmic HBM bytes of one launch of each operator-gather kernel, and
    of one CG iteration.

    edge_gather (k_spmm_edge): read the P rows of the vertices that lie in
    some hyperedge (`covered`), write Z (E x k); edge_ptr, edge_vtx, c, s.
    vertex_gather (k_spmm_vertex applying M, one launch): read every Z row
    once, read P and write Q for the N - hubs rows it finishes itself (hub
    rows, more hyperedges than the hub threshold, are finished by a separate
    launch); vtx_ptr, vtx_edge, s.
    vertex_step (k_spmm_vertex as the fused CG step): read every Z row once,
    read P, F, R and write F, R for the rows it finishes itself: N less the
    hub rows and the `decoupled` rows (s_v = 0, solved at the start of the
    solve and skipped); vtx_ptr, vtx_edge, s of every row.
    direction (k_cg_direction): read R and P, write P, for the rows that
    iterate (N - decoupled).
    cg_iteration: a lower bound, F, R, P read and written once, the E x k
    intermediate written and read once, both CSR index arrays read once, over
    all N rows (the definition the iteration's bandwidth fraction uses).
    cg_iteration_as_run: the same over the N - decoupled rows that iterate."""
    covered = N if covered is None else covered
    idx = 4 * (N + 1 + nnz + (N - hubs))
    vertex = elem * k * (E + 2 * (N - hubs)) + idx
    step = elem * k * (E + 5 * (N - hubs - decoupled)) + 4 * (N + 1 + nnz + N)
    edge = elem * k * (covered + E) + 4 * (2 * E + 1 + nnz + covered)
    per_iter = elem * k * (6 * N + 2 * E) + 4 * (2 * nnz + 2 * N + 2 * E)
    as_run = elem * k * (6 * (N - decoupled) + 2 * E) + 4 * (2 * nnz + 2 * N + 2 * E)
    return {"vertex_gather": vertex, "vertex_step": step, "edge_gather": edge, "cg_iteration": per_iter,
            "direction": 3 * elem * k * (N - decoupled), "cg_iteration_as_run": as_run}


def decoupled_rows(p):
    """Rows with delta(v) = 0 (no hyperedge of positive weight): s_v = 0, so
    the fused solve fixes them at the start and skips them."""
    per_entry = np.repeat(np.asarray(p.w, dtype=np.float64), np.diff(p.edge_ptr))
    dv = np.bincount(p.edge_vtx, weights=per_entry, minlength=p.N)
    return int(np.count_nonzero(dv == 0))


# ------------------------------------------------------- profile summaries

PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = ["paper_1908_08281_amd/csrc/spmm.hip", "paper_1908_08281_amd/csrc/kernels.h",
                  "paper_1908_08281_amd/csrc/common.h", "paper_1908_08281_amd/csrc/cg.hip"]


def sources_digest():
    """SHA-256 over the sources of the operator and CG kernels: a stored
    counter figure is used only while the kernels it measured are unchanged."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _short(name):
    return name.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "").strip()


def summarize_counters(fetch_csv, write_csv, kernel, workload, command, calib_bytes=1 << 30):
    """Per-dispatch HBM traffic of `kernel` (base name, e.g. k_spmm_vertex;
    its most-dispatched instance) from two rocprofv3 --pmc runs (FETCH_SIZE,
    WRITE_SIZE; KiB per dispatch), each scaled by what the same counter reads
    for the calibration copy of `calib_bytes` (the largest
    __amd_rocclr_copyBuffer dispatch of the run)."""
    import collections
    import csv

    def per_kernel(path, counter):
        vals, calib = collections.defaultdict(list), []
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            v = float(r["Counter_Value"])
            name = _short(r["Kernel_Name"])
            if "copyBuffer" in name:
                calib.append(v)
            elif name.split("::")[-1].startswith(kernel + "<") or name.split("::")[-1] == kernel:
                vals[name].append(v)
        inst = max(vals, key=lambda n2: len(vals[n2]))
        factor = calib_bytes / (max(calib) * 1024.0)
        return sum(vals[inst]) / len(vals[inst]) * 1024.0 * factor, factor, len(vals[inst]), inst

    fb, ff, nf, inst = per_kernel(fetch_csv, "FETCH_SIZE")
    wb, wf, nw, _ = per_kernel(write_csv, "WRITE_SIZE")
    return {"kernel": kernel, "instance": inst, "workload": workload, "fetch_bytes_per_launch": round(fb),
            "write_bytes_per_launch": round(wb), "traffic_bytes_per_launch": round(fb + wb),
            "fetch_scale": round(ff, 4), "write_scale": round(wf, 4), "dispatches": [nf, nw],
            "calibration": f"{calib_bytes} B device-to-device copy (bench.py --calib)",
            "sources_sha256": sources_digest(), "command": command}


def summarize_stats(stats_csv, workload, command, top=16):
    """Text table of a rocprofv3 --kernel-trace --stats run."""
    import csv
    rows = list(csv.DictReader(open(stats_csv)))
    lines = [f"# rocprofv3 kernel statistics: {workload}", "", f"command: {command}", "",
             f"{'kernel':70s} {'calls':>6s} {'avg_us':>9s} {'total_ms':>9s} {'pct':>6s}"]
    for r in rows[:top]:
        lines.append(f"{_short(r['Name'])[:70]:70s} {r['Calls']:>6s} {float(r['AverageNs']) / 1e3:9.2f} "
                     f"{float(r['TotalDurationNs']) / 1e6:9.3f} {float(r['Percentage']):6.2f}")
    return "\n".join(lines) + "\n"


def stored_traffic(kernel, workload, instance):
    """Traffic per launch from the committed counter summary, or None when
    there is none, the kernel sources changed since it was taken, or it was
    taken of another template instance (column shape) of the kernel."""
    path = os.path.join(PROFILES, f"{workload}_{kernel}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel") != kernel or rec.get("sources_sha256") != sources_digest():
        return None
    if rec.get("instance", "").split("::")[-1] != instance:
        return None
    return rec["traffic_bytes_per_launch"]


def _roof(name, n, ms, alg, bound="hbm", traffic=None, dtype="bf16"):
    avg = ms / max(n, 1)
    if bound == "hbm":
        ach = alg / (avg * 1e-3) / 1e9
        return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": name,
                "avg_launch_us": round(avg * 1e3, 2), "launches": n, "algorithmic_bytes_per_launch": int(alg)}
    ach = alg / (avg * 1e-3) / 1e12
    peak = BF16_PEAK_TFLOPS if dtype == "bf16" else FP32_MFMA_PEAK_TFLOPS
    return {"bound": "mfma", "achieved": round(ach, 2), "peak": peak, "unit": "TFLOP/s", "dtype": dtype,
            "frac": round(ach / peak, 5), "traffic": None, "kernel": name,
            "avg_launch_us": round(avg * 1e3, 2), "launches": n, "algorithmic_flops_per_launch": int(alg)}


def _breakdown(h, fn, n):
    """Every kernel of `n` further steps timed by launch events (diagnostics,
    outside the timed region: stamping every launch costs dispatch time)."""
    import torch

    from paper_1908_08281_amd import hgl
    hgl.profile(h, True)
    for _ in range(n):
        fn()
    torch.cuda.synchronize()
    prof = hgl.profile_read(h)
    hgl.profile(h, False)
    return _kernel_ms(prof)


def _kernel_ms(prof):
    return {k2: [n2, round(m2, 3)] for k2, (n2, m2) in prof.items() if n2}


def _upload(p, dev):
    import torch
    return tuple(torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in (p.edge_ptr, p.edge_vtx, p.w))


def _host_info():
    """The host the CPU baseline ran on: CPU model, cores in this process's
    affinity mask, and the BLAS threads the oracle was limited to."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "affinity_cores": len(os.sched_getaffinity(0)), "blas_threads": 1}


def _line(metric, value, unit, steps, warmup, ms, dtype, config, roof, extra=None, higher=True):
    out = {"metric": metric, "value": round(value, 3), "unit": unit, "n_gpus": 1, "steps": steps,
           "warmup": warmup, "ms_per_step": round(ms, 4), "higher_is_better": higher, "scaling": "weak",
           "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config, "roofline": roof}
    if extra:
        out.update(extra)
    if isinstance(out.get("cpu_baseline"), dict):
        out["cpu_baseline"]["host"] = _host_info()
    return out


def _timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = [fn() for _ in range(steps)]
    torch.cuda.synchronize()
    return time.perf_counter() - t0, res


# ------------------------------------------------------------------ workloads

def cpu_cg_baseline(p, tol, budget_s=15.0):
    """Oracle FP64 matrix-free CG (one thread) on a bounded sample of the
    workload: the first columns of Y, or whole solves of all of them repeated
    until about budget_s of CPU time."""
    from threadpoolctl import threadpool_limits

    from oracle import laplacian as lap
    from oracle import solve
    op = lap.SparseOperator(p.N, p.E, p.edge_ptr, p.edge_vtx, p.w, p.lam)
    cols = 4
    k = p.Y.shape[1]
    with threadpool_limits(1):
        t0 = time.perf_counter()
        solve.cg_ranking(op, p.w, p.lam, p.Y[:, :cols], tol=tol)
        probe = time.perf_counter() - t0
        ncols = int(max(cols, min(k, cols * budget_s / max(probe, 1e-3))))
        reps, dt = 0, 0.0
        t0 = time.perf_counter()
        while reps == 0 or (ncols == k and dt < budget_s * 0.6 and reps < 8):
            solve.cg_ranking(op, p.w, p.lam, p.Y[:, :ncols], tol=tol)
            reps += 1
            dt = time.perf_counter() - t0
    what = f"first {ncols} of {k} columns" if ncols < k else f"all {k} columns, {reps} solves"
    return {"value": round(reps * ncols / dt, 2), "unit": "RHS/s", "cores": 1, "kind": "oracle",
            "sample": f"{what} of the same workload, FP64 matrix-free CG (eqs. 16-20) to the same relres, "
                      f"one thread, {dt:.1f} s"}


# The oracle on every core of the host: worker processes (started fresh, so
# none of them touches the GPU), each running the unchanged oracle on its
# share of independent units (columns, graphs, blocks).  The pool is sized to
# the process's affinity mask, at most 16.
_POOL_STATE = {}


def _pool_cores():
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _pool_init_cg(N, E, edge_ptr, edge_vtx, w, lam, Y_u8, tol):
    from threadpoolctl import threadpool_limits

    from oracle import laplacian as lap
    _POOL_STATE["limit"] = threadpool_limits(1)
    _POOL_STATE["op"] = lap.SparseOperator(N, E, edge_ptr, edge_vtx, w, lam)
    _POOL_STATE["Y"] = Y_u8
    _POOL_STATE["w"] = w
    _POOL_STATE["lam"] = lam
    _POOL_STATE["tol"] = tol


def _pool_cg_cols(c01):
    from oracle import solve
    c0, c1 = c01
    st = _POOL_STATE
    solve.cg_ranking(st["op"], st["w"], st["lam"], st["Y"][:, c0:c1].astype(np.float64), tol=st["tol"])
    return c1 - c0


def _pool_init_learn(N, E, edge_ptr, edge_vtx, w, lam, mu, Y_u8, tol):
    _pool_init_cg(N, E, edge_ptr, edge_vtx, w, lam, Y_u8, tol)
    _POOL_STATE["mu"] = mu


def _pool_learn_cols(c01):
    from oracle import grad as ograd
    from oracle import solve
    c0, c1 = c01
    st = _POOL_STATE
    Yc = st["Y"][:, c0:c1].astype(np.float64)
    F, _, _ = solve.cg_ranking(st["op"], st["w"], st["lam"], Yc, tol=st["tol"])
    ograd.objective_grad_sparse(st["op"], st["w"], st["lam"], st["mu"], Yc, F, tol=st["tol"])
    return c1 - c0


def _pool_graph(args):
    from threadpoolctl import threadpool_limits

    from oracle import laplacian as lap
    from oracle import solve
    n, e, ep, ev, w, lam, Y_u8, tol = args
    with threadpool_limits(1):
        op = lap.SparseOperator(n, e, ep, ev, w, lam)
        solve.cg_ranking(op, w, lam, Y_u8.astype(np.float64), tol=tol)
    return Y_u8.shape[1]


def _pool_init_rsvd(N, E, edge_ptr, edge_vtx, w, lam, omega, q, scheme):
    from threadpoolctl import threadpool_limits

    from oracle import laplacian as lap
    _POOL_STATE["limit"] = threadpool_limits(1)
    _POOL_STATE["op"] = lap.SparseOperator(N, E, edge_ptr, edge_vtx, w, lam)
    _POOL_STATE["omega"] = omega
    _POOL_STATE["q"] = q
    _POOL_STATE["scheme"] = scheme


def _pool_block(o01):
    """One block as the one-thread baseline does it: A_bb extracted through the
    sparse operator, then Algorithm 1 (or the power scheme)."""
    from oracle import rsvd
    o0, o1 = o01
    st = _POOL_STATE
    P = np.zeros((st["op"].N, o1 - o0))
    P[o0:o1] = np.eye(o1 - o0)
    Ab = st["op"].adjacency_apply(P)[o0:o1]
    (rsvd.randomized_svd if st["scheme"] == "subspace" else rsvd.randomized_svd_power)(Ab, st["omega"][o0:o1],
                                                                                       st["q"])
    return 1


def _pool_noop(i):
    import scipy.sparse  # noqa: F401  (the oracle's imports, paid before the timing)
    time.sleep(0.05)
    return i


def _pool_run(init, initargs, fn, tasks, budget_s):
    """Run tasks (repeating the list until about budget_s has passed, at
    least once) on the pool; returns (units done, seconds, workers)."""
    import multiprocessing as mp
    n = _pool_cores()
    ctx = mp.get_context("spawn")
    with ctx.Pool(n, initializer=init, initargs=initargs) as pool:
        # every worker started and initialised (imports, operator) outside the timing
        pool.map(_pool_noop, range(4 * n), chunksize=1)
        done, reps = 0, 0
        t0 = time.perf_counter()
        while reps == 0 or (time.perf_counter() - t0 < budget_s * 0.5 and reps < 8):
            done += sum(pool.map(fn, tasks, chunksize=1))
            reps += 1
        dt = time.perf_counter() - t0
    return done, dt, n


def _col_tasks(k, parts):
    step = max(1, -(-k // parts))
    return [(c, min(k, c + step)) for c in range(0, k, step)]


def cpu_cg_all_cores(p, tol, budget_s=8.0):
    """The same oracle CG on every core: columns split over the workers."""
    Yu8 = np.ascontiguousarray(p.Y.astype(np.uint8))
    k = p.Y.shape[1]
    done, dt, n = _pool_run(_pool_init_cg, (p.N, p.E, p.edge_ptr, p.edge_vtx, p.w, p.lam, Yu8, tol), _pool_cg_cols,
                            _col_tasks(k, 4 * _pool_cores()), budget_s)
    return {"value": round(done / dt, 2), "unit": "RHS/s", "cores": n, "kind": "oracle",
            "sample": f"all {k} columns split over {n} worker processes (one thread each), repeated "
                      f"{done // k} times, {dt:.1f} s"}


def bench_cg(a, name, p, mode, tol, rr_period=0, with_cpu=True):
    import torch

    from paper_1908_08281_amd import hgl
    dev = torch.device("cuda:0")
    k = p.Y.shape[1]
    dtype = torch.float32 if mode == "f32" else torch.float64
    ep, ev, w = _upload(p, dev)
    h = (hgl.build_laplacian_batched(p.vtx_offsets, p.edge_offsets, ep, ev, w) if p.vtx_offsets is not None
         else hgl.build_laplacian(ep, ev, w, p.N))
    Y = torch.from_numpy(p.Y).to(dev, dtype)
    batched = p.vtx_offsets is not None
    state = {"ok": True, "iters": [], "ms": []}
    out = torch.empty_like(Y)  # one output buffer, so that a recorded graph is replayed
    graph = bool(a.graph)
    tune = bool(a.tune)

    def step():
        t0 = time.perf_counter()  # each solve synchronises before it returns
        if batched:
            F, it, rel, st = hgl.cg_solve_batched(h, p.lams, Y, mode=mode, tol=tol, rr_period=rr_period,
                                                  graph=graph, out=out, tune=tune)
        else:
            F, it, rel, st = hgl.cg_solve(h, p.lam, Y, mode=mode, tol=tol, rr_period=rr_period, graph=graph,
                                          out=out, tune=tune)
        state["ms"].append(1e3 * (time.perf_counter() - t0))
        state["ok"] = state["ok"] and st == 0 and bool(np.all(rel <= tol))
        state["iters"].append(int(it.max()))

    for _ in range(a.warmup):
        step()
    state["iters"].clear()
    state["ms"].clear()
    # in the timed steps every 4th launch of the two gather kernels carries
    # launch events (stamping every launch would slow the stream by ~7%)
    hgl.profile(h, True, kinds=["vertex_gather", "edge_gather"], every=4)
    dt, _ = _timed(step, a.steps, 0)
    prof = hgl.profile_read(h)
    hgl.profile(h, False)
    breakdown = _breakdown(h, step, max(2, a.steps // 5))
    G = h.G
    ms = 1e3 * dt / a.steps
    value = a.steps * k * G / dt if state["ok"] else 0.0
    elem = 4 if mode == "f32" else 8
    part = h.partition()
    covered = int(np.unique(p.edge_vtx).size)
    dec = decoupled_rows(p)
    ab = gather_bytes(p.N, p.E, p.nnz, k, elem, covered, part["hub_rows"], dec)
    nv, mv = prof["vertex_gather"]
    ne, me = prof["edge_gather"]
    # template instances the solves ran (the column shape may be autotuned)
    shp = h.gather_shape()
    t = "float" if mode == "f32" else "double"
    inst_v = f"k_spmm_vertex<{t}, {t}, {shp['vertex'][0]}, {shp['vertex'][1]}, 3>"
    inst_e = f"k_spmm_edge<{t}, {t}, {shp['edge'][0]}, {shp['edge'][1]}, true>"
    if mv >= me:
        roof = _roof("k_spmm_vertex", nv, mv, ab["vertex_step"],
                     traffic=stored_traffic("k_spmm_vertex", name, inst_v))
        roof["instance"] = inst_v
    else:
        roof = _roof("k_spmm_edge", ne, me, ab["edge_gather"], traffic=stored_traffic("k_spmm_edge", name, inst_e))
        roof["instance"] = inst_e
    it_mean = float(np.mean(state["iters"]))
    cfg = {"workload": name, "N": p.N, "E": p.E, "nnz": p.nnz, "k": k, "graphs": G,
           "lambda": float(p.lam), "relres_tol": tol,
           "cg": f"{mode} vectors, fp64 inner products, residual replacement at convergence checks"
                 + (", first chunk of iterations as a replayed HIP graph" if graph else "")
                 + (f" and every {rr_period}" if rr_period else ""),
           "iterations": it_mean, "all_columns_converged": state["ok"], "partition": part}
    it_gbs = ab["cg_iteration"] * it_mean / (ms * 1e-3) / 1e9
    run_gbs = ab["cg_iteration_as_run"] * it_mean / (ms * 1e-3) / 1e9
    extra = {"cg_iteration_gbs": round(it_gbs, 1), "cg_iteration_frac": round(it_gbs / HBM_PEAK_GBS, 4),
             "cg_iteration_as_run": {"decoupled_rows": dec, "bytes": int(ab["cg_iteration_as_run"]),
                                     "gbs": round(run_gbs, 1), "frac": round(run_gbs / HBM_PEAK_GBS, 4)},
             "ms_per_step_median": round(float(np.median(state["ms"][:a.steps])), 4),
             "kernel_ms": breakdown}
    if batched and not a.no_extra:
        # the same graphs as G separate single-graph solves, one after another
        # (handles built outside the timing)
        subs = []
        for g in range(G):
            v0, v1 = int(p.vtx_offsets[g]), int(p.vtx_offsets[g + 1])
            e0, e1 = int(p.edge_offsets[g]), int(p.edge_offsets[g + 1])
            sep = (p.edge_ptr[e0:e1 + 1] - p.edge_ptr[e0]).astype(np.int32)
            sev = (p.edge_vtx[p.edge_ptr[e0]:p.edge_ptr[e1]] - v0).astype(np.int32)
            hg = hgl.build_laplacian(torch.from_numpy(sep).to(dev), torch.from_numpy(sev).to(dev),
                                     torch.from_numpy(np.ascontiguousarray(p.w[e0:e1])).to(dev), v1 - v0)
            subs.append((hg, float(p.lams[g]), Y[v0:v1].contiguous()))

        def separate():
            for hg, lam_g, Yg in subs:
                hgl.cg_solve(hg, lam_g, Yg, mode=mode, tol=tol, rr_period=rr_period, tune=tune)

        d_sep, _ = _timed(separate, 2, 1)
        extra["separate_solves"] = {"graphs": G, "ms": round(1e3 * d_sep / 2, 3),
                                    "batched_speedup": round((d_sep / 2) / (dt / a.steps), 3)}
    if mode == "f32" and not batched and not a.no_extra:
        # the plain FP64 solve on the GPU to the same FP64-checked relres (equal
        # accuracy), after the timed steps
        Y64 = Y.double()
        out64 = torch.empty_like(Y64)
        d64, r64 = _timed(lambda: hgl.cg_solve(h, p.lam, Y64, mode="f64", tol=tol, out=out64), 3, 1)
        extra["plain_f64_solve"] = {
            "ms_per_solve": round(1e3 * d64 / 3, 4), "iterations": int(r64[-1][1].max()),
            "converged": all(r[3] == 0 and bool(np.all(r[2] <= tol)) for r in r64),
            "f32_speedup": round((d64 / 3) / (dt / a.steps), 3)}
    if with_cpu and not a.no_cpu:
        if batched:
            extra["cpu_baseline"] = cpu_batch_baseline(p, tol)
        else:
            extra["cpu_baseline"] = cpu_cg_baseline(p, tol)
            extra["cpu_baseline"]["all_cores"] = cpu_cg_all_cores(p, tol)
    return _line("solved RHS/s at relres 1e-6" if mode == "f32" else "solved RHS/s at relres 1e-10",
                 value, "RHS/s", a.steps, a.warmup, ms, mode, cfg, roof, extra)


def _graph_parts(p):
    """The batch's graphs as separate problems (local ids), in order."""
    out = []
    for g in range(len(p.lams)):
        v0, v1 = int(p.vtx_offsets[g]), int(p.vtx_offsets[g + 1])
        e0, e1 = int(p.edge_offsets[g]), int(p.edge_offsets[g + 1])
        ep = (p.edge_ptr[e0:e1 + 1] - p.edge_ptr[e0]).astype(np.int32)
        ev = (p.edge_vtx[p.edge_ptr[e0]:p.edge_ptr[e1]] - v0).astype(np.int32)
        out.append((v1 - v0, e1 - e0, ep, ev, np.ascontiguousarray(p.w[e0:e1]), float(p.lams[g]),
                    np.ascontiguousarray(p.Y[v0:v1].astype(np.uint8))))
    return out


def cpu_batch_baseline(p, tol, budget_s=12.0):
    """Oracle FP64 CG graph by graph (all columns of each) on one thread until
    about budget_s, and all graphs over every core."""
    from threadpoolctl import threadpool_limits

    from oracle import laplacian as lap
    from oracle import solve
    parts = _graph_parts(p)
    G, k = len(parts), p.Y.shape[1]
    with threadpool_limits(1):
        t0 = time.perf_counter()
        done = 0
        for n, e, ep, ev, w, lam, Yg in parts:
            op = lap.SparseOperator(n, e, ep, ev, w, lam)
            solve.cg_ranking(op, w, lam, Yg.astype(np.float64), tol=tol)
            done += 1
            if time.perf_counter() - t0 > budget_s:
                break
        dt = time.perf_counter() - t0
    out = {"value": round(done * k / dt, 2), "unit": "RHS/s", "cores": 1, "kind": "oracle",
           "sample": f"first {done} of {G} graphs, all {k} columns each, FP64 matrix-free CG (eqs. 16-20) "
                     f"to the same relres, one thread, {dt:.1f} s"}
    tasks = [(n, e, ep, ev, w, lam, Yg, tol) for n, e, ep, ev, w, lam, Yg in parts]
    tasks.sort(key=lambda t: -t[0])  # largest first
    cdone, cdt, nw = _pool_run(None, (), _pool_graph, tasks, budget_s * 0.75)
    out["all_cores"] = {"value": round(cdone / cdt, 2), "unit": "RHS/s", "cores": nw, "kind": "oracle",
                        "sample": f"all {G} graphs over {nw} worker processes (one thread each, largest first), "
                                  f"{cdt:.1f} s"}
    return out


def bench_schur(a, min_block=50):
    """The Schur-complement block inverse (eqs. 12-14, nested tessellation
    down to min_block, exact leaves) of the 50 tessellated blocks, then the
    solve it preconditions."""
    import torch

    import synth
    from paper_1908_08281_amd import hgl
    dev = torch.device("cuda:0")
    p = synth.tessellated()
    nb = len(p.blocks) - 1
    ep, ev, w = _upload(p, dev)
    h = hgl.build_laplacian(ep, ev, w, p.N)
    run = lambda: hgl.block_schur_inverse(h, p.lam, p.blocks, min_block)  # noqa: E731
    for _ in range(a.warmup):
        run()
    flops = hgl.block_schur_plan(p.blocks, min_block)["flops"]
    # the calls replay the recorded HIP graph; the roofline comes from the
    # same number of calls launched directly with the products timed
    dt, _ = _timed(run, a.steps, 0)
    hgl.profile(h, True, kinds=["dense_gemm"])
    _timed(run, a.steps, 0)
    prof = hgl.profile_read(h)
    hgl.profile(h, False)
    breakdown = _breakdown(h, run, max(2, a.steps // 5))
    n_g, ms_g = prof["dense_gemm"]
    roof = _roof("k_schur_gemm", n_g, ms_g, flops * a.steps / max(n_g, 1), bound="mfma", dtype="fp32")
    ms = 1e3 * dt / a.steps
    Y = torch.from_numpy(p.Y).to(dev, torch.float32)
    tol = 1e-6 / (1 + 1 / p.lam)
    hgl.block_schur_invert(h, p.lam, p.blocks, Y, min_block=min_block, refine_tol=tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    F, it, rel, st = hgl.block_schur_invert(h, p.lam, p.blocks, Y, min_block=min_block, refine_tol=tol)
    torch.cuda.synchronize()
    t_inv = time.perf_counter() - t0
    hgl.block_rsvd_invert(h, p.lam, p.blocks, Y, 64, 10, 2, refine_tol=tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, it_r, rel_r, _, st_r = hgl.block_rsvd_invert(h, p.lam, p.blocks, Y, 64, 10, 2, refine_tol=tol)
    torch.cuda.synchronize()
    t_rsvd = time.perf_counter() - t0
    cfg = {"workload": "block_schur", "N": p.N, "blocks": nb, "block_rows": "U[500,1500]", "min_block": min_block,
           "products": "fp32 MFMA 16x16x4, fp32 accumulation", "leaves": "fp32 Gauss-Jordan in registers"}
    extra = {"kernel_ms": breakdown, "flops_per_batch": flops,
             "refined_solve": {"nrhs": Y.shape[1], "pcg_iters": int(it.max()), "seconds": round(t_inv, 4),
                               "converged": st == 0 and bool(np.all(rel <= tol)),
                               "rsvd_pcg_iters": int(it_r.max()), "rsvd_seconds": round(t_rsvd, 4),
                               "rsvd_converged": st_r == 0 and bool(np.all(rel_r <= tol))}}
    if not a.no_cpu:
        from threadpoolctl import threadpool_limits

        from oracle import laplacian as lap
        from oracle import schur
        Hs = lap.incidence_sparse(p.N, p.E, p.edge_ptr, p.edge_vtx)
        with threadpool_limits(1):
            t0 = time.perf_counter()
            done = 0
            for b in range(nb):
                schur.schur_inverse(schur.system_block(Hs, p.w, p.lam, p.blocks[b], p.blocks[b + 1]), min_block)
                done += 1
                if time.perf_counter() - t0 > 20.0:
                    break
            dtc = time.perf_counter() - t0
        extra["cpu_baseline"] = {"value": round(done / dtc, 3), "unit": "blocks/s", "cores": 1, "kind": "oracle",
                                 "sample": f"first {done} of {nb} blocks, FP64 eqs. 12-15 with SVD leaves "
                                           f"(block extraction included), one thread, {dtc:.1f} s"}
    return _line("Schur block inverses/s", a.steps * nb / dt, "blocks/s", a.steps, a.warmup, ms, "f32", cfg, roof,
                 extra)


def bench_rsvd(a, scheme="subspace"):
    import torch

    import synth
    from paper_1908_08281_amd import hgl
    dev = torch.device("cuda:0")
    p = synth.tessellated()
    k, pp, q = 64, 10, 2
    l = k + pp
    nb = len(p.blocks) - 1
    ep, ev, w = _upload(p, dev)
    h = hgl.build_laplacian(ep, ev, w, p.N)
    om = torch.from_numpy(synth.gaussian_sketch(p.N, l, 11)[0].view(np.int16).copy()).to(dev)
    run = lambda: hgl.block_rsvd(h, p.blocks, k, pp, q, omega=om, scheme=scheme)  # noqa: E731
    for _ in range(a.warmup):
        run()
    hgl.profile(h, True, kinds=["dense_gemm"])
    dt, _ = _timed(run, a.steps, 0)
    prof = hgl.profile_read(h)
    hgl.profile(h, False)
    breakdown = _breakdown(h, run, max(2, a.steps // 5))
    sizes = np.diff(p.blocks).astype(np.float64)
    gemm_flops = float(np.sum(2.0 * sizes * sizes * l))           # one product A_bb S, every block
    n_g, ms_g = prof["dense_gemm"]
    # 2q + 2 products per call; the library splits the blocks into groups
    # with a launch each, so a launch covers the products' share n_prod / n_g
    n_prod = (2 * q + 2) * a.steps
    per_launch = n_prod / max(n_g, 1)
    roof = _roof("rsvd_gemm", n_g, ms_g, gemm_flops * per_launch, bound="mfma")
    nbp = np.ceil(sizes / 64) * 64
    gemm_bytes = float(np.sum(2 * nbp * nbp + 2 * 2 * nbp * 80 + 4 * nbp * 80))
    hbm = _roof("rsvd_gemm", n_g, ms_g, gemm_bytes * per_launch)
    ms = 1e3 * dt / a.steps
    # refined solve beside it
    Y = torch.from_numpy(p.Y).to(dev, torch.float32)
    tol = 1e-6 / (1 + 1 / p.lam)
    t0 = time.perf_counter()
    F, it, rel, sig, st = hgl.block_rsvd_invert(h, p.lam, p.blocks, Y, k, pp, q, omega=om, refine_tol=tol,
                                                scheme=scheme)
    torch.cuda.synchronize()
    t_inv = time.perf_counter() - t0
    t0 = time.perf_counter()
    F2, it2, rel2, st2 = hgl.cg_solve(h, p.lam, Y, tol=tol)
    torch.cuda.synchronize()
    t_cg = time.perf_counter() - t0
    cfg = {"workload": "block_rsvd" if scheme == "subspace" else "block_rsvd_power", "N": p.N, "blocks": nb,
           "block_rows": "U[500,1500]", "k": k, "p": pp, "q": q,
           "sketch": "bf16 A_bb, split-bf16 basis, fp32 accumulation, fp64 CholQR2, fp32 tridiagonal eigensolver",
           "scheme": "Algorithm 1 (orthonormalised after every product)" if scheme == "subspace" else
                     "power scheme of eq. 10 (2q+1 products, one CholQR2)"}
    extra = {"roofline_hbm": hbm, "kernel_ms": breakdown,
             "refined_solve": {"nrhs": Y.shape[1], "pcg_iters": int(it.max()), "seconds": round(t_inv, 4),
                               "converged": st == 0 and bool(np.all(rel <= tol)),
                               "plain_cg_iters": int(it2.max()), "plain_cg_seconds": round(t_cg, 4)}}
    if scheme == "subspace" and not a.no_extra:
        # the FP64 sketch (every product in FP64) on the same inputs: its time,
        # and the refined solve it gives (equal accuracy: the same tolerance)
        d64, _ = _timed(lambda: hgl.block_rsvd(h, p.blocks, k, pp, q, sketch="f64", omega=om), 3, 1)
        F6, it6, rel6, sig6, st6 = hgl.block_rsvd_invert(h, p.lam, p.blocks, Y, k, pp, q, sketch="f64", omega=om,
                                                         refine_tol=tol)
        extra["f64_sketch"] = {"ms_per_batch": round(1e3 * d64 / 3, 4),
                               "bf16_speedup": round((d64 / 3) / (dt / a.steps), 3),
                               "pcg_iters": int(it6.max()),
                               "converged": st6 == 0 and bool(np.all(rel6 <= tol))}
    if scheme == "power":
        # accuracy against Algorithm 1 on the same sketch: relative deviation
        # of the kept singular values, worst block
        _, s_pow = run()
        _, s_sub = hgl.block_rsvd(h, p.blocks, k, pp, q, omega=om)
        dev_rel = ((s_pow - s_sub).abs() / s_sub.abs()).max().item()
        extra["sigma_vs_algorithm1"] = {"max_rel_dev": dev_rel, "blocks": nb, "k": k}
    if not a.no_cpu:
        from threadpoolctl import threadpool_limits

        from oracle import laplacian as lap
        from oracle import rsvd
        op = lap.SparseOperator(p.N, p.E, p.edge_ptr, p.edge_vtx, p.w, p.lam)
        vals = synth.gaussian_sketch(p.N, l, 11)[1]
        with threadpool_limits(1):
            t0 = time.perf_counter()
            done = 0
            for b in range(nb):
                o0, o1 = p.blocks[b], p.blocks[b + 1]
                P = np.zeros((p.N, o1 - o0))
                P[o0:o1] = np.eye(o1 - o0)
                Ab = op.adjacency_apply(P)[o0:o1]
                (rsvd.randomized_svd if scheme == "subspace" else rsvd.randomized_svd_power)(Ab, vals[o0:o1], q)
                done += 1
                if time.perf_counter() - t0 > 20.0:
                    break
            dtc = time.perf_counter() - t0
        extra["cpu_baseline"] = {"value": round(done / dtc, 3), "unit": "blocks/s", "cores": 1, "kind": "oracle",
                                 "sample": f"first {done} of {nb} blocks, FP64 "
                                           + ("Algorithm 1" if scheme == "subspace" else "eq. 10 power scheme")
                                           + f" with Householder QR (block extraction included), one thread, "
                                             f"{dtc:.1f} s"}
        # every block over every core, each as the one-thread run does it
        blocks = sorted(((int(p.blocks[b]), int(p.blocks[b + 1])) for b in range(nb)), key=lambda t: t[0] - t[1])
        cdone, cdt, nw = _pool_run(_pool_init_rsvd, (p.N, p.E, p.edge_ptr, p.edge_vtx, p.w, p.lam, vals, q, scheme),
                                   _pool_block, blocks, 0.0)
        extra["cpu_baseline"]["all_cores"] = {
            "value": round(cdone / cdt, 3), "unit": "blocks/s", "cores": nw, "kind": "oracle",
            "sample": f"all {nb} blocks over {nw} worker processes (one thread each, largest first, block "
                      f"extraction included), {cdt:.1f} s"}
    return _line("rSVD blocks/s", a.steps * nb / dt, "blocks/s", a.steps, a.warmup, ms, "bf16", cfg, roof, extra)


def bench_single(a):
    """The paper's query shape (section 4): one RHS per test image on a
    5,867-vertex graph; latency of one query through the one-workgroup
    solver, and the 1292 queries of the paper's test set in one call."""
    import torch

    import synth
    from paper_1908_08281_amd import hgl
    dev = torch.device("cuda:0")
    p = synth.single_query()
    k = p.Y.shape[1]
    tol = 1e-6 / (1 + 1 / p.lam)
    ep, ev, w = _upload(p, dev)
    h = hgl.build_laplacian(ep, ev, w, p.N)
    Y = torch.from_numpy(p.Y).to(dev, torch.float32)
    Y1 = Y[:, :1].contiguous()
    out1, outk = torch.empty_like(Y1), torch.empty_like(Y)
    steps1 = max(a.steps, 20)
    stepsk = max(a.steps // 4, 5)
    dt1, r1 = _timed(lambda: hgl.cg_solve_wg(h, p.lam, Y1, tol=tol, out=out1), steps1, max(a.warmup, 3))
    dtk, rk = _timed(lambda: hgl.cg_solve_wg(h, p.lam, Y, tol=tol, out=outk), stepsk, max(a.warmup, 1))
    ok = all(r[3] == 0 and bool(np.all(r[2] <= tol)) for r in r1 + rk)
    mk1, _ = _timed(lambda: hgl.cg_solve(h, p.lam, Y1, tol=tol), steps1, 3)
    mkk, _ = _timed(lambda: hgl.cg_solve(h, p.lam, Y, tol=tol), stepsk, 1)
    lat_ms = 1e3 * dt1 / steps1
    # compulsory bytes of one query: y and f (4 N each), s (4 N), c (4 E),
    # and the per-thread tables of both CSRs (read once per gather, from L2)
    alg = 4.0 * (3 * p.N + p.E)
    roof = _roof("k_cg_wg", 1, lat_ms, alg)
    roof["note"] = ("one workgroup per query: bound by the latency of its gathers and barriers, not by HBM; "
                    "achieved counts the compulsory bytes over the whole call")
    cfg = {"workload": "single_query_cg", "N": p.N, "E": p.E, "nnz": p.nnz, "k": 1, "lambda": p.lam,
           "tol": tol, "solver": "one-workgroup CG (hgl_cg_solve_wg), FP32 vectors, FP64 sums and checks"}
    extra = {"converged": ok, "iterations": int(r1[-1][1].max()),
             "multi_kernel_latency_us": round(1e6 * mk1 / steps1, 1),
             "throughput": {"queries": k, "one_workgroup_rhs_per_s": round(stepsk * k / dtk, 1),
                            "multi_kernel_rhs_per_s": round(stepsk * k / mkk, 1)}}
    if not a.no_cpu:
        from threadpoolctl import threadpool_limits

        from oracle import laplacian as lap
        from oracle import solve
        op = lap.SparseOperator(p.N, p.E, p.edge_ptr, p.edge_vtx, p.w, p.lam)
        with threadpool_limits(1):
            t0 = time.perf_counter()
            done = 0
            while done < k and time.perf_counter() - t0 < 10.0:
                solve.cg_ranking(op, p.w, p.lam, p.Y[:, done:done + 1], tol=tol)
                done += 1
            dtc = time.perf_counter() - t0
        extra["cpu_baseline"] = {"value": round(1e6 * dtc / done, 1), "unit": "us per query", "cores": 1,
                                 "kind": "oracle",
                                 "sample": f"first {done} of {k} queries one at a time, FP64 matrix-free CG "
                                           f"(eqs. 16-20) to the same relres, one thread, {dtc:.1f} s"}
    return _line("single-query solve latency", 1e3 * lat_ms, "us", steps1, max(a.warmup, 3), lat_ms, "f32", cfg,
                 roof, extra, higher=False)


def bench_batch_small(a):
    """Many small independent problems: 64 G2 graphs of 2000-6000 vertices
    (the batch workload's recipe at the one-workgroup solver's sizes), 100
    RHS each; every (graph, column) pair one workgroup of one launch, and
    the multi-kernel batched solver on the same inputs."""
    import torch

    import synth
    from paper_1908_08281_amd import hgl
    dev = torch.device("cuda:0")
    p = synth.batch_of_graphs(G=64, nlo=2000, nhi=6000, k=100)
    G, k = len(p.lams), p.Y.shape[1]
    tol = 1e-6 / (1 + 1 / 0.5)
    ep, ev, w = _upload(p, dev)
    h = hgl.build_laplacian_batched(p.vtx_offsets, p.edge_offsets, ep, ev, w)
    Y = torch.from_numpy(p.Y).to(dev, torch.float32)
    out = torch.empty_like(Y)
    steps = max(a.steps // 2, 5)
    dt, r = _timed(lambda: hgl.cg_solve_wg_batched(h, p.lams, Y, tol=tol, out=out), steps, max(a.warmup, 1))
    ok = all(x[3] == 0 and bool(np.all(x[2] <= tol)) for x in r)
    dm, _ = _timed(lambda: hgl.cg_solve_batched(h, p.lams, Y, tol=tol), steps, 1)
    ms = 1e3 * dt / steps
    alg = 4.0 * (3 * p.N + p.E) * k  # compulsory bytes: y, f, s per vertex row and column, c per hyperedge
    roof = _roof("k_cg_wg", 1, ms, alg)
    roof["note"] = ("one workgroup per (graph, column): bound by the latency of its gathers and barriers, "
                    "not by HBM; achieved counts the compulsory bytes over the whole call")
    cfg = {"workload": "batched_small_graphs_wg", "graphs": G, "N": p.N, "E": p.E, "nnz": p.nnz, "k": k,
           "graph_sizes": "N_g ~ U[2000,6000], E_g = 0.8 N_g", "lambda": 0.5, "tol": tol,
           "solver": "one-workgroup CG per (graph, column) (hgl_cg_solve_wg_batched)"}
    extra = {"converged": ok, "iterations": int(r[-1][1].max()),
             "multi_kernel_rhs_per_s": round(steps * G * k / dm, 1)}
    return _line("solved RHS/s at relres 1e-6", steps * G * k / dt if ok else 0.0, "RHS/s", steps,
                 max(a.warmup, 1), ms, "f32", cfg, roof, extra)


def bench_learn(a):
    import torch

    import synth
    from paper_1908_08281_amd import hgl
    from paper_1908_08281_amd.learn import learn_weights
    dev = torch.device("cuda:0")
    p = synth.weight_learning()
    mu = 0.01
    k = p.Y.shape[1]
    ep, ev, w = _upload(p, dev)
    h = hgl.build_laplacian(ep, ev, w, p.N)
    Y = torch.from_numpy(p.Y).to(dev, torch.float32)
    tol = 1e-6 / (1 + 1 / p.lam)
    w0 = w.clone()
    wl, recs = learn_weights(h, Y, p.lam, mu, max(a.warmup, 1), w0, tol=tol, history=True, strict=False)
    eta = recs[0]["eta"]
    hgl.profile(h, True, kinds=["vertex_gather"])
    t0 = time.perf_counter()
    wl, recs = learn_weights(h, Y, p.lam, mu, a.steps, wl, eta=eta, tol=tol, history=True, strict=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # only steps whose forward and adjoint solves both met tol count
    ok_steps = sum(1 for r in recs if r["cg_status"] == 0 and r["adjoint_status"] == 0)
    prof = hgl.profile_read(h)
    hgl.profile(h, False)
    part = h.partition()
    ab = gather_bytes(p.N, p.E, p.nnz, k, 4, int(np.unique(p.edge_vtx).size), part["hub_rows"], decoupled_rows(p))
    nv, mv = prof["vertex_gather"]
    roof = _roof("k_spmm_vertex", nv, mv, ab["vertex_step"])
    shp = h.gather_shape()
    roof["instance"] = f"k_spmm_vertex<float, float, {shp['vertex'][0]}, {shp['vertex'][1]}, 3>"
    cfg = {"workload": "weight_learning", "N": p.N, "E": p.E, "nnz": p.nnz, "k": k, "lambda": p.lam, "mu": mu,
           "eta": eta, "cg": "f32 vectors, fp64 inner products, residual replacement at convergence checks; "
                             "forward solve, adjoint solve, FP64 gradient contractions, simplex projection per step",
           "cg_iters_last": recs[-1]["cg_iters"], "adjoint_iters_last": recs[-1]["adjoint_iters"]}
    extra = {"converged_steps": ok_steps,
             "kernel_ms": _breakdown(h, lambda: learn_weights(h, Y, p.lam, mu, 1, wl, eta=eta, tol=tol), 1)}
    if not a.no_extra:
        # the paper's active-set rule of eq. 5 in the same loop, after the timed
        # steps, and the two step kernels alone on one gradient
        t0 = time.perf_counter()
        wa, ra = learn_weights(h, Y, p.lam, mu, a.steps, wl.clone(), eta=eta, tol=tol, history=True,
                               rule="active_set")
        torch.cuda.synchronize()
        dta = time.perf_counter() - t0
        hgl.set_weights(h, wl)
        F, _, _, _ = hgl.cg_solve(h, p.lam, Y, tol=tol)
        g, _, _, _, _ = hgl.weight_grad(h, p.lam, F, Y=Y, mu=mu, tol=tol)
        d_proj, _ = _timed(lambda: hgl.projected_gradient_step(wl, g, eta), 20, 2)
        d_act, _ = _timed(lambda: hgl.active_set_step(wl, g, eta), 20, 2)
        extra["active_set_rule"] = {"steps_per_s": round(a.steps / dta, 3), "mu_eff_last": ra[-1]["mu_eff"],
                                    "released_last": ra[-1]["released"], "active_last": ra[-1]["active"],
                                    "step_us": round(1e6 * d_act / 20, 2),
                                    "projection_step_us": round(1e6 * d_proj / 20, 2)}
    if not a.no_cpu:
        extra["cpu_baseline"] = cpu_learn_baseline(p, mu, tol)
    return _line("projected-gradient steps/s", ok_steps / dt, "steps/s", a.steps, a.warmup, 1e3 * dt / a.steps,
                 "f32", cfg, roof, extra)


def cpu_learn_baseline(p, mu, tol, budget_s=12.0):
    """The oracle's outer step (FP64 matrix-free CG forward solve, the adjoint
    CG and the edge contractions of eq. 4's gradient) on a sample of the tag
    columns, one thread; the objective sums over the columns, so the step's
    time is the sample's scaled to all of them (the E-length projection is
    negligible beside it).  Also all columns over every core."""
    from threadpoolctl import threadpool_limits

    from oracle import grad as ograd
    from oracle import laplacian as lap
    from oracle import solve
    op = lap.SparseOperator(p.N, p.E, p.edge_ptr, p.edge_vtx, p.w, p.lam)
    k = p.Y.shape[1]
    cols = 2
    with threadpool_limits(1):
        while True:
            t0 = time.perf_counter()
            Yc = p.Y[:, :cols].astype(np.float64)
            F, _, _ = solve.cg_ranking(op, p.w, p.lam, Yc, tol=tol)
            ograd.objective_grad_sparse(op, p.w, p.lam, mu, Yc, F, tol=tol)
            dt = time.perf_counter() - t0
            if dt > budget_s / 3 or cols >= k:
                break
            cols = min(k, cols * 2)
    per_step = dt * k / cols
    out = {"value": round(1.0 / per_step, 5), "unit": "steps/s", "cores": 1, "kind": "oracle",
           "sample": f"first {cols} of {k} columns (forward CG, adjoint CG, gradient contractions in FP64, "
                     f"to the same relres), {dt:.1f} s on one thread, scaled to {k} columns"}
    Yu8 = np.ascontiguousarray(p.Y.astype(np.uint8))
    nw = _pool_cores()
    tasks = _col_tasks(k, 2 * nw)
    # one pass over a share of the tasks (the whole step takes minutes on one thread)
    share = tasks[:nw]
    cdone, cdt, nw = _pool_run(_pool_init_learn, (p.N, p.E, p.edge_ptr, p.edge_vtx, p.w, p.lam, mu, Yu8, tol),
                               _pool_learn_cols, share, 0.0)
    out["all_cores"] = {"value": round(cdone / cdt / k, 5), "unit": "steps/s", "cores": nw, "kind": "oracle",
                        "sample": f"{cdone} of {k} columns over {nw} worker processes (one thread each), "
                                  f"{cdt:.1f} s, scaled to {k} columns"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the comparison runs after the timed steps (plain FP64 solve, FP64 sketch, "
                         "separate solves of the batch, the active-set loop), so that a profiled run holds the "
                         "measured kernels only")
    ap.add_argument("--workload", default=None,
                    help="multi_rhs, small, rsvd, rsvd_power, schur, single, batch_small, learn, batch, or a comma "
                         "list (one line each).  Default: one line for multi_rhs with the small, rsvd, learn and "
                         "batch results nested under 'workloads'")
    ap.add_argument("--rr-period", type=int, default=0)
    ap.add_argument("--tune", type=int, default=1,
                    help="1: column shapes of the CG kernels picked by the library's autotuner (default)")
    ap.add_argument("--graph", type=int, default=0,
                    help="1: run the first CG iteration chunk as a recorded HIP graph (off while kernels are "
                         "timed), 0: direct launches (default)")
    ap.add_argument("--summarize", nargs="+", metavar="ARG",
                    help="write profile summaries and exit: 'stats STATS_CSV WORKLOAD COMMAND' or "
                         "'counters FETCH_CSV WRITE_CSV KERNEL WORKLOAD COMMAND'")
    ap.add_argument("--peaks", type=int, default=1,
                    help="1: measure the achievable HBM GB/s and BF16 MFMA TFLOP/s with the library's probes "
                         "first and report each roofline against them too (frac_measured)")
    ap.add_argument("--calib", action="store_true",
                    help="first copy 1 GiB device to device (the known-size kernel that scales the "
                         "FETCH_SIZE / WRITE_SIZE counters of a profiled run)")
    a = ap.parse_args()
    if a.summarize:
        os.makedirs(PROFILES, exist_ok=True)
        kind = a.summarize[0]
        if kind == "stats":
            stats_csv, workload, command = a.summarize[1:4]
            out = os.path.join(PROFILES, f"{workload}_kernel_stats.txt")
            with open(out, "w") as fh:
                fh.write(summarize_stats(stats_csv, workload, command))
        else:
            fetch_csv, write_csv, kernel, workload, command = a.summarize[1:6]
            out = os.path.join(PROFILES, f"{workload}_{kernel}_traffic.json")
            with open(out, "w") as fh:
                json.dump(summarize_counters(fetch_csv, write_csv, kernel, workload, command), fh, indent=1)
        print(out)
        return
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {a.gpus}): the solves shard by columns, "
              "blocks or graphs with no communication, so no multi-GPU figure is produced", file=sys.stderr)
        sys.exit(2)
    import synth
    if a.calib:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    peaks = None
    if a.peaks:
        # the device's achievable peaks, measured with the library's own probes
        from paper_1908_08281_amd import hgl
        peaks = hgl.measure_peaks("cuda:0")
    def run(wl):
        if wl == "multi_rhs":
            p = synth.multi_rhs()
            out = bench_cg(a, "multi_rhs_cg", p, "f32", 1e-6 / (1 + 1 / p.lam), a.rr_period)
        elif wl == "small":
            p = synth.small_plain()
            out = bench_cg(a, "small_plain_cg_f64", p, "f64", 1e-10)
        elif wl == "batch":
            p = synth.batch_of_graphs()
            out = bench_cg(a, "batched_64_graphs", p, "f32", 1e-6 / (1 + 1 / 0.5))
        elif wl == "rsvd":
            out = bench_rsvd(a)
        elif wl == "rsvd_power":
            out = bench_rsvd(a, scheme="power")
        elif wl == "schur":
            out = bench_schur(a)
        elif wl == "single":
            out = bench_single(a)
        elif wl == "batch_small":
            out = bench_batch_small(a)
        elif wl == "learn":
            out = bench_learn(a)
        else:
            print(f"unknown workload {wl}", file=sys.stderr)
            sys.exit(2)
        for key in ("roofline", "roofline_hbm"):
            roof = out.get(key)
            if peaks and isinstance(roof, dict) and (roof["bound"] == "hbm" or roof.get("dtype") == "bf16"):
                meas = peaks["hbm_gbs"] if roof["bound"] == "hbm" else peaks["bf16_mfma_tflops"]
                roof["measured_peak"] = meas
                roof["frac_measured"] = round(roof["achieved"] / meas, 4)
        return out

    if a.workload is None:
        # the headline line, with the other configurations' results nested
        head = run("multi_rhs")
        head["workloads"] = {}
        for wl in NESTED:
            print(f"bench: {wl}", file=sys.stderr, flush=True)
            sub = run(wl)
            for key in ("n_gpus", "scaling", "data"):
                sub.pop(key, None)
            head["workloads"][wl] = sub
        print(json.dumps(head), flush=True)
        return
    for wl in a.workload.split(","):
        print(json.dumps(run(wl)), flush=True)


if __name__ == "__main__":
    main()
