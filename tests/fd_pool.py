"""Finite differences of the adaptive-weight objective at full size on every
host core (test infrastructure): worker processes, started fresh so that none
of them touches the GPU, each build the FP64 sparse oracle once and return
Richardson-extrapolated central differences for their share of the edges.

J(w) = tr(F' L F) + lambda ||F - Y||^2 + mu ||w||^2 with F = (I + L/lambda)^-1 Y
(section 2, eq. 4, reading R14), F by the oracle's FP64 CG to relres 1e-13."""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np

_STATE = {}


def _init(N, E, edge_ptr, edge_vtx, w, lam, mu, Y):
    from threadpoolctl import threadpool_limits

    from oracle import laplacian as lap
    _STATE["limit"] = threadpool_limits(1)
    op = lap.SparseOperator(N, E, edge_ptr, edge_vtx, w, lam)
    _STATE.update(op=op, de=lap.edge_degrees(op.H), lam=lam, mu=mu, Y=Y, w=np.asarray(w, dtype=np.float64))


def _objective(w):
    from oracle import laplacian as lap
    from oracle import solve
    st = _STATE
    op = st["op"]
    op.s = lap.inv_sqrt_degrees(lap.vertex_degrees(op.H, w))
    op.c = w / st["de"]
    F, _, _ = solve.cg_ranking(op, w, st["lam"], st["Y"], tol=1e-13)
    AF = op.adjacency_apply(F)
    return float(np.sum(F * (F - AF)) + st["lam"] * np.sum((F - st["Y"]) ** 2) + st["mu"] * (w @ w))


def _richardson(args):
    from oracle import grad as ograd
    e, h = args
    return ograd.richardson_difference(_objective, _STATE["w"], int(e), h)


def richardson_gradient(p, mu, edges, h=1e-6, workers=None):
    """dJ/dw_e by (4 D(h/2) - D(h))/3 for each edge in `edges`."""
    n = workers or max(1, min(16, len(os.sched_getaffinity(0))))
    ctx = mp.get_context("spawn")
    Y = np.asarray(p.Y, dtype=np.float64)
    with ctx.Pool(n, initializer=_init, initargs=(p.N, p.E, p.edge_ptr, p.edge_vtx, p.w, p.lam, mu, Y)) as pool:
        return np.array(pool.map(_richardson, [(int(e), h) for e in edges], chunksize=1))
