"""The FP64 oracle over many points in a process pool (test infrastructure).

Workers are started with the "spawn" method, so they share no state with a
parent that has initialised the GPU, and each runs NumPy on one thread.
Every worker walks its chunk of points with oracle.estep_point and returns
the per-point outputs plus its share of the M-step sums; the parent adds
the shares in FP64.  The selection gap (H'-th minus (H'+1)-th score) is kept
per point for the near-tie checks.
"""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np

WORKERS = 16  # the host CPU share of one GPU on the test machines


def n_workers() -> int:
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return max(1, min(WORKERS, avail))


def _one_thread():
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:
        pass


def _chunk(args):
    from oracle import prosper_oracle as O
    model, Y, W, pi, sigma, Hp, gamma, sel = args
    Y = np.asarray(Y, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    n, D = Y.shape
    H = W.shape[1]
    tab = O.state_table(model, Hp, gamma)
    out = {"sel": np.zeros((n, Hp), np.int64), "flagged": np.zeros(n, bool),
           "s_mean": np.zeros((n, Hp)), "logL": np.zeros(n), "gap": np.zeros(n),
           "rH": np.zeros(n)}
    A = np.zeros((D, H))
    B = np.zeros((D, H)) if model in O.MAX_MODELS else np.zeros((H, H))
    scal = np.zeros(5)
    for i in range(n):
        p = O.estep_point(model, Y[i], W, pi, sigma, Hp, gamma, tab=tab,
                          sel=None if sel is None else sel[i])
        c = p["sel"]
        out["sel"][i], out["flagged"][i] = c, p["flagged"]
        out["s_mean"][i], out["logL"][i] = p["s_mean"], p["logL"]
        r = p["scores"]
        order = np.lexsort((np.arange(H), -r))
        out["rH"][i] = r[order[Hp - 1]]
        out["gap"][i] = r[order[Hp - 1]] - r[order[Hp]] if Hp < H else np.inf
        if model in O.MAX_MODELS:
            A[:, c] += p["R"] * Y[i][:, None]
            B[:, c] += p["R"]
            scal[3] += p["res_mean"]
        else:
            A[:, c] += np.outer(Y[i], p["s_mean"])
            B[np.ix_(c, c)] += p["ss_mean"]
        scal[0] += p["k_mean"]
        scal[1] += p["logL"]
        scal[2] += float(Y[i] @ Y[i])
        scal[4] += 1
    return out, A, B, scal


def oracle_pool(model, Y, W, pi, sigma, Hp, gamma, sel=None, workers=None):
    """Oracle E-step over every row of Y: per-point outputs and the sums
    A, B, scal (as oracle.estep), with the selection gap per point."""
    workers = workers or n_workers()
    N = Y.shape[0]
    parts = np.array_split(np.arange(N), workers * 4)
    jobs = [(model, Y[ix], W, pi, sigma, Hp, gamma, None if sel is None else sel[ix])
            for ix in parts if len(ix)]
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers, initializer=_one_thread) as pool:
        res = pool.map(_chunk, jobs)
    out = {k: np.concatenate([r[0][k] for r in res]) for k in res[0][0]}
    out["A"] = sum(r[1] for r in res)
    out["B"] = sum(r[2] for r in res)
    out["scal"] = sum(r[3] for r in res)
    return out
