"""The Lasso definition (``oracle.lasso.solve``) and the method reference
(``oracle.screening.fast_l1``) over many signals in worker processes -- TEST
INFRASTRUCTURE.

Parity checks of a whole batch need one oracle solve per signal; these run in
spawned processes, each with a share of the host's BLAS threads.  The dictionary is sent once per
worker; each task is one signal.  Nothing here adds arithmetic: every result is
exactly what the serial call returns.
"""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np

_SHARED = {}


def _init(shared):
    _SHARED.clear()
    _SHARED.update(shared)


def _solve_one(task):
    from . import lasso
    b, y, lam = task
    r = lasso.solve(_SHARED["A"], y, lam, L=_SHARED["L"], tol=_SHARED["tol"])
    return b, r["x"], r["P"], r["kkt"], r["margin"]


def _method_one(task):
    from . import screening
    b, y, lam, kw = task
    r = screening.fast_l1(_SHARED["stages"], _SHARED["atom_norm"], y, lam, _SHARED["rc"], **kw)
    return b, r


def _pool(shared, workers, threads=1):
    # BLAS threads per worker: the environment is read when numpy loads in the child
    keys = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
    saved = {k: os.environ.get(k) for k in keys}
    for k in keys:
        os.environ[k] = str(max(1, int(threads)))
    try:
        return mp.get_context("spawn").Pool(workers, initializer=_init, initargs=(shared,))
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def default_workers():
    """Workers and BLAS threads per worker: four workers sharing the host's cores (at
    most 16), which keeps each worker's products multi-threaded."""
    cores = max(1, min(16, os.cpu_count() or 1))
    w = min(4, cores)
    return w, max(1, cores // w)


def solve_batch(A, Y, lam, L, indices=None, tol=1e-13, workers=None, threads=None, progress=None):
    """{b: (x*, P*, kkt residual, complementarity margin)} of oracle.lasso.solve for
    the signals Y[b], lam[b], b in indices (default: all).  progress(done, total) is
    called as results arrive."""
    idx = range(len(Y)) if indices is None else indices
    tasks = [(int(b), np.asarray(Y[b], dtype=np.float64), float(lam[b])) for b in idx]
    shared = dict(A=np.asarray(A, dtype=np.float64), L=float(L), tol=float(tol))
    res = {}
    dw, dt = default_workers()
    with _pool(shared, workers or dw, threads or dt) as pool:
        for b, x, P, kkt, m in pool.imap_unordered(_solve_one, tasks, chunksize=1):
            res[b] = (x, P, kkt, m)
            if progress is not None:
                progress(len(res), len(tasks))
    return res


def method_batch(stages, atom_norm, Y, lam, rc, indices=None, workers=None, threads=None, **kw):
    """{b: Result} of oracle.screening.fast_l1 for the signals b in indices."""
    idx = range(len(Y)) if indices is None else indices
    tasks = [(int(b), np.asarray(Y[b], dtype=np.float64), float(lam[b]), kw) for b in idx]
    shared = dict(stages=stages, atom_norm=np.asarray(atom_norm), rc=list(rc))
    dw, dt = default_workers()
    with _pool(shared, workers or dw, threads or dt) as pool:
        out = pool.map(_method_one, tasks, chunksize=1)
    return dict(out)
