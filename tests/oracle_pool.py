"""Per-tube oracle runs in worker processes (test infrastructure).

The batched workload has hundreds of small independent tubes; the oracle's
OpenMP loops gain little on one small tube, so the tests run one tube per
worker process, each with one thread.  Workers import only numpy, the
seeded workload generators and the oracle (no GPU library, no torch).
"""
import concurrent.futures as cf
import multiprocessing as mp
import os

import numpy as np


def _physical(U):
    rho = U[0]
    u = U[1] / rho
    th = (2.0 * U[2] - rho * u * u) / rho
    return bool(np.all(np.isfinite(U)) and np.all(rho > 0) and np.all(th > 0))


def run_tube(args):
    """(tube, steps) -> (U after `steps` steps or None, first failing step or 0).
    A step fails when the oracle raises (non-physical state met during the
    step) or when the moments it produces are non-physical."""
    tube, steps = args
    import workloads as W
    from oracle import Oracle, OracleError, set_threads
    set_threads(1)
    o = Oracle(1, (tube.nx,), tube.dx, tube.nv, tube.dv, bc=(1,), tau=tube.tau)
    r, uu, tt = W.sod_tube(tube.nx, left=tube.left, right=tube.right)
    o.init_macro(r, uu, tt)
    for n in range(1, steps + 1):
        try:
            o.step(1)
        except OracleError:
            return None, n
        U = o.U
        if not _physical(U):
            return None, n
    return U, 0


def run_tubes(tubes, steps, workers=None):
    workers = workers or min(16, os.cpu_count() or 1)
    env = dict(os.environ)
    os.environ["OMP_NUM_THREADS"] = "1"
    try:
        with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
            return list(ex.map(run_tube, [(t, steps) for t in tubes], chunksize=4))
    finally:
        os.environ.clear()
        os.environ.update(env)
