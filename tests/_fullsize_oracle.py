"""The oracle's FP64 butterfly of the full-size workloads, computed in
worker processes so that the GPU tests can compare every output entry.

Each job is one vector of one workload (its seeded batch, the complex64
values widened to complex128, with the amplitude factors as the GPU holds
them) through oracle.butterfly (Algorithm 4.1 step by step, eq. (eqn:tg)).
prefetch() starts every job when the session collects the full-size tests,
so the oracle runs while the other GPU tests use the device; result() waits
for one, reporting progress while it waits."""

import concurrent.futures as cf
import multiprocessing as mp
import time

# workload -> vectors compared over all N entries (vector 0 and the last)
JOBS = {
    "radon2d_n256": (0, 15),
    "fio1d_n262144_batched": (0, 63),
    "radon2d_n512": (0, 15),
    "fio1d_n1048576_sweep": (0, 255),
}

_pool = None
_futures = {}


def _butterfly(name, v):
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle.butterfly import butterfly_apply, butterfly_matvec
    from synthetic import CONFIGS, amplitude_factors, gaussian_vectors
    w = CONFIGS[name]
    f = gaussian_vectors(w.N, w.nvec, w.seed)[v:v + 1]
    f = f.astype(np.complex64).astype(np.complex128)
    with threadpool_limits(2):
        if w.amplitude == "one":
            g = butterfly_apply(w.dim, w.n, w.phase_kind, w.phase_params,
                                w.q, f)
        else:
            a, b = amplitude_factors(w.amplitude, w.dim, w.n, w.r,
                                     w.amp_seed)
            a = a.astype(np.complex64).astype(np.complex128)
            b = b.astype(np.complex64).astype(np.complex128)
            g = butterfly_matvec(w.dim, w.n, w.phase_kind, w.phase_params,
                                 w.q, a, b, f)
    return g[0]


def prefetch():
    """Start every job (idempotent)."""
    global _pool
    if _pool is not None:
        return
    _pool = cf.ProcessPoolExecutor(max_workers=8,
                                   mp_context=mp.get_context("spawn"))
    for name, vs in JOBS.items():
        for v in vs:
            _futures[(name, v)] = _pool.submit(_butterfly, name, v)


def result(name, v, log=print):
    """The oracle butterfly of vector v of workload name, complex128 [N]."""
    prefetch()
    fut = _futures[(name, v)]
    t0 = time.time()
    while True:
        try:
            return fut.result(timeout=20)
        except cf.TimeoutError:
            log(f"  waiting for the oracle butterfly of {name} vector {v} "
                f"({time.time() - t0:.0f} s)")


def shutdown():
    global _pool
    if _pool is not None:
        _pool.shutdown(wait=False, cancel_futures=True)
        _pool = None
        _futures.clear()
