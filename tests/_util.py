"""Shared helpers of the GPU tests: seeded inputs for a workload, the HIP
apply through the C ABI binding, and the oracle references."""

import sys
import time

import numpy as np

from synthetic import gaussian_vectors, amplitude_factors


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def inputs(dim, n, nvec, seed, amp="one", r=1, amp_seed=11):
    """f as complex64 (what the GPU gets) and its exact complex128 copy
    (what the oracle gets), plus amplitude factors or None."""
    N = n ** dim
    f64 = gaussian_vectors(N, nvec, seed)
    f32 = f64.astype(np.complex64)
    ab = None
    if amp != "one":
        ab = amplitude_factors(amp, dim, n, r, amp_seed)
        # the GPU stores the factors in complex64; the oracle sees the same
        ab = tuple(x.astype(np.complex64).astype(np.complex128) for x in ab)
    return f32, f32.astype(np.complex128), ab


def gpu_apply(plan, f32, repeat=1):
    """Apply through the binding; returns (complex128 result, seconds)."""
    import torch
    ft = torch.from_numpy(np.ascontiguousarray(f32)).to("cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(repeat):
        g = plan.apply(ft)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / repeat
    return g.cpu().numpy().astype(np.complex128), dt


def rel(a, b):
    a = np.atleast_2d(a)
    b = np.atleast_2d(b)
    return np.sqrt(np.sum(np.abs(a - b) ** 2, -1) /
                   np.sum(np.abs(b) ** 2, -1))
