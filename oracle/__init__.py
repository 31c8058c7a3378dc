"""Oracle: plain, slow, FP64 CPU reference for g = K f.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU
library never calls it, and it shares no code with the GPU library (no
kernels, headers, helpers, tables or constants); both sides take their inputs
from ``synthetic`` only.

Contents (each function cites the passage of Yang, "A Unified Framework for
Oscillatory Integral Transforms: When to use NUFFT or Butterfly
Factorization?", arXiv:1803.04128, that it follows):

* ``kernel``    the grid, the phase functions, the amplitude, and the kernel
                entries K(x, xi) = alpha(x, xi) exp(2 pi i Phi(x, xi)).
* ``dense``     the exact matvec g = K f on chosen rows (dense, O(N) per row).
* ``butterfly`` the butterfly algorithm of Section 4 (Algorithm 4.1) taken
                step by step with the interpolative low-rank factors of
                Algorithm 2 (Section 2.1), in FP64, plus the amplitude split
                of eq. (eqn:tg).

Parity status: every function is pinned by ``tests/test_oracle_*.py`` (closed
forms, brute force, exactness cases, the paper's printed errors as an order of
magnitude).  The interpolation error of the butterfly on the non-separable
phases of the workloads is measured, not pinned: the paper prints no value for
those phases.
"""
