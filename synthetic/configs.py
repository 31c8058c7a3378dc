"""Workload table: shapes, phase parameters, seeds.  Numbers only.

Phase kinds (the formulas are implemented separately by the oracle and by the
HIP library; here they are only named and parameterised):

* ``dft``       Phi = x . xi
* ``fio1d``     Phi = x xi + c(x) |xi|, c(x) = (p0 + p1 sin 2 pi x) / p2
* ``fio1d_warp`` Phi = x xi + c(x) xi with the same c(x) (the composition
                example, eq. (eqn:FIOK2))
* ``radon2d``   Phi = x . xi + sqrt(c1(x)^2 xi1^2 + c2(x)^2 xi2^2),
                c1 = (p0 + p1 sin 2 pi x1 sin 2 pi x2) / p2,
                c2 = (p3 + p4 cos 2 pi x1 cos 2 pi x2) / p5
* ``separable`` Phi = p0 sin(2 pi x1) (1 + x2) + p1 |xi| + p2 |xi|^2 / n
                (x2 = 0 in 1D; |xi| is the Euclidean norm), an additively
                separable phase for which the butterfly factorization is exact.
"""

from dataclasses import dataclass, field
from typing import Tuple

PHASE_PARAMS = {
    "dft": (),
    # c(x) = (2 + sin 2 pi x) / 8
    "fio1d": (2.0, 1.0, 8.0),
    # the paper's 1D FIO experiment: c(x) = (2 + 0.2 sin 2 pi x) / 16
    "fio1d_paper": (2.0, 0.2, 16.0),
    "radon2d": (2.0, 1.0, 16.0, 2.0, 1.0, 16.0),
    # the composition example: Phi = x xi + c(x) xi,
    # c(x) = (2 + 0.2 sin 2 pi x) / 16
    "fio1d_warp": (2.0, 0.2, 16.0),
    "separable": (3.7, 0.37, 0.011),
}


@dataclass(frozen=True)
class Workload:
    name: str
    dim: int
    n: int                      # points per dimension; N = n ** dim
    phase: str                  # key of PHASE_PARAMS (kind is the prefix)
    amplitude: str              # "one" | "sincos"
    r: int                      # amplitude rank
    q: int                      # interpolation points per box per dimension
    nvec: int
    seed: int                   # seed of the input vectors
    rows: int                   # rows checked against the dense oracle
    row_seed: int
    amp_seed: int = 11
    note: str = ""
    extra: Tuple = field(default_factory=tuple)

    @property
    def N(self):
        return self.n ** self.dim

    @property
    def phase_kind(self):
        return "fio1d" if self.phase == "fio1d_paper" else self.phase

    @property
    def phase_params(self):
        return PHASE_PARAMS[self.phase]


CONFIGS = {
    # 1D FIO, plain method, one vector, all rows against the dense oracle.
    "fio1d_n1024": Workload("fio1d_n1024", 1, 1024, "fio1d", "one", 1, 8, 1,
                            seed=0, rows=1024, row_seed=100),
    # 1D FIO batched: N = 2^18, r = 4 amplitude, q = 10, 64 vectors.
    "fio1d_n262144_batched": Workload("fio1d_n262144_batched", 1, 1 << 18,
                                      "fio1d", "sincos", 4, 10, 64, seed=1,
                                      rows=512, row_seed=101),
    # 2D generalized Radon FIO: n = 256 (N = 65536), q = 7, 16 vectors.
    "radon2d_n256": Workload("radon2d_n256", 2, 256, "radon2d", "one", 1, 7,
                             16, seed=2, rows=1024, row_seed=102),
    # 2D generalized Radon FIO at n = 512 (N = 262144), the largest 2D grid
    # of the serving mix: a parity case (16 vectors).
    "radon2d_n512": Workload("radon2d_n512", 2, 512, "radon2d", "one", 1, 7,
                             16, seed=5, rows=1024, row_seed=105),
    # precision sweep: N = 2^20, r = 4, q = 10, 256 vectors.
    "fio1d_n1048576_sweep": Workload("fio1d_n1048576_sweep", 1, 1 << 20,
                                     "fio1d", "sincos", 4, 10, 256, seed=3,
                                     rows=1024, row_seed=103),
}


# Serving mix: plan shapes (dim, n, phase, amplitude, r, q) and their weights
# in the request stream.  1D FIO plans at every N = 2^12 ... 2^20 (odd and
# even depths) and 2D Radon plans at n = 64 ... 512, each with amplitude
# rank r = 1, 2 or 4; smaller transforms are requested more often (weight
# halving per doubling of N).
def _serving_shapes():
    shapes = []
    for k in range(12, 21):
        w = max(1, 2 ** (20 - k) // 16)
        for r in (1, 2, 4):
            shapes.append(((1, 1 << k, "fio1d", "one" if r == 1 else "sincos",
                            r, 8), w))
    for n in (64, 128, 256, 512):
        w = {64: 8, 128: 4, 256: 2, 512: 1}[n]
        for r in (1, 2, 4):
            shapes.append(((2, n, "radon2d", "one" if r == 1 else "sincos",
                            r, 7), w))
    return tuple(shapes)


SERVING_SHAPES = _serving_shapes()
# vectors per request: 1 ... 32, weights proportional to 1 / nvec
SERVING_NVEC = tuple(range(1, 33))
SERVING_NVEC_WEIGHTS = tuple(1.0 / v for v in SERVING_NVEC)


def serving_requests(count, seed, rate=None, shapes=SERVING_SHAPES):
    """Request stream: [(arrival_s, shape_index, nvec)], Poisson arrivals at
    ``rate`` requests/s (all at t = 0 when rate is None), shapes and vector
    counts drawn with the weights above (PCG64, ``seed``)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    w = np.array([s[1] for s in shapes], float)
    kinds = rng.choice(len(shapes), size=count, p=w / w.sum())
    wv = np.array(SERVING_NVEC_WEIGHTS, float)
    nv = rng.choice(SERVING_NVEC, size=count, p=wv / wv.sum())
    if rate is None:
        t = np.zeros(count)
    else:
        t = np.cumsum(rng.exponential(1.0 / rate, size=count))
    return [(float(t[i]), int(kinds[i]), int(nv[i])) for i in range(count)]
