"""Write tests/golden/fullsize_oracle.json: exact FP64 matvec values at
seeded sampled rows of the full-size workloads, for test_gpu_fullsize.py.

For each workload: the rows (sample_rows with the workload's row count and
row seed) and, for vector 0 and the last vector of its seeded input batch
(the complex64 values widened to complex128, as the GPU sees them), the
exact FP64 matvec at those rows (dense_rows, alpha from its formula).  The
oracle butterfly of the same vectors is computed over all N entries by the
tests themselves.  Only oracle/ and synthetic/ are used.  Run from the
repository root:
    python tests/golden/make_fullsize.py
(a few minutes on 8 cores; the N = 2^20 rows dominate).
"""

import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(
    os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.dense import dense_rows  # noqa: E402
from synthetic import CONFIGS, gaussian_vectors, sample_rows  # noqa: E402

WORKLOADS = ("fio1d_n262144_batched", "radon2d_n256", "radon2d_n512",
             "fio1d_n1048576_sweep")


def vectors(w, picks):
    """Vectors `picks` of the workload's seeded batch, as the GPU sees them
    (complex64 widened to complex128)."""
    f = gaussian_vectors(w.N, w.nvec, w.seed)
    return np.stack([f[v].astype(np.complex64).astype(np.complex128)
                     for v in picks])


def pack(z):
    return [[float(c.real), float(c.imag)] for c in np.ravel(z)]


def main():
    out = {}
    for name in WORKLOADS:
        w = CONFIGS[name]
        picks = [0, w.nvec - 1]
        fs = vectors(w, picks)
        rows = sample_rows(w.N, w.rows, w.row_seed)
        dense = dense_rows(w.dim, w.n, w.phase_kind, w.phase_params,
                           w.amplitude, fs, rows)
        out[name] = {"rows": rows.tolist(), "vectors": picks,
                     "dense": {str(v): pack(dense[k])
                               for k, v in enumerate(picks)}}
        print(name, rows.size, "rows done", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                        "fullsize_oracle.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print("wrote", path)


if __name__ == "__main__":
    main()
