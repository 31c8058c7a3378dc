"""Write tests/golden/fullsize_oracle.json: oracle values at seeded sampled
rows of the full-size workloads, for the GPU tests of test_gpu_fullsize.py.

For each workload: the rows (sample_rows with the workload's row seed),
and for vector 0 and the last vector of its seeded input batch (the
complex64 values widened to complex128, as the GPU sees them):
  * "bf": the oracle's step-by-step FP64 butterfly (Algorithm 4.1 with
    eq. (eqn:tg)) at those rows — the same factorization the GPU applies;
  * "dense": the exact FP64 matvec at those rows (alpha from its formula).
Only oracle/ and synthetic/ are used.  Run from the repository root:
    python tests/golden/make_fullsize.py
(a few minutes on 8 cores; the N = 2^20 butterfly dominates).
"""

import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(
    os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.butterfly import butterfly_apply, butterfly_matvec  # noqa: E402
from oracle.dense import dense_rows  # noqa: E402
from synthetic import (CONFIGS, amplitude_factors, gaussian_vectors,  # noqa: E402
                       sample_rows)

# workload -> (rows, vectors whose butterfly is stored)
PLAN = {
    "fio1d_n262144_batched": (512, "both"),
    "radon2d_n256": (512, "both"),
    "fio1d_n1048576_sweep": (128, "first"),
}


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
    for name, (nrows, which) in PLAN.items():
        w = CONFIGS[name]
        picks = [0, w.nvec - 1]
        fs = vectors(w, picks)
        ab = None
        if w.amplitude != "one":
            ab = amplitude_factors(w.amplitude, w.dim, w.n, w.r, w.amp_seed)
            ab = tuple(x.astype(np.complex64).astype(np.complex128)
                       for x in ab)
        rows = sample_rows(w.N, nrows, w.row_seed)
        amp = "one" if ab is None else w.amplitude
        dense = dense_rows(w.dim, w.n, w.phase_kind, w.phase_params, amp,
                           fs, rows)
        entry = {"rows": rows.tolist(), "vectors": picks, "dense": {},
                 "bf": {}}
        for k, v in enumerate(picks):
            entry["dense"][str(v)] = pack(dense[k])
            if which == "first" and k > 0:
                continue
            if ab is None:
                bf = butterfly_apply(w.dim, w.n, w.phase_kind,
                                     w.phase_params, w.q, fs[k:k + 1])[0]
            else:
                bf = butterfly_matvec(w.dim, w.n, w.phase_kind,
                                      w.phase_params, w.q, ab[0], ab[1],
                                      fs[k:k + 1])[0]
            entry["bf"][str(v)] = pack(bf[rows])
            print(name, "vector", v, "done", flush=True)
        out[name] = entry
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                        "fullsize_oracle.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print("wrote", path)


if __name__ == "__main__":
    main()
