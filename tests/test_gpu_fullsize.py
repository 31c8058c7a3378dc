"""GPU parity at the workloads' full sizes, in the launch configuration the
benchmark times (the plan built for the whole batch, its default execution
form, one apply of every vector).

For vector 0 and the last vector of each workload's seeded batch, every one
of the N output entries is compared with the oracle's step-by-step FP64
butterfly (the same factorization, computed over all N by worker processes
started at collection, tests/_fullsize_oracle.py):
  * relative l2 over all N entries, and max |GPU - oracle| / max |oracle|,
    each <= 1e-5 in FP32 (and the split precisions' bars below);
and at the workload's seeded sampled rows, with the exact FP64 matvec values
tests/golden/make_fullsize.py stored (oracle/ alone):
  * relative l2 <= eps_BF + the bar, eps_BF the oracle butterfly's own error
    at those rows, stated in the log.
Workloads: the batched 1D FIO (N = 2^18, r = 4, 64 vectors), the 2D Radon
FIO at n = 256 and n = 512 (16 vectors), the precision sweep (N = 2^20,
r = 4, 256 vectors); the split precisions at both 1D sizes and the 2D
Radon size (per-step MFMA kernels); the batched
plan built for a single vector (both passes in 512-thread workgroups)."""

import json
import os

import numpy as np
import pytest

import _fullsize_oracle as fo
from _util import rel, log
from synthetic import CONFIGS, gaussian_vectors, amplitude_factors

pytestmark = [pytest.mark.gpu, pytest.mark.fullsize_oracle,
              pytest.mark.timeout(1800)]

TOL = 1e-5
BARS = {"fp32": TOL, "bf16x3": 1e-4, "fp16x3": 1e-5}
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "fullsize_oracle.json")


def _golden():
    with open(GOLDEN) as fh:
        return json.load(fh)


def _unpack(pairs):
    a = np.asarray(pairs, np.float64)
    return a[:, 0] + 1j * a[:, 1]


def _gpu(name, precision, picks, nvec=None):
    """GPU results (complex128 [N]) of vectors `picks` of one apply of the
    first nvec vectors (default: the whole batch)."""
    import torch
    import paper_1803_04128_amd as bfm
    w = CONFIGS[name]
    nvec = nvec or w.nvec
    # the first nvec vectors of the workload's seeded batch
    f32 = gaussian_vectors(w.N, w.nvec, w.seed)[:nvec].astype(np.complex64)
    ab = None
    if w.amplitude != "one":
        ab = amplitude_factors(w.amplitude, w.dim, w.n, w.r, w.amp_seed)
        ab = tuple(x.astype(np.complex64).astype(np.complex128) for x in ab)
    with bfm.Plan(w.dim, w.n, w.phase_kind, w.phase_params, q=w.q,
                  amplitude=ab, precision=precision, max_nvec=nvec) as pl:
        f = torch.from_numpy(f32).to("cuda")
        del f32
        g = pl.apply(f)
        torch.cuda.synchronize()
        return {v: g[v].cpu().numpy().astype(np.complex128) for v in picks}


def _compare(name, precision, g, picks):
    bar = BARS[precision]
    ref = _golden()[name]
    rows = np.asarray(ref["rows"], np.int64)
    for v in picks:
        bf = fo.result(name, v, log)
        e2 = rel(g[v], bf)[0]
        einf = np.max(np.abs(g[v] - bf)) / np.max(np.abs(bf))
        dense = _unpack(ref["dense"][str(v)])
        eps = rel(bf[rows], dense)[0]
        ed = rel(g[v][rows], dense)[0]
        log(f"  {name} {precision} vector {v}: all {bf.size} entries rel l2 "
            f"{e2:.3e}, max {einf:.3e}; {rows.size} rows vs dense {ed:.3e} "
            f"(eps_BF {eps:.3e})")
        assert e2 < bar and einf < bar
        assert ed < eps + bar


@pytest.mark.parametrize("name", ["radon2d_n256", "fio1d_n262144_batched",
                                  "radon2d_n512", "fio1d_n1048576_sweep"])
def test_full_size_fp32_all_entries(name):
    picks = list(fo.JOBS[name])
    log(f"case full size {name} fp32, vectors {picks}")
    _compare(name, "fp32", _gpu(name, "fp32", picks), picks)


@pytest.mark.parametrize("name", ["fio1d_n262144_batched",
                                  "fio1d_n1048576_sweep", "radon2d_n256"])
@pytest.mark.parametrize("precision", ["bf16x3", "fp16x3"])
def test_split_precision_all_entries(name, precision):
    picks = list(fo.JOBS[name])
    log(f"case full size {name} {precision}, vectors {picks}")
    _compare(name, precision, _gpu(name, precision, picks), picks)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp16x3"])
def test_single_vector_at_full_size(precision):
    # the batched workload's plan built for one vector (four amplitude
    # columns): a narrower tile, both passes in 512-thread workgroups
    name = "fio1d_n262144_batched"
    log(f"case full size {name}, one vector, {precision}")
    _compare(name, precision, _gpu(name, precision, [0], nvec=1), [0])
