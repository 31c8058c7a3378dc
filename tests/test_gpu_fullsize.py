"""GPU parity at the workloads' full sizes, in the launch configuration the
benchmark times (the plan built for the whole batch, its default execution
form, one apply of every vector), checked on seeded sampled rows whose
oracle values `tests/golden/make_fullsize.py` computed with oracle/ alone:

* vector 0 (and the last vector where stored) against the oracle's
  step-by-step FP64 butterfly at those rows (the same factorization):
  relative l2 <= 1e-5 in FP32;
* vector 0 and the last vector against the dense FP64 matvec at those rows:
  relative l2 <= eps_BF + 1e-5, eps_BF the oracle butterfly's own error
  there (vector 0);
* the batched workload's plan built for a single vector, vector 0 against
  the same butterfly rows (FP32 <= 1e-5, BF16x3 <= 1e-4, FP16x3 <= 1e-5);
* the split precisions at the batched size and at the precision-sweep size
  (N = 2^20, 256 vectors) against the stored butterfly rows: BF16x3 <= 1e-4,
  FP16x3 <= 1e-5."""

import json
import os

import numpy as np
import pytest

from _util import rel, log
from synthetic import CONFIGS, gaussian_vectors, amplitude_factors

pytestmark = pytest.mark.gpu

TOL = 1e-5
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "fullsize_oracle.json")


def _golden():
    with open(GOLDEN) as fh:
        return json.load(fh)


def _unpack(pairs):
    a = np.asarray(pairs, np.float64)
    return a[:, 0] + 1j * a[:, 1]


def _gpu_rows(name, precision, rows, picks, nvec=None):
    import torch
    import paper_1803_04128_amd as bfm
    w = CONFIGS[name]
    nvec = nvec or w.nvec
    f32 = gaussian_vectors(w.N, w.nvec, w.seed).astype(np.complex64)[:nvec]
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
        idx = torch.as_tensor(rows, device="cuda")
        return {v: g[v][idx].cpu().numpy().astype(np.complex128)
                for v in picks}


@pytest.mark.parametrize("name", ["fio1d_n262144_batched", "radon2d_n256",
                                  "fio1d_n1048576_sweep"])
def test_full_size_against_oracle(name):
    ref = _golden()[name]
    rows = np.asarray(ref["rows"], np.int64)
    picks = ref["vectors"]
    log(f"case full size {name}, {rows.size} rows, vectors {picks}")
    g = _gpu_rows(name, "fp32", rows, picks)
    dense0 = _unpack(ref["dense"][str(picks[0])])
    eps = rel(_unpack(ref["bf"][str(picks[0])]), dense0)[0]
    log(f"  eps_BF (oracle butterfly vs dense, vector 0) = {eps:.3e}")
    for v in picks:
        if str(v) in ref["bf"]:
            e = rel(g[v], _unpack(ref["bf"][str(v)]))[0]
            log(f"  vector {v}: GPU vs oracle butterfly {e:.3e}")
            assert e < TOL
        e = rel(g[v], _unpack(ref["dense"][str(v)]))[0]
        log(f"  vector {v}: GPU vs dense {e:.3e}")
        assert e < eps + TOL


@pytest.mark.parametrize("precision,tol", [("bf16x3", 1e-4),
                                           ("fp16x3", 1e-5)])
def test_split_precision_at_batched_size(precision, tol):
    # the batched workload in the launch configuration the benchmark times
    # (head gathered into the state tile, two workgroups per CU)
    name = "fio1d_n262144_batched"
    ref = _golden()[name]
    rows = np.asarray(ref["rows"], np.int64)
    picks = ref["vectors"]
    log(f"case batched size {precision}, vectors {picks}")
    g = _gpu_rows(name, precision, rows, picks)
    for v in picks:
        if str(v) in ref["bf"]:
            e = rel(g[v], _unpack(ref["bf"][str(v)]))[0]
            log(f"  {precision} vector {v} vs oracle butterfly {e:.3e}")
            assert e < tol


@pytest.mark.parametrize("precision,tol", [("bf16x3", 1e-4),
                                           ("fp16x3", 1e-5)])
def test_split_precision_at_sweep_size(precision, tol):
    name = "fio1d_n1048576_sweep"
    ref = _golden()[name]
    rows = np.asarray(ref["rows"], np.int64)
    log(f"case sweep size {precision}")
    g = _gpu_rows(name, precision, rows, [0])
    e = rel(g[0], _unpack(ref["bf"]["0"]))[0]
    log(f"  {precision} vs oracle butterfly (vector 0) {e:.3e}")
    assert e < tol


@pytest.mark.parametrize("precision,tol", [("fp32", TOL), ("bf16x3", 1e-4),
                                           ("fp16x3", 1e-5)])
def test_single_vector_at_full_size(precision, tol):
    # the batched workload's plan built for one vector (four amplitude
    # columns): a narrower tile, and both passes in 512-thread workgroups
    name = "fio1d_n262144_batched"
    ref = _golden()[name]
    rows = np.asarray(ref["rows"], np.int64)
    log(f"case full size {name}, one vector, {precision}")
    g = _gpu_rows(name, precision, rows, [0], nvec=1)
    e = rel(g[0], _unpack(ref["bf"]["0"]))[0]
    log(f"  vector 0 alone: GPU vs oracle butterfly {e:.3e}")
    assert e < tol
