"""GPU parity for phases given as low-rank factors (BF_PHASE_LOWRANK, the
input form of Algorithm 2): against the oracle's dense rows where the
butterfly is exact and its butterfly of the same phase otherwise (relative
l2 <= 1e-5), through every execution form, the transposed operators and the
on-the-fly switch; and the exact factors of the FIO phase of Section 5
against the built-in FIO plan at the benchmark size."""

import numpy as np
import pytest

from _util import inputs, gpu_apply, rel, log
from oracle.butterfly import butterfly_apply, butterfly_matvec
from oracle.dense import dense_rows
from synthetic import gaussian_vectors, lowrank_phase, orthogonal_mix, \
    PHASE_PARAMS

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(autouse=True, params=["fused", "per_step", "per_step_mfma"])
def apply_path(request, monkeypatch):
    monkeypatch.setenv("BF_FUSED", "1" if request.param == "fused" else "0")
    monkeypatch.setenv("BF_MFMA", "0" if request.param == "per_step" else "1")
    return request.param


def _plan(dim, n, UV, q, op="N", ab=None, nvec=1):
    import paper_1803_04128_amd as bfm
    return bfm.Plan(dim, n, "lowrank", UV, q=q, amplitude=ab, max_nvec=nvec,
                    op=op)


@pytest.mark.parametrize("op", ["N", "H"])
@pytest.mark.parametrize("dim,n,q", [(1, 64, 8), (2, 16, 7)])
def test_exact_small(dim, n, q, op):
    log(f"case lowrank exact dim={dim} n={n} op={op}")
    UV = lowrank_phase(dim, n, dim + 2, 4000 + n)
    N = n ** dim
    f32, f, _ = inputs(dim, n, 2, 4001)
    with _plan(dim, n, UV, q, op, nvec=2) as pl:
        g, _ = gpu_apply(pl, f32)
    ref = dense_rows(dim, n, "lowrank", UV, "one", f, np.arange(N),
                     transpose=op == "H", conjugate=op == "H")
    assert np.max(rel(g, ref)) < TOL


@pytest.mark.parametrize("op", ["N", "T"])
@pytest.mark.parametrize("dim,n,q,rank", [(1, 4096, 10, 4),
                                          (1, 1 << 14, 8, 6),
                                          (2, 64, 7, 5), (2, 128, 5, 3)])
def test_parity_vs_oracle_butterfly(dim, n, q, rank, op):
    log(f"case lowrank parity dim={dim} n={n} q={q} rank={rank} op={op}")
    UV = lowrank_phase(dim, n, rank, 4100 + rank)
    f32, f, _ = inputs(dim, n, 2, 4101)
    with _plan(dim, n, UV, q, op, nvec=2) as pl:
        g, _ = gpu_apply(pl, f32)
    ref = butterfly_apply(dim, n, "lowrank", UV, q, f, transpose=op == "T")
    assert np.max(rel(g, ref)) < TOL


@pytest.mark.parametrize("dim,n,q", [(1, 2048, 8), (2, 32, 7)])
def test_parity_with_amplitude(dim, n, q):
    log(f"case lowrank amplitude dim={dim} n={n}")
    UV = lowrank_phase(dim, n, dim + 2, 4200)
    f32, f, ab = inputs(dim, n, 2, 4201, amp="sincos", r=2)
    with _plan(dim, n, UV, q, ab=ab, nvec=2) as pl:
        g, _ = gpu_apply(pl, f32)
    ref = butterfly_matvec(dim, n, "lowrank", UV, q, ab[0], ab[1], f)
    assert np.max(rel(g, ref)) < TOL


def test_on_the_fly_switch(apply_path):
    if apply_path != "per_step_mfma":
        pytest.skip("the on-the-fly switch exists in the per-step MFMA form")
    dim, n, q = 2, 64, 7
    log("case lowrank otf")
    UV = lowrank_phase(dim, n, 5, 4300)
    f32, f, _ = inputs(dim, n, 2, 4301)
    with _plan(dim, n, UV, q, nvec=2) as pl:
        pl.set_config("per_step_mfma", switch_otf=True)
        g, _ = gpu_apply(pl, f32)
    ref = butterfly_apply(dim, n, "lowrank", UV, q, f)
    assert np.max(rel(g, ref)) < TOL


def test_fio_factors_match_builtin_fio_at_size(apply_path):
    # the same phase given two ways at N = 2^18, q = 10
    import paper_1803_04128_amd as bfm
    n, q = 1 << 18, 10
    log(f"case lowrank vs builtin fio n={n}")
    p0, p1, p2 = PHASE_PARAMS["fio1d"]
    i = np.arange(n)
    x, xi = i / n, (i - n // 2).astype(np.float64)
    U = np.stack([x, (p0 + p1 * np.sin(2 * np.pi * x)) / p2,
                  np.zeros(n)], 1) @ orthogonal_mix(3, 4400)
    V = np.stack([xi, np.abs(xi), np.zeros(n)], 1) @ orthogonal_mix(3, 4400)
    f32 = gaussian_vectors(n, 2, 4401).astype(np.complex64)
    with _plan(1, n, (U, V), q, nvec=2) as pl:
        g, _ = gpu_apply(pl, f32)
    with bfm.Plan(1, n, "fio1d", PHASE_PARAMS["fio1d"], q=q,
                  max_nvec=2) as pl:
        ref, _ = gpu_apply(pl, f32)
    e = np.max(rel(g, ref))
    log(f"  lowrank vs builtin {e:.3e}")
    assert e < 1e-6
