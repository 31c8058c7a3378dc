"""GPU tests of the on-the-fly switch blocks (BF_PATH_PER_STEP_MFMA with
switch_otf): the blocks generated during the apply from the FP64 phase
(Algorithm 4.1's switch step, eq. (eqn:RAB)) instead of read from storage.

Bars: against the oracle's butterfly of the same operator, relative l2
<= 1e-5 (the FP32 bar); against the stored-block apply of the same plan
<= 3e-6 (the generated entries differ from the stored FP32-rounded ones by
the error of an FP32 sincospi, ~1e-7 per entry); a plan built for the
on-the-fly form stores no switch blocks until a form that reads them is
selected."""

import json
import os

import numpy as np
import pytest

from _util import inputs, rel, log
from oracle.butterfly import butterfly_apply, butterfly_matvec
from synthetic import CONFIGS, PHASE_PARAMS, gaussian_vectors

pytestmark = pytest.mark.gpu

TOL = 1e-5
VS_STORED = 3e-6


def _bfm():
    import paper_1803_04128_amd as bfm
    return bfm


def _to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _host(t):
    return t.cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("dim,n,kind,q,op,amp", [
    (2, 64, "radon2d", 7, "N", False),
    (2, 128, "radon2d", 5, "H", False),
    (2, 32, "radon2d", 7, "T", True),
    (2, 32, "dft", 6, "N", False),
    (2, 64, "separable", 7, "N", False),
    (1, 4096, "fio1d", 10, "N", True),
    (1, 8192, "fio1d_warp", 12, "H", False),
    (1, 2048, "dft", 8, "T", False),
])
def test_otf_against_oracle_and_stored(dim, n, kind, q, op, amp):
    bfm = _bfm()
    log(f"case otf dim={dim} n={n} kind={kind} q={q} op={op} amp={amp}")
    nvec = 3
    f32, f, ab = inputs(dim, n, nvec, 3100 + q,
                        amp="sincos" if amp else "one", r=4 if amp else 1)
    t, c = op in ("T", "H"), op in ("C", "H")
    params = PHASE_PARAMS[kind]
    if ab is None:
        ref = butterfly_apply(dim, n, kind, params, q, f, transpose=t,
                              conjugate=c)
    else:
        ref = butterfly_matvec(dim, n, kind, params, q, ab[0], ab[1], f,
                               transpose=t, conjugate=c)
    with bfm.Plan(dim, n, kind, params, q=q, amplitude=ab, max_nvec=nvec,
                  op=op) as pl:
        ft = _to_dev(f32)
        pl.set_config("per_step_mfma")
        g_st = _host(pl.apply(ft))
        pl.set_config("per_step_mfma", switch_otf=True)
        assert pl.config()["switch_otf"]
        g = _host(pl.apply(ft))
    e_or, e_st = np.max(rel(g, ref)), np.max(rel(g, g_st))
    log(f"  vs oracle {e_or:.3e}  vs stored {e_st:.3e}")
    assert e_or < TOL
    assert e_st < VS_STORED


def test_otf_plan_stores_no_switch_blocks_until_needed(monkeypatch):
    bfm = _bfm()
    n, q = 64, 7
    f32, f, _ = inputs(2, n, 2, 3200)
    ref = butterfly_apply(2, n, "radon2d", PHASE_PARAMS["radon2d"], q, f)
    with bfm.Plan(2, n, "radon2d", PHASE_PARAMS["radon2d"], q=q,
                  max_nvec=2) as stored:
        full = stored.info()["factor_bytes"]
    monkeypatch.setenv("BF_SWITCH_OTF", "1")
    with bfm.Plan(2, n, "radon2d", PHASE_PARAMS["radon2d"], q=q,
                  max_nvec=2) as pl:
        c = pl.config()
        assert c["path"] == "per_step_mfma" and c["switch_otf"]
        lean = pl.info()["factor_bytes"]
        # the switch blocks: N pairs x q^4 complex64 entries
        assert full - lean >= n * n * q ** 4 * 8
        ft = _to_dev(f32)
        g0 = _host(pl.apply(ft))
        assert np.max(rel(g0, ref)) < TOL
        pl.set_config("per_step_mfma")            # stored: built now
        assert pl.info()["factor_bytes"] == full
        g1 = _host(pl.apply(ft))
        assert np.max(rel(g1, ref)) < TOL
        assert np.max(rel(g0, g1)) < VS_STORED
        with pytest.raises(bfm.BfError) as ei:
            pl.set_config("per_step", switch_otf=True)
        assert ei.value.code == bfm._lib.BF_EUNSUPPORTED
        with pytest.raises(bfm.BfError) as ei:
            pl.set_config("fused", switch_otf=True)
        assert ei.value.code == bfm._lib.BF_EUNSUPPORTED
        assert pl.config() == dict(path="per_step_mfma", tile_cols=0,
                                   tile_cols_used=0, switch_otf=False,
                                   max_pass_levels=0, twiddle_otf=False)


def test_otf_fused_env_is_ignored(monkeypatch):
    # the environment default applies to the per-step MFMA form only
    bfm = _bfm()
    monkeypatch.setenv("BF_SWITCH_OTF", "1")
    with bfm.Plan(1, 4096, "fio1d", PHASE_PARAMS["fio1d"], q=10) as pl:
        assert pl.config()["path"] == "fused"
        assert not pl.config()["switch_otf"]


def test_otf_autotune_candidate_and_graph():
    import torch
    bfm = _bfm()
    n, q, nvec = 64, 7, 2
    log("case otf autotune + graph")
    f32, f, _ = inputs(2, n, nvec, 3300)
    ref = butterfly_apply(2, n, "radon2d", PHASE_PARAMS["radon2d"], q, f)
    with bfm.Plan(2, n, "radon2d", PHASE_PARAMS["radon2d"], q=q,
                  max_nvec=nvec) as pl:
        ft = _to_dev(f32)
        res = pl.autotune(ft, reps=2)
        for e in res:
            log("  ", e)
        otf = [e for e in res if e["switch_otf"] and not e["twiddle_otf"]]
        assert len(otf) == 1 and otf[0]["ms"] > 0
        pl.set_config("per_step_mfma", switch_otf=True)
        eager = pl.apply(ft)
        assert np.max(rel(_host(eager), ref)) < TOL
        gout = torch.zeros_like(ft)
        gr = pl.graph(ft, gout)
        try:
            for _ in range(3):
                junk = torch.randn(1 << 18, device="cuda").sum()
                torch.cuda.synchronize()
                gr.launch()
                torch.cuda.synchronize()
                assert torch.equal(gout, eager)
                assert float(junk) == float(junk)
        finally:
            gr.close()


@pytest.mark.fullsize_oracle
@pytest.mark.timeout(1800)
def test_otf_at_full_size_2d():
    # the 2D Radon workload (n = 256, 16 vectors) at full size: every entry
    # of vectors 0 and 15 against the oracle's butterfly
    import _fullsize_oracle as fo
    bfm = _bfm()
    name = "radon2d_n256"
    w = CONFIGS[name]
    log(f"case otf full size {name}")
    f32 = gaussian_vectors(w.N, w.nvec, w.seed).astype(np.complex64)
    with bfm.Plan(w.dim, w.n, w.phase_kind, w.phase_params, q=w.q,
                  max_nvec=w.nvec) as pl:
        pl.set_config("per_step_mfma", switch_otf=True)
        g = pl.apply(_to_dev(f32))
        for v in fo.JOBS[name]:
            bf = fo.result(name, v, log)
            e = rel(_host(g[v]), bf)[0]
            log(f"  vector {v}: all {bf.size} entries vs oracle butterfly "
                f"{e:.3e}")
            assert e < TOL
