"""GPU tests of the twiddles evaluated during the apply
(BF_PATH_PER_STEP_MFMA with twiddle_otf): every twiddle entry a per-step
kernel would read from storage is evaluated where it is read, by the device
function that writes the stored array (the entry's FP64 phase terms,
reduced modulo 1, FP64 sincospi, rounded to complex64).

Bars: the apply equals the stored-twiddle apply of the same plan bit for
bit (the same entries meet the same arithmetic); with the switch blocks
generated too, no precomputed factor is read (Algorithm 4.1 as Section 4
states it, without precomputation) and the result is held to the oracle's
butterfly at the FP32 bar 1e-5, and to the stored apply at 3e-6 (the
generated switch entries use an FP32 sincospi).  A plan built with
BF_TWIDDLE_OTF=1 stores no twiddles and refuses the forms that read them."""

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


def _reference(dim, n, kind, q, f, ab, op):
    t, c = op in ("T", "H"), op in ("C", "H")
    params = PHASE_PARAMS[kind]
    if ab is None:
        return butterfly_apply(dim, n, kind, params, q, f, transpose=t,
                               conjugate=c)
    return butterfly_matvec(dim, n, kind, params, q, ab[0], ab[1], f,
                            transpose=t, conjugate=c)


# 2D: the head level as the last xi level (n = 64: the fused xi + switch
# launch reads f), separable levels at 7 and 8 points per dimension, every
# op; 1D: the per-step MFMA kernels with amplitude terms, even and odd depth
@pytest.mark.parametrize("dim,n,kind,q,op,amp", [
    (2, 64, "radon2d", 7, "N", False),
    (2, 256, "radon2d", 7, "H", False),
    (2, 32, "radon2d", 7, "T", True),
    (2, 64, "separable", 8, "N", False),
    (2, 32, "dft", 6, "C", False),
    (1, 4096, "fio1d", 10, "N", True),
    (1, 8192, "fio1d_warp", 12, "H", False),
    (1, 2048, "dft", 8, "T", False),
])
def test_generated_twiddles_equal_stored(dim, n, kind, q, op, amp):
    bfm = _bfm()
    log(f"case twiddle-otf dim={dim} n={n} kind={kind} q={q} op={op} "
        f"amp={amp}")
    nvec = 3
    f32, f, ab = inputs(dim, n, nvec, 3400 + q,
                        amp="sincos" if amp else "one", r=4 if amp else 1)
    ref = _reference(dim, n, kind, q, f, ab, op)
    with bfm.Plan(dim, n, kind, PHASE_PARAMS[kind], q=q, amplitude=ab,
                  max_nvec=nvec, op=op) as pl:
        ft = _to_dev(f32)
        pl.set_config("per_step_mfma")
        g_st = _host(pl.apply(ft))
        pl.set_config("per_step_mfma", twiddle_otf=True)
        assert pl.config()["twiddle_otf"]
        g_tw = _host(pl.apply(ft))
        pl.set_config("per_step_mfma", switch_otf=True, twiddle_otf=True)
        g_all = _host(pl.apply(ft))
    e_or = np.max(rel(g_all, ref))
    e_st = np.max(rel(g_all, g_st))
    log(f"  twiddles generated == stored: {np.array_equal(g_tw, g_st)}; "
        f"all factors generated vs oracle {e_or:.3e}, vs stored {e_st:.3e}")
    assert np.array_equal(g_tw, g_st)
    assert e_or < TOL
    assert e_st < VS_STORED


def test_plan_without_stored_factors(monkeypatch):
    bfm = _bfm()
    n, q, nvec = 64, 7, 2
    kind = "radon2d"
    log("case plan built with BF_TWIDDLE_OTF and BF_SWITCH_OTF")
    f32, f, _ = inputs(2, n, nvec, 3500)
    ref = butterfly_apply(2, n, kind, PHASE_PARAMS[kind], q, f)
    with bfm.Plan(2, n, kind, PHASE_PARAMS[kind], q=q,
                  max_nvec=nvec) as stored:
        stored.set_config("per_step_mfma")
        full = stored.info()["factor_bytes"]
        tw_bytes = 8 * sum(s["tw_entries"] for s in stored.steps())
        g_st = _host(stored.apply(_to_dev(f32)))
    assert tw_bytes > 0
    monkeypatch.setenv("BF_FUSED", "0")
    monkeypatch.setenv("BF_TWIDDLE_OTF", "1")
    monkeypatch.setenv("BF_SWITCH_OTF", "1")
    with bfm.Plan(2, n, kind, PHASE_PARAMS[kind], q=q,
                  max_nvec=nvec) as pl:
        c = pl.config()
        assert c["path"] == "per_step_mfma"
        assert c["twiddle_otf"] and c["switch_otf"]
        assert all(s["tw_entries"] == 0 and s["S_entries"] == 0
                   for s in pl.steps())
        lean = pl.info()["factor_bytes"]
        # no twiddles and no switch blocks in storage
        assert full - lean >= tw_bytes + n * n * q ** 4 * 8
        ft = _to_dev(f32)
        g = _host(pl.apply(ft))
        e_or, e_st = np.max(rel(g, ref)), np.max(rel(g, g_st))
        log(f"  vs oracle {e_or:.3e}, vs stored {e_st:.3e}; factor bytes "
            f"{lean} against {full}")
        assert e_or < TOL and e_st < VS_STORED
        # the twiddles are generated with the stored switch blocks as well
        pl.set_config("per_step_mfma", twiddle_otf=True)
        g1 = _host(pl.apply(ft))
        assert np.array_equal(g1, g_st)
        for path, kw in (("fused", {}), ("per_step", {}),
                         ("per_step_mfma", {}),
                         ("per_step_mfma", dict(switch_otf=True))):
            with pytest.raises(bfm.BfError) as ei:
                pl.set_config(path, **kw)
            assert ei.value.code == bfm._lib.BF_EUNSUPPORTED
        assert pl.config()["twiddle_otf"]
        with pytest.raises(bfm.BfError):
            pl.factor_entries(0, "twiddle", [0])
        # the autotuner times the forms that can run the plan
        res = pl.autotune(ft, reps=2)
        for e in res:
            log("  ", e)
        timed = [e for e in res if e["ms"] > 0]
        assert timed and all(e["twiddle_otf"] for e in timed)
        assert pl.config()["twiddle_otf"]
        assert np.max(rel(_host(pl.apply(ft)), ref)) < TOL


def test_twiddle_otf_refused_off_per_step_mfma(monkeypatch):
    bfm = _bfm()
    with bfm.Plan(1, 4096, "fio1d", PHASE_PARAMS["fio1d"], q=10) as pl:
        for path in ("fused", "fused_valu", "per_step"):
            with pytest.raises(bfm.BfError) as ei:
                pl.set_config(path, twiddle_otf=True)
            assert ei.value.code == bfm._lib.BF_EUNSUPPORTED
        assert not pl.config()["twiddle_otf"]
    with bfm.Plan(2, 32, "radon2d", PHASE_PARAMS["radon2d"], q=7,
                  precision="bf16x3") as pl:
        with pytest.raises(bfm.BfError) as ei:
            pl.set_config("per_step_mfma", twiddle_otf=True)
        assert ei.value.code == bfm._lib.BF_EUNSUPPORTED
    # the environment default applies to the FP32 per-step MFMA form only
    monkeypatch.setenv("BF_TWIDDLE_OTF", "1")
    with bfm.Plan(1, 4096, "fio1d", PHASE_PARAMS["fio1d"], q=10) as pl:
        assert pl.config()["path"] == "fused"
        assert not pl.config()["twiddle_otf"]
        assert all(s["tw_entries"] > 0 for s in pl.steps()
                   if s["kind"] != 1)


@pytest.mark.fullsize_oracle
@pytest.mark.timeout(1800)
def test_all_factors_generated_at_full_size_2d(monkeypatch):
    # the 2D Radon workload (n = 256, 16 vectors) built without stored
    # factors: every entry of vectors 0 and 15 against the oracle's butterfly
    import _fullsize_oracle as fo
    bfm = _bfm()
    name = "radon2d_n256"
    w = CONFIGS[name]
    log(f"case all factors generated, full size {name}")
    monkeypatch.setenv("BF_FUSED", "0")
    monkeypatch.setenv("BF_TWIDDLE_OTF", "1")
    monkeypatch.setenv("BF_SWITCH_OTF", "1")
    f32 = gaussian_vectors(w.N, w.nvec, w.seed).astype(np.complex64)
    with bfm.Plan(w.dim, w.n, w.phase_kind, w.phase_params, q=w.q,
                  max_nvec=w.nvec) as pl:
        assert pl.config()["twiddle_otf"] and pl.config()["switch_otf"]
        g = pl.apply(_to_dev(f32))
        for v in fo.JOBS[name]:
            bf = fo.result(name, v, log)
            e = rel(_host(g[v]), bf)[0]
            log(f"  vector {v}: all {bf.size} entries vs oracle butterfly "
                f"{e:.3e}")
            assert e < TOL
