"""GPU parity: the HIP apply (through the C ABI) against the FP64 oracle.

Bars (FP32 apply): relative l2 <= 1e-5 per vector against the oracle's
step-by-step butterfly on the same points (the same factorization), and
<= eps_BF + 1e-5 against the dense matvec, eps_BF being the oracle
butterfly's own error on the same rows.  Exact cases (small grids, separable
phases) must match the dense matvec to <= 1e-5.
"""

import numpy as np
import pytest

from _util import inputs, gpu_apply, rel, log
from oracle.butterfly import butterfly_apply, butterfly_matvec
from oracle.dense import dense_rows
from synthetic import sample_rows, PHASE_PARAMS, CONFIGS

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(autouse=True, params=["fused", "per_step", "per_step_mfma"])
def apply_path(request, monkeypatch):
    """Run every parity case through the level-fused passes, the
    one-launch-per-level vector-ALU kernels and the one-launch-per-level MFMA
    kernels (BF_FUSED and BF_MFMA are read when a plan is built)."""
    monkeypatch.setenv("BF_FUSED", "1" if request.param == "fused" else "0")
    monkeypatch.setenv("BF_MFMA", "0" if request.param == "per_step" else "1")
    return request.param


def _plan(dim, n, kind, q, ab=None, nvec=1, precision="fp32", phase=None):
    import paper_1803_04128_amd as bfm
    params = PHASE_PARAMS[phase or kind]
    return bfm.Plan(dim, n, kind, params, q=q, amplitude=ab,
                    precision=precision, max_nvec=nvec)


@pytest.mark.parametrize("n", [2, 4, 8, 16, 32, 64])
@pytest.mark.parametrize("kind", ["fio1d", "dft", "separable"])
def test_exact_small_1d(n, kind):
    log(f"case exact_small_1d n={n} kind={kind}")
    f32, f, _ = inputs(1, n, 3, 100 + n)
    with _plan(1, n, kind, 8, nvec=3) as pl:
        g, _ = gpu_apply(pl, f32)
    ref = dense_rows(1, n, kind, PHASE_PARAMS[kind], "one", f, np.arange(n))
    assert np.max(rel(g, ref)) < TOL


@pytest.mark.parametrize("n", [2, 4, 8, 16])
@pytest.mark.parametrize("kind", ["radon2d", "dft"])
def test_exact_small_2d(n, kind):
    log(f"case exact_small_2d n={n} kind={kind}")
    f32, f, _ = inputs(2, n, 2, 200 + n)
    with _plan(2, n, kind, 7, nvec=2) as pl:
        g, _ = gpu_apply(pl, f32)
    ref = dense_rows(2, n, kind, PHASE_PARAMS[kind], "one", f,
                     np.arange(n * n))
    assert np.max(rel(g, ref)) < TOL


@pytest.mark.parametrize("n,q", [(1024, 6), (1024, 8), (2048, 8), (4096, 10),
                                 (8192, 12), (512, 16), (16384, 8)])
@pytest.mark.parametrize("kind", ["fio1d", "dft"])
def test_parity_vs_oracle_butterfly_1d(n, q, kind):
    log(f"case parity_1d n={n} q={q} kind={kind}")
    f32, f, _ = inputs(1, n, 2, 300 + q)
    with _plan(1, n, kind, q, nvec=2) as pl:
        g, _ = gpu_apply(pl, f32)
    ref = butterfly_apply(1, n, kind, PHASE_PARAMS[kind], q, f)
    assert np.max(rel(g, ref)) < TOL


@pytest.mark.parametrize("n,q,r", [(1024, 8, 2), (4096, 10, 4), (2048, 6, 3)])
def test_parity_amplitude_1d(n, q, r):
    log(f"case parity_amp_1d n={n} q={q} r={r}")
    f32, f, ab = inputs(1, n, 3, 400 + r, amp="sincos", r=r)
    with _plan(1, n, "fio1d", q, ab=ab, nvec=3) as pl:
        g, _ = gpu_apply(pl, f32)
    ref = butterfly_matvec(1, n, "fio1d", PHASE_PARAMS["fio1d"], q, ab[0],
                           ab[1], f)
    assert np.max(rel(g, ref)) < TOL


@pytest.mark.parametrize("n,q", [(32, 7), (64, 7), (128, 5), (64, 4),
                                 (128, 7)])
def test_parity_vs_oracle_butterfly_2d(n, q):
    log(f"case parity_2d n={n} q={q}")
    f32, f, _ = inputs(2, n, 2, 500 + n)
    with _plan(2, n, "radon2d", q, nvec=2) as pl:
        g, _ = gpu_apply(pl, f32)
    ref = butterfly_apply(2, n, "radon2d", PHASE_PARAMS["radon2d"], q, f)
    assert np.max(rel(g, ref)) < TOL


def test_parity_amplitude_2d():
    log("case parity_amp_2d")
    n, q = 64, 7
    f32, f, ab = inputs(2, n, 2, 600, amp="sincos", r=2)
    with _plan(2, n, "radon2d", q, ab=ab, nvec=2) as pl:
        g, _ = gpu_apply(pl, f32)
    ref = butterfly_matvec(2, n, "radon2d", PHASE_PARAMS["radon2d"], q,
                           ab[0], ab[1], f)
    assert np.max(rel(g, ref)) < TOL


@pytest.mark.parametrize("dim,n,q", [(1, 1 << 18, 10), (1, 1 << 20, 8),
                                     (2, 256, 7), (2, 512, 7)])
def test_separable_phase_exact_at_full_size(dim, n, q):
    # exact factorization at any size: compare with the dense matvec on
    # sampled rows (every level's twiddles and index math at full size)
    log(f"case separable_full dim={dim} n={n} q={q}")
    N = n ** dim
    f32, f, _ = inputs(dim, n, 2, 700 + dim)
    with _plan(dim, n, "separable", q, nvec=2) as pl:
        g, _ = gpu_apply(pl, f32)
    rows = sample_rows(N, 256, 701)
    ref = dense_rows(dim, n, "separable", PHASE_PARAMS["separable"], "one", f,
                     rows)
    assert np.max(rel(g[:, rows], ref)) < TOL


@pytest.mark.parametrize("dim,n,q", [(1, 1 << 22, 8), (2, 1 << 11, 4)])
def test_separable_phase_exact_at_maximum_size(dim, n, q):
    # the largest grids bf_plan accepts (1D N = 2^22, 2D 2048 x 2048 = 2^22
    # points): the factorization is exact for a separable phase, so sampled
    # dense rows bound the FP32 apply at the maximum depth of the trees
    log(f"case separable_max dim={dim} n={n} q={q}")
    N = n ** dim
    f32, f, _ = inputs(dim, n, 2, 710 + dim)
    with _plan(dim, n, "separable", q, nvec=2) as pl:
        g, _ = gpu_apply(pl, f32)
    rows = sample_rows(N, 64, 711)
    ref = dense_rows(dim, n, "separable", PHASE_PARAMS["separable"], "one", f,
                     rows)
    err = np.max(rel(g[:, rows], ref))
    log(f"  rel err {err:.3e}")
    assert err < TOL


def test_dft_against_fft_full_size():
    n, q = 1 << 16, 10
    log(f"case dft_fft n={n} q={q}")
    f32, f, _ = inputs(1, n, 1, 800)
    with _plan(1, n, "dft", q) as pl:
        g, _ = gpu_apply(pl, f32)
    ref = ((-1.0) ** np.arange(n)) * n * np.fft.ifft(f, axis=-1)
    rows = sample_rows(n, 256, 801)
    e_bf = rel(butterfly_apply(1, 4096, "dft", (), q, f[:, :4096]),
               ((-1.0) ** np.arange(4096)) * 4096 *
               np.fft.ifft(f[:, :4096], axis=-1))[0]
    assert rel(g, ref)[0] < max(10 * e_bf, 1e-6) + TOL


def test_config_fio1d_n1024():
    w = CONFIGS["fio1d_n1024"]
    log(f"case config {w.name}")
    f32, f, _ = inputs(w.dim, w.n, w.nvec, w.seed)
    with _plan(w.dim, w.n, w.phase_kind, w.q, nvec=w.nvec,
               phase=w.phase) as pl:
        g, _ = gpu_apply(pl, f32)
    rows = np.arange(w.N)
    dense = dense_rows(w.dim, w.n, w.phase_kind, w.phase_params, "one", f,
                       rows)
    bf = butterfly_apply(w.dim, w.n, w.phase_kind, w.phase_params, w.q, f)
    eps_bf = np.max(rel(bf, dense))
    log(f"  eps_BF={eps_bf:.3e} gpu-vs-bf={np.max(rel(g, bf)):.3e} "
        f"gpu-vs-dense={np.max(rel(g, dense)):.3e}")
    assert np.max(rel(g, bf)) < TOL
    assert np.max(rel(g, dense)) < eps_bf + TOL


def test_batch_invariance_and_chunking(monkeypatch):
    # each column of a batched apply equals the vector applied alone (same
    # kernels, so bitwise), and a workspace cap that forces ragged vector
    # chunks changes nothing
    import paper_1803_04128_amd as bfm
    n, q, nvec = 4096, 10, 7
    log("case batch_invariance")
    f32, f, ab = inputs(1, n, nvec, 900, amp="sincos", r=4)
    with _plan(1, n, "fio1d", q, ab=ab, nvec=nvec) as pl:
        g_all, _ = gpu_apply(pl, f32)
        singles = [gpu_apply(pl, f32[v:v + 1])[0] for v in range(nvec)]
    for v in range(nvec):
        assert np.array_equal(g_all[v], singles[v][0])
    per_vec = 2 * n * 10 * 4 * 8 + 64
    monkeypatch.setenv("BF_WS_CAP_BYTES", str(3 * per_vec))
    with _plan(1, n, "fio1d", q, ab=ab, nvec=nvec) as pl:
        assert pl.info()["chunk_nvec"] == 3
        g_chunk, _ = gpu_apply(pl, f32)
    assert np.array_equal(g_all, g_chunk)


def test_apply_rejects_overlap_and_bad_nvec():
    import torch
    import paper_1803_04128_amd as bfm
    log("case apply_errors")
    with _plan(1, 1024, "fio1d", 8, nvec=2) as pl:
        f = torch.zeros((2, 1024), dtype=torch.complex64, device="cuda")
        with pytest.raises(bfm.BfError) as e:
            pl.apply(f, out=f)
        assert e.value.code == -1
        with pytest.raises(bfm.BfError):
            pl.apply(torch.zeros((3, 1024), dtype=torch.complex64,
                                 device="cuda"))


# split precisions: hi + lo parts represent each operand to 2^-18 (bfloat16)
# or 2^-22 (half) relative; over the ~13 contraction steps of these plans the
# errors add to a few 1e-5 (BF16) or 1e-6 (FP16).  The bars are stated
# against the FP64 oracle butterfly on the same points.
SPLIT_TOL = {"bf16x3": 1e-4, "fp16x3": 1e-5}


@pytest.mark.parametrize("precision", ["bf16x3", "fp16x3"])
@pytest.mark.parametrize("n,q,r,nvec", [(4096, 10, 4, 3), (1 << 14, 8, 1, 2),
                                        (1 << 13, 10, 2, 5), (1 << 13, 7, 1, 3),
                                        (1 << 12, 13, 2, 2)])
def test_split_precision_accuracy(apply_path, precision, n, q, r, nvec):
    if apply_path != "fused":
        pytest.skip("split precisions run on the fused MFMA passes only")
    log(f"case split {precision} n={n} q={q} r={r} nvec={nvec}")
    amp = "sincos" if r > 1 else "one"
    f32, f, ab = inputs(1, n, nvec, 950 + r, amp=amp, r=r)
    with _plan(1, n, "fio1d", q, ab=ab, nvec=nvec, precision=precision) as pl:
        g, _ = gpu_apply(pl, f32)
    if ab is None:
        ref = butterfly_apply(1, n, "fio1d", PHASE_PARAMS["fio1d"], q, f)
    else:
        ref = butterfly_matvec(1, n, "fio1d", PHASE_PARAMS["fio1d"], q, ab[0],
                               ab[1], f)
    err = np.max(rel(g, ref))
    log(f"  {precision} rel err vs FP64 butterfly = {err:.3e}")
    assert err < SPLIT_TOL[precision]


@pytest.mark.parametrize("precision", ["bf16x3", "fp16x3"])
@pytest.mark.parametrize("scale", [1e6, 1e-6])
def test_split_precision_any_input_scale(apply_path, precision, scale):
    # half parts have a narrow range: the panel columns are scaled by powers
    # of two inside the products, so the relative error does not depend on
    # the magnitude of f (1e6 * |f| overflows half without the scaling)
    if apply_path != "fused":
        pytest.skip("split precisions run on the fused MFMA passes only")
    n, q = 4096, 10
    log(f"case split scale {precision} {scale:g}")
    f32, f, _ = inputs(1, n, 2, 960)
    f32 = (f32 * np.float32(scale)).astype(np.complex64)
    with _plan(1, n, "fio1d", q, nvec=2, precision=precision) as pl:
        g, _ = gpu_apply(pl, f32)
    ref = butterfly_apply(1, n, "fio1d", PHASE_PARAMS["fio1d"], q,
                          f32.astype(np.complex128))
    assert np.all(np.isfinite(g))
    err = np.max(rel(g, ref))
    log(f"  rel err {err:.3e}")
    assert err < SPLIT_TOL[precision]


@pytest.mark.parametrize("precision", ["bf16x3", "fp16x3"])
@pytest.mark.parametrize("n,q,amp,r,nvec", [(32, 7, "one", 1, 3),
                                            (64, 7, "sincos", 2, 2),
                                            (128, 6, "one", 1, 17)])
def test_split_precision_2d(apply_path, precision, n, q, amp, r, nvec):
    # 2D plans run the split products in the per-step MFMA kernels (the
    # Lagrange matrices and the stored switch blocks split at plan time)
    if apply_path != "per_step_mfma":
        pytest.skip("2D split precisions run on the per-step MFMA kernels")
    log(f"case split 2D {precision} n={n} q={q} r={r} nvec={nvec}")
    f32, f, ab = inputs(2, n, nvec, 970 + n, amp=amp, r=r)
    with _plan(2, n, "radon2d", q, ab=ab, nvec=nvec,
               precision=precision) as pl:
        g, _ = gpu_apply(pl, f32)
    if ab is None:
        ref = butterfly_apply(2, n, "radon2d", PHASE_PARAMS["radon2d"], q, f)
    else:
        ref = butterfly_matvec(2, n, "radon2d", PHASE_PARAMS["radon2d"], q,
                               ab[0], ab[1], f)
    err = np.max(rel(g, ref))
    log(f"  {precision} 2D rel err vs FP64 butterfly = {err:.3e}")
    assert err < SPLIT_TOL[precision]


@pytest.mark.parametrize("scale", [1e6, 1e-6])
def test_split_precision_2d_any_input_scale(apply_path, scale):
    if apply_path != "per_step_mfma":
        pytest.skip("2D split precisions run on the per-step MFMA kernels")
    n, q = 64, 7
    log(f"case split 2D scale fp16x3 {scale:g}")
    f32, f, _ = inputs(2, n, 2, 990)
    f32 = (f32 * np.float32(scale)).astype(np.complex64)
    with _plan(2, n, "radon2d", q, nvec=2, precision="fp16x3") as pl:
        g, _ = gpu_apply(pl, f32)
    ref = butterfly_apply(2, n, "radon2d", PHASE_PARAMS["radon2d"], q,
                          f32.astype(np.complex128))
    assert np.all(np.isfinite(g))
    err = np.max(rel(g, ref))
    log(f"  rel err {err:.3e}")
    assert err < SPLIT_TOL["fp16x3"]


def test_split_precision_rejected_where_not_built(apply_path):
    # split products exist in the 1D fused passes and the 2D per-step MFMA
    # kernels; every other form refuses them instead of computing in FP32
    import paper_1803_04128_amd as bfm
    if apply_path != "per_step_mfma":
        with pytest.raises(bfm.BfError):
            bfm.Plan(2, 64, "radon2d", PHASE_PARAMS["radon2d"], q=7,
                     precision="bf16x3")
    if apply_path != "fused":
        with pytest.raises(bfm.BfError):
            bfm.Plan(1, 4096, "fio1d", PHASE_PARAMS["fio1d"], q=8,
                     precision="fp16x3")
    if apply_path == "per_step_mfma":
        with bfm.Plan(2, 64, "radon2d", PHASE_PARAMS["radon2d"], q=7,
                      precision="bf16x3") as pl:
            with pytest.raises(bfm.BfError):
                pl.set_config("per_step_mfma", switch_otf=True)
            with pytest.raises(bfm.BfError):
                pl.set_config("fused")
