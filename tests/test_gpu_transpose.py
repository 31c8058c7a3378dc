"""GPU parity of the transposed and conjugate operators (bf_plan_op):
K^T, conj(K) and K^H, needed by the solvers of Scenario 2 in Section 1.

Same bars as the forward apply: relative l2 <= 1e-5 per vector against the
oracle's butterfly of the same operator (same factorization), <= 1e-5
against the dense matvec where the factorization is exact, the BF16x3 and
FP16x3 bars of the forward apply for the split precisions, and at sizes the
oracle cannot finish, the FFT closed form and the adjoint identity.  The
factorization of K^T is the exact transpose of K's (the oracle pins it to
rounding): as matrices the GPU's BF_{K^T} and BF_{K^H} equal BF_K^T and
BF_K^H to FP32 rounding, at odd and even depth."""

import numpy as np
import pytest

from _util import inputs, gpu_apply, rel, log
from oracle.butterfly import butterfly_apply, butterfly_matvec
from oracle.dense import dense_rows
from synthetic import gaussian_vectors, sample_rows, PHASE_PARAMS

pytestmark = pytest.mark.gpu

TOL = 1e-5
FLAGS = {"T": (True, False), "C": (False, True), "H": (True, True)}


@pytest.fixture(autouse=True, params=["fused", "per_step", "per_step_mfma"])
def apply_path(request, monkeypatch):
    monkeypatch.setenv("BF_FUSED", "1" if request.param == "fused" else "0")
    monkeypatch.setenv("BF_MFMA", "0" if request.param == "per_step" else "1")
    return request.param


def _plan(dim, n, kind, q, op, ab=None, nvec=1, precision="fp32"):
    import paper_1803_04128_amd as bfm
    return bfm.Plan(dim, n, kind, PHASE_PARAMS[kind], q=q, amplitude=ab,
                    precision=precision, max_nvec=nvec, op=op)


@pytest.mark.parametrize("op", ["T", "C", "H"])
@pytest.mark.parametrize("n", [16, 64])
@pytest.mark.parametrize("kind", ["fio1d", "dft"])
def test_exact_small_1d(n, kind, op):
    log(f"case transpose exact_small_1d n={n} kind={kind} op={op}")
    f32, f, _ = inputs(1, n, 2, 1100 + n)
    with _plan(1, n, kind, 8, op, nvec=2) as pl:
        assert pl.info()["op"] == "NTCH".index(op)
        g, _ = gpu_apply(pl, f32)
    t, c = FLAGS[op]
    ref = dense_rows(1, n, kind, PHASE_PARAMS[kind], "one", f, np.arange(n),
                     transpose=t, conjugate=c)
    assert np.max(rel(g, ref)) < TOL


@pytest.mark.parametrize("op", ["T", "H"])
@pytest.mark.parametrize("n", [8, 16])
def test_exact_small_2d(n, op):
    log(f"case transpose exact_small_2d n={n} op={op}")
    f32, f, _ = inputs(2, n, 2, 1200 + n)
    with _plan(2, n, "radon2d", 7, op, nvec=2) as pl:
        g, _ = gpu_apply(pl, f32)
    t, c = FLAGS[op]
    ref = dense_rows(2, n, "radon2d", PHASE_PARAMS["radon2d"], "one", f,
                     np.arange(n * n), transpose=t, conjugate=c)
    assert np.max(rel(g, ref)) < TOL


@pytest.mark.parametrize("op", ["T", "C", "H"])
@pytest.mark.parametrize("n,q,kind", [(4096, 10, "fio1d"), (2048, 8, "dft"),
                                      (8192, 12, "fio1d")])
def test_parity_vs_oracle_butterfly_1d(n, q, kind, op):
    log(f"case transpose parity_1d n={n} q={q} kind={kind} op={op}")
    f32, f, _ = inputs(1, n, 2, 1300 + q)
    with _plan(1, n, kind, q, op, nvec=2) as pl:
        g, _ = gpu_apply(pl, f32)
    t, c = FLAGS[op]
    ref = butterfly_apply(1, n, kind, PHASE_PARAMS[kind], q, f,
                          transpose=t, conjugate=c)
    assert np.max(rel(g, ref)) < TOL


@pytest.mark.parametrize("op", ["T", "H"])
@pytest.mark.parametrize("n,q,r", [(4096, 10, 4), (2048, 6, 3)])
def test_parity_amplitude_1d(n, q, r, op):
    log(f"case transpose amp_1d n={n} q={q} r={r} op={op}")
    f32, f, ab = inputs(1, n, 3, 1400 + r, amp="sincos", r=r)
    with _plan(1, n, "fio1d", q, op, ab=ab, nvec=3) as pl:
        g, _ = gpu_apply(pl, f32)
    t, c = FLAGS[op]
    ref = butterfly_matvec(1, n, "fio1d", PHASE_PARAMS["fio1d"], q, ab[0],
                           ab[1], f, transpose=t, conjugate=c)
    assert np.max(rel(g, ref)) < TOL


@pytest.mark.parametrize("op", ["T", "H"])
@pytest.mark.parametrize("n,q", [(64, 7), (128, 5)])
def test_parity_vs_oracle_butterfly_2d(n, q, op):
    log(f"case transpose parity_2d n={n} q={q} op={op}")
    f32, f, _ = inputs(2, n, 1, 1500 + q)
    with _plan(2, n, "radon2d", q, op) as pl:
        g, _ = gpu_apply(pl, f32)
    t, c = FLAGS[op]
    ref = butterfly_apply(2, n, "radon2d", PHASE_PARAMS["radon2d"], q, f,
                          transpose=t, conjugate=c)
    assert np.max(rel(g, ref)) < TOL


@pytest.mark.parametrize("op", ["T", "H"])
def test_parity_amplitude_2d(op):
    n, q = 32, 7
    log(f"case transpose amp_2d op={op}")
    f32, f, ab = inputs(2, n, 2, 1600, amp="sincos", r=2)
    with _plan(2, n, "radon2d", q, op, ab=ab, nvec=2) as pl:
        g, _ = gpu_apply(pl, f32)
    t, c = FLAGS[op]
    ref = butterfly_matvec(2, n, "radon2d", PHASE_PARAMS["radon2d"], q,
                           ab[0], ab[1], f, transpose=t, conjugate=c)
    assert np.max(rel(g, ref)) < TOL


@pytest.mark.parametrize("op", ["T", "H"])
def test_separable_phase_exact_at_size(op):
    # separable phases stay separable under transposition: the butterfly is
    # exact, so the dense rows bound the FP32 apply directly
    for dim, n, q in [(1, 1 << 18, 10), (2, 256, 6)]:
        log(f"case transpose separable dim={dim} n={n} op={op}")
        N = n ** dim
        f32, f, _ = inputs(dim, n, 1, 1700 + dim)
        with _plan(dim, n, "separable", q, op) as pl:
            g, _ = gpu_apply(pl, f32)
        rows = sample_rows(N, 256, 1701)
        t, c = FLAGS[op]
        ref = dense_rows(dim, n, "separable", PHASE_PARAMS["separable"],
                         "one", f, rows, transpose=t, conjugate=c)
        assert np.max(rel(g[:, rows], ref)) < TOL


def test_dft_adjoint_against_fft_full_size():
    # K^H h = fft((-1)^i h) for the DFT phase (closed form at any size)
    n, q = 1 << 16, 10
    log(f"case transpose dft_fft n={n}")
    f32, f, _ = inputs(1, n, 1, 1800)
    s = (-1.0) ** np.arange(n)
    with _plan(1, n, "dft", q, "H") as pl:
        g, _ = gpu_apply(pl, f32)
    with _plan(1, n, "dft", q, "T") as pl:
        gt, _ = gpu_apply(pl, f32)
    m = 4096
    e_bf = rel(butterfly_apply(1, m, "dft", (), q, f[:, :m], transpose=True,
                               conjugate=True),
               np.fft.fft(s[:m] * f[:, :m], axis=-1))[0]
    bound = max(10 * e_bf, 1e-6) + TOL
    assert rel(g, np.fft.fft(s * f, axis=-1))[0] < bound
    assert rel(gt, n * np.fft.ifft(s * f, axis=-1))[0] < bound


@pytest.mark.parametrize("dim,n,q,kind", [(1, 2048, 8, "fio1d"),
                                          (1, 1024, 8, "fio1d"),
                                          (2, 32, 5, "radon2d")])
def test_transpose_is_exact_transpose_of_forward(dim, n, q, kind):
    # depth L = 11, 10 (1D), 5 (2D): columns of the operators from applies
    # to the unit vectors, BF_{K^T} against BF_K^T and BF_{K^H} against
    # BF_K^H; the same FP32 factors in transposed order, so only rounding
    # separates them (FP32 bar 1e-5 relative in Frobenius norm)
    N = n ** dim
    log(f"case exact transpose dim={dim} n={n} q={q}")
    eye = np.eye(N, dtype=np.complex64)
    mats = {}
    for op in ("N", "T", "H"):
        with _plan(dim, n, kind, q, op, nvec=N) as pl:
            g, _ = gpu_apply(pl, eye)
        mats[op] = g.T                      # column v = BF applied to e_v
    nb = np.linalg.norm(mats["N"])
    eT = np.linalg.norm(mats["T"] - mats["N"].T) / nb
    eH = np.linalg.norm(mats["H"] - mats["N"].conj().T) / nb
    log(f"  ||BF_T - BF^T|| {eT:.2e}, ||BF_H - BF^H|| {eH:.2e} (relative)")
    assert eT < TOL and eH < TOL


@pytest.mark.parametrize("n", [1 << 19, 1 << 20])
def test_adjoint_identity_at_full_size(n):
    # <K f, h> = <f, K^H h>: the factorization of K^H is the exact adjoint
    # of K's at odd and even depth, so the FP32 applies agree to rounding
    import torch
    q = 10
    log(f"case adjoint identity n={n}")
    f = gaussian_vectors(n, 1, 1900).astype(np.complex64)
    h = gaussian_vectors(n, 1, 1901).astype(np.complex64)
    with _plan(1, n, "fio1d", q, "N") as pl:
        Kf, _ = gpu_apply(pl, f)
    with _plan(1, n, "fio1d", q, "H") as pl:
        KHh, _ = gpu_apply(pl, h)
    f, h = f.astype(np.complex128), h.astype(np.complex128)
    lhs, rhs = np.vdot(h, Kf), np.vdot(KHh, f)
    scale = np.linalg.norm(Kf) * np.linalg.norm(h)
    log(f"  |<Kf,h> - <f,K^H h>| / (|Kf||h|) = {abs(lhs - rhs) / scale:.3e}")
    assert abs(lhs - rhs) < 1e-6 * scale
    torch.cuda.synchronize()


SPLIT_TOL = {"bf16x3": 1e-4, "fp16x3": 1e-5}


@pytest.mark.parametrize("op", ["T", "H"])
@pytest.mark.parametrize("precision", ["bf16x3", "fp16x3"])
def test_split_precision(apply_path, precision, op):
    if apply_path != "fused":
        pytest.skip("split precisions run on the fused MFMA passes only")
    n, q, r = 4096, 10, 4
    log(f"case transpose split {precision} op={op}")
    f32, f, ab = inputs(1, n, 3, 2000, amp="sincos", r=r)
    with _plan(1, n, "fio1d", q, op, ab=ab, nvec=3,
               precision=precision) as pl:
        g, _ = gpu_apply(pl, f32)
    t, c = FLAGS[op]
    ref = butterfly_matvec(1, n, "fio1d", PHASE_PARAMS["fio1d"], q, ab[0],
                           ab[1], f, transpose=t, conjugate=c)
    err = np.max(rel(g, ref))
    log(f"  rel err {err:.3e}")
    assert err < SPLIT_TOL[precision]
