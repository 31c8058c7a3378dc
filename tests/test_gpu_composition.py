"""GPU parity of the composition example (eq. (eq:example4)): the phase of
eq. (eqn:FIOK2) through every execution form, the Fourier-coefficient plan
(the DFT-phase adjoint with amplitude 1/n) and chained applies
(bf_apply_chain) against the oracle's dense and chained-butterfly
compositions, and at full size against the FFT closed form of a constant
shift."""

import numpy as np
import pytest

from _util import inputs, gpu_apply, rel, log
from oracle.butterfly import butterfly_apply, butterfly_composition
from oracle.dense import composition_rows, dense_rows
from synthetic import gaussian_vectors, sample_rows, PHASE_PARAMS

pytestmark = pytest.mark.gpu

TOL = 1e-5
WARP = PHASE_PARAMS["fio1d_warp"]


@pytest.fixture(autouse=True, params=["fused", "per_step", "per_step_mfma"])
def apply_path(request, monkeypatch):
    monkeypatch.setenv("BF_FUSED", "1" if request.param == "fused" else "0")
    monkeypatch.setenv("BF_MFMA", "0" if request.param == "per_step" else "1")
    return request.param


def _warp(n, q, nvec=1, params=WARP, op="N"):
    import paper_1803_04128_amd as bfm
    return bfm.Plan(1, n, "fio1d_warp", params, q=q, max_nvec=nvec, op=op)


def _chain(plans, f32):
    import torch
    import paper_1803_04128_amd as bfm
    f = torch.from_numpy(np.ascontiguousarray(f32)).to("cuda")
    g = bfm.apply_chain(plans, f)
    torch.cuda.synchronize()
    return g.cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("n", [16, 64])
def test_warp_exact_small(n):
    log(f"case warp exact n={n}")
    f32, f, _ = inputs(1, n, 2, 2100 + n)
    with _warp(n, 8, 2) as pl:
        g, _ = gpu_apply(pl, f32)
    ref = dense_rows(1, n, "fio1d_warp", WARP, "one", f, np.arange(n))
    assert np.max(rel(g, ref)) < TOL


@pytest.mark.parametrize("op", ["N", "H"])
@pytest.mark.parametrize("n,q", [(4096, 10), (1 << 14, 8), (2048, 12)])
def test_warp_parity_vs_oracle_butterfly(n, q, op):
    log(f"case warp parity n={n} q={q} op={op}")
    f32, f, _ = inputs(1, n, 2, 2200 + q)
    with _warp(n, q, 2, op=op) as pl:
        g, _ = gpu_apply(pl, f32)
    ref = butterfly_apply(1, n, "fio1d_warp", WARP, q, f,
                          transpose=op == "H", conjugate=op == "H")
    assert np.max(rel(g, ref)) < TOL


def test_fourier_coefficients_plan():
    import paper_1803_04128_amd as bfm
    n, q = 1 << 16, 10
    log(f"case fourier coefficients n={n}")
    f32, f, _ = inputs(1, n, 2, 2300)
    with bfm.fourier_coefficients_plan(n, q, max_nvec=2) as pl:
        g, _ = gpu_apply(pl, f32)
    ref = np.fft.fftshift(np.fft.fft(f, axis=-1), axes=-1) / n
    assert np.max(rel(g, ref)) < TOL
    m = 4096
    f32, f, _ = inputs(1, m, 1, 2301)
    with bfm.fourier_coefficients_plan(m, q) as pl:
        g, _ = gpu_apply(pl, f32)
    bf = butterfly_apply(1, m, "dft", (), q, f, transpose=True,
                         conjugate=True) / m
    assert rel(g, bf)[0] < TOL


@pytest.mark.parametrize("n,q", [(64, 8), (4096, 10), (2048, 8)])
def test_composition_against_oracle(n, q):
    import paper_1803_04128_amd as bfm
    log(f"case composition n={n} q={q}")
    f32, f, _ = inputs(1, n, 2, 2400 + q)
    with _warp(n, q, 2) as L, bfm.fourier_coefficients_plan(
            n, q, max_nvec=2) as F:
        g = _chain([L, F, L], f32)
    bf = butterfly_composition(n, "fio1d_warp", WARP, q, f)
    rows = sample_rows(n, min(n, 256), 2401)
    dense = composition_rows(n, "fio1d_warp", WARP, f, rows)
    eps = np.max(rel(bf[:, rows], dense))
    log(f"  eps_BF(composition) {eps:.3e}  gpu-vs-bf "
        f"{np.max(rel(g, bf)):.3e}")
    assert np.max(rel(g, bf)) < TOL
    assert np.max(rel(g[:, rows], dense)) < eps + TOL


def test_chain_equals_sequential_applies():
    # the ping-pong through tmp and g changes nothing: chains of 1 to 4
    # applies are bitwise the applies issued one by one
    import paper_1803_04128_amd as bfm
    n, q = 4096, 8
    log("case chain vs sequential")
    f32, _, _ = inputs(1, n, 3, 2500)
    with _warp(n, q, 3) as L, bfm.fourier_coefficients_plan(
            n, q, max_nvec=3) as F:
        seq = [L, F, L, F]
        for m in range(1, 5):
            g = _chain(seq[:m], f32)
            h = f32
            for p in seq[:m]:
                h, _ = gpu_apply(p, h.astype(np.complex64))
            assert np.array_equal(g, h), m


def test_chain_rejects_bad_arguments():
    import torch
    import paper_1803_04128_amd as bfm
    log("case chain errors")
    with _warp(1024, 8) as L, _warp(2048, 8) as L2:
        f = torch.zeros((1, 1024), dtype=torch.complex64, device="cuda")
        with pytest.raises(bfm.BfError):
            bfm.apply_chain([L, L2], f)
        with pytest.raises(bfm.BfError):
            bfm.apply_chain([L, L], f, tmp=f)
        with pytest.raises(bfm.BfError):
            bfm.apply_chain([L], f, out=f)
        with pytest.raises(bfm.BfError):
            bfm.apply_chain([L], torch.zeros((2, 1024), dtype=torch.complex64,
                                             device="cuda"))


def test_composition_constant_shift_full_size():
    # c(x) = c: L(L f) = K_dft (exp(4 pi i c xi) f), an FFT closed form at
    # any size (N = 2^20, 4 vectors, three chained applies)
    import paper_1803_04128_amd as bfm
    n, q, c, nvec = 1 << 20, 10, 0.3, 4
    log(f"case composition constant shift n={n}")
    f = gaussian_vectors(n, nvec, 2600).astype(np.complex64)
    with _warp(n, q, nvec, params=(c, 0.0, 1.0)) as L, \
            bfm.fourier_coefficients_plan(n, q, max_nvec=nvec) as F:
        g = _chain([L, F, L], f)
    xi = np.arange(n) - n // 2
    ref = ((-1.0) ** np.arange(n)) * n * np.fft.ifft(
        np.exp(4j * np.pi * c * xi) * f.astype(np.complex128), axis=-1)
    err = np.max(rel(g, ref))
    log(f"  rel err {err:.3e}")
    assert err < TOL


def test_chain_graph_replays_match_eager():
    # bf_graph_create_chain: one graph for [L, F, L]; every replay equals the
    # eager chain bit for bit, with fresh input and other device work in
    # between; the plans stay locked while the graph exists
    import torch
    import paper_1803_04128_amd as bfm
    n, q, nvec = 4096, 8, 2
    log("case chain graph")
    rng = np.random.default_rng(2700)
    with _warp(n, q, nvec) as L, bfm.fourier_coefficients_plan(
            n, q, max_nvec=nvec) as F:
        f = torch.zeros((nvec, n), dtype=torch.complex64, device="cuda")
        gout = torch.zeros_like(f)
        gr = bfm.graph_chain([L, F, L], f, gout)
        try:
            for rep in range(4):
                x = (rng.standard_normal((nvec, n)) +
                     1j * rng.standard_normal((nvec, n))).astype(np.complex64)
                f.copy_(torch.from_numpy(x).to("cuda"))
                eager = bfm.apply_chain([L, F, L], f)
                junk = torch.randn(1 << 18, device="cuda").sum()
                torch.cuda.synchronize()
                gr.launch()
                torch.cuda.synchronize()
                assert torch.equal(gout, eager), rep
                assert float(junk) == float(junk)
            for pl in (L, F):
                with pytest.raises(bfm.BfError) as ei:
                    pl.set_config("per_step")
                assert ei.value.code == bfm._lib.BF_EBUSY
        finally:
            gr.close()
        L.set_config("per_step")          # released
