"""Pins for the oracle's transposed and adjoint operators.

Scenario 2 of Section 1 (solving with K by an iterative method, or a
preconditioner built from K) needs applies of K^T and K^H as well as of K.
The transposed kernel K^T(xi_j, x_i) = alpha(x_i, xi_j) exp(2 pi i
Phi(x_i, xi_j)) is again of the form of eq. (eqn:FIO), with the roles of x
and xi exchanged, so Algorithm 4.1 factorizes it unchanged.  The pins here
fix the dense flags to the plain matrix transpose and conjugate, the DFT
case to the FFT, and the transposed butterfly to the dense transpose where
it is exact and to the paper's error order where it is not.  As matrices,
the factorization of K^T is the exact transpose of K's (its recursion in
xi is the transpose of K's recursion in x, its switch the mirror level
L - floor(L / 2)): pinned to rounding at odd and even depth, where only
the mirrored switch level makes it so."""

import os

import numpy as np
import pytest

import oracle.butterfly as bfo
import oracle.kernel as kern
from oracle.butterfly import butterfly_apply, butterfly_matvec
from oracle.dense import dense_rows, kernel_rows, rel_err
from synthetic import (gaussian_vectors, amplitude_factors, sample_rows,
                       PHASE_PARAMS)

FLAGS = [(True, False), (False, True), (True, True)]


def _full(dim, n, kind, amp, transpose=False, conjugate=False):
    return kernel_rows(dim, n, kind, PHASE_PARAMS[kind], amp,
                       np.arange(n ** dim), transpose, conjugate)


@pytest.mark.parametrize("dim,n,kind,amp", [(1, 32, "fio1d", "sincos"),
                                            (1, 16, "dft", "one"),
                                            (2, 8, "radon2d", "sincos"),
                                            (2, 4, "separable", "one")])
def test_dense_flags_are_matrix_transpose_and_conjugate(dim, n, kind, amp):
    K = _full(dim, n, kind, amp)
    np.testing.assert_allclose(_full(dim, n, kind, amp, True, False), K.T,
                               rtol=0, atol=1e-14)
    np.testing.assert_allclose(_full(dim, n, kind, amp, False, True),
                               np.conj(K), rtol=0, atol=1e-14)
    np.testing.assert_allclose(_full(dim, n, kind, amp, True, True),
                               np.conj(K).T, rtol=0, atol=1e-14)
    # the adjoint identity <K f, h> = <f, K^H h> through dense_rows
    N = n ** dim
    f, h = gaussian_vectors(N, 2, 60)
    rows = np.arange(N)
    Kf = dense_rows(dim, n, kind, PHASE_PARAMS[kind], amp, f, rows)[0]
    KHh = dense_rows(dim, n, kind, PHASE_PARAMS[kind], amp, h, rows,
                     transpose=True, conjugate=True)[0]
    lhs, rhs = np.vdot(h, Kf), np.vdot(KHh, f)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


@pytest.mark.parametrize("n", [16, 64, 256])
def test_dense_dft_transpose_and_adjoint_match_fft(n):
    # Phi = x xi on the grid x_i = i/n, xi_j = j - n/2: K_ij = (-1)^i
    # exp(2 pi i ij/n), so K^T h = n ifft((-1)^i h) and K^H h = fft((-1)^i h)
    h = gaussian_vectors(n, 2, 61)
    s = (-1.0) ** np.arange(n)
    rows = np.arange(n)
    KT = dense_rows(1, n, "dft", (), "one", h, rows, transpose=True)
    KH = dense_rows(1, n, "dft", (), "one", h, rows, transpose=True,
                    conjugate=True)
    assert np.max(rel_err(KT, n * np.fft.ifft(s * h, axis=-1))) < 1e-13
    assert np.max(rel_err(KH, np.fft.fft(s * h, axis=-1))) < 1e-13


@pytest.mark.parametrize("n", [8, 16])
def test_dense_dft_2d_adjoint_matches_fft2(n):
    h = gaussian_vectors(n * n, 1, 62)
    i1, i2 = np.divmod(np.arange(n * n), n)
    s = ((-1.0) ** (i1 + i2))
    KH = dense_rows(2, n, "dft", (), "one", h, np.arange(n * n),
                    transpose=True, conjugate=True)
    ref = np.fft.fft2((s * h).reshape(-1, n, n)).reshape(1, -1)
    assert rel_err(KH, ref)[0] < 1e-13


@pytest.mark.parametrize("transpose,conjugate", FLAGS)
@pytest.mark.parametrize("n", [4, 16, 64])
@pytest.mark.parametrize("kind", ["fio1d", "dft", "separable"])
def test_butterfly_exact_small_1d(n, kind, transpose, conjugate):
    # every box at the switch holds <= q indices: the interpolations go
    # through all points and the factorization of K^T (K^H) is exact.
    f = gaussian_vectors(n, 2, 63)
    g = butterfly_apply(1, n, kind, PHASE_PARAMS[kind], 8, f,
                        transpose=transpose, conjugate=conjugate)
    ref = dense_rows(1, n, kind, PHASE_PARAMS[kind], "one", f, np.arange(n),
                     transpose=transpose, conjugate=conjugate)
    assert np.max(rel_err(g, ref)) < 1e-13


@pytest.mark.parametrize("transpose,conjugate", FLAGS)
@pytest.mark.parametrize("n", [4, 16])
def test_butterfly_exact_small_2d(n, transpose, conjugate):
    f = gaussian_vectors(n * n, 2, 64)
    g = butterfly_apply(2, n, "radon2d", PHASE_PARAMS["radon2d"], 7, f,
                        transpose=transpose, conjugate=conjugate)
    ref = dense_rows(2, n, "radon2d", PHASE_PARAMS["radon2d"], "one", f,
                     np.arange(n * n), transpose=transpose,
                     conjugate=conjugate)
    assert np.max(rel_err(g, ref)) < 1e-13


@pytest.mark.parametrize("transpose,conjugate", FLAGS)
@pytest.mark.parametrize("dim,n,q", [(1, 4096, 8), (2, 64, 7)])
def test_butterfly_exact_for_separable_phase(dim, n, q, transpose,
                                             conjugate):
    # an additively separable phase stays separable under transposition and
    # conjugation: R(A, B) of eq. (eqn:RAB) vanishes and the butterfly is
    # exact at any size.
    N = n ** dim
    f = gaussian_vectors(N, 1, 65)
    g = butterfly_apply(dim, n, "separable", PHASE_PARAMS["separable"], q, f,
                        transpose=transpose, conjugate=conjugate)
    rows = sample_rows(N, 256, 66)
    ref = dense_rows(dim, n, "separable", PHASE_PARAMS["separable"], "one",
                     f, rows, transpose=transpose, conjugate=conjugate)
    assert np.max(rel_err(g[:, rows], ref)) < 1e-12


@pytest.mark.parametrize("conjugate", [False, True])
def test_butterfly_dft_transpose_error_decays_in_q(conjugate):
    n = 4096
    f = gaussian_vectors(n, 1, 67)
    s = (-1.0) ** np.arange(n)
    ref = (np.fft.fft(s * f, axis=-1) if conjugate
           else n * np.fft.ifft(s * f, axis=-1))
    errs = []
    for q in (4, 6, 8, 10, 12):
        g = butterfly_apply(1, n, "dft", (), q, f, transpose=True,
                            conjugate=conjugate)
        errs.append(rel_err(g, ref)[0])
    for e0, e1 in zip(errs, errs[1:]):
        assert e1 < e0 / 20
    assert errs[-1] < 1e-9


def _paper_table(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "paper_tab_1d_fio.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                N, q, e = line.split()
                rows.append((int(N), int(q), float(e)))
    return rows


@pytest.mark.parametrize("conjugate", [False, True])
@pytest.mark.parametrize("N", [1024, 4096])
def test_butterfly_transpose_error_order_matches_paper_table(N, conjugate,
                                                             golden_dir):
    # Table (tab:1D-FIO) prints the forward error only; the transposed
    # kernel's phase is exactly as smooth in each variable, with the same
    # rank bounds (Section 3), so its error must be of the same order:
    # within a factor of 4 of the printed forward values.
    params = PHASE_PARAMS["fio1d_paper"]
    f = gaussian_vectors(N, 1, 68)
    rows = sample_rows(N, 256, 69)
    ref = dense_rows(1, N, "fio1d", params, "one", f, rows, transpose=True,
                     conjugate=conjugate)
    for (n_, q, eps) in _paper_table(golden_dir):
        if n_ != N:
            continue
        g = butterfly_apply(1, N, "fio1d", params, q, f, transpose=True,
                            conjugate=conjugate)
        e = rel_err(g[:, rows], ref)[0]
        assert eps / 4 < e < eps * 4, (N, q, e, eps)


@pytest.mark.parametrize("conjugate", [False, True])
def test_butterfly_transpose_radon_2d(conjugate):
    n = 64
    f = gaussian_vectors(n * n, 1, 70)
    rows = sample_rows(n * n, 256, 71)
    params = PHASE_PARAMS["radon2d"]
    ref = dense_rows(2, n, "radon2d", params, "one", f, rows, transpose=True,
                     conjugate=conjugate)
    e = [rel_err(butterfly_apply(2, n, "radon2d", params, q, f,
                                 transpose=True,
                                 conjugate=conjugate)[:, rows], ref)[0]
         for q in (5, 7)]
    assert e[1] < e[0] / 5
    assert e[1] < 1e-4


@pytest.mark.parametrize("transpose,conjugate", FLAGS)
@pytest.mark.parametrize("dim,n,kind,q", [(1, 1024, "fio1d", 8),
                                          (2, 32, "radon2d", 7)])
def test_amplitude_split_transposed(dim, n, kind, q, transpose, conjugate):
    # with alpha = sum_k a_k(x) b_k(xi) (eq. (eqn:tg)), K^T takes b_k on its
    # output (xi) side and a_k on its input (x) side; the sincos amplitude is
    # not symmetric in x and xi, so swapping them wrongly is caught.
    N = n ** dim
    params = PHASE_PARAMS[kind]
    f = gaussian_vectors(N, 2, 72)
    a, b = amplitude_factors("sincos", dim, n, 4, 73)
    g = butterfly_matvec(dim, n, kind, params, q, a, b, f,
                         transpose=transpose, conjugate=conjugate)
    rows = sample_rows(N, 256, 74)
    ref = dense_rows(dim, n, kind, params, "sincos", f, rows,
                     transpose=transpose, conjugate=conjugate)
    e_amp = np.max(rel_err(g[:, rows], ref))
    e_one = np.max(rel_err(
        butterfly_apply(dim, n, kind, params, q, f, transpose=transpose,
                        conjugate=conjugate)[:, rows],
        dense_rows(dim, n, kind, params, "one", f, rows, transpose=transpose,
                   conjugate=conjugate)))
    assert e_amp < 3 * e_one + 1e-13


def _pins_pass():
    ok = True
    n = 64
    params = PHASE_PARAMS["fio1d"]
    for t, c in FLAGS:
        f = gaussian_vectors(n, 1, 75)
        g = bfo.butterfly_apply(1, n, "fio1d", params, 8, f, transpose=t,
                                conjugate=c)
        ref = dense_rows(1, n, "fio1d", params, "one", f, np.arange(n),
                         transpose=t, conjugate=c)
        ok &= rel_err(g, ref)[0] < 1e-13
    return bool(ok)


def _unswapped_roles(kind, params, ix, jx, n, sign=1):
    # the transposed phase evaluated with the index roles not exchanged
    return kern.expi_phase(kind, params, jx, ix, n, sign)


def _dropped_conjugation(kind, params, ix, jx, n, sign=1):
    return kern.expi_phase(kind, params, ix, jx, n, abs(sign))


def _bf_matrix(dim, n, kind, q, transpose=False, conjugate=False):
    """The butterfly operator as a matrix: column v = BF applied to e_v."""
    N = n ** dim
    cols = butterfly_apply(dim, n, kind, PHASE_PARAMS[kind], q,
                           np.eye(N, dtype=np.complex128),
                           transpose=transpose, conjugate=conjugate)
    return cols.T


@pytest.mark.parametrize("dim,n,q,kind", [(1, 512, 6, "fio1d"),
                                          (1, 256, 5, "fio1d"),
                                          (1, 128, 4, "dft"),
                                          (2, 32, 5, "radon2d"),
                                          (2, 16, 3, "radon2d")])
def test_butterfly_of_transpose_is_exact_transpose(dim, n, q, kind):
    # depth L = 9, 8, 7 (1D) and 5, 4 (2D): BF_{K^T} = (BF_K)^T and
    # BF_{K^H} = (BF_K)^H to rounding, not merely to eps_BF
    B = _bf_matrix(dim, n, kind, q)
    Bt = _bf_matrix(dim, n, kind, q, transpose=True)
    Bh = _bf_matrix(dim, n, kind, q, transpose=True, conjugate=True)
    nb = np.linalg.norm(B)
    assert np.linalg.norm(Bt - B.T) < 1e-13 * nb
    assert np.linalg.norm(Bh - B.conj().T) < 1e-13 * nb


def test_unmirrored_switch_level_is_not_the_transpose(monkeypatch):
    # the transposed factorization switching at floor(L / 2) like K's (odd
    # L = 9) is a different approximation: the pin above would fail
    B = _bf_matrix(1, 512, "fio1d", 6)
    monkeypatch.setattr(bfo, "switch_level", lambda L, transpose: L // 2)
    Bt = _bf_matrix(1, 512, "fio1d", 6, transpose=True)
    assert np.linalg.norm(Bt - B.T) > 1e-4 * np.linalg.norm(B)


def test_unmutated_transpose_pins_pass():
    assert _pins_pass()


@pytest.mark.parametrize("name,mutant", [
    ("unswapped index roles", _unswapped_roles),
    ("dropped conjugation", _dropped_conjugation),
])
def test_transpose_pins_reject_mutant(monkeypatch, name, mutant):
    monkeypatch.setattr(bfo, "expi_phase", mutant)
    assert not _pins_pass(), name
