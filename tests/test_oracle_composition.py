"""Pins for the oracle's composition of two FIOs (eq. (eq:example4), the
phase of eq. (eqn:FIOK2)) and for that phase itself: closed forms through
the FFT, 50-digit brute force, exactness of the butterflies at small sizes
and the error of the chained butterflies."""

import mpmath
import numpy as np
import pytest

from oracle.butterfly import butterfly_apply, butterfly_composition
from oracle.dense import (composition_rows, dense_rows, fourier_coefficients,
                          rel_err)
from synthetic import gaussian_vectors, sample_rows, PHASE_PARAMS

WARP = PHASE_PARAMS["fio1d_warp"]


@pytest.mark.parametrize("n", [16, 256, 4096])
def test_fourier_coefficients_match_fft_and_invert_the_dft_kernel(n):
    h = gaussian_vectors(n, 2, 80)
    c = fourier_coefficients(n, h)
    # hat_j = (1/n) fft(h)[(j - n/2) mod n]
    ref = np.fft.fftshift(np.fft.fft(h, axis=-1), axes=-1) / n
    assert np.max(rel_err(c, ref)) < 1e-13
    if n <= 256:
        back = dense_rows(1, n, "dft", (), "one", c, np.arange(n))
        assert np.max(rel_err(back, h)) < 1e-13


@pytest.mark.parametrize("n", [16, 64])
def test_warp_phase_brute_force_mpmath(n):
    # Phi = x xi + c(x) xi in 50 digits, summed in a plain double loop
    f = gaussian_vectors(n, 1, 81)[0]
    g = dense_rows(1, n, "fio1d_warp", WARP, "one", f[None], np.arange(n))[0]
    mpmath.mp.dps = 50
    p0, p1, p2 = [mpmath.mpf(v) for v in WARP]
    for i in range(n):
        x = mpmath.mpf(i) / n
        c = (p0 + p1 * mpmath.sin(2 * mpmath.pi * x)) / p2
        acc = mpmath.mpc(0)
        for j in range(n):
            xi = mpmath.mpf(j - n // 2)
            acc += mpmath.expjpi(2 * (x * xi + c * xi)) * mpmath.mpc(
                f[j].real, f[j].imag)
        assert abs(complex(acc) - g[i]) < 1e-13 * max(1.0, abs(complex(acc)))


@pytest.mark.parametrize("c", [0.0, 0.125, 0.3])
def test_warp_phase_with_constant_shift_is_a_modulated_dft(c):
    # c(x) = c: K_ij = exp(2 pi i x_i xi_j) exp(2 pi i c xi_j)
    n = 1024
    f = gaussian_vectors(n, 2, 82)
    xi = np.arange(n) - n // 2
    g = dense_rows(1, n, "fio1d_warp", (c, 0.0, 1.0), "one", f, np.arange(n))
    ref = ((-1.0) ** np.arange(n)) * n * np.fft.ifft(
        np.exp(2j * np.pi * c * xi) * f, axis=-1)
    assert np.max(rel_err(g, ref)) < 1e-12


def test_composition_without_warp_is_one_dft_apply():
    # c = 0: L is the DFT-phase kernel K, and (1/n) K^H K = I, so L(L f) = K f
    n = 512
    f = gaussian_vectors(n, 2, 83)
    g = composition_rows(n, "fio1d_warp", (0.0, 0.0, 1.0), f, np.arange(n))
    ref = ((-1.0) ** np.arange(n)) * n * np.fft.ifft(f, axis=-1)
    assert np.max(rel_err(g, ref)) < 1e-12


@pytest.mark.parametrize("c", [0.125, 0.3])
def test_composition_with_constant_shift_doubles_the_shift(c):
    n = 512
    f = gaussian_vectors(n, 2, 84)
    xi = np.arange(n) - n // 2
    g = composition_rows(n, "fio1d_warp", (c, 0.0, 1.0), f, np.arange(n))
    ref = ((-1.0) ** np.arange(n)) * n * np.fft.ifft(
        np.exp(4j * np.pi * c * xi) * f, axis=-1)
    assert np.max(rel_err(g, ref)) < 1e-12


@pytest.mark.parametrize("n", [16, 64])
def test_butterfly_composition_exact_small(n):
    f = gaussian_vectors(n, 2, 85)
    g = butterfly_composition(n, "fio1d_warp", WARP, 8, f)
    ref = composition_rows(n, "fio1d_warp", WARP, f, np.arange(n))
    assert np.max(rel_err(g, ref)) < 1e-13


def test_butterfly_composition_error_decays_in_q():
    # three chained factorizations: the composed error stays within a small
    # multiple of the largest single-operator error and falls with q
    n = 4096
    f = gaussian_vectors(n, 1, 86)
    rows = sample_rows(n, 256, 87)
    ref = composition_rows(n, "fio1d_warp", WARP, f, rows)
    errs = []
    for q in (6, 8, 10):
        g = butterfly_composition(n, "fio1d_warp", WARP, q, f)
        e_one = max(
            rel_err(butterfly_apply(1, n, "fio1d_warp", WARP, q, f)[:, rows],
                    dense_rows(1, n, "fio1d_warp", WARP, "one", f, rows))[0],
            rel_err(butterfly_apply(1, n, "dft", (), q, f, transpose=True,
                                    conjugate=True)[:, rows],
                    dense_rows(1, n, "dft", (), "one", f, rows,
                               transpose=True, conjugate=True))[0])
        e = rel_err(g[:, rows], ref)[0]
        assert e < 4 * e_one, (q, e, e_one)
        errs.append(e)
    assert errs[1] < errs[0] / 20 and errs[2] < errs[1] / 20
