"""Pins for the oracle's phase in low-rank form (Algorithm 2's input,
Phi(m, n) = U(m, :) V(n, :)^T): exact factorizations of the built-in
phases reproduce their kernels, 50-digit brute force, and the butterfly on
a low-rank phase (exact cases, decay in q)."""

import mpmath
import numpy as np
import pytest

from oracle.butterfly import butterfly_apply
from oracle.dense import dense_rows, rel_err
from synthetic import (gaussian_vectors, lowrank_phase, orthogonal_mix,
                       sample_rows, PHASE_PARAMS)


def _fio_factors(n, params, rank=4, seed=90):
    # Phi = x xi + c(x) |xi| with c(x) = (p0 + p1 sin 2 pi x) / p2 (Section
    # 5, eq. (eqn:1D-FIO-kernal)) is exactly U V^T for U = [x, c(x)],
    # V = [xi, |xi|]; zero-padded to rank columns and mixed by Q
    p0, p1, p2 = params
    i = np.arange(n)
    x, xi = i / n, (i - n // 2).astype(np.float64)
    U = np.zeros((n, rank))
    V = np.zeros((n, rank))
    U[:, 0], U[:, 1] = x, (p0 + p1 * np.sin(2 * np.pi * x)) / p2
    V[:, 0], V[:, 1] = xi, np.abs(xi)
    Q = orthogonal_mix(rank, seed)
    return U @ Q, V @ Q


def _dft2_factors(n):
    g = np.arange(n * n)
    x = np.stack([g // n, g % n], 1) / n
    xi = (np.stack([g // n, g % n], 1) - n // 2).astype(np.float64)
    return x, xi


@pytest.mark.parametrize("n", [64, 1024, 1 << 14])
def test_exact_factors_reproduce_fio_kernel(n):
    params = PHASE_PARAMS["fio1d"]
    U, V = _fio_factors(n, params)
    f = gaussian_vectors(n, 1, 91)
    rows = sample_rows(n, 64, 92)
    g = dense_rows(1, n, "lowrank", (U, V), "one", f, rows)
    ref = dense_rows(1, n, "fio1d", params, "one", f, rows)
    # the products reach n/2 in magnitude: the reduction modulo 1 of the
    # FP64 sum loses about n * 2^-52 of a cycle
    assert rel_err(g, ref)[0] < 1e-12 * n


@pytest.mark.parametrize("n", [8, 32])
def test_exact_factors_reproduce_2d_dft(n):
    U, V = _dft2_factors(n)
    f = gaussian_vectors(n * n, 1, 93)
    g = dense_rows(2, n, "lowrank", (U, V), "one", f, np.arange(n * n))
    i1, i2 = np.divmod(np.arange(n * n), n)
    ref = ((-1.0) ** (i1 + i2)) * (n * n) * np.fft.ifft2(
        f.reshape(1, n, n)).reshape(1, -1)
    assert rel_err(g, ref)[0] < 1e-12


@pytest.mark.parametrize("dim,n,rank", [(1, 16, 4), (2, 4, 5)])
def test_lowrank_brute_force_mpmath(dim, n, rank):
    U, V = lowrank_phase(dim, n, rank, 94)
    N = n ** dim
    f = gaussian_vectors(N, 1, 95)[0]
    g = dense_rows(dim, n, "lowrank", (U, V), "one", f[None],
                   np.arange(N))[0]
    mpmath.mp.dps = 50
    for i in range(N):
        acc = mpmath.mpc(0)
        for j in range(N):
            ph = mpmath.fsum(mpmath.mpf(U[i, k]) * mpmath.mpf(V[j, k])
                             for k in range(rank))
            acc += mpmath.expjpi(2 * ph) * mpmath.mpc(f[j].real, f[j].imag)
        assert abs(complex(acc) - g[i]) < 1e-12 * max(1.0, abs(complex(acc)))


def test_synthetic_lowrank_phase_has_the_stated_form():
    # mixing by Q leaves U V^T = x . xi + sum_k u_k(x) w_k(xi) with small
    # smooth u_k: the bilinear part dominates and the rest is bounded by
    # 0.12 |xi| per term
    n, rank = 64, 4
    U, V = lowrank_phase(1, n, rank, 96)
    Phi = U @ V.T
    i = np.arange(n)
    bil = np.outer(i / n, i - n // 2)
    rest = Phi - bil
    assert np.max(np.abs(rest)) <= 0.12 * (rank - 1) * (n // 2) + 1e-9
    assert np.linalg.matrix_rank(rest, tol=1e-9) <= rank - 1


@pytest.mark.parametrize("transpose,conjugate", [(False, False),
                                                 (True, True)])
@pytest.mark.parametrize("dim,n,q", [(1, 64, 8), (2, 16, 7)])
def test_butterfly_exact_small(dim, n, q, transpose, conjugate):
    U, V = lowrank_phase(dim, n, dim + 2, 97)
    N = n ** dim
    f = gaussian_vectors(N, 2, 98)
    g = butterfly_apply(dim, n, "lowrank", (U, V), q, f,
                        transpose=transpose, conjugate=conjugate)
    ref = dense_rows(dim, n, "lowrank", (U, V), "one", f, np.arange(N),
                     transpose=transpose, conjugate=conjugate)
    assert np.max(rel_err(g, ref)) < 1e-12


def test_butterfly_with_fio_factors_matches_fio_butterfly():
    # the same phase in two forms: the factorizations agree to the phase
    # rounding of the low-rank form
    n, q = 4096, 8
    params = PHASE_PARAMS["fio1d"]
    U, V = _fio_factors(n, params)
    f = gaussian_vectors(n, 1, 99)
    g = butterfly_apply(1, n, "lowrank", (U, V), q, f)
    ref = butterfly_apply(1, n, "fio1d", params, q, f)
    assert rel_err(g, ref)[0] < 1e-12 * n


@pytest.mark.parametrize("dim,n", [(1, 4096), (2, 64)])
def test_butterfly_lowrank_error_decays_in_q(dim, n):
    U, V = lowrank_phase(dim, n, dim + 3, 100)
    N = n ** dim
    f = gaussian_vectors(N, 1, 101)
    rows = sample_rows(N, 256, 102)
    ref = dense_rows(dim, n, "lowrank", (U, V), "one", f, rows)
    # measured: 1D 3.9e-3, 1.0e-4, 1.5e-6, 2.4e-8 at q = 6, 8, 10, 12;
    # 2D 3.0e-2, 7.8e-3, 1.7e-4 at q = 4, 5, 7
    qs = (6, 8, 10, 12) if dim == 1 else (4, 5, 7)
    errs = [rel_err(butterfly_apply(dim, n, "lowrank", (U, V), q, f)[:, rows],
                    ref)[0] for q in qs]
    for e0, e1 in zip(errs, errs[1:]):
        assert e1 < e0 / 3
    assert errs[-1] < (1e-7 if dim == 1 else 1e-3)
