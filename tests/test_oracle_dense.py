"""Pins for the dense oracle g = K f (Section 4 problem statement; Section 5,
eq. (eqn:1D-FIO) and eq. (eqn:1D-xandxi)) against closed forms, brute force
and invariants that do not reuse its code."""

import cmath
import math

import mpmath
import numpy as np
import pytest

from oracle.dense import dense_rows, kernel_rows, rel_err
from oracle.kernel import phase_mod1
from synthetic import gaussian_vectors, amplitude_factors, PHASE_PARAMS


def _all(dim, n, kind, params, amp, f):
    return dense_rows(dim, n, kind, params, amp, f, np.arange(n ** dim))


@pytest.mark.parametrize("n", [8, 64, 1024, 4096])
def test_dft_1d_matches_fft(n):
    # Phi = x xi: K_ij = exp(2 pi i i (j - n/2)/n) = (-1)^i exp(2 pi i ij/n),
    # so g_i = (-1)^i n ifft(f)_i.
    f = gaussian_vectors(n, 2, 7)
    g = _all(1, n, "dft", (), "one", f)
    ref = ((-1.0) ** np.arange(n)) * n * np.fft.ifft(f, axis=-1)
    assert np.max(rel_err(g, ref)) < 1e-12


@pytest.mark.parametrize("n", [4, 16, 64])
def test_dft_2d_matches_fft(n):
    f = gaussian_vectors(n * n, 2, 8)
    g = _all(2, n, "dft", (), "one", f)
    i1, i2 = np.divmod(np.arange(n * n), n)
    sign = (-1.0) ** (i1 + i2)
    ref = sign * (n * n) * np.fft.ifft2(f.reshape(2, n, n)).reshape(2, -1)
    assert np.max(rel_err(g, ref)) < 1e-12


@pytest.mark.parametrize("k", [0, 5, 511, 1000])
def test_dft_impulse_is_pure_exponential(k):
    # f = e_k gives a geometric sequence with ratio exp(2 pi i (k - n/2)/n)
    # starting at 1 (row 0 has x = 0).
    n = 1024
    f = np.zeros((1, n), complex)
    f[0, k] = 1.0
    g = _all(1, n, "dft", (), "one", f)[0]
    assert abs(g[0] - 1) < 1e-14
    ratio = g[1:] / g[:-1]
    w = cmath.exp(2j * math.pi * (k - n // 2) / n)
    assert np.max(np.abs(ratio - w)) < 1e-12
    assert np.max(np.abs(np.abs(g) - 1)) < 1e-14


def test_dft_parseval():
    n = 2048
    f = gaussian_vectors(n, 3, 9)
    g = _all(1, n, "dft", (), "one", f)
    assert np.allclose(np.sum(np.abs(g) ** 2, -1),
                       n * np.sum(np.abs(f) ** 2, -1), rtol=1e-12)


@pytest.mark.parametrize("dim,kind", [(1, "fio1d"), (2, "radon2d"),
                                      (1, "separable"), (2, "separable")])
def test_linearity(dim, kind):
    n = 256 if dim == 1 else 16
    N = n ** dim
    f = gaussian_vectors(N, 2, 10)
    a, b = 0.3 - 1.7j, 2.1 + 0.4j
    params = PHASE_PARAMS[kind]
    rows = np.arange(0, N, 3)
    g = dense_rows(dim, n, kind, params, "one", np.vstack(
        [f, a * f[0] + b * f[1]]), rows)
    assert np.max(np.abs(g[2] - (a * g[0] + b * g[1]))) < 1e-12 * np.max(
        np.abs(g[2]))


@pytest.mark.parametrize("dim,n", [(1, 512), (2, 32)])
def test_separable_phase_is_rank_one(dim, n):
    # Phi = p(x) + s(xi) makes K = exp(2 pi i p(x)) exp(2 pi i s(xi))^T, so
    # every row is the same functional times a unit phase.
    N = n ** dim
    f = gaussian_vectors(N, 1, 11)
    rows = np.arange(N)
    g = dense_rows(dim, n, "separable", PHASE_PARAMS["separable"], "one", f,
                   rows)[0]
    p0, p1, p2 = PHASE_PARAMS["separable"]
    idx = np.arange(N)
    if dim == 1:
        x1, x2, xi = idx / n, 0.0, (idx - n // 2)[:, None]
    else:
        x1, x2 = (idx // n) / n, (idx % n) / n
        xi = np.stack([idx // n - n // 2, idx % n - n // 2], -1)
    px = p0 * np.sin(2 * np.pi * x1) * (1 + x2)
    nrm2 = np.sum(xi.astype(float) ** 2, -1)
    sx = p1 * np.sqrt(nrm2) + p2 * nrm2 / n
    total = np.sum(np.exp(2j * np.pi * sx) * f[0])
    assert np.max(np.abs(g - np.exp(2j * np.pi * px) * total)) < 1e-9 * abs(
        total)


def _mp_phase(kind, params, ix, jx, n):
    """The phase in 50-digit arithmetic from the workload definitions."""
    mpmath.mp.dps = 50
    x = [mpmath.mpf(int(i)) / n for i in ix]
    xi = [mpmath.mpf(int(j) - n // 2) for j in jx]
    bil = sum(a * b for a, b in zip(x, xi))
    tp = 2 * mpmath.pi
    if kind == "dft":
        return bil
    if kind == "fio1d":
        p0, p1, p2 = [mpmath.mpf(v) for v in params]
        return bil + (p0 + p1 * mpmath.sin(tp * x[0])) / p2 * abs(xi[0])
    if kind == "radon2d":
        p = [mpmath.mpf(v) for v in params]
        c1 = (p[0] + p[1] * mpmath.sin(tp * x[0]) * mpmath.sin(tp * x[1])) / p[2]
        c2 = (p[3] + p[4] * mpmath.cos(tp * x[0]) * mpmath.cos(tp * x[1])) / p[5]
        return bil + mpmath.sqrt(c1 ** 2 * xi[0] ** 2 + c2 ** 2 * xi[1] ** 2)
    if kind == "separable":
        p0, p1, p2 = [mpmath.mpf(v) for v in params]
        x2 = x[1] if len(x) > 1 else 0
        nrm2 = sum(v * v for v in xi)
        return p0 * mpmath.sin(tp * x[0]) * (1 + x2) + p1 * mpmath.sqrt(
            nrm2) + p2 * nrm2 / n
    raise ValueError(kind)


@pytest.mark.parametrize("dim,n,kind,amp", [
    (1, 16, "fio1d", "one"), (1, 16, "fio1d", "sincos"), (1, 8, "dft", "one"),
    (1, 16, "separable", "one"), (2, 4, "radon2d", "one"),
    (2, 4, "radon2d", "sincos"), (2, 4, "separable", "one")])
def test_brute_force_mpmath(dim, n, kind, amp):
    # plain double loop in 50-digit arithmetic, sharing nothing with the
    # vectorised oracle but the workload definitions.
    N = n ** dim
    params = PHASE_PARAMS[kind]
    f = gaussian_vectors(N, 1, 12)[0]
    g = dense_rows(dim, n, kind, params, amp, f[None], np.arange(N))[0]
    mpmath.mp.dps = 50
    for i in range(N):
        ix = [i] if dim == 1 else [i // n, i % n]
        acc = mpmath.mpc(0)
        for j in range(N):
            jx = [j] if dim == 1 else [j // n, j % n]
            ph = _mp_phase(kind, params, ix, jx, n)
            al = mpmath.mpf(1)
            if amp == "sincos":
                al = 1 + mpmath.mpf(0.5) * mpmath.sin(
                    2 * mpmath.pi * mpmath.mpf(ix[0]) / n) * mpmath.cos(
                    2 * mpmath.pi * (jx[0] - n // 2) / mpmath.mpf(n))
            acc += al * mpmath.expjpi(2 * ph) * mpmath.mpc(f[j].real,
                                                           f[j].imag)
        assert abs(complex(acc) - g[i]) < 1e-13 * max(1.0, abs(complex(acc)))


@pytest.mark.parametrize("n", [1 << 18, 1 << 20])
def test_phase_reduction_large_grid(n):
    # the exactly reduced bilinear part plus the FP64 smooth part stays
    # within 1e-9 of a cycle of the 50-digit phase at the largest grids.
    rng = np.random.default_rng(13)
    i = rng.integers(0, n, 40)
    j = rng.integers(0, n, 40)
    t = phase_mod1("fio1d", PHASE_PARAMS["fio1d"], i[:, None], j[:, None], n)
    for k in range(40):
        ref = _mp_phase("fio1d", PHASE_PARAMS["fio1d"], [i[k]], [j[k]], n)
        ref = ref - mpmath.nint(ref)
        d = float(ref) - t[k]
        assert abs(d - round(d)) < 1e-9


@pytest.mark.parametrize("dim,n", [(1, 512), (2, 16)])
def test_amplitude_split_reproduces_alpha(dim, n):
    # eq. (eqn:tg): with alpha = sum_k a_k(x) b_k(xi) the matvec equals
    # sum_k a_k * (K_{alpha=1} (b_k * f)).
    N = n ** dim
    kind = "fio1d" if dim == 1 else "radon2d"
    params = PHASE_PARAMS[kind]
    f = gaussian_vectors(N, 2, 14)
    a, b = amplitude_factors("sincos", dim, n, 4, 15)
    rows = np.arange(0, N, 5)
    g = dense_rows(dim, n, kind, params, "sincos", f, rows)
    acc = 0
    for k in range(4):
        acc = acc + a[k, rows][None, :] * dense_rows(
            dim, n, kind, params, "one", b[k][None, :] * f, rows)
    assert np.max(rel_err(acc, g)) < 1e-13


def test_kernel_entries_unit_modulus_and_block_identity():
    # eq. (eqn:terms): K(A, B) = e^{-2pi i Phi(cA,cB)} diag(e^{2pi i Phi(A,cB)})
    # e^{2pi i R(A,B)} diag(e^{2pi i Phi(cA,B)}) with R from eq. (eqn:RAB).
    n = 256
    K = kernel_rows(1, n, "fio1d", PHASE_PARAMS["fio1d"], "one",
                    np.arange(32, 48))[:, 96:112]
    assert np.allclose(np.abs(K), 1, atol=1e-14)
    A, B = np.arange(32, 48), np.arange(96, 112)
    cA, cB = 32 + 7, 96 + 7
    ph = lambda i, j: phase_mod1("fio1d", PHASE_PARAMS["fio1d"],
                                 np.asarray(i)[..., None],
                                 np.asarray(j)[..., None], n)
    R = (ph(A[:, None], B[None, :]) - ph(cA, B)[None, :]
         - ph(A, cB)[:, None] + ph(cA, cB))
    rebuilt = (np.exp(-2j * np.pi * ph(cA, cB))
               * np.exp(2j * np.pi * ph(A, cB))[:, None]
               * np.exp(2j * np.pi * R)
               * np.exp(2j * np.pi * ph(cA, B))[None, :])
    assert np.allclose(rebuilt, K, atol=1e-12)
