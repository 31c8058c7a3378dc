"""Pins of the dimension-lifting oracle (oracle/lifting.py: Section 3,
Algorithms 6 and 1, eq. (eqn:tg3)) against what the mathematics fixes:
a library SVD of the dense matrix, exact low-rank matrices, the FFT closed
form of the DFT kernel, the dense FP64 matvec of oracle/dense.py, and
brute-force sums."""

import numpy as np
import pytest

from oracle.dense import dense_rows
from oracle.lifting import (alg1, decide, leading_svd, lifted_matvec,
                            numerical_rank, nufft3_direct, residual_entries)


def _grid(N):
    x = np.arange(N) / N
    xi = (np.arange(N) - N // 2).astype(float)
    return x, xi


def _samples(rng, N, r, q, rounds=2, extra=4):
    rows = [rng.choice(N, r * q, replace=False) for _ in range(rounds)]
    cols = [rng.choice(N, r * q, replace=False) for _ in range(rounds)]
    return (rows, cols, rng.choice(N, extra, replace=False),
            rng.choice(N, extra, replace=False))


def fio_factors(N, delta=0.0):
    """Phi = x xi + c(x)|xi| (+ delta cos(2 pi x) (xi / (N/2))^2), c(x) = (2 +
    sin 2 pi x)/8, as real factors [N][3]; delta = 0 gives an exactly rank-2
    phase with a zero third column, delta > 0 a rank-3 phase whose third
    term stays below delta cycles."""
    x, xi = _grid(N)
    c = (2 + np.sin(2 * np.pi * x)) / 8
    U1 = np.stack([x, c, delta * np.cos(2 * np.pi * x)], 1)
    V1 = np.stack([xi, np.abs(xi), (xi / (N / 2)) ** 2], 1)
    return U1, V1


def sincos_factors(N):
    """alpha = 1 + 0.5 sin(2 pi x) cos(2 pi xi / N) as real factors [N][2]."""
    x, xi = _grid(N)
    return (np.stack([np.ones(N), 0.5 * np.sin(2 * np.pi * x)], 1),
            np.stack([np.ones(N), np.cos(2 * np.pi * xi / N)], 1))


def test_leading_svd_is_the_truncated_svd():
    rng = np.random.default_rng(0)
    N = 96
    U1, V1 = rng.standard_normal((N, 4)), rng.standard_normal((N, 4))
    P, Q, s = leading_svd(U1, V1, 2, rng.standard_normal((N, 7)))
    u, sv, vt = np.linalg.svd(U1 @ V1.T)
    ref = (u[:, :2] * sv[:2]) @ vt[:2]
    assert np.allclose(s[:4], sv[:4], rtol=1e-12)
    assert np.max(np.abs(P @ Q.T - ref)) < 1e-10 * sv[0]
    assert np.allclose(Q.T @ Q, np.eye(2), atol=1e-12)


def test_numerical_rank_of_exact_low_rank_matrices():
    rng = np.random.default_rng(1)
    for k in (1, 3, 6):
        M = (rng.standard_normal((80, k)) + 1j * rng.standard_normal((80, k))) \
            @ rng.standard_normal((k, 20))
        assert numerical_rank(M, 1e-10) == k


def test_alg1_reproduces_a_low_rank_matrix():
    rng = np.random.default_rng(2)
    m, n, k = 120, 100, 5
    A = (rng.standard_normal((m, k)) + 1j * rng.standard_normal((m, k))) @ \
        (rng.standard_normal((k, n)) + 1j * rng.standard_normal((k, n)))

    def entries(rows, cols):
        return A[np.ix_(rows, cols)]

    for r in (5, 8):
        rows = [rng.choice(m, 4 * r, replace=False) for _ in range(2)]
        cols = [rng.choice(n, 4 * r, replace=False) for _ in range(2)]
        U0, s, V0 = alg1(entries, m, n, r, rows, cols,
                         rng.choice(m, 5, replace=False),
                         rng.choice(n, 5, replace=False))
        err = np.linalg.norm(U0 @ np.diag(s) @ V0.conj().T - A) / \
            np.linalg.norm(A)
        assert err < 1e-10, (r, err)
        assert np.allclose(s[:k], np.linalg.svd(A, compute_uv=False)[:k],
                           rtol=1e-9)


def test_exact_rank_two_phase_lifts_to_rank_one_residual():
    # the FIO phase of the 1D workloads is exactly x xi + c(x)|xi|: with a
    # zero third factor column, P Q^T reproduces it, the residual kernel is
    # the amplitude (alpha = 1: all ones), and the NUFFT path applies with
    # r_eps = 1; its apply equals the dense matvec
    rng = np.random.default_rng(3)
    N = 256
    U1, V1 = fio_factors(N, 0.0)
    U2, V2 = np.ones((N, 1)), np.ones((N, 1))
    y, P, Q, a, b, n = decide(U1, V1, U2, V2, 2, 1, 1e-10,
                              rng.standard_normal((N, 6)),
                              rng.choice(N, 8, replace=False),
                              _samples(rng, N, 1, 4))
    assert y == 1 and n == 1
    f = rng.standard_normal((2, N)) + 1j * rng.standard_normal((2, N))
    g = lifted_matvec(P, Q, a, b, f)
    ref = dense_rows(1, N, "fio1d", (2.0, 1.0, 8.0), "one", f, np.arange(N))
    assert np.linalg.norm(g - ref) / np.linalg.norm(ref) < 1e-9


def test_dft_phase_matches_the_fft_closed_form():
    # Phi = x xi (rank 1, padded by a zero column): K f = N (-1)^i ifft(f)
    rng = np.random.default_rng(4)
    N = 128
    x, xi = _grid(N)
    U1 = np.stack([x, np.zeros(N)], 1)
    V1 = np.stack([xi, np.zeros(N)], 1)
    ones = np.ones((N, 1))
    y, P, Q, a, b, _ = decide(U1, V1, ones, ones, 1, 1, 1e-10,
                              rng.standard_normal((N, 4)),
                              rng.choice(N, 4, replace=False),
                              _samples(rng, N, 1, 4))
    assert y == 1
    f = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    g = lifted_matvec(P, Q, a, b, f)[0]
    ref = N * (-1.0) ** np.arange(N) * np.fft.ifft(f)
    assert np.linalg.norm(g - ref) / np.linalg.norm(ref) < 1e-10


def test_perturbed_phase_with_amplitude_against_dense():
    # rank-3 phase x xi + c(x)|xi| + delta cos(2 pi x)(xi/(N/2))^2 and the
    # sincos amplitude (rank 2): lifting to r = 2 leaves a smooth residual of
    # small numerical rank; eq. (eqn:tg3) with Algorithm 1's factors matches
    # the dense matvec to the factorization's accuracy
    rng = np.random.default_rng(5)
    N = 512
    U1, V1 = fio_factors(N, 0.4)
    U2, V2 = sincos_factors(N)
    r_eps = 16
    y, P, Q, a, b, n = decide(U1, V1, U2, V2, 2, r_eps, 1e-9,
                              rng.standard_normal((N, 8)),
                              rng.choice(N, 4 * r_eps, replace=False),
                              _samples(rng, N, r_eps, 3))
    assert y == 1 and 2 <= n <= r_eps
    f = rng.standard_normal((2, N)) + 1j * rng.standard_normal((2, N))
    g = lifted_matvec(P, Q, a, b, f)
    rows = np.arange(N)
    from oracle.kernel import amplitude  # noqa: F401  (formula amplitude)
    ref = dense_rows(1, N, "lowrank", (U1, V1), "sincos", f, rows)
    err = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    assert err < 1e-7, err
    # the residual entries themselves: exactly alpha exp(2 pi i (Phi - PQ^T))
    i, j = rng.integers(0, N, 5), rng.integers(0, N, 5)
    e = residual_entries(U1, V1, U2, V2, P, Q, i, j)
    x, xi = _grid(N)
    alpha = 1 + 0.5 * np.sin(2 * np.pi * x[i])[:, None] * \
        np.cos(2 * np.pi * xi[j] / N)[None, :]
    phi = U1[i] @ V1[j].T
    assert np.allclose(e, alpha * np.exp(2j * np.pi * (phi - P[i] @ Q[j].T)),
                       rtol=1e-12, atol=1e-12)


def test_fio_phase_without_lifting_is_refused():
    # r = 1 keeps only x xi-like part: exp(2 pi i c(x)|xi|) with c ~ 1/4
    # oscillates about N/8 times across the matrix, far beyond a small rank
    rng = np.random.default_rng(6)
    N = 512
    U1, V1 = fio_factors(N, 0.0)
    ones = np.ones((N, 1))
    r_eps = 8
    y, *_ , n = decide(U1, V1, ones, ones, 1, r_eps, 1e-9,
                       rng.standard_normal((N, 6)),
                       rng.choice(N, 4 * r_eps, replace=False),
                       _samples(rng, N, r_eps, 3))
    assert y == 0 and n > r_eps


def test_nufft3_direct_brute_force():
    rng = np.random.default_rng(7)
    t = rng.uniform(-3, 3, (5, 2))
    s = rng.uniform(-20, 20, (7, 2))
    c = rng.standard_normal(7) + 1j * rng.standard_normal(7)
    g = nufft3_direct(t, s, c)[0]
    for i in range(5):
        ref = sum(c[j] * np.exp(2j * np.pi * (t[i] @ s[j])) for j in range(7))
        assert abs(g[i] - ref) < 1e-12


def test_mutant_dropped_residual_is_caught():
    # planting P Q^T = U1 V1^T minus its third singular component as the
    # whole phase (dropping the residual exponential) misses the dense
    # matvec: the pins above would fail on such a mistake
    rng = np.random.default_rng(8)
    N = 256
    U1, V1 = fio_factors(N, 0.4)
    ones = np.ones((N, 1))
    P, Q, _ = leading_svd(U1, V1, 2, rng.standard_normal((N, 6)))
    f = rng.standard_normal((1, N)) + 1j * rng.standard_normal((1, N))
    g_bad = lifted_matvec(P, Q, np.ones((1, N)), np.ones((1, N)), f)
    ref = dense_rows(1, N, "lowrank", (U1, V1), "one", f, np.arange(N))
    assert np.linalg.norm(g_bad - ref) / np.linalg.norm(ref) > 1e-2
