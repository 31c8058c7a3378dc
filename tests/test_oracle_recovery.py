"""Pins for the oracle's phase recovery under indirect access (Section 3.2:
Algorithms 3, 4 and 5 with the factorization of Algorithm 1): unwrapping
of known smooth and piecewise-smooth vectors, exact recovery of low-rank
matrices from sampled rows and columns, and end-to-end recovery of known
phases from their values modulo 1."""

import numpy as np
import pytest

import oracle.recovery as rec
from oracle.butterfly import butterfly_apply
from oracle.kernel import coords, phase_mod1
from oracle.dense import rel_err
from synthetic import PHASE_PARAMS, gaussian_vectors


def _frac(x):
    return x - np.round(x)


def test_unwrap_smooth_vector_up_to_an_integer():
    # slope 0.37 per step plus smooth terms: the continuation returns v
    # itself up to one integer constant
    i = np.arange(3000)
    t = i / i.size
    v = 0.37 * i + 40 * t * t + 3 * np.sin(4 * np.pi * t)
    w, S = rec.unwrap_vector(_frac(v), np.pi / 2)
    d = w - v
    assert np.all(S == [0])
    assert np.max(np.abs(d - np.round(d[0]))) < 1e-9


def test_unwrap_aliased_slope_stays_smooth():
    # a slope of 0.7 cycles per step is seen as -0.3: the result agrees with
    # v modulo 1 and keeps a constant first difference
    i = np.arange(2000)
    v = 0.7 * i + 0.123
    w, S = rec.unwrap_vector(_frac(v), np.pi / 2)
    assert np.max(np.abs(_frac(w - v))) < 1e-9
    assert np.max(np.abs(np.diff(w, 2))) < 1e-9
    assert np.allclose(np.diff(w), -0.3)


def test_unwrap_detects_a_kink_and_restarts():
    # slope 0.1 then 0.45: the second difference 0.35 cycles (2.2 rad)
    # exceeds tau = pi/2 at the kink; both pieces come back exactly
    i = np.arange(1000)
    v = np.where(i < 500, 0.1 * i, 0.1 * 499 + 0.45 * (i - 499))
    w, S = rec.unwrap_vector(_frac(v), np.pi / 2)
    assert list(S) == [0, 500]
    d = w - v
    assert np.max(np.abs(d - np.round(d[0]))) < 1e-9


def test_unwrap_keeps_fixed_entries():
    i = np.arange(200)
    v = 0.2 * i + 0.01 * i * i / 200
    u = _frac(v)
    w, _ = rec.unwrap_vector(u, 2 * np.pi, fixed={0: v[0] + 5, 1: v[1] + 5,
                                                  2: v[2] + 5})
    assert np.max(np.abs(w - (v + 5))) < 1e-9


def test_nearest_representative():
    assert rec.nearest(0.25, 3.1) == 3.25
    assert rec.nearest(0.25, 2.6) == 2.25
    assert rec.nearest(-0.4, 0.3) == 0.6


@pytest.mark.parametrize("rank", [1, 3, 6])
def test_lowrank_from_samples_exact_for_low_rank(rank):
    # Algorithm 1 on a matrix of exact rank k reproduces it everywhere
    rng = np.random.default_rng(120 + rank)
    N = 2000
    A = rng.standard_normal((N, rank))
    B = rng.standard_normal((N, rank))
    Psi = A @ B.T
    Cs = np.sort(rng.choice(N, 3 * rank + 4, replace=False))
    Rs = np.sort(rng.choice(N, 3 * rank + 4, replace=False))
    U, V = rec.lowrank_from_samples(Psi[:, Cs], Psi[Rs, :], Cs, Rs, 8)
    assert U.shape[1] == rank
    assert np.max(np.abs(U @ V.T - Psi)) < 1e-9 * np.max(np.abs(Psi))


def _samplers(kind, params, N):
    allx = coords(np.arange(N), 1, N)

    def cols(idx):
        j = coords(np.asarray(idx), 1, N)
        return phase_mod1(kind, params, allx[:, None, :], j[None, :, :], N)

    def rows(idx):
        i = coords(np.asarray(idx), 1, N)
        return phase_mod1(kind, params, i[:, None, :], allx[None, :, :], N)
    return cols, rows


def _true_phase(kind, params, N, i, j):
    x = np.asarray(i) / N
    xi = np.asarray(j) - N // 2
    ph = np.outer(x, xi).astype(np.float64)
    if kind == "fio1d":
        c = (params[0] + params[1] * np.sin(2 * np.pi * x)) / params[2]
        ph = ph + np.outer(c, np.abs(xi))
    return ph


@pytest.mark.parametrize("params", [PHASE_PARAMS["fio1d_paper"],
                                    PHASE_PARAMS["fio1d"]])
def test_unwrap_samples_consistent_and_integer_offset(params):
    N = 4096
    sc, sr = _samplers("fio1d", params, N)
    rng = np.random.default_rng(130)
    C = np.sort(rng.choice(N, 20, replace=False))
    R = np.sort(rng.choice(N, 20, replace=False))
    Cs, cols, Rs, rows = rec.unwrap_samples(C, R, np.pi / 2, sc, sr)
    assert set(C) <= set(Cs) and set(R) <= set(Rs)
    # rows and columns agree where they meet
    assert np.array_equal(cols[Rs, :], rows[:, Cs])
    # equal to the samples modulo 1
    assert np.max(np.abs(_frac(cols - sc(Cs)))) < 1e-9
    assert np.max(np.abs(_frac(rows - sr(Rs)))) < 1e-9
    # an integer-valued offset from the true phase, of low rank
    E = cols - _true_phase("fio1d", params, N, np.arange(N), Cs)
    assert np.max(np.abs(E - np.round(E))) < 1e-8
    s = np.linalg.svd(rows[:, Cs], compute_uv=False)
    assert np.sum(s > 1e-9 * s[0]) <= 4


@pytest.mark.parametrize("kind,params", [("fio1d", PHASE_PARAMS["fio1d_paper"]),
                                         ("fio1d", PHASE_PARAMS["fio1d"]),
                                         ("dft", ())])
@pytest.mark.parametrize("N", [1024, 4096])
def test_recover_phase_reproduces_the_kernel(kind, params, N):
    # Algorithm 5 end to end: exp(2 pi i U V^T) equals exp(2 pi i Phi) on
    # entries that were never sampled
    sc, sr = _samplers(kind, params, N)
    U, V = rec.recover_phase(N, 8, 3, 5, sc, sr)
    assert U.shape[1] <= 4
    rng = np.random.default_rng(140)
    i, j = rng.integers(0, N, 4000), rng.integers(0, N, 4000)
    psi = np.sum(U[i] * V[j], axis=1)
    ph = phase_mod1(kind, params, coords(i, 1, N), coords(j, 1, N), N)
    assert np.max(np.abs(np.exp(2j * np.pi * psi) -
                         np.exp(2j * np.pi * ph))) < 1e-9


def test_recovered_factors_drive_the_butterfly():
    # the butterfly of the recovered low-rank phase equals the butterfly of
    # the original phase (same kernel, same factorization)
    N, q = 4096, 8
    params = PHASE_PARAMS["fio1d_paper"]
    sc, sr = _samplers("fio1d", params, N)
    U, V = rec.recover_phase(N, 8, 3, 6, sc, sr)
    f = gaussian_vectors(N, 1, 141)
    g = butterfly_apply(1, N, "lowrank", (U, V), q, f)
    ref = butterfly_apply(1, N, "fio1d", params, q, f)
    assert rel_err(g, ref)[0] < 1e-8


def test_threshold_read_in_cycles_fails_for_the_wide_fio(monkeypatch):
    # the pins separate the readings of tau: compared with the second
    # difference in cycles, the kink of the wider FIO phase goes undetected
    # and the recovery breaks
    orig = rec.unwrap_vector

    def cycles(u, tau, fixed=None):
        return orig(u, 2 * np.pi * tau, fixed)
    monkeypatch.setattr(rec, "unwrap_vector", cycles)
    N = 4096
    sc, sr = _samplers("fio1d", PHASE_PARAMS["fio1d"], N)
    U, V = rec.recover_phase(N, 8, 3, 5, sc, sr)
    rng = np.random.default_rng(142)
    i, j = rng.integers(0, N, 2000), rng.integers(0, N, 2000)
    psi = np.sum(U[i] * V[j], axis=1)
    ph = phase_mod1("fio1d", PHASE_PARAMS["fio1d"], coords(i, 1, N),
                    coords(j, 1, N), N)
    assert np.max(np.abs(np.exp(2j * np.pi * psi) -
                         np.exp(2j * np.pi * ph))) > 1e-3
