"""The library's Algorithm 6 with Algorithm 1 (bf_lift_decide, host C++)
against the oracle's (oracle/lifting.py) on the same random draws (CPU):
the decision and the sampled numerical rank exactly, the lifted phase
P Q^T (unique: the truncated SVD), and the residual factorization through
what is unique about it, its accuracy on the residual kernel's entries."""

import numpy as np
import pytest

import paper_1803_04128_amd as bfm
from oracle import lifting as ol
from test_oracle_lifting import fio_factors, sincos_factors


def _draws(seed, N, r1, r_eps, q=3, rounds=2, extra=4):
    rng = np.random.default_rng(seed)
    omega = rng.standard_normal((N, r1 + 3))
    test = rng.choice(N, min(N, r_eps * q), replace=False)
    rows = np.stack([rng.choice(N, r_eps * q, replace=False)
                     for _ in range(rounds)])
    cols = np.stack([rng.choice(N, r_eps * q, replace=False)
                     for _ in range(rounds)])
    xr = rng.choice(N, extra, replace=False)
    xc = rng.choice(N, extra, replace=False)
    return omega, test, (rows, cols, xr, xc)


def _approx_err(U1, V1, U2, V2, P, Q, a, b, seed):
    rng = np.random.default_rng(seed)
    N = U1.shape[0]
    i = rng.choice(N, 64, replace=False)
    j = rng.choice(N, 64, replace=False)
    ex = ol.residual_entries(U1, V1, U2, V2, P, Q, i, j)
    ap = a[:, i].T @ b[:, j]
    return np.linalg.norm(ap - ex) / np.linalg.norm(ex)


@pytest.mark.parametrize("case", ["perturbed", "exact_rank2", "refused"])
def test_library_decision_matches_oracle(case):
    N = 512
    if case == "perturbed":
        U1, V1 = fio_factors(N, 0.4)
        U2, V2 = sincos_factors(N)
        r, r_eps, eps = 2, 16, 1e-9
    elif case == "exact_rank2":
        U1, V1 = fio_factors(N, 0.0)
        U2, V2 = np.ones((N, 1)), np.ones((N, 1))
        r, r_eps, eps = 2, 2, 1e-10
    else:
        U1, V1 = fio_factors(N, 0.0)
        U2, V2 = np.ones((N, 1)), np.ones((N, 1))
        r, r_eps, eps = 1, 8, 1e-9
    omega, test, samples = _draws(11, N, U1.shape[1], r_eps)
    y, n, P, Q, a, b = bfm.lift_decide(U1, V1, U2, V2, r, r_eps, eps, omega,
                                       test, samples)
    yo, Po, Qo, ao, bo, no = ol.decide(U1, V1, U2, V2, r, r_eps, eps, omega,
                                       test, (list(samples[0]),
                                              list(samples[1]),
                                              samples[2], samples[3]))
    assert (y, n) == (yo, no)
    PQ, PQo = P @ Q.T, Po @ Qo.T
    assert np.max(np.abs(PQ - PQo)) <= 1e-10 * np.max(np.abs(PQo))
    if case == "refused":
        assert y == 0 and a is None
        return
    assert y == 1
    e_lib = _approx_err(U1, V1, U2, V2, P, Q, a, b, 3)
    e_or = _approx_err(U1, V1, U2, V2, Po, Qo, ao, bo, 3)
    assert e_lib < 1e-7 and e_or < 1e-7, (e_lib, e_or)


def test_lift_decide_argument_errors():
    N = 64
    U1, V1 = fio_factors(N, 0.4)
    ones = np.ones((N, 1))
    omega, test, samples = _draws(1, N, 3, 4)
    with pytest.raises(bfm.BfError):      # r must be below r1
        bfm.lift_decide(U1, V1, ones, ones, 3, 4, 1e-9, omega, test, samples)
    with pytest.raises(bfm.BfError):      # omega needs more than r1 columns
        bfm.lift_decide(U1, V1, ones, ones, 2, 4, 1e-9, omega[:, :3], test,
                        samples)
    bad = np.array(test)
    bad[0] = N
    with pytest.raises(bfm.BfError):      # index out of range
        bfm.lift_decide(U1, V1, ones, ones, 2, 4, 1e-9, omega, bad, samples)
