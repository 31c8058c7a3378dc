"""Plant plausible mistakes in the oracle (on the CPU, by monkeypatching) and
check that its pins reject each one.  Nothing here touches the GPU path."""

import numpy as np
import pytest

import oracle.butterfly as bfo
import oracle.kernel as kern
from oracle.dense import dense_rows, rel_err
from synthetic import gaussian_vectors, sample_rows, PHASE_PARAMS


def _pins_pass():
    """A compact subset of the butterfly pins; True when all hold."""
    ok = True
    # exactness at small N (all boxes interpolate through all points)
    for n in (16, 64):
        f = gaussian_vectors(n, 1, 40)
        g = bfo.butterfly_apply(1, n, "fio1d", PHASE_PARAMS["fio1d"], 8, f)
        ref = dense_rows(1, n, "fio1d", PHASE_PARAMS["fio1d"], "one", f,
                         np.arange(n))
        ok &= rel_err(g, ref)[0] < 1e-13
    # separable exactness at a size with interpolating levels
    n = 1024
    f = gaussian_vectors(n, 1, 41)
    g = bfo.butterfly_apply(1, n, "separable", PHASE_PARAMS["separable"], 8, f)
    rows = sample_rows(n, 128, 42)
    ref = dense_rows(1, n, "separable", PHASE_PARAMS["separable"], "one", f,
                     rows)
    ok &= rel_err(g[:, rows], ref)[0] < 1e-12
    # paper's printed error, N = 1024, r_eps = 8: 2.60e-6 (Table tab:1D-FIO)
    params = PHASE_PARAMS["fio1d_paper"]
    g = bfo.butterfly_apply(1, n, "fio1d", params, 8, f)
    ref = dense_rows(1, n, "fio1d", params, "one", f, rows)
    e = rel_err(g[:, rows], ref)[0]
    ok &= 2.6e-6 / 4 < e < 2.6e-6 * 4
    return bool(ok)


def test_unmutated_oracle_passes():
    assert _pins_pass()


def _printed_grid(size, r):
    if size <= r:
        return np.arange(size, dtype=np.int64)
    return bfo.mock_chebyshev_as_printed(size, r) - 1


def _drop_conjugate_twiddles(kind, params, ix, jx, n, sign=1):
    # a lost minus sign: every exp(-2 pi i Phi) becomes exp(+2 pi i Phi)
    return np.exp(2j * np.pi * kern.phase_mod1(kind, params, ix, jx, n))


def _shifted_lagrange(nodes, y):
    # an off-by-one in the node set used by the basis polynomials
    return _ORIG_LAGRANGE(np.asarray(nodes, float) + 1.0, y)


def _contract_drop_imag(Lag, z):
    return _ORIG_CONTRACT(Lag, z.real.astype(complex))


_ORIG_LAGRANGE = bfo.lagrange_1d
_ORIG_CONTRACT = bfo._contract


@pytest.mark.parametrize("name,attr,mutant", [
    ("printed grid formula", "mock_chebyshev", _printed_grid),
    ("lost conjugate sign", "expi_phase", _drop_conjugate_twiddles),
    ("shifted Lagrange nodes", "lagrange_1d", _shifted_lagrange),
    ("dropped imaginary part", "_contract", _contract_drop_imag),
])
def test_pins_reject_mutant(monkeypatch, name, attr, mutant):
    monkeypatch.setattr(bfo, attr, mutant)
    assert not _pins_pass(), name
