"""Factor construction on the GPU, entry by entry.

Every stored twiddle and switch-block entry is exp(2 pi i theta) of a
difference of phase values at interpolation points and box centers (the
xi-level factor of eq. (eqn:2), the switch block of Algorithm 4.1 step 4,
the x-level factor of eq. (eqn:3), regrouped around one real matrix per
level and child), built on the device with an FP64 phase reduced modulo 1
before sincospi and stored as complex64.  For seeded samples of the entries
of every step (bf_factor_entries) this test

* decodes each entry index from the documented layout and derives its boxes,
  points (the oracle's mock_chebyshev) and centers (the lower-middle index)
  from the tree definitions of Section 4: the phase-term indices the library
  reports must equal them exactly;
* evaluates theta in FP64 with the oracle's phase (oracle.kernel.phase_mod1,
  exact bilinear reduction) and requires the stored value to be the
  complex64 rounding of exp(2 pi i theta): per component within half an
  FP32 ulp plus 2e-9 (the FP64 rounding of theta at |Phi| ~ 7e5).

An FP32 phase, a reduction after sincos or a wrong box or point would miss
this bound by orders of magnitude; at N = 2^20 the phase reaches about
0.69 N cycles, where an FP32 ulp is 0.06 of a cycle."""

import numpy as np
import pytest

from _util import log
from oracle.butterfly import mock_chebyshev
from oracle.kernel import phase_mod1
from synthetic import PHASE_PARAMS

pytestmark = pytest.mark.gpu


def _compact(m):
    m = np.asarray(m, np.int64) & 0x55555555
    m = (m | (m >> 1)) & 0x33333333
    m = (m | (m >> 2)) & 0x0F0F0F0F
    m = (m | (m >> 4)) & 0x00FF00FF
    m = (m | (m >> 8)) & 0x0000FFFF
    return m


def _box(m, dim):
    """Box index at a tree level -> per-dimension box coordinates (..., dim)
    (2D: Morton order, first coordinate on the odd bits)."""
    m = np.asarray(m, np.int64)
    if dim == 1:
        return m[..., None]
    return np.stack([_compact(m >> 1), _compact(m)], axis=-1)


def _user(g, n):
    return g[..., 0] if g.shape[-1] == 1 else g[..., 0] * n + g[..., 1]


def _center(bc, side):
    return bc * side + (side - 1) // 2


def _point(bc, side, q, t, dim):
    off = mock_chebyshev(side, q)
    r1 = off.size
    digits = [t] if dim == 1 else [t // r1, t % r1]
    return np.stack([bc[..., d] * side + off[digits[d]] for d in range(dim)],
                    axis=-1)


def _expected_terms(kind, level, L, n, dim, q, idx, r_in, r_out, reads_f,
                    writes_lambda):
    """Phase terms [(x grid coords, xi grid coords)] of entries idx, from
    the layouts of include/bf.h and the trees of Section 4."""
    R = 1 << dim
    if kind == 1:                      # switch at level h: [p][t][s]
        s = idx % r_in
        t = (idx // r_in) % r_out
        p = idx // r_in // r_out
        sh = dim * (L - level)
        A, B = _box(p >> sh, dim), _box(p & ((1 << sh) - 1), dim)
        sA, sB = n >> level, n >> (L - level)
        xt = _point(A, sA, q, t, dim)
        xs = _point(B, sB, q, s, dim)
        terms = [(xt, xs)]
        if not reads_f:
            terms.append((_center(A, sA), xs))
        if not writes_lambda:
            terms.append((xt, _center(B, sB)))
        return terms
    r = r_in if kind == 0 else r_out
    e = idx % r
    rest = idx // r
    c = rest % R
    i = (rest // R) % R
    u = rest // R // R
    sh = dim * (L - level)
    ap, b = u >> sh, u & ((1 << sh) - 1)
    A = _box(ap * R + i, dim)
    if kind == 0:                      # xi level l: [u][i][c][s]
        P = _box(ap, dim)
        C = _box(b * R + c, dim)
        xs = _point(C, n >> (L - level + 1), q, e, dim)
        terms = [(_center(A, n >> level), xs)]
        if not reads_f:
            terms.append((_center(P, n >> (level - 1)), xs))
        return terms
    B = _box(b, dim)                   # x level l: [u][i][c][t]
    C = _box(b * R + c, dim)
    xt = _point(A, n >> level, q, e, dim)
    terms = [(xt, _center(C, n >> (L - level + 1)))]
    if not writes_lambda:
        terms.append((xt, _center(B, n >> (L - level))))
    return terms


def _check_plan(plan, dim, n, kind, params, q, samples, seed):
    import math
    rng = np.random.default_rng(seed)
    L = int(math.log2(n))
    steps = plan.steps()
    xi_steps = [k for k, s in enumerate(steps) if s["kind"] == 0]
    worst = 0.0
    for k, st in enumerate(steps):
        for which, total in (("twiddle", st["tw_entries"]),
                             ("switch", st["S_entries"])):
            if total == 0:
                continue
            m = min(samples, total)
            idx = np.unique(np.concatenate([
                rng.integers(0, total, m), [0, total - 1]])).astype(np.int64)
            x, xi, val = plan.factor_entries(k, which, idx)
            # the schedule: the first xi level reads f (the levels below it
            # are exact copies); the last x level emits lambda
            reads_f = (st["kind"] == 0 and k == xi_steps[0]) or \
                (st["kind"] == 1 and not xi_steps)
            assert bool(st["reads_f"]) == reads_f, (k, st)
            terms = _expected_terms(st["kind"], st["level"], L, n, dim, q,
                                    idx, st["r_in"], st["r_out"],
                                    st["reads_f"], st["writes_lambda"])
            for j in range(3):
                if j < len(terms):
                    assert np.array_equal(x[:, j], _user(terms[j][0], n)), \
                        (k, which, j)
                    assert np.array_equal(xi[:, j], _user(terms[j][1], n)), \
                        (k, which, j)
                else:
                    assert np.all(x[:, j] == -1) and np.all(xi[:, j] == -1)
            theta = phase_mod1(kind, params, terms[0][0], terms[0][1], n)
            for gx, gxi in terms[1:]:
                theta = theta - phase_mod1(kind, params, gx, gxi, n)
            theta = theta - np.round(theta)
            exact = np.exp(2j * np.pi * theta)
            e32 = exact.astype(np.complex64)
            for comp in (np.real, np.imag):
                half_ulp = 0.5 * np.spacing(np.abs(comp(e32)).astype(
                    np.float32)).astype(np.float64)
                d = np.abs(comp(val).astype(np.float64) - comp(exact))
                assert np.all(d <= half_ulp + 2e-9), \
                    (k, which, float(np.max(d - half_ulp)))
                worst = max(worst, float(np.max(d)))
            log(f"  step {k} (kind {st['kind']}, level {st['level']}) "
                f"{which}: {idx.size} of {total} entries exact")
    return worst


@pytest.mark.parametrize("dim,n,kind,q,op", [
    (1, 1 << 20, "fio1d", 10, "N"),     # |Phi| up to ~7e5 cycles
    (1, 1024, "fio1d", 8, "N"),
    (1, 1 << 16, "dft", 10, "N"),
    (2, 256, "radon2d", 7, "N"),
    (2, 64, "separable", 7, "N"),
])
def test_stored_factors_are_exactly_rounded(dim, n, kind, q, op):
    import paper_1803_04128_amd as bfm
    params = PHASE_PARAMS[kind]
    log(f"case factors dim={dim} n={n} {kind} q={q} op={op}")
    with bfm.Plan(dim, n, kind, params, q=q, max_nvec=1, op=op) as pl:
        worst = _check_plan(pl, dim, n, kind, params, q, 4096, 7)
    log(f"  largest |stored - exact| component {worst:.3e}")


def test_factor_entries_argument_errors():
    import paper_1803_04128_amd as bfm
    from paper_1803_04128_amd import BfError
    with bfm.Plan(1, 1024, "fio1d", PHASE_PARAMS["fio1d"], q=8) as pl:
        st = pl.steps()
        sw = next(k for k, s in enumerate(st) if s["kind"] == 1)
        xi0 = next(k for k, s in enumerate(st) if s["kind"] == 0)
        with pytest.raises(BfError):
            pl.factor_entries(xi0, "twiddle", [st[xi0]["tw_entries"]])
        with pytest.raises(BfError):
            pl.factor_entries(xi0, "switch", [0])
        with pytest.raises(BfError):
            pl.factor_entries(len(st), "twiddle", [0])
        pl.factor_entries(sw, "switch", [0, st[sw]["S_entries"] - 1])
