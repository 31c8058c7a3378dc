"""Grid, phase, amplitude and kernel entries in FP64 (test infrastructure).

Discretisation (Section 5, eq. (eqn:1D-FIO) and eq. (eqn:1D-xandxi)): per
dimension x_i = i / n and xi_j = j - n/2 for 0-based i, j in [0, n).  The 2D
grids use the same rule in each coordinate; a 2D point is addressed by its
row-major user index i1 * n + i2.

The phase is evaluated from integer grid indices.  Its bilinear part
x . xi = sum_d i_d (j_d - n/2) / n is reduced modulo 1 exactly, with the
integer product taken modulo n before the division; the remaining smooth part
is added in FP64 and the sum is reduced to [-1/2, 1/2] before the exponential.
Only the fractional part of the phase matters for exp(2 pi i Phi).

Phase kind "lowrank" (Algorithm 2's input form) takes params = (U, V), real
[N][rank] factors in user index order, and Phi(x_i, xi_j) = U[i] . V[j] in
FP64 with no separate bilinear term.
"""

import numpy as np

TWO_PI = 2.0 * np.pi
# phase kinds whose formula contains the bilinear term x . xi
BILINEAR_KINDS = ("dft", "fio1d", "radon2d", "fio1d_warp")


def coords(user_idx, dim, n):
    """User index -> per-dimension grid index, shape (..., dim)."""
    user_idx = np.asarray(user_idx, dtype=np.int64)
    if dim == 1:
        return user_idx[..., None]
    return np.stack([user_idx // n, user_idx % n], axis=-1)


def _bilinear_frac(ix, jx, n):
    """Fractional part of x . xi for integer x-index ix and xi-index jx, both
    of shape (..., dim); exact (the product is an integer reduced mod n)."""
    prod = np.zeros(np.broadcast_shapes(ix.shape, jx.shape)[:-1], np.int64)
    for d in range(ix.shape[-1]):
        prod = (prod + ix[..., d] * (jx[..., d] - n // 2)) % n
    return prod.astype(np.float64) / n


def _user_index(g, n):
    """Per-dimension grid index (..., dim) -> user index (row-major in 2D)."""
    return g[..., 0] if g.shape[-1] == 1 else g[..., 0] * n + g[..., 1]


def _smooth(kind, params, ix, jx, n):
    """Non-bilinear part of the phase (FP64).  ix, jx: (..., dim) integers."""
    if kind == "lowrank":
        # Algorithm 2's input form: Phi(m, n) = U(m, :) V(n, :)^T with real
        # factors, evaluated entry by entry
        U, V = params
        i, j = _user_index(ix, n), _user_index(jx, n)
        return np.sum(U[i] * V[j], axis=-1)
    x = ix.astype(np.float64) / n
    xi = (jx - n // 2).astype(np.float64)
    if kind == "dft":
        return np.zeros(np.broadcast_shapes(ix.shape, jx.shape)[:-1])
    if kind == "fio1d":
        p0, p1, p2 = params
        c = (p0 + p1 * np.sin(TWO_PI * x[..., 0])) / p2
        return c * np.abs(xi[..., 0])
    if kind == "fio1d_warp":
        # eq. (eqn:FIOK2): Phi = x xi + c(x) xi (the composition example)
        p0, p1, p2 = params
        c = (p0 + p1 * np.sin(TWO_PI * x[..., 0])) / p2
        return c * xi[..., 0]
    if kind == "radon2d":
        p0, p1, p2, p3, p4, p5 = params
        s1, s2 = np.sin(TWO_PI * x[..., 0]), np.sin(TWO_PI * x[..., 1])
        k1, k2 = np.cos(TWO_PI * x[..., 0]), np.cos(TWO_PI * x[..., 1])
        c1 = (p0 + p1 * s1 * s2) / p2
        c2 = (p3 + p4 * k1 * k2) / p5
        return np.sqrt(c1 * c1 * xi[..., 0] ** 2 + c2 * c2 * xi[..., 1] ** 2)
    if kind == "separable":
        p0, p1, p2 = params
        x2 = x[..., 1] if x.shape[-1] > 1 else 0.0
        px = p0 * np.sin(TWO_PI * x[..., 0]) * (1.0 + x2)
        nrm2 = np.sum(xi * xi, axis=-1)
        return px + p1 * np.sqrt(nrm2) + p2 * nrm2 / n
    raise ValueError(kind)


def phase_mod1(kind, params, ix, jx, n):
    """Phi(x_ix, xi_jx) reduced to [-1/2, 1/2]; ix, jx integer (..., dim)."""
    ix = np.asarray(ix, np.int64)
    jx = np.asarray(jx, np.int64)
    t = _smooth(kind, params, ix, jx, n)
    if kind in BILINEAR_KINDS:
        t = t + _bilinear_frac(ix, jx, n)
    return t - np.round(t)


def expi_phase(kind, params, ix, jx, n, sign=1):
    """exp(sign * 2 pi i Phi(x_ix, xi_jx)) in complex128."""
    t = phase_mod1(kind, params, ix, jx, n)
    return np.exp((sign * TWO_PI) * 1j * t)


def amplitude(kind, ix, jx, n):
    """alpha(x_ix, xi_jx) from its formula (not from low-rank factors)."""
    ix = np.asarray(ix, np.int64)
    jx = np.asarray(jx, np.int64)
    shape = np.broadcast_shapes(ix.shape, jx.shape)[:-1]
    if kind == "one":
        return np.ones(shape)
    if kind == "sincos":
        x1 = ix[..., 0] / n
        xi1 = (jx[..., 0] - n // 2).astype(np.float64)
        return 1.0 + 0.5 * np.sin(TWO_PI * x1) * np.cos(TWO_PI * xi1 / n)
    raise ValueError(kind)
