"""Exact matvec g = K f on selected rows, FP64 (test infrastructure).

Problem statement (Section 4, the potential g(x) = sum over xi of
K(x, xi) f(xi); Section 5, eq. (eqn:1D-FIO)): the sum is plain, with no
quadrature weight and no 1/N, and the kernel is
K(x, xi) = alpha(x, xi) exp(2 pi i Phi(x, xi)) with alpha taken from its
formula.  Rows are computed one block at a time and accumulated with a BLAS
product in complex128.
"""

import numpy as np

from .kernel import coords, expi_phase, amplitude


def kernel_rows(dim, n, phase_kind, phase_params, amp_kind, rows,
                transpose=False, conjugate=False):
    """Rows ``rows`` of K as a complex128 array (len(rows), N).

    transpose: rows of the transposed matrix K^T (row j holds
    K(x_i, xi_j) for every i); conjugate: conjugated entries (with
    transpose, rows of the adjoint K^H)."""
    N = n ** dim
    r_idx = coords(np.asarray(rows), dim, n)[:, None, :]
    a_idx = coords(np.arange(N), dim, n)[None, :, :]
    ix, jx = (a_idx, r_idx) if transpose else (r_idx, a_idx)
    K = expi_phase(phase_kind, phase_params, ix, jx, n)
    if amp_kind != "one":
        K = K * amplitude(amp_kind, ix, jx, n)
    return np.conj(K) if conjugate else K


def dense_rows(dim, n, phase_kind, phase_params, amp_kind, f, rows,
               block=8, transpose=False, conjugate=False):
    """g[v, rows] = sum_j K[rows, j] f[v, j] for every vector v of ``f``
    (K^T, conj K or K^H with the flags of kernel_rows).

    f: complex array [nvec][N].  Returns complex128 [nvec][len(rows)].
    """
    f = np.atleast_2d(np.asarray(f, np.complex128))
    rows = np.asarray(rows, np.int64)
    out = np.empty((f.shape[0], rows.size), np.complex128)
    for s in range(0, rows.size, block):
        K = kernel_rows(dim, n, phase_kind, phase_params, amp_kind,
                        rows[s:s + block], transpose, conjugate)
        out[:, s:s + block] = f @ K.T
    return out


def rel_err(approx, exact):
    """Relative l2 error over the sampled rows, per vector (Section 5,
    definition of epsilon^b).  approx, exact: [nvec][rows]."""
    approx = np.atleast_2d(approx)
    exact = np.atleast_2d(exact)
    num = np.sqrt(np.sum(np.abs(approx - exact) ** 2, axis=-1))
    den = np.sqrt(np.sum(np.abs(exact) ** 2, axis=-1))
    return num / den


def fourier_coefficients(n, h):
    """Coefficients of the 1D grid function h [nvec][n] in the basis of the
    DFT-phase kernel: hat_j = (1/n) sum_i h_i exp(-2 pi i x_i xi_j) on the
    grid of eq. (eqn:1D-xandxi), so that h_i = sum_j hat_j exp(2 pi i x_i
    xi_j).  This is the transform that turns the output of one FIO of the
    form of eq. (eq:example3) into the input of the next."""
    return dense_rows(1, n, "dft", (), "one", h, np.arange(n),
                      transpose=True, conjugate=True) / n


def composition_rows(n, phase_kind, phase_params, fhat, rows):
    """Rows ``rows`` of g = L(L f) (eq. (eq:example4)), L the FIO of eq.
    (eq:example3) discretized as eq. (eqn:1D-FIO): L maps coefficients hat f
    to grid values K hat f; the inner result is re-expanded into Fourier
    coefficients before the outer L.  fhat: [nvec][n]."""
    inner = dense_rows(1, n, phase_kind, phase_params, "one", fhat,
                       np.arange(n))
    return dense_rows(1, n, phase_kind, phase_params, "one",
                      fourier_coefficients(n, inner), rows)

