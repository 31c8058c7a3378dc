"""NUFFT by dimension lifting and the decision between it and the butterfly
(Section 3, eqs. (eqn:tg2), (eqn:tg3), (eqn:minexp); Algorithm 6
(alg:dc); Algorithm 1 (alg:rlr)), in plain NumPy/SciPy, FP64.  Test
infrastructure only: tests/ and the benchmark's CPU baseline use it; the
library never does.

The method, for a kernel K(x_i, xi_j) = alpha(x_i, xi_j) exp(2 pi i
Phi(x_i, xi_j)) on N x N points given by real low-rank factors of its phase,
Phi ~ U1 V1^T (rank r1), and of its amplitude, A ~ U2 V2^T (rank r2):

1. the leading rank-r part P Q^T of U1 V1^T (randomized truncated SVD with
   a test matrix of more than r1 columns, P scaled by the singular values);
2. the residual kernel Kres = (U2 V2^T) . exp(2 pi i (U1 V1^T - P Q^T));
   the numerical rank of sampled columns of Kres (pivoted QR) decides
   whether the NUFFT path applies;
3. if it does, Algorithm 1 factors Kres ~ sum_k a_k b_k^T (rank r_eps), and
   g = K f ~ sum_k a_k . E (b_k . f) with E(i, j) = exp(2 pi i P_i . Q_j):
   r_eps applications of an r-dimensional type-3 NUFFT (eq. (eqn:tg3)).

Every random choice (the test matrix, the sampled columns, the sampled rows
and columns of Algorithm 1) is an input.  Reading: the printed test
samples r q columns and accepts when their numerical rank n is below r, the
lifting dimension; with r = 1 that could never succeed, and the rank that
matters is the r_eps of the sum in eq. (eqn:tg3) the algorithm returns.  It
is read as: sample r_eps q columns, accept when n <= r_eps.
"""

import numpy as np
import scipy.linalg

TWO_PI = 2.0 * np.pi


def leading_svd(U1, V1, r, omega):
    """Step 1 of Algorithm 6: the rank-r truncated SVD of the rank-r1 matrix
    U1 V1^T by a randomized range finder with test matrix omega [N][m],
    m > r1 (the range of U1 V1^T is captured exactly).  Returns P [N][r]
    (left singular vectors times singular values), Q [N][r] (right singular
    vectors) and the singular values."""
    Y = U1 @ (V1.T @ omega)                      # N x m, range of U1 V1^T
    Qy, _ = np.linalg.qr(Y)
    B = (Qy.T @ U1) @ V1.T                       # m x N
    Ub, s, Vt = np.linalg.svd(B, full_matrices=False)
    P = (Qy @ Ub[:, :r]) * s[:r]
    Q = Vt[:r].T
    return P, Q, s


def residual_entries(U1, V1, U2, V2, P, Q, rows, cols):
    """Kres(rows, cols) = (U2 V2^T) . exp(2 pi i (U1 V1^T - P Q^T)) on the
    given index sets (outer product), complex128."""
    rows = np.asarray(rows, np.int64)
    cols = np.asarray(cols, np.int64)
    ph = U1[rows] @ V1[cols].T - P[rows] @ Q[cols].T
    amp = U2[rows] @ V2[cols].T
    return amp * np.exp(TWO_PI * 1j * ph)


def numerical_rank(M, eps):
    """Number of diagonal entries of R in the pivoted QR of M larger than
    |R(1,1)| eps (step 3 of Algorithm 6)."""
    R = scipy.linalg.qr(M, mode="r", pivoting=True)[0]
    d = np.abs(np.diag(R))
    return int(np.sum(d > d[0] * eps)) if d.size and d[0] > 0 else 0


def _pivots(M, count):
    """Indices of the first `count` pivot columns of a pivoted QR of M."""
    piv = scipy.linalg.qr(M, mode="r", pivoting=True)[1]
    return piv[:count]


def alg1(entries, m, n, r, row_samples, col_samples, extra_rows,
         extra_cols):
    """Algorithm 1 (randomized sampling for a rank-r approximate SVD) of an
    m x n matrix known through entries(rows, cols).  row_samples[t],
    col_samples[t]: the random rows and columns of round t (each round
    alternates once between finding important columns from sampled rows
    and important rows from sampled columns); extra_rows, extra_cols: the
    extra samples of the core matrix.  Returns U0 [m][k], s [k], V0 [n][k] with K ~ U0
    diag(s) V0^H, k <= r."""
    pi_col = np.zeros(0, np.int64)
    pi_row = np.zeros(0, np.int64)
    all_r = np.arange(m)
    all_c = np.arange(n)
    for rs, cs in zip(row_samples, col_samples):
        I = np.union1d(rs, pi_row)
        # important columns: pivots of a pivoted QR of K(I, :)
        pi_col = np.sort(_pivots(entries(I, all_c), r))
        J = np.union1d(cs, pi_col)
        # important rows: pivots of a pivoted LQ of K(:, J), i.e. of the
        # pivoted QR of K(:, J)^H
        pi_row = np.sort(_pivots(entries(all_r, J).conj().T, r))
    Kc = entries(all_r, pi_col)
    Qc = scipy.linalg.qr(Kc, mode="economic", pivoting=True)[0][:, :r]
    Kr = entries(pi_row, all_c)
    Qr = scipy.linalg.qr(Kr.conj().T, mode="economic", pivoting=True)[0][:, :r]
    J = np.union1d(pi_col, extra_cols)
    I = np.union1d(pi_row, extra_rows)
    M = np.linalg.pinv(Qc[I]) @ entries(I, J) @ np.linalg.pinv(Qr.conj().T[:, J])
    Um, s, Vmh = np.linalg.svd(M)
    k = min(r, s.size)
    return Qc @ Um[:, :k], s[:k], (Vmh[:k] @ Qr.conj().T).conj().T


def decide(U1, V1, U2, V2, r, r_eps, eps, omega, test_cols, alg1_samples):
    """Algorithm 6.  alg1_samples = (row_samples, col_samples, extra_rows,
    extra_cols) for Algorithm 1.  Returns (y, P, Q, a, b, n): y = 1 when the
    numerical rank n of the sampled residual columns test_cols is at most
    r_eps, and then a, b [k][N] (complex) with Kres ~ sum_k a_k b_k^T
    (k <= r_eps); else a = b = None."""
    N = U1.shape[0]
    P, Q, _ = leading_svd(U1, V1, r, omega)
    M = residual_entries(U1, V1, U2, V2, P, Q, np.arange(N), test_cols)
    n = numerical_rank(M, eps)
    if n > r_eps:
        return 0, P, Q, None, None, n

    def entries(rows, cols):
        return residual_entries(U1, V1, U2, V2, P, Q, rows, cols)

    U0, s, V0 = alg1(entries, N, N, r_eps, *alg1_samples)
    a = (U0 * s).T                     # a_k(x_i)
    b = V0.conj().T                    # b_k(xi_j): Kres ~ U0 S V0^H
    return 1, P, Q, a, b, n


def lifted_matvec(P, Q, a, b, f, rows=None, block=256):
    """Eq. (eqn:tg3) summed directly: g_v = sum_k a_k . E (b_k . f_v),
    E(i, j) = exp(2 pi i P_i . Q_j), FP64 (the exact result the r-dimensional
    type-3 NUFFTs approximate), at the given rows (default all).
    f: [nvec][N]; returns [nvec][len(rows)]."""
    f = np.atleast_2d(np.asarray(f, np.complex128))
    N = P.shape[0]
    rows = np.arange(N) if rows is None else np.asarray(rows, np.int64)
    g = np.zeros((f.shape[0], rows.size), np.complex128)
    for s in range(0, rows.size, block):
        ri = rows[s:s + block]
        E = np.exp(TWO_PI * 1j * (P[ri] @ Q.T))      # the block's rows of E
        for k in range(a.shape[0]):
            g[:, s:s + block] += a[k, ri] * ((f * b[k]) @ E.T)
    return g


def nufft3_direct(t, s, c):
    """The type-3 sum g_i = sum_j c_j exp(2 pi i t_i . s_j) directly (t [M][r],
    s [N][r], c [nvec][N]); the NUFFT's own oracle."""
    c = np.atleast_2d(np.asarray(c, np.complex128))
    E = np.exp(TWO_PI * 1j * (np.atleast_2d(t) @ np.atleast_2d(s).T))
    return c @ E.T
