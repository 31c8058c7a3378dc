"""Low-rank phase recovery under indirect access (test infrastructure only:
tests/ and the benchmark's CPU baseline may use it; the library never does).

Section 3.2 recovers a low-rank phase Psi with exp(2 pi i Psi) = K / |K|
from O(1) sampled rows and columns of K (Scenarios 1 and 2 of Table
(tab:sc)), since the samples only fix Phi modulo 1:

* ``unwrap_vector``: Algorithm 3 (alg:sst2), vector recovery by
  third-order continuation with discontinuity detection;
* ``unwrap_samples``: Algorithm 4 (alg:sst), rows and columns that agree
  where they intersect (1D phases);
* ``lowrank_from_samples``: the randomized factorization of Algorithm 1
  (alg:rlr) restricted to the sampled rows and columns;
* ``recover_phase``: Algorithm 5 (alg:idrLR).

Phases are in cycles (the fraction of Phi that exp(2 pi i Phi) sees), indices
are 0-based.  The plain NumPy/SciPy steps follow the algorithms' order; they
share no code with the library.
"""

import numpy as np
import scipy.linalg


def nearest(u, target):
    """The representative of u modulo 1 nearest to target: u + round(target
    - u) (ties away from zero)."""
    d = target - u
    return u + np.copysign(np.floor(np.abs(d) + 0.5), d)


def unwrap_vector(u, tau, fixed=None):
    """Algorithm 3: v with v = u modulo 1, continued with matched second
    differences, and the discontinuity set S (0-based, S[0] = 0).

    fixed: optional {index: value} of entries already assigned (equal to u
    modulo 1); they replace the continuation where they occur, as Algorithm
    4 requires when rows and columns must agree on their intersections.
    """
    u = np.asarray(u, np.float64)
    N = u.size
    v = np.empty(N)
    fixed = fixed or {}
    S = [0]
    c = 0

    def put(a, value):
        v[a] = fixed[a] if a in fixed else value

    while c < len(S):
        st = S[c]
        ed = S[c + 1] - 1 if c + 1 < len(S) else N - 1
        if c == 0:
            # the first two entries as close as possible
            put(st, fixed.get(st, u[st]))
            if st + 1 <= ed:
                put(st + 1, nearest(u[st + 1], v[st]))
            # the third continues the first difference
            if st + 2 <= ed:
                put(st + 2, nearest(u[st + 2], 2 * v[st + 1] - v[st]))
            bg = st + 3
        else:
            # the entry after a discontinuity closest to its predecessor,
            # the next one continuing that difference
            put(st, nearest(u[st], v[st - 1]))
            if st + 1 <= ed:
                put(st + 1, nearest(u[st + 1], 2 * v[st] - v[st - 1]))
            bg = st + 2
        for a in range(bg, ed + 1):
            # equal second differences: v(a) - 2 v(a-1) + v(a-2) as close as
            # possible to v(a-1) - 2 v(a-2) + v(a-3)
            p = 3 * v[a - 1] - 3 * v[a - 2] + v[a - 3]
            put(a, nearest(u[a], p))
            # tau is an angle (the paper's value is pi / 2): compared with
            # the second difference of the phase in radians
            if 2 * np.pi * abs(v[a] + v[a - 2] - 2 * v[a - 1]) > tau:
                S.append(a)
                break
        c += 1
    return v, np.asarray(S, np.int64)


def _block_bounds(S, N):
    b = list(S) + [N]
    return [(b[i], b[i + 1]) for i in range(len(S))]


def unwrap_samples(C, R, tau, sample_cols, sample_rows):
    """Algorithm 4 for a 1D phase (x along rows, xi along columns).

    Samples come through the callbacks sample_cols(idx) -> [N][len(idx)]
    and sample_rows(idx) -> [len(idx)][N], phases modulo 1.  C, R: the randomly sampled column and row indices.
    Returns (Cs, cols, Rs, rows): sorted index arrays and the recovered
    columns Psi(:, Cs) [N][|Cs|] and rows Psi(Rs, :) [|Rs|][N], equal to the
    samples modulo 1 and to each other where they intersect."""
    C = [int(c) for c in C]
    R = [int(r) for r in R]
    first_col = sample_cols([C[0]])[:, 0]
    N = first_col.size
    # discontinuities down the first column split the rows ...
    _, Sr = unwrap_vector(first_col, tau)
    R = sorted(set(R) | set(int(s) for s in Sr))
    first_row = sample_rows([R[0]])[0]
    # ... and along the first row the columns
    _, Sc = unwrap_vector(first_row, tau)
    row_blocks = _block_bounds(Sr, N)
    col_blocks = _block_bounds(Sc, N)
    # every block's first three columns and first three rows are needed
    extra = set(int(s) for s in Sc)
    for c0, c1 in col_blocks:
        extra |= {c for c in (c0 + 1, c0 + 2) if c < c1}
    extra_r = set()
    for r0, r1 in row_blocks:
        extra_r |= {r for r in (r0 + 1, r0 + 2) if r < r1}
    Cs = np.asarray(sorted(set(C) | extra), np.int64)
    Rs = np.asarray(sorted(set(R) | extra_r), np.int64)
    ucol = sample_cols(Cs)
    urow = sample_rows(Rs)
    cpos = {int(c): k for k, c in enumerate(Cs)}
    rpos = {int(r): k for k, r in enumerate(Rs)}
    cols = np.full(ucol.shape, np.nan)
    rows = np.full(urow.shape, np.nan)
    big = 2 * np.pi          # Algorithm 4: no detection inside a block
    for r0, r1 in row_blocks:
        for c0, c1 in col_blocks:
            # first row and first column of the block (they share u at the
            # corner and both start there)
            v, _ = unwrap_vector(urow[rpos[r0], c0:c1], big)
            rows[rpos[r0], c0:c1] = v
            v, _ = unwrap_vector(ucol[r0:r1, cpos[c0]], big,
                                 fixed={0: rows[rpos[r0], c0]})
            cols[r0:r1, cpos[c0]] = v
            # second and third columns, starting from the first row
            for c in (c0 + 1, c0 + 2):
                if c < c1:
                    v, _ = unwrap_vector(ucol[r0:r1, cpos[c]], big,
                                         fixed={0: rows[rpos[r0], c]})
                    cols[r0:r1, cpos[c]] = v
            # the sampled rows of the block, their first three entries taken
            # from those columns
            for r in Rs[(Rs > r0) & (Rs < r1)]:
                fx = {k: cols[r, cpos[c0 + k]] for k in range(3)
                      if c0 + k < c1}
                v, _ = unwrap_vector(urow[rpos[r], c0:c1], big, fixed=fx)
                rows[rpos[r], c0:c1] = v
            # the sampled columns of the block, agreeing with the rows where
            # they intersect: the first three entries come from the block's
            # first three rows (as the rows' come from its first three
            # columns), so the column continues on the rows' branch
            rin = Rs[(Rs >= r0) & (Rs < r1)]
            for c in Cs[(Cs > c0 + 2) & (Cs < c1)]:
                fx = {int(r - r0): rows[rpos[int(r)], c] for r in rin}
                v, _ = unwrap_vector(ucol[r0:r1, cpos[int(c)]], big,
                                     fixed=fx)
                cols[r0:r1, cpos[int(c)]] = v
    # rows outside the first ones of a block are filled by the row loop;
    # columns in Sc or the first three of a block by the block loop
    return Cs, cols, Rs, rows


def lowrank_from_samples(cols, rows, Cs, Rs, rank, tol=1e-12):
    """Algorithm 1 on the sampled columns Psi(:, Cs) and rows Psi(Rs, :):
    the important columns and rows are the pivots of pivoted QR / LQ of the
    sampled block Psi(Rs, Cs) (truncated where the pivots fall below tol
    times the largest, at most ``rank``); Q_col and Q_row are orthonormal
    bases of Psi(:, Pi_col) and Psi(Pi_row, :)^T; M = Q_col(I, :)^+ Psi(I, J)
    (Q_row(J, :)^T)^+ with I = Rs, J = Cs; M = U_M S V_M^T.  Returns U, V
    [N][k] with Psi ~ U V^T (U = Q_col U_M S, V = Q_row V_M)."""
    W = rows[:, Cs]                          # Psi(Rs, Cs)
    _, Rq, pc = scipy.linalg.qr(W, pivoting=True, mode="economic")
    d = np.abs(np.diag(Rq))
    k = int(min(rank, np.sum(d > tol * d[0]))) if d.size and d[0] > 0 else 1
    pi_col = pc[:k]
    _, Rl, pr = scipy.linalg.qr(W.T, pivoting=True, mode="economic")
    pi_row = pr[:k]
    Qc, _ = np.linalg.qr(cols[:, pi_col])
    Qr, _ = np.linalg.qr(rows[pi_row, :].T)
    M = np.linalg.pinv(Qc[Rs, :]) @ W @ np.linalg.pinv(Qr[Cs, :].T)
    Um, s, Vmt = np.linalg.svd(M)
    U = Qc @ (Um * s)
    V = Qr @ Vmt.T
    return U, V


def recover_phase(N, rank, oversample, seed, sample_cols, sample_rows,
                  tau=np.pi / 2):
    """Algorithm 5: rank * oversample random columns and rows, Algorithm 4,
    then the factorization of Algorithm 1.  Returns U, V [N][k]."""
    rng = np.random.default_rng(seed)
    m = min(N, rank * oversample)
    C = np.sort(rng.choice(N, m, replace=False))
    R = np.sort(rng.choice(N, m, replace=False))
    Cs, cols, Rs, rows = unwrap_samples(C, R, tau, sample_cols, sample_rows)
    return lowrank_from_samples(cols, rows, Cs, Rs, rank)
