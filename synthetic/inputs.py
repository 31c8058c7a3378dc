"""Seeded input generators (PCG64).  No method arithmetic lives here."""

import numpy as np


def gaussian_vectors(N, nvec, seed):
    """``nvec`` complex128 vectors of length ``N``; real and imaginary parts
    i.i.d. N(0, 1).  Layout ``[nvec][N]``, C-contiguous."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal((nvec, N))
    im = rng.standard_normal((nvec, N))
    return (re + 1j * im).astype(np.complex128)


def sample_rows(N, count, seed):
    """``count`` distinct row indices in ``[0, N)``, sorted (all rows when
    ``count >= N``)."""
    if count >= N:
        return np.arange(N, dtype=np.int64)
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(N, size=count, replace=False)).astype(np.int64)


def orthogonal_mix(r, seed):
    """A seeded real ``r x r`` orthogonal matrix (QR of a Gaussian matrix with
    the sign of R's diagonal folded into Q)."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((r, r))
    q, rr = np.linalg.qr(g)
    return q * np.sign(np.diag(rr))[None, :]


def amplitude_factors(kind, dim, n, r, seed):
    """Rank-``r`` factors ``a[r][N]``, ``b[r][N]`` (complex128, user index
    order) of the amplitude ``alpha(x, xi) = sum_k a_k(x) b_k(xi)``.

    kind ``"one"``: alpha = 1, which needs r = 1 (a = b = 1).
    kind ``"sincos"``: alpha = 1 + 0.5 sin(2 pi x1) cos(2 pi xi1 / n), an
    exact rank-2 function of (x1, xi1); the factors [1, sin/2] and [1, cos]
    are zero-padded to ``r`` columns and mixed by a seeded orthogonal matrix
    Q (A <- A Q, B <- B Q), so every column is non-trivial while
    sum_k a_k b_k is unchanged.  r = 1 is not possible for this kind.

    The grid is x = i/n, xi = j - n/2 per dimension; for dim = 2 the user
    index is row-major i1 * n + i2 and only the first coordinate enters.
    """
    N = n ** dim
    idx = np.arange(N, dtype=np.int64)
    first = idx // n if dim == 2 else idx          # first coordinate index
    if kind == "one":
        if r != 1:
            raise ValueError("amplitude 'one' has rank 1")
        return np.ones((1, N), np.complex128), np.ones((1, N), np.complex128)
    if kind != "sincos":
        raise ValueError(kind)
    if r < 2:
        raise ValueError("amplitude 'sincos' needs r >= 2")
    x1 = first / n
    xi1 = first - n // 2
    A = np.zeros((N, r))
    B = np.zeros((N, r))
    A[:, 0] = 1.0
    A[:, 1] = 0.5 * np.sin(2 * np.pi * x1)
    B[:, 0] = 1.0
    B[:, 1] = np.cos(2 * np.pi * xi1 / n)
    Q = orthogonal_mix(r, seed)
    A = A @ Q
    B = B @ Q
    return (np.ascontiguousarray(A.T).astype(np.complex128),
            np.ascontiguousarray(B.T).astype(np.complex128))


def lowrank_phase(dim, n, rank, seed):
    """Real factors ``U[N][rank]``, ``V[N][rank]`` (float64, user index
    order) of a phase given in low-rank form, Phi(x_i, xi_j) = sum_k U[i, k]
    V[j, k]: x . xi plus ``rank - dim`` terms u_k(x) w_k(xi), each u_k a
    small smooth periodic function of x (0.02 to 0.08 times 1 + sin/2 of a
    random low frequency and shift) and w_k the Euclidean norm |xi| or one
    coordinate of xi, so that the phase is smooth in x and homogeneous of
    degree 1 in xi like the workloads' phases.  The columns are mixed by a
    seeded orthogonal matrix (U <- U Q, V <- V Q), which leaves U V^T
    unchanged.  Grid: x = i/n, xi = j - n/2 per dimension, 2D user index
    i1 * n + i2."""
    if rank < dim:
        raise ValueError("rank must be at least dim")
    N = n ** dim
    rng = np.random.default_rng(seed)
    idx = np.arange(N, dtype=np.int64)
    g = idx[:, None] if dim == 1 else np.stack([idx // n, idx % n], axis=1)
    x = g / n
    xi = (g - n // 2).astype(np.float64)
    nrm = np.sqrt(np.sum(xi * xi, axis=1))
    cu = [x[:, d] for d in range(dim)]
    cv = [xi[:, d] for d in range(dim)]
    for k in range(rank - dim):
        m = rng.integers(1, 3, size=dim)
        th = rng.uniform(0.0, 2 * np.pi)
        amp = rng.uniform(0.02, 0.08)
        cu.append(amp * (1.0 + 0.5 * np.sin(2 * np.pi * (x @ m) + th)))
        cv.append(nrm if k % 2 == 0 else xi[:, k % dim])
    Q = orthogonal_mix(rank, seed + 1)
    U = np.stack(cu, axis=1) @ Q
    V = np.stack(cv, axis=1) @ Q
    return np.ascontiguousarray(U), np.ascontiguousarray(V)

