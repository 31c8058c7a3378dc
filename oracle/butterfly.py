"""The butterfly algorithm of Section 4 in FP64, step by step (test
infrastructure).

What is computed: the butterfly algorithm (Algorithm 4.1: preliminaries,
initialization, recursion in xi, switch, recursion in x, termination) built on
the interpolative low-rank factors of Algorithm 2 (Section 2.1), for 1D and,
through tensor products of the 1D rules, 2D grids.  The amplitude enters
through eq. (eqn:tg): g = sum_k a_k * BF(b_k * f).

Readings taken where the text is silent or does not work as printed:

* Interpolation points (eqs. (eqn:gdA)/(eqn:gdB)).  As printed, the offset t
  is paired with a descending Chebyshev node and the set collapses (a box of
  16 with r = 8 gives {7, 8, 9, 10}).  We pair t with the ascending node:
  x_t = Round(t + (N_A - r) s_t), s_t = (1 - cos((t-1) pi / (r-1))) / 2,
  1-based in the box, which is strictly increasing from 1 to N_A.
* Round is half away from zero; a value within 1e-9 of a half-integer is
  treated as an exact tie (so floating-point noise in cos cannot flip it).
* A box with N_A <= r uses all of its indices (the paper keeps one copy of
  repeated points), so its rank is min(r, N_A) per dimension.
* The center c_A (the index of A closest to the mean of its indices) is the
  lower middle index, start + floor((N_A - 1) / 2).
* Trees are dyadic down to single-index leaves (the 16 x 16 illustration of
  Section 4); the switch level is h = floor(L / 2) when L is odd, and
  L - floor(L / 2) for the transposed kernel (see butterfly_apply).
* Inside Algorithm 4.1 the input vector is called g; here it is f and the
  output is g.

Lagrange weights depend only on index differences, which are exact integers in
FP64, so one matrix per (level, child position) is computed in box-relative
coordinates; the paper notes that a box not starting at index 1 is handled by
shifting the grid points.
"""

import numpy as np

from .kernel import coords as user_coords, expi_phase

TIE_SNAP = 1e-9


# ---------------------------------------------------------------- geometry

def mock_chebyshev(size, r):
    """0-based interpolation offsets in a box of ``size`` indices
    (eqs. (eqn:gdA)/(eqn:gdB) with the ascending-node reading)."""
    if r < 2:
        raise ValueError("need at least 2 interpolation points")
    if size <= r:
        return np.arange(size, dtype=np.int64)
    t = np.arange(1, r + 1, dtype=np.float64)
    s = (1.0 - np.cos((t - 1.0) * np.pi / (r - 1))) / 2.0
    v = t + (size - r) * s
    x = np.floor(v + 0.5 + TIE_SNAP).astype(np.int64)   # 1-based
    return np.unique(x) - 1


def mock_chebyshev_as_printed(size, r):
    """The printed formula taken literally (descending node with the +t
    offset); used only to document why it is not the reading adopted."""
    t = np.arange(1, r + 1, dtype=np.float64)
    z = 0.5 * np.cos((t - 1.0) * np.pi / (r - 1))
    v = t + (size - r) * (z + 0.5)
    return np.unique(np.floor(v + 0.5 + TIE_SNAP).astype(np.int64))


def lagrange_1d(nodes, y):
    """Matrix [len(y), len(nodes)] of M_t(y_k) = prod_{j != t}
    (y_k - x_j) / (x_t - x_j) (Section 2.1, Lagrange polynomials)."""
    nodes = np.asarray(nodes, np.float64)
    y = np.asarray(y, np.float64)
    out = np.ones((y.size, nodes.size))
    for t in range(nodes.size):
        for j in range(nodes.size):
            if j != t:
                out[:, t] *= (y - nodes[j]) / (nodes[t] - nodes[j])
    return out


class Trees:
    """Dyadic trees T_X and T_Omega of depth L over an n^dim grid
    (Section 4).  A box at tree level l has side n >> l per dimension and is
    named by its integer box coordinates, flattened row-major."""

    def __init__(self, dim, n, q):
        L = int(n).bit_length() - 1
        if n != 1 << L or L < 1:
            raise ValueError("n must be a power of two >= 2")
        self.dim, self.n, self.L, self.q = dim, n, L, q

    def side(self, level):
        return self.n >> level

    def box_coords(self, level):
        m = 1 << level
        g = np.indices((m,) * self.dim).reshape(self.dim, -1).T
        return g.astype(np.int64)

    def flat(self, level, c):
        m = 1 << level
        idx = np.zeros(c.shape[:-1], np.int64)
        for d in range(self.dim):
            idx = idx * m + c[..., d]
        return idx

    def offsets(self, level):
        """Tensor-product interpolation offsets of a box at this level,
        shape (r, dim), t flattened row-major over (t_1, ..., t_dim)."""
        off = mock_chebyshev(self.side(level), self.q)
        grids = np.meshgrid(*([off] * self.dim), indexing="ij")
        return np.stack(grids, -1).reshape(-1, self.dim)

    def points(self, level):
        """Interpolation points of every box: (nbox, r, dim) grid indices."""
        base = self.box_coords(level) * self.side(level)
        return base[:, None, :] + self.offsets(level)[None, :, :]

    def centers(self, level):
        s = self.side(level)
        return self.box_coords(level) * s + (s - 1) // 2

    def child_positions(self):
        return np.indices((2,) * self.dim).reshape(self.dim, -1).T

    def lagrange(self, node_level, eval_rel):
        """M_t^{box}(y) for a box at ``node_level`` (nodes in box-relative
        coordinates) at box-relative points ``eval_rel`` (m, dim).
        Returns (r_box, m): row t, column k."""
        off1 = mock_chebyshev(self.side(node_level), self.q)
        tmulti = self.offsets(node_level)           # multi-index via values
        tidx = np.searchsorted(off1, tmulti)        # (r, dim) positions
        M = np.ones((tmulti.shape[0], eval_rel.shape[0]))
        for d in range(self.dim):
            Ld = lagrange_1d(off1, eval_rel[:, d])  # (m, r1)
            M *= Ld[:, tidx[:, d]].T
        return M


# ------------------------------------------------------------- arithmetic

def _contract(Lag, z):
    """out[..., t, v] = sum_s Lag[t, s] z[..., s, v] (real Lag, complex z),
    as two real BLAS products."""
    zt = np.moveaxis(z, -2, -1)
    lead = zt.shape[:-1]
    zr = np.ascontiguousarray(zt.real).reshape(-1, zt.shape[-1])
    zi = np.ascontiguousarray(zt.imag).reshape(-1, zt.shape[-1])
    out = (zr @ Lag.T) + 1j * (zi @ Lag.T)
    return np.moveaxis(out.reshape(lead + (Lag.shape[0],)), -1, -2)


def switch_level(L, transpose):
    """Level h of the switch (Algorithm 4.1, step 4): floor(L / 2) for odd L
    (the paper takes L even).  The factorization of the transposed kernel
    mirrors K's levels (its recursion in xi is the transpose of K's
    recursion in x, and the other way round), so it switches at
    L - floor(L / 2); the two factorizations are then exact transposes of
    each other at every depth."""
    return L - L // 2 if transpose else L // 2


def butterfly_apply(dim, n, phase_kind, phase_params, q, f, a_block=None,
                    transpose=False, conjugate=False):
    """Butterfly algorithm (Algorithm 4.1) applied to the columns of
    ``f`` ([V][N], user index order) for the kernel exp(2 pi i Phi).

    Returns complex128 [V][N].  ``a_block`` bounds the number of T_X boxes
    handled at once in the switch (memory only, not arithmetic order).

    transpose: factorize the transposed kernel instead (the operator of
    Scenario 2 in Section 1, applied to vectors indexed by x, giving values
    indexed by xi): its entry at output index j and input index i is
    exp(2 pi i Phi(x_i, xi_j)).  The algorithm is unchanged; only the phase
    evaluation swaps its index roles.  conjugate: the conjugate kernel
    (with transpose, the adjoint K^H).
    """
    T = Trees(dim, n, q)
    L = T.L
    h = switch_level(L, transpose)
    f = np.atleast_2d(np.asarray(f, np.complex128))
    V = f.shape[0]
    sgn = -1 if conjugate else 1

    def E(ix, jx, sign=1):
        # ix: indices of the output tree, jx: of the input tree
        if transpose:
            return expi_phase(phase_kind, phase_params, jx, ix, n, sgn * sign)
        return expi_phase(phase_kind, phase_params, ix, jx, n, sgn * sign)

    # -- Step 2, initialization: A = root of T_X, B = every leaf of T_Omega
    # (eq. (eqn:1)).  A single-index leaf has one point and M_1 = 1.
    cA = T.centers(0)                                  # (1, dim)
    xiB = T.points(L)                                  # (N, 1, dim)
    leaf_user = T.flat(L, xiB[:, 0, :])                # leaf -> user index
    # user index of a 2D grid point (j1, j2) is j1 * n + j2: the same value
    assert np.array_equal(user_coords(leaf_user, dim, n), xiB[:, 0, :])
    fB = f[:, leaf_user].T                             # (N, V)
    M1 = T.lagrange(L, np.zeros((1, dim), np.int64))[0, 0]
    c4, x4 = cA[:, None, None, :], xiB[None, :, :, :]
    lam = (E(c4, x4, -1)[..., None]                    # (1, N, 1, 1)
           * (M1 * E(c4, x4, +1)[..., None]
              * fB[None, :, None, :]))                 # (1, N, 1, V)

    # -- Step 3, recursion in xi for l = 1..h (eq. (eqn:2)).
    for l in range(1, h + 1):
        lB, lC = L - l, L - l + 1
        cA = T.centers(l)                              # (nA, dim)
        parA = T.flat(l - 1, T.box_coords(l) >> 1)     # (nA,)
        xiB = T.points(lB)                             # (nB, rB, dim)
        xiC = T.points(lC)                             # (nC, rC, dim)
        bco = T.box_coords(lB)
        sideC = T.side(lC)
        new = 0
        for cpos in T.child_positions():
            child = T.flat(lC, bco * 2 + cpos)         # (nB,)
            # M_t^B(xi_s^C) in B-relative coordinates
            rel = cpos * sideC + T.offsets(lC)         # (rC, dim)
            Lag = T.lagrange(lB, rel)                  # (rB, rC)
            ph = E(cA[:, None, None, :], xiC[child][None, :, :, :], +1)
            z = ph[..., None] * lam[parA][:, child]    # (nA, nB, rC, V)
            new = new + _contract(Lag, z)
        lam = E(cA[:, None, None, :], xiB[None, :, :, :], -1)[..., None] * new

    # -- Step 4, switch at l = h: lambda_t <- sum_s exp(2 pi i Phi(x_t^A,
    # xi_s^B)) lambda_s.
    xA = T.points(h)                                   # (nA, rA, dim)
    xiB = T.points(L - h)                              # (nB, rB, dim)
    nA = xA.shape[0]
    step = a_block or max(1, (1 << 22) // max(1, xiB.shape[0] * xiB.shape[1]
                                                 * xA.shape[1]))
    out = np.empty((nA, xiB.shape[0], xA.shape[1], V), np.complex128)
    for s0 in range(0, nA, step):
        K = E(xA[s0:s0 + step, None, :, None, :],
              xiB[None, :, None, :, :], +1)           # (a, b, rA, rB)
        out[s0:s0 + step] = np.einsum("abts,absv->abtv", K,
                                      lam[s0:s0 + step])
    lam = out

    # -- Step 5, recursion in x for l = h+1..L (eq. (eqn:3)).
    for l in range(h + 1, L + 1):
        lB, lC = L - l, L - l + 1
        xA = T.points(l)                               # (nA, rA, dim)
        xP = T.points(l - 1)                           # (nP, rP, dim)
        cC = T.centers(lC)                             # (nC, dim)
        aco = T.box_coords(l)
        bco = T.box_coords(lB)
        sideA = T.side(l)
        nA = aco.shape[0]
        new = 0
        for cpos in T.child_positions():
            child = T.flat(lC, bco * 2 + cpos)         # (nB,)
            cc = cC[child]                             # (nB, dim)
            # exp(-2 pi i Phi(x_s^P, c_C)) lambda_s^{PC}
            src = (E(xP[:, None, :, :], cc[None, :, None, :], -1)[..., None]
                   * lam[:, child])                    # (nP, nB, rP, V)
            tmp = np.empty((nA, bco.shape[0], xA.shape[1], V), np.complex128)
            for apos in T.child_positions():
                sel = np.nonzero(np.all((aco & 1) == apos, axis=1))[0]
                par = T.flat(l - 1, aco[sel] >> 1)
                # M_s^P(x_t^A) in P-relative coordinates: (rP, rA)
                rel = apos * sideA + T.offsets(l)
                Lag = T.lagrange(l - 1, rel).T         # (rA, rP)
                tmp[sel] = _contract(Lag, src[par])
            new = new + (E(xA[:, None, :, :], cc[None, :, None, :], +1)
                         [..., None] * tmp)
        lam = new

    # -- Step 6, termination: B = root of T_Omega, A = every leaf of T_X
    # (eq. (eqn:bf3)); a single-index leaf has one point and M_1 = 1.
    cB = T.centers(0)                                  # (1, dim)
    xA = T.points(L)                                   # (N, 1, dim)
    M1 = T.lagrange(L, np.zeros((1, dim), np.int64))[0, 0]
    u = (E(xA[:, 0, :], cB, +1)[:, None]
         * (M1 * E(xA[:, 0, :], cB, -1)[:, None] * lam[:, 0, 0, :]))
    g = np.empty((V, xA.shape[0]), np.complex128)
    g[:, T.flat(L, xA[:, 0, :])] = u.T
    return g


def butterfly_matvec(dim, n, phase_kind, phase_params, q, a, b, f,
                     transpose=False, conjugate=False):
    """g_v = sum_k a_k * BF(b_k * f_v) (eq. (eqn:tg)) for f [nvec][N] and
    amplitude factors a, b [r][N].  Returns complex128 [nvec][N].

    transpose: the transposed operator, alpha(x_i, xi_j) exp(2 pi i
    Phi(x_i, xi_j)) at output j, input i, so the b_k (functions of xi)
    weight the output and the a_k (functions of x) the input; conjugate:
    all of it conjugated (with transpose, the adjoint K^H)."""
    f = np.atleast_2d(np.asarray(f, np.complex128))
    a = np.atleast_2d(np.asarray(a, np.complex128))
    b = np.atleast_2d(np.asarray(b, np.complex128))
    if transpose:
        a, b = b, a
    if conjugate:
        a, b = np.conj(a), np.conj(b)
    r = a.shape[0]
    cols = (b[None, :, :] * f[:, None, :]).reshape(-1, f.shape[1])
    u = butterfly_apply(dim, n, phase_kind, phase_params, q, cols,
                        transpose=transpose, conjugate=conjugate)
    u = u.reshape(f.shape[0], r, f.shape[1])
    return np.sum(a[None, :, :] * u, axis=1)


def butterfly_composition(n, phase_kind, phase_params, q, fhat):
    """g = L(L f) (eq. (eq:example4)) with every operator applied by its
    butterfly factorization: the FIO of eq. (eq:example3), then the
    Fourier coefficients of its output (the DFT-phase kernel's adjoint,
    scaled by 1/n), then the FIO again.  Each factor has the error of
    Algorithm 4.1 at q points; the composed error adds them."""
    inner = butterfly_apply(1, n, phase_kind, phase_params, q, fhat)
    coef = butterfly_apply(1, n, "dft", (), q, inner, transpose=True,
                           conjugate=True) / n
    return butterfly_apply(1, n, phase_kind, phase_params, q, coef)

