// NUFFT by dimension lifting, host side: Algorithm 6 (alg:dc), the O(N)
// test of whether a kernel alpha exp(2 pi i Phi) given by low-rank factors
// of its phase (Phi ~ U1 V1^T) and amplitude (A ~ U2 V2^T) can be applied
// as r_eps r-dimensional type-3 NUFFTs (eq. (eqn:tg3)), and Algorithm 1
// (alg:rlr), the randomized factorization of the residual kernel
// Kres = A . exp(2 pi i (U1 V1^T - P Q^T)) that eq. (eqn:tg3) needs.
//
// FP64, complex where the residual is complex; small dense linear algebra
// of its own (column-pivoted Gram-Schmidt QR with exact norm updates,
// one-sided Jacobi SVD, pseudo-inverses through the SVD).  Every random
// choice of the method (the test matrix of the randomized SVD, the sampled
// columns of the test, the sampled rows and columns of Algorithm 1) is an
// input.
#include <algorithm>
#include <cmath>
#include <complex>
#include <string>
#include <vector>

#include "bf_internal.h"

namespace bfi {

namespace {

using cd = std::complex<double>;
constexpr double kTwoPi = 6.283185307179586476925286766559;

// Column-major complex matrix.
struct CMat {
    int m = 0, n = 0;
    std::vector<cd> a;
    CMat() = default;
    CMat(int m_, int n_) : m(m_), n(n_), a((size_t)m_ * n_) {}
    cd& operator()(int i, int j) { return a[(size_t)j * m + i]; }
    cd operator()(int i, int j) const { return a[(size_t)j * m + i]; }
    cd* col(int j) { return a.data() + (size_t)j * m; }
    const cd* col(int j) const { return a.data() + (size_t)j * m; }
};

double col_norm2(const cd* x, int m) {
    double s = 0;
    for (int i = 0; i < m; ++i) s += std::norm(x[i]);
    return s;
}

// Column-pivoted QR by modified Gram-Schmidt (twice per column): the first
// kmax pivots, |R(i, i)| and the orthonormal columns Q (m x k).  Norms of the
// remaining columns are recomputed at every step, so small diagonal entries
// are measured without cancellation.
struct PivQR {
    std::vector<int> piv;
    std::vector<double> diag;
    CMat Q;
};

PivQR pivoted_qr(CMat A, int kmax) {
    PivQR out;
    const int m = A.m, n = A.n;
    const int kk = std::min({kmax, m, n});
    std::vector<int> order(n);
    for (int j = 0; j < n; ++j) order[j] = j;
    out.Q = CMat(m, kk);
    int k = 0;
    for (; k < kk; ++k) {
        int best = -1;
        double bn = -1;
        for (int j = k; j < n; ++j) {
            const double v = col_norm2(A.col(j), m);
            if (v > bn) {
                bn = v;
                best = j;
            }
        }
        if (best != k) {
            std::swap_ranges(A.col(k), A.col(k) + m, A.col(best));
            std::swap(order[k], order[best]);
        }
        cd* q = out.Q.col(k);
        std::copy(A.col(k), A.col(k) + m, q);
        for (int pass = 0; pass < 2; ++pass)
            for (int p = 0; p < k; ++p) {
                const cd* qp = out.Q.col(p);
                cd d = 0;
                for (int i = 0; i < m; ++i) d += std::conj(qp[i]) * q[i];
                for (int i = 0; i < m; ++i) q[i] -= d * qp[i];
            }
        const double nr = std::sqrt(col_norm2(q, m));
        out.piv.push_back(order[k]);
        out.diag.push_back(nr);
        if (nr == 0.0) {
            ++k;
            break;
        }
        for (int i = 0; i < m; ++i) q[i] /= nr;
        for (int j = k + 1; j < n; ++j) {
            cd* aj = A.col(j);
            for (int pass = 0; pass < 2; ++pass) {
                cd d = 0;
                for (int i = 0; i < m; ++i) d += std::conj(q[i]) * aj[i];
                for (int i = 0; i < m; ++i) aj[i] -= d * q[i];
            }
        }
    }
    out.Q.n = k;
    out.Q.a.resize((size_t)m * k);
    return out;
}

// One-sided Jacobi SVD of A (m x n, m >= n): A = U diag(s) V^H, singular
// values in decreasing order.
void jacobi_svd(CMat A, CMat& U, std::vector<double>& s, CMat& V) {
    const int m = A.m, n = A.n;
    V = CMat(n, n);
    for (int j = 0; j < n; ++j) V(j, j) = 1.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        bool rotated = false;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                cd* ap = A.col(p);
                cd* aq = A.col(q);
                const double al = col_norm2(ap, m), be = col_norm2(aq, m);
                cd g = 0;
                for (int i = 0; i < m; ++i) g += std::conj(ap[i]) * aq[i];
                const double ga = std::abs(g);
                if (ga <= 1e-15 * std::sqrt(al * be) || ga == 0.0) continue;
                rotated = true;
                // column q times conj(phase of g) makes the inner product
                // real; then the real rotation of the symmetric 2 x 2 case
                const cd ph = g / ga;
                const double zeta = (be - al) / (2.0 * ga);
                const double t = (zeta >= 0 ? 1.0 : -1.0) /
                                 (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / std::sqrt(1.0 + t * t), sn = c * t;
                for (int i = 0; i < m; ++i) {
                    const cd x = ap[i], y = aq[i] * std::conj(ph);
                    ap[i] = c * x - sn * y;
                    aq[i] = sn * x + c * y;
                }
                cd* vp = V.col(p);
                cd* vq = V.col(q);
                for (int i = 0; i < n; ++i) {
                    const cd x = vp[i], y = vq[i] * std::conj(ph);
                    vp[i] = c * x - sn * y;
                    vq[i] = sn * x + c * y;
                }
            }
        if (!rotated) break;
    }
    std::vector<int> idx(n);
    std::vector<double> nr(n);
    for (int j = 0; j < n; ++j) {
        idx[j] = j;
        nr[j] = std::sqrt(col_norm2(A.col(j), m));
    }
    std::sort(idx.begin(), idx.end(), [&](int x, int y) { return nr[x] > nr[y]; });
    U = CMat(m, n);
    CMat V2(n, n);
    s.assign(n, 0.0);
    for (int k = 0; k < n; ++k) {
        const int j = idx[k];
        s[k] = nr[j];
        for (int i = 0; i < m; ++i)
            U(i, k) = nr[j] > 0 ? A(i, j) / nr[j] : cd(0.0);
        for (int i = 0; i < n; ++i) V2(i, k) = V(i, j);
    }
    V = V2;
}

// Moore-Penrose pseudo-inverse (n x m) of A (m x n), through the SVD of A
// (or of A^H when A is wide); singular values below 1e-14 of the largest
// are dropped.
CMat pinv(const CMat& A) {
    const bool wide = A.m < A.n;
    CMat B = A;
    if (wide) {
        B = CMat(A.n, A.m);
        for (int i = 0; i < A.m; ++i)
            for (int j = 0; j < A.n; ++j) B(j, i) = std::conj(A(i, j));
    }
    CMat U, V;
    std::vector<double> s;
    jacobi_svd(B, U, s, V);                  // B = U S V^H, B^+ = V S^-1 U^H
    CMat Bp(B.n, B.m);
    const double cut = s.empty() ? 0.0 : s[0] * 1e-14;
    for (int k = 0; k < (int)s.size(); ++k) {
        if (s[k] <= cut) continue;
        for (int i = 0; i < B.n; ++i)
            for (int j = 0; j < B.m; ++j)
                Bp(i, j) += V(i, k) * (1.0 / s[k]) * std::conj(U(j, k));
    }
    if (!wide) return Bp;
    CMat Ap(A.n, A.m);                       // (A^H)^+ = (A^+)^H
    for (int i = 0; i < Bp.m; ++i)
        for (int j = 0; j < Bp.n; ++j) Ap(j, i) = std::conj(Bp(i, j));
    return Ap;
}

CMat matmul(const CMat& A, const CMat& B) {
    CMat C(A.m, B.n);
    for (int j = 0; j < B.n; ++j)
        for (int k = 0; k < A.n; ++k) {
            const cd b = B(k, j);
            if (b == cd(0.0)) continue;
            for (int i = 0; i < A.m; ++i) C(i, j) += A(i, k) * b;
        }
    return C;
}

// The problem: factors of the phase and the amplitude, and the leading
// rank-r part P Q^T of the phase.
struct Lift {
    long long N;
    int r1, r2, r;
    const double *U1, *V1, *U2, *V2;
    std::vector<double> P, Q;     // [N][r]

    // Kres(i, j) = (U2 V2^T)(i, j) exp(2 pi i (U1 V1^T - P Q^T)(i, j))
    cd entry(long long i, long long j) const {
        double ph = 0, am = 0;
        for (int k = 0; k < r1; ++k) ph += U1[i * r1 + k] * V1[j * r1 + k];
        for (int k = 0; k < r; ++k) ph -= P[i * r + k] * Q[j * r + k];
        for (int k = 0; k < r2; ++k) am += U2[i * r2 + k] * V2[j * r2 + k];
        ph -= std::nearbyint(ph);
        return am * cd(std::cos(kTwoPi * ph), std::sin(kTwoPi * ph));
    }
    CMat block(const std::vector<long long>& I,
               const std::vector<long long>& J) const {
        CMat M((int)I.size(), (int)J.size());
        for (int b = 0; b < (int)J.size(); ++b)
            for (int a = 0; a < (int)I.size(); ++a) M(a, b) = entry(I[a], J[b]);
        return M;
    }
};

std::vector<long long> iota_ll(long long n) {
    std::vector<long long> v(n);
    for (long long i = 0; i < n; ++i) v[i] = i;
    return v;
}

std::vector<long long> merged(const long long* a, int na,
                              const std::vector<long long>& b) {
    std::vector<long long> v(a, a + na);
    v.insert(v.end(), b.begin(), b.end());
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    return v;
}

// Step 1 of Algorithm 6: the rank-r truncated SVD of U1 V1^T from the range
// of U1 (V1^T Omega), Omega [N][m] with m > r1 columns.
std::string leading_part(Lift& L, const double* omega, int m) {
    const long long N = L.N;
    const int r1 = L.r1;
    // W = V1^T Omega (r1 x m), Y = U1 W (N x m)
    std::vector<double> W((size_t)r1 * m, 0.0);
    for (long long j = 0; j < N; ++j)
        for (int a = 0; a < r1; ++a)
            for (int b = 0; b < m; ++b)
                W[(size_t)a * m + b] += L.V1[j * r1 + a] * omega[j * m + b];
    CMat Y((int)N, m);
    for (long long i = 0; i < N; ++i)
        for (int b = 0; b < m; ++b) {
            double v = 0;
            for (int a = 0; a < r1; ++a) v += L.U1[i * r1 + a] * W[(size_t)a * m + b];
            Y((int)i, b) = v;
        }
    PivQR qr = pivoted_qr(Y, m);            // orthonormal range basis Qy
    const int k = qr.Q.n;
    if (k < L.r) return "the phase has numerical rank below r";
    // B^T = V1 (U1^T Qy) (N x k); its SVD gives B's singular triplets
    std::vector<double> T((size_t)r1 * k, 0.0);
    for (long long i = 0; i < N; ++i)
        for (int a = 0; a < r1; ++a)
            for (int b = 0; b < k; ++b)
                T[(size_t)a * k + b] += L.U1[i * r1 + a] * qr.Q((int)i, b).real();
    CMat Bt((int)N, k);
    for (long long j = 0; j < N; ++j)
        for (int b = 0; b < k; ++b) {
            double v = 0;
            for (int a = 0; a < r1; ++a) v += L.V1[j * r1 + a] * T[(size_t)a * k + b];
            Bt((int)j, b) = v;
        }
    CMat Ub, Vb;
    std::vector<double> s;
    jacobi_svd(Bt, Ub, s, Vb);   // B^T = Ub S Vb^H: B = Vb S Ub^T (real)
    L.P.assign((size_t)N * L.r, 0.0);
    L.Q.assign((size_t)N * L.r, 0.0);
    for (int c = 0; c < L.r; ++c) {
        for (long long j = 0; j < N; ++j) L.Q[j * L.r + c] = Ub((int)j, c).real();
        for (long long i = 0; i < N; ++i) {
            double v = 0;
            for (int b = 0; b < k; ++b) v += qr.Q((int)i, b).real() * Vb(b, c).real();
            L.P[i * L.r + c] = v * s[c];
        }
    }
    return "";
}

}  // namespace

int lift_decide(long long N, int r1, const double* U1, const double* V1,
                int r2, const double* U2, const double* V2, int r, int r_eps,
                double eps, const double* omega, int omega_cols,
                const long long* test_cols, int n_test, int rounds,
                const long long* rows_s, const long long* cols_s,
                int per_round, const long long* extra_rows,
                const long long* extra_cols, int n_extra, int* y, int* n_rank,
                double* P, double* Q, double* a, double* b, int* k_out,
                std::string& err) {
    Lift L{N, r1, r2, r, U1, V1, U2, V2, {}, {}};
    err = leading_part(L, omega, omega_cols);
    if (!err.empty()) return BF_EINVAL;
    std::copy(L.P.begin(), L.P.end(), P);
    std::copy(L.Q.begin(), L.Q.end(), Q);
    // step 2-3: numerical rank of the sampled residual columns
    const std::vector<long long> all = iota_ll(N);
    std::vector<long long> tc(test_cols, test_cols + n_test);
    PivQR t = pivoted_qr(L.block(all, tc), n_test);
    int n = 0;
    for (double d : t.diag)
        if (!t.diag.empty() && d > t.diag[0] * eps) ++n;
    *n_rank = n;
    *y = n <= r_eps ? 1 : 0;
    *k_out = 0;
    if (!*y) return BF_OK;
    // step 4: Algorithm 1 on the residual kernel, rank r_eps
    std::vector<long long> pi_col, pi_row;
    for (int t2 = 0; t2 < rounds; ++t2) {
        std::vector<long long> I = merged(rows_s + (size_t)t2 * per_round,
                                          per_round, pi_row);
        // important columns: pivots of the pivoted QR of Kres(I, :)
        PivQR qc = pivoted_qr(L.block(I, all), r_eps);
        pi_col.assign(qc.piv.begin(), qc.piv.end());
        std::sort(pi_col.begin(), pi_col.end());
        std::vector<long long> J = merged(cols_s + (size_t)t2 * per_round,
                                          per_round, pi_col);
        // important rows: pivots of the pivoted LQ of Kres(:, J), i.e. of
        // the pivoted QR of its conjugate transpose
        CMat KJ = L.block(all, J);
        CMat KJh((int)J.size(), (int)N);
        for (int i = 0; i < KJ.m; ++i)
            for (int j = 0; j < KJ.n; ++j) KJh(j, i) = std::conj(KJ(i, j));
        PivQR qr_ = pivoted_qr(KJh, r_eps);
        pi_row.assign(qr_.piv.begin(), qr_.piv.end());
        std::sort(pi_row.begin(), pi_row.end());
    }
    // column and row bases
    PivQR bc = pivoted_qr(L.block(all, pi_col), r_eps);
    CMat Kr = L.block(pi_row, all);
    CMat Krh((int)N, Kr.m);
    for (int i = 0; i < Kr.m; ++i)
        for (int j = 0; j < Kr.n; ++j) Krh(j, i) = std::conj(Kr(i, j));
    PivQR br = pivoted_qr(Krh, r_eps);
    const CMat& Qc = bc.Q;                  // N x kc
    const CMat& Qr = br.Q;                  // N x kr
    std::vector<long long> J = merged(extra_cols, n_extra, pi_col);
    std::vector<long long> I = merged(extra_rows, n_extra, pi_row);
    // M = Qc(I, :)^+ Kres(I, J) (Qr^H(:, J))^+
    CMat QcI((int)I.size(), Qc.n);
    for (int a2 = 0; a2 < (int)I.size(); ++a2)
        for (int c = 0; c < Qc.n; ++c) QcI(a2, c) = Qc((int)I[a2], c);
    CMat QrhJ(Qr.n, (int)J.size());
    for (int c = 0; c < Qr.n; ++c)
        for (int b2 = 0; b2 < (int)J.size(); ++b2)
            QrhJ(c, b2) = std::conj(Qr((int)J[b2], c));
    CMat M = matmul(matmul(pinv(QcI), L.block(I, J)), pinv(QrhJ));
    CMat Um, Vm;
    std::vector<double> sm;
    if (M.m >= M.n) {
        jacobi_svd(M, Um, sm, Vm);
    } else {
        CMat Mh(M.n, M.m);
        for (int i = 0; i < M.m; ++i)
            for (int j = 0; j < M.n; ++j) Mh(j, i) = std::conj(M(i, j));
        jacobi_svd(Mh, Vm, sm, Um);          // M^H = Vm S Um^H
    }
    const int k = std::min<int>(r_eps, (int)sm.size());
    // Kres ~ (Qc Um) S (Qr Vm)^H: a_k = (Qc Um)(:, k) s_k, b_k = conj(Qr Vm)
    for (int c = 0; c < k; ++c) {
        for (long long i = 0; i < N; ++i) {
            cd u = 0, v = 0;
            for (int q = 0; q < Qc.n; ++q) u += Qc((int)i, q) * Um(q, c);
            for (int q = 0; q < Qr.n; ++q) v += Qr((int)i, q) * Vm(q, c);
            u *= sm[c];
            v = std::conj(v);
            a[2 * ((size_t)c * N + i)] = u.real();
            a[2 * ((size_t)c * N + i) + 1] = u.imag();
            b[2 * ((size_t)c * N + i)] = v.real();
            b[2 * ((size_t)c * N + i) + 1] = v.imag();
        }
    }
    *k_out = k;
    return BF_OK;
}

}  // namespace bfi
