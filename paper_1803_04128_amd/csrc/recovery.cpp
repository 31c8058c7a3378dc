// Low-rank phase recovery under indirect access (Section 3.2), host C++:
// Algorithm 3 (vector unwrapping with discontinuity detection), Algorithm 4
// (rows and columns of the unwrapped phase that agree where they meet, 1D)
// and the factorization of Algorithm 1 restricted to the sampled rows and
// columns, composed as in Algorithm 5.  All arithmetic is FP64; the samples
// come through a caller callback (Scenario 1: entry evaluation; Scenario 2:
// applies of K and its transpose to unit vectors).
//
// Phases are in cycles.  Two readings where the paper is loose: the
// detection threshold tau is an angle, compared with 2 pi times the second
// difference; the recovered columns take their first three entries from
// their block's first three rows, as the rows take theirs from its first
// three columns, so both follow one branch of the phase.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <set>
#include <string>
#include <vector>

#include "bf_internal.h"

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;

// representative of u modulo 1 nearest to target (ties away from zero)
inline double nearest(double u, double target) {
    const double d = target - u;
    return u + std::copysign(std::floor(std::fabs(d) + 0.5), d);
}

// Algorithm 3 (Section 3.2) on u[0..n) with stride 1, as one forward pass.
// Each entry takes the representative of u modulo 1 nearest to a
// prediction from the entries before it in its smooth piece: the very first
// entry keeps u; with one entry of history the prediction is that entry
// (the smallest jump), with two the linear continuation, with three or more
// the continuation of the second difference (the smallest change of the
// third difference, the TV^3 criterion).  A piece after a discontinuity has
// the last entry of the previous piece as its first history entry.  Once an
// entry is assigned from three entries of history, a second difference of
// more than tau / (2 pi) cycles marks a discontinuity there: the entry
// starts a new piece and is assigned again from one entry of history.
// fix: optional per-entry values already assigned (NaN = free).  S receives
// the piece starts (S[0] = 0).
void unwrap(const double* u, long long n, double tau, const double* fix,
            double* v, std::vector<long long>& S) {
    S.assign(1, 0);
    int hist = 0;                       // usable entries before a
    for (long long a = 0; a < n; ++a) {
        double value;
        if (hist == 0)
            value = u[a];
        else if (hist == 1)
            value = nearest(u[a], v[a - 1]);
        else if (hist == 2)
            value = nearest(u[a], 2.0 * v[a - 1] - v[a - 2]);
        else
            value = nearest(u[a], 3.0 * v[a - 1] - 3.0 * v[a - 2] + v[a - 3]);
        v[a] = (fix && !std::isnan(fix[a])) ? fix[a] : value;
        if (hist >= 3 &&
            kTwoPi * std::fabs(v[a] + v[a - 2] - 2.0 * v[a - 1]) > tau) {
            // a discontinuity: a piece starts here, continued from v[a - 1]
            S.push_back(a);
            const double again = nearest(u[a], v[a - 1]);
            v[a] = (fix && !std::isnan(fix[a])) ? fix[a] : again;
            hist = 2;
            continue;
        }
        ++hist;
    }
}

// ---- small dense linear algebra (row-major, FP64) ----------------------

// Householder QR with column pivoting of A (m x n, row-major, overwritten):
// returns the column order and |R_kk| for k < min(m, n).
void pivoted_qr(std::vector<double> A, int m, int n, std::vector<int>& piv,
                std::vector<double>& rdiag) {
    piv.resize(n);
    for (int j = 0; j < n; ++j) piv[j] = j;
    std::vector<double> norms(n, 0.0);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < m; ++i) norms[j] += A[(size_t)i * n + j] * A[(size_t)i * n + j];
    const int kmax = std::min(m, n);
    rdiag.assign(kmax, 0.0);
    std::vector<double> w(m);
    for (int k = 0; k < kmax; ++k) {
        // column of largest remaining norm (recomputed: the sizes are small)
        int best = k;
        double bn = -1.0;
        for (int j = k; j < n; ++j) {
            double s = 0.0;
            for (int i = k; i < m; ++i) s += A[(size_t)i * n + j] * A[(size_t)i * n + j];
            norms[j] = s;
            if (s > bn) { bn = s; best = j; }
        }
        if (best != k) {
            for (int i = 0; i < m; ++i) std::swap(A[(size_t)i * n + k], A[(size_t)i * n + best]);
            std::swap(piv[k], piv[best]);
        }
        const double alpha = std::sqrt(std::max(bn, 0.0));
        rdiag[k] = alpha;
        if (alpha == 0.0) continue;
        // reflector v = x + sign(x0) |x| e0 on rows k..m-1 of column k
        const double x0 = A[(size_t)k * n + k];
        const double s0 = x0 >= 0 ? 1.0 : -1.0;
        for (int i = k; i < m; ++i) w[i] = A[(size_t)i * n + k];
        w[k] += s0 * alpha;
        double vv = 0.0;
        for (int i = k; i < m; ++i) vv += w[i] * w[i];
        if (vv == 0.0) continue;
        for (int j = k; j < n; ++j) {
            double d = 0.0;
            for (int i = k; i < m; ++i) d += w[i] * A[(size_t)i * n + j];
            d = 2.0 * d / vv;
            for (int i = k; i < m; ++i) A[(size_t)i * n + j] -= d * w[i];
        }
    }
}

// Orthonormal basis of the k columns of X (N x k, column j at X[j * N ..]):
// Gram-Schmidt applied twice per column; returns Q in the same layout.
std::vector<double> orthonormal_basis(std::vector<double> X, long long N, int k) {
    for (int j = 0; j < k; ++j) {
        double* xj = &X[(size_t)j * N];
        for (int pass = 0; pass < 2; ++pass)
            for (int i = 0; i < j; ++i) {
                const double* qi = &X[(size_t)i * N];
                double d = 0.0;
                for (long long t = 0; t < N; ++t) d += qi[t] * xj[t];
                for (long long t = 0; t < N; ++t) xj[t] -= d * qi[t];
            }
        double nr = 0.0;
        for (long long t = 0; t < N; ++t) nr += xj[t] * xj[t];
        nr = std::sqrt(nr);
        if (nr > 0)
            for (long long t = 0; t < N; ++t) xj[t] /= nr;
    }
    return X;
}

// Pseudo-inverse of A (m x k, full column rank, m >= k): R^-1 Q^T from a
// Gram-Schmidt QR; returns k x m row-major.
std::vector<double> pinv_tall(const std::vector<double>& A, int m, int k) {
    std::vector<double> Q((size_t)k * m), R((size_t)k * k, 0.0);
    for (int j = 0; j < k; ++j)
        for (int i = 0; i < m; ++i) Q[(size_t)j * m + i] = A[(size_t)i * k + j];
    for (int j = 0; j < k; ++j) {
        double* qj = &Q[(size_t)j * m];
        for (int pass = 0; pass < 2; ++pass)
            for (int i = 0; i < j; ++i) {
                const double* qi = &Q[(size_t)i * m];
                double d = 0.0;
                for (int t = 0; t < m; ++t) d += qi[t] * qj[t];
                R[(size_t)i * k + j] += d;
                for (int t = 0; t < m; ++t) qj[t] -= d * qi[t];
            }
        double nr = 0.0;
        for (int t = 0; t < m; ++t) nr += qj[t] * qj[t];
        nr = std::sqrt(nr);
        R[(size_t)j * k + j] = nr;
        if (nr > 0)
            for (int t = 0; t < m; ++t) qj[t] /= nr;
    }
    // P = R^-1 Q^T: back substitution per column of Q^T
    std::vector<double> P((size_t)k * m, 0.0);
    for (int t = 0; t < m; ++t)
        for (int i = k - 1; i >= 0; --i) {
            double s = Q[(size_t)i * m + t];
            for (int j = i + 1; j < k; ++j) s -= R[(size_t)i * k + j] * P[(size_t)j * m + t];
            P[(size_t)i * m + t] = R[(size_t)i * k + i] != 0 ? s / R[(size_t)i * k + i] : 0.0;
        }
    return P;
}

// One-sided Jacobi SVD of M (k x k, row-major): M = U diag(s) V^T.
void jacobi_svd(const std::vector<double>& M, int k, std::vector<double>& U,
                std::vector<double>& s, std::vector<double>& V) {
    // columns of A = M rotated until orthogonal; V accumulates the rotations
    std::vector<double> A(M);
    V.assign((size_t)k * k, 0.0);
    for (int i = 0; i < k; ++i) V[(size_t)i * k + i] = 1.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < k; ++p)
            for (int q = p + 1; q < k; ++q) {
                double a = 0, b = 0, c = 0;
                for (int i = 0; i < k; ++i) {
                    const double x = A[(size_t)i * k + p], y = A[(size_t)i * k + q];
                    a += x * x;
                    b += y * y;
                    c += x * y;
                }
                if (c == 0.0 || std::fabs(c) <= 1e-15 * std::sqrt(a * b)) continue;
                off = std::max(off, std::fabs(c) / std::sqrt(a * b));
                const double zeta = (b - a) / (2.0 * c);
                const double t = (zeta >= 0 ? 1.0 : -1.0) /
                                 (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
                const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = cs * t;
                for (int i = 0; i < k; ++i) {
                    const double x = A[(size_t)i * k + p], y = A[(size_t)i * k + q];
                    A[(size_t)i * k + p] = cs * x - sn * y;
                    A[(size_t)i * k + q] = sn * x + cs * y;
                    const double vx = V[(size_t)i * k + p], vy = V[(size_t)i * k + q];
                    V[(size_t)i * k + p] = cs * vx - sn * vy;
                    V[(size_t)i * k + q] = sn * vx + cs * vy;
                }
            }
        if (off < 1e-15) break;
    }
    s.assign(k, 0.0);
    U.assign((size_t)k * k, 0.0);
    for (int j = 0; j < k; ++j) {
        double nr = 0.0;
        for (int i = 0; i < k; ++i) nr += A[(size_t)i * k + j] * A[(size_t)i * k + j];
        nr = std::sqrt(nr);
        s[j] = nr;
        for (int i = 0; i < k; ++i)
            U[(size_t)i * k + j] = nr > 0 ? A[(size_t)i * k + j] / nr : 0.0;
    }
}

thread_local std::string g_rec_error;

}  // namespace

namespace bfi {

const char* recovery_error() { return g_rec_error.c_str(); }

int lowrank_fit(long long N, const double* colsp, const long long* Cs,
                int mc, const double* rowsp, const long long* Rs, int mr,
                int rank, int cap_rank, double* U, double* V, int* rank_out);

// Algorithm 4 + Algorithm 1 (see bf.h, bf_recover_phase).
int recover_phase(long long N, const long long* C0, int nc,
                  const long long* R0, int nr, int rank, double tau,
                  bf_phase_sampler sample, void* ctx, int cap_rank, double* U,
                  double* V, int* rank_out) {
    auto err = [](const char* m) {
        g_rec_error = m;
        return BF_EINVAL;
    };
    // --- Algorithm 4: discontinuities of the first column and first row
    std::vector<double> first((size_t)N), tmp((size_t)N);
    std::vector<long long> Sr, Sc;
    if (sample(ctx, 0, 1, &C0[0], first.data()) != 0) return err("sampler failed");
    unwrap(first.data(), N, tau, nullptr, tmp.data(), Sr);
    std::set<long long> Rset(R0, R0 + nr);
    Rset.insert(Sr.begin(), Sr.end());
    const long long r_first = *Rset.begin();
    if (sample(ctx, 1, 1, &r_first, first.data()) != 0) return err("sampler failed");
    unwrap(first.data(), N, tau, nullptr, tmp.data(), Sc);
    auto blocks = [N](const std::vector<long long>& S) {
        std::vector<std::pair<long long, long long>> b;
        for (size_t i = 0; i < S.size(); ++i)
            b.push_back({S[i], i + 1 < S.size() ? S[i + 1] : N});
        return b;
    };
    const auto rb = blocks(Sr), cb = blocks(Sc);
    std::set<long long> Cset(C0, C0 + nc);
    Cset.insert(Sc.begin(), Sc.end());
    for (auto& b : cb)
        for (long long c = b.first + 1; c <= b.first + 2; ++c)
            if (c < b.second) Cset.insert(c);
    for (auto& b : rb)
        for (long long r = b.first + 1; r <= b.first + 2; ++r)
            if (r < b.second) Rset.insert(r);
    std::vector<long long> Cs(Cset.begin(), Cset.end()), Rs(Rset.begin(), Rset.end());
    const int mc = (int)Cs.size(), mr = (int)Rs.size();
    // samples: ucol[i][k] = Phi(i, Cs[k]) mod 1, urow[k][j] = Phi(Rs[k], j)
    std::vector<double> ucol((size_t)N * mc), urow((size_t)mr * N);
    if (sample(ctx, 0, mc, Cs.data(), ucol.data()) != 0 ||
        sample(ctx, 1, mr, Rs.data(), urow.data()) != 0)
        return err("sampler failed");
    std::map<long long, int> cpos, rpos;
    for (int k = 0; k < mc; ++k) cpos[Cs[k]] = k;
    for (int k = 0; k < mr; ++k) rpos[Rs[k]] = k;
    // recovered columns, column-major [mc][N], and rows [mr][N]
    std::vector<double> cols((size_t)mc * N, NAN), rows((size_t)mr * N, NAN);
    std::vector<double> colbuf((size_t)N), fix((size_t)N);
    std::vector<long long> S;
    const double big = kTwoPi;   // no detection inside a block
    auto unwrap_col = [&](int k, long long r0, long long r1, const double* fx) {
        for (long long i = r0; i < r1; ++i) colbuf[i - r0] = ucol[(size_t)i * mc + k];
        unwrap(colbuf.data(), r1 - r0, big, fx, &cols[(size_t)k * N + r0], S);
    };
    for (auto& R : rb) {
        const long long r0 = R.first, r1 = R.second;
        for (auto& Cb : cb) {
            const long long c0 = Cb.first, c1 = Cb.second;
            const long long nn = c1 - c0;
            // first row, then the first three columns from it
            const int p0 = rpos[r0];
            unwrap(&urow[(size_t)p0 * N + c0], nn, big, nullptr,
                   &rows[(size_t)p0 * N + c0], S);
            for (long long c = c0; c <= c0 + 2 && c < c1; ++c) {
                std::fill(fix.begin(), fix.begin() + (r1 - r0), NAN);
                fix[0] = rows[(size_t)p0 * N + c];
                unwrap_col(cpos[c], r0, r1, fix.data());
            }
            // the block's other sampled rows from the first three columns
            for (int kr = 0; kr < mr; ++kr) {
                const long long r = Rs[kr];
                if (r <= r0 || r >= r1) continue;
                std::fill(fix.begin(), fix.begin() + nn, NAN);
                for (long long c = c0; c <= c0 + 2 && c < c1; ++c)
                    fix[c - c0] = cols[(size_t)cpos[c] * N + r];
                unwrap(&urow[(size_t)kr * N + c0], nn, big, fix.data(),
                       &rows[(size_t)kr * N + c0], S);
            }
            // the block's other sampled columns, fixed where they meet rows
            for (int kc = 0; kc < mc; ++kc) {
                const long long c = Cs[kc];
                if (c <= c0 + 2 || c >= c1) continue;
                std::fill(fix.begin(), fix.begin() + (r1 - r0), NAN);
                for (int kr = 0; kr < mr; ++kr) {
                    const long long r = Rs[kr];
                    if (r >= r0 && r < r1) fix[r - r0] = rows[(size_t)kr * N + c];
                }
                unwrap_col(kc, r0, r1, fix.data());
            }
        }
    }
    return lowrank_fit(N, cols.data(), Cs.data(), mc, rows.data(), Rs.data(),
                       mr, rank, cap_rank, U, V, rank_out);
}

// Algorithm 1 on sampled columns cols [mc][N] (column-major, column k =
// Psi(:, Cs[k])) and rows rows [mr][N] (row k = Psi(Rs[k], :)): important
// columns and rows by pivoted QR / LQ of Psi(Rs, Cs), orthonormal bases of
// the important columns and rows, M = Qc(Rs, :)^+ Psi(Rs, Cs) (Qr(Cs, :)^T)^+
// and its SVD; Psi ~ U V^T with U = Qc U_M S, V = Qr V_M.
int lowrank_fit(long long N, const double* colsp, const long long* Cs,
                int mc, const double* rowsp, const long long* Rs, int mr,
                int rank, int cap_rank, double* U, double* V, int* rank_out) {
    auto err = [](const char* m) {
        g_rec_error = m;
        return BF_EINVAL;
    };
    std::vector<double> W((size_t)mr * mc);     // Psi(Rs, Cs)
    for (int a = 0; a < mr; ++a)
        for (int b = 0; b < mc; ++b) W[(size_t)a * mc + b] = rowsp[(size_t)a * N + Cs[b]];
    std::vector<int> pc, pr;
    std::vector<double> dc, dr;
    pivoted_qr(W, mr, mc, pc, dc);
    std::vector<double> Wt((size_t)mc * mr);
    for (int a = 0; a < mr; ++a)
        for (int b = 0; b < mc; ++b) Wt[(size_t)b * mr + a] = W[(size_t)a * mc + b];
    pivoted_qr(Wt, mc, mr, pr, dr);
    int k = 0;
    if (!dc.empty() && dc[0] > 0)
        for (double d : dc) k += d > 1e-12 * dc[0];
    k = std::max(1, std::min(k, std::min(rank, cap_rank)));
    if (k > mr || k > mc) return err("too few samples for the rank");
    // bases of Psi(:, Pi_col) and Psi(Pi_row, :)^T
    std::vector<double> X((size_t)k * N), Y((size_t)k * N);
    for (int j = 0; j < k; ++j) {
        std::memcpy(&X[(size_t)j * N], &colsp[(size_t)pc[j] * N], sizeof(double) * N);
        std::memcpy(&Y[(size_t)j * N], &rowsp[(size_t)pr[j] * N], sizeof(double) * N);
    }
    const std::vector<double> Qc = orthonormal_basis(X, N, k);
    const std::vector<double> Qr = orthonormal_basis(Y, N, k);
    // M = Qc(Rs, :)^+ W (Qr(Cs, :)^T)^+
    std::vector<double> A((size_t)mr * k), B((size_t)mc * k);
    for (int a = 0; a < mr; ++a)
        for (int j = 0; j < k; ++j) A[(size_t)a * k + j] = Qc[(size_t)j * N + Rs[a]];
    for (int b = 0; b < mc; ++b)
        for (int j = 0; j < k; ++j) B[(size_t)b * k + j] = Qr[(size_t)j * N + Cs[b]];
    const std::vector<double> PA = pinv_tall(A, mr, k);   // k x mr
    const std::vector<double> PB = pinv_tall(B, mc, k);   // k x mc; (B^T)^+ = PB^T
    std::vector<double> T((size_t)k * mc, 0.0), M((size_t)k * k, 0.0);
    for (int i = 0; i < k; ++i)
        for (int a = 0; a < mr; ++a) {
            const double pa = PA[(size_t)i * mr + a];
            for (int b = 0; b < mc; ++b) T[(size_t)i * mc + b] += pa * W[(size_t)a * mc + b];
        }
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) {
            double s = 0.0;
            for (int b = 0; b < mc; ++b) s += T[(size_t)i * mc + b] * PB[(size_t)j * mc + b];
            M[(size_t)i * k + j] = s;
        }
    std::vector<double> Um, sv, Vm;
    jacobi_svd(M, k, Um, sv, Vm);
    // U = Qc Um diag(s), V = Qr Vm, row stride cap_rank, zero past k
    for (long long t = 0; t < N; ++t) {
        for (int j = 0; j < cap_rank; ++j) {
            double u = 0.0, v = 0.0;
            if (j < k)
                for (int i = 0; i < k; ++i) {
                    u += Qc[(size_t)i * N + t] * Um[(size_t)i * k + j];
                    v += Qr[(size_t)i * N + t] * Vm[(size_t)i * k + j];
                }
            U[(size_t)t * cap_rank + j] = u * (j < k ? sv[j] : 0.0);
            V[(size_t)t * cap_rank + j] = v;
        }
    }
    *rank_out = k;
    return BF_OK;
}

int unwrap_vector(const double* u, long long n, double tau, double* v,
                  long long* disc, int cap, int* ndisc) {
    std::vector<long long> S;
    unwrap(u, n, tau, nullptr, v, S);
    *ndisc = (int)S.size();
    for (int i = 0; i < (int)S.size() && i < cap; ++i) disc[i] = S[i];
    return BF_OK;
}

}  // namespace bfi
