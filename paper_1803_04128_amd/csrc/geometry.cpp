// Plan geometry on the host: interpolation points, Lagrange matrices and the
// level schedule of the butterfly apply.
//
// Points (Section 2.1, eqs. (eqn:gdA)/(eqn:gdB)): in a box of N_A indices
// with r points, x_t = Round(t + (N_A - r) s_t), 1-based, with the ascending
// Chebyshev node s_t = (1 - cos((t-1) pi / (r-1))) / 2.  (Printed, the +t
// offset is paired with the descending node, which collapses the set.)
// Round is half away from zero and a value within 1e-9 of a half-integer is
// an exact tie.  A box with N_A <= r uses all of its indices.
//
// Lagrange weights (Section 2.1): M_t(y) = prod_{j != t} (y - x_j) /
// (x_t - x_j), in FP64 from integer differences; they depend only on
// positions relative to the box, so each level holds one matrix per child
// position (the paper shifts the grid of a box not starting at index 1).
//
// Schedule: with single-index leaves a box of at most q indices per
// dimension interpolates through all of its points, so the xi levels with
// 2^l <= q are copies of f and the x levels whose parent box has at most q
// indices are plain sums (Algorithm 4.1, steps 2-3 and 5-6 specialised).
// Only levels l0 = floor(log2 q) + 1 .. h (xi) and h+1 .. L+1-l0 (x) are
// computed, plus the switch at h = floor(L / 2) (L - floor(L / 2) for the
// transposed kernel, whose factorization is then the exact transpose of
// K's).
#include <cmath>
#include <cstring>

#include "bf_internal.h"

namespace bfi {

int mock_chebyshev(int side, int q, int* off) {
    if (side <= q) {
        for (int i = 0; i < side; ++i) off[i] = i;
        return side;
    }
    int cnt = 0;
    long prev = -1;
    for (int t = 1; t <= q; ++t) {
        double s = (1.0 - std::cos((t - 1.0) * M_PI / (q - 1))) / 2.0;
        double v = t + (double)(side - q) * s;
        long x = (long)std::floor(v + 0.5 + 1e-9) - 1;
        if (x != prev) {
            off[cnt++] = (int)x;
            prev = x;
        }
    }
    return cnt;
}

void lagrange_1d(const int* nodes, int r, const double* y, int m,
                 double* out) {
    for (int k = 0; k < m; ++k) {
        for (int t = 0; t < r; ++t) {
            double v = 1.0;
            for (int j = 0; j < r; ++j) {
                if (j == t) continue;
                v *= (y[k] - (double)nodes[j]) /
                     (double)(nodes[t] - nodes[j]);
            }
            out[k * r + t] = v;
        }
    }
}

Axis make_axis(int side, int q) {
    Axis a{};
    a.side = side;
    a.r1 = mock_chebyshev(side, q, a.off);
    return a;
}

// multi-index digit d (0 = first dimension) of a flattened point index
static inline int digit(int t, int r1, int dim, int d) {
    for (int k = dim - 1; k > d; --k) t /= r1;
    return t % r1;
}

// child position bit for dimension d (child c = c1 * 2 + c2 in 2D)
static inline int child_bit(int c, int dim, int d) {
    return (c >> (dim - 1 - d)) & 1;
}

static int ipow(int b, int e) {
    int v = 1;
    for (int i = 0; i < e; ++i) v *= b;
    return v;
}

// XI matrices: M_c[t][s] = M_t^B(xi_s^C), B nodes = ax_out, C points =
// child offset + ax_in (box-relative to B).
static void xi_matrices(Step& s, int dim, int R) {
    const Axis& B = s.ax_out;
    const Axis& C = s.ax_in;
    s.mats_host.assign((size_t)R * s.r_out * s.r_in, 0.0);
    std::vector<double> w(B.r1);
    // the 1D factors L^c[t][s] = M_t^B(c side_C + off_C[s]) (2D only)
    s.lag1_host.clear();
    if (dim == 2) {
        s.lag1_host.assign((size_t)2 * B.r1 * C.r1, 0.0);
        for (int c = 0; c < 2; ++c)
            for (int si = 0; si < C.r1; ++si) {
                double y = c * C.side + C.off[si];
                lagrange_1d(B.off, B.r1, &y, 1, w.data());
                for (int t = 0; t < B.r1; ++t)
                    s.lag1_host[((size_t)c * B.r1 + t) * C.r1 + si] = w[t];
            }
    }
    for (int c = 0; c < R; ++c)
        for (int t = 0; t < s.r_out; ++t)
            for (int si = 0; si < s.r_in; ++si) {
                double v = 1.0;
                for (int d = 0; d < dim; ++d) {
                    double y = child_bit(c, dim, d) * C.side +
                               C.off[digit(si, C.r1, dim, d)];
                    lagrange_1d(B.off, B.r1, &y, 1, w.data());
                    v *= w[digit(t, B.r1, dim, d)];
                }
                s.mats_host[((size_t)c * s.r_out + t) * s.r_in + si] = v;
            }
}

// X matrices: M_i[t][s] = M_s^P(x_t^A), P nodes = ax_in, A points = child
// offset + ax_out (box-relative to P).
static void x_matrices(Step& s, int dim, int R) {
    const Axis& P = s.ax_in;
    const Axis& A = s.ax_out;
    s.mats_host.assign((size_t)R * s.r_out * s.r_in, 0.0);
    std::vector<double> w(P.r1);
    // the 1D factors L^i[t][s] = M_s^P(i side_A + off_A[t]) (2D only)
    s.lag1_host.clear();
    if (dim == 2) {
        s.lag1_host.assign((size_t)2 * A.r1 * P.r1, 0.0);
        for (int i = 0; i < 2; ++i)
            for (int t = 0; t < A.r1; ++t) {
                double y = i * A.side + A.off[t];
                lagrange_1d(P.off, P.r1, &y, 1, w.data());
                for (int si = 0; si < P.r1; ++si)
                    s.lag1_host[((size_t)i * A.r1 + t) * P.r1 + si] = w[si];
            }
    }
    for (int i = 0; i < R; ++i)
        for (int t = 0; t < s.r_out; ++t)
            for (int si = 0; si < s.r_in; ++si) {
                double v = 1.0;
                for (int d = 0; d < dim; ++d) {
                    double y = child_bit(i, dim, d) * A.side +
                               A.off[digit(t, A.r1, dim, d)];
                    lagrange_1d(P.off, P.r1, &y, 1, w.data());
                    v *= w[digit(si, P.r1, dim, d)];
                }
                s.mats_host[((size_t)i * s.r_out + t) * s.r_in + si] = v;
            }
}

std::string build_schedule(Plan& p) {
    const int d = p.dim;
    p.L = ilog2(p.n);
    // switch level floor(L / 2); the factorization of K^T mirrors K's (its
    // recursion in xi is the transpose of K's recursion in x), so it
    // switches at L - floor(L / 2) and is the exact transpose of K's
    p.h = p.phase.transpose ? p.L - p.L / 2 : p.L / 2;
    p.R = 1 << d;
    p.N = 1;
    for (int k = 0; k < d; ++k) p.N *= p.n;
    p.l0 = ilog2(p.q) + 1;
    p.l1 = p.L + 1 - p.l0;
    p.lend = p.l1 >= p.h + 1 ? p.l1 : p.h;
    p.steps.clear();
    const int R = p.R;
    p.max_rank = 1;

    for (int l = p.l0; l <= p.h; ++l) {
        Step s;
        s.kind = STEP_XI;
        s.level = l;
        s.ax_in = make_axis(1 << (l - 1), p.q);
        s.ax_out = make_axis(1 << l, p.q);
        s.r_in = ipow(s.ax_in.r1, d);
        s.r_out = ipow(s.ax_out.r1, d);
        s.reads_f = (l == p.l0);
        s.units = p.N / R;
        s.tw_elems = (size_t)s.units * R * R * s.r_in;
        s.mat_elems = (size_t)R * s.r_out * s.r_in;
        s.amat_elems = (size_t)R * ((s.r_out + 15) / 16) * ((s.r_in + 3) / 4) * 64;
        if (p.dim == 1 && s.r_out <= 16)
            s.amat_xi_elems = (size_t)((s.r_in + 1) / 2) * 64;
        xi_matrices(s, d, R);
        p.steps.push_back(s);
    }
    {
        Step s;
        s.kind = STEP_SWITCH;
        s.level = p.h;
        s.ax_in = make_axis(1 << p.h, p.q);            // B at level L-h
        s.ax_out = make_axis(1 << (p.L - p.h), p.q);   // A at level h
        s.r_in = ipow(s.ax_in.r1, d);
        s.r_out = ipow(s.ax_out.r1, d);
        s.reads_f = p.l0 > p.h;
        s.writes_lambda = p.l1 < p.h + 1;
        s.units = p.N;
        s.S_elems = (size_t)p.N * s.r_out * s.r_in;
        p.steps.push_back(s);
    }
    for (int l = p.h + 1; l <= p.l1; ++l) {
        Step s;
        s.kind = STEP_X;
        s.level = l;
        s.ax_in = make_axis(1 << (p.L - l + 1), p.q);  // P
        s.ax_out = make_axis(1 << (p.L - l), p.q);     // A
        s.r_in = ipow(s.ax_in.r1, d);
        s.r_out = ipow(s.ax_out.r1, d);
        s.writes_lambda = (l == p.l1);
        s.units = p.N / R;
        s.tw_elems = (size_t)s.units * R * R * s.r_out;
        s.mat_elems = (size_t)R * s.r_out * s.r_in;
        s.amat_elems = (size_t)R * ((s.r_out + 15) / 16) * ((s.r_in + 3) / 4) * 64;
        x_matrices(s, d, R);
        p.steps.push_back(s);
    }
    for (auto& s : p.steps) {
        if (s.r_in > kMaxRank || s.r_out > kMaxRank)
            return "rank exceeds the supported maximum";
        p.max_rank = std::max(p.max_rank, std::max(s.r_in, s.r_out));
    }
    p.head_step_side = p.l0 <= p.h ? (1 << (p.l0 - 1)) : (1 << p.h);
    p.tail_side = 1 << (p.L - p.lend);

    // algorithmic work per apply column and factor bytes streamed per apply
    double fl = 0, by = 0;
    for (auto& s : p.steps) {
        fl += step_alg_flops(p, s, 1.0);
        by += s.kind == STEP_SWITCH ? s.S_elems * 8.0 : s.tw_elems * 8.0;
        by += s.mat_elems * 4.0;
    }
    const double nb = std::pow((double)R, p.L - p.lend);
    fl += (double)p.N * (nb * 2.0 + 8.0);
    p.flops_per_column = fl;
    p.factor_stream_bytes = by;
    return "";
}

}  // namespace bfi
