// The entries of the stored factors as functions of their index: each
// twiddle W, T (Algorithm 4.1, eqs. (eqn:2), (eqn:3) regrouped) and switch
// entry S is exp(2 pi i [sum of phase terms]) at grid points and centers
// that the entry's index determines.  The construction kernels evaluate
// them into the factor arrays, the diagnostic read-back decodes stored
// entries with them, and the per-step apply kernels of a plan that stores
// no twiddles evaluate them where they would read the array.
#pragma once

#include "bf_device.h"

namespace bfi {

struct TwArgs {
    PhaseSpec P;
    Axis ax_in, ax_out;
    int L, level, reads_f, writes_lambda;
    long long total;
    float2* out;
};

// The phase terms of one stored factor entry: the entry is
// exp(2 pi i [Phi(ix_0, jx_0) - Phi(ix_1, jx_1) - Phi(ix_2, jx_2)]) over the
// first `count` terms (grid coordinates; ix on the output tree, jx on the
// input tree, as phase_value takes them).  The construction kernels and the
// diagnostic read-back (factor_entries) decode entries with these functions.
struct Terms {
    int count;
    int ix[3][2];
    int jx[3][2];
};

// point_grid / center_grid with the dimension loop at a fixed trip count,
// so that the term arrays stay in registers (a loop over the run-time
// dimension indexes them dynamically, which puts them in scratch memory)
__device__ __forceinline__ void term_point(const int* bc, const Axis& ax,
                                           int t, int dim, int* g) {
#pragma unroll
    for (int d = 0; d < 2; ++d)
        if (d < dim)
            g[d] = bc[d] * ax.side + ax.off[point_digit(t, ax.r1, dim, d)];
}

__device__ __forceinline__ void term_center(const int* bc, int side, int dim,
                                            int* g) {
#pragma unroll
    for (int d = 0; d < 2; ++d)
        if (d < dim) g[d] = bc[d] * side + (side - 1) / 2;
}

__device__ __forceinline__ void term_copy(const int* from, int dim, int* to) {
#pragma unroll
    for (int d = 0; d < 2; ++d)
        if (d < dim) to[d] = from[d];
}

// W (or D+ when the step reads f): [u][i][c][s]
__device__ __forceinline__ Terms xi_terms(const TwArgs& a, long long idx) {
    const int dim = a.P.dim, R = 1 << dim, n = a.P.n;
    const int r_in = a.ax_in.r1 * (dim == 2 ? a.ax_in.r1 : 1);
    const int shiftB = dim * (a.L - a.level);
    int s = (int)(idx % r_in);
    long long rest = idx / r_in;
    int c = (int)(rest % R);
    rest /= R;
    int i = (int)(rest % R);
    long long u = rest / R;
    long long ap = u >> shiftB, b = u & ((1LL << shiftB) - 1);
    int Ac[2], Pc[2], Cc[2];
    Terms T;
    box_coords(ap * R + i, dim, Ac);
    box_coords(ap, dim, Pc);
    box_coords(b * R + c, dim, Cc);
    term_point(Cc, a.ax_in, s, dim, T.jx[0]);
    term_center(Ac, n >> a.level, dim, T.ix[0]);
    T.count = 1;
    if (!a.reads_f) {
        term_center(Pc, n >> (a.level - 1), dim, T.ix[1]);
        term_copy(T.jx[0], dim, T.jx[1]);
        T.count = 2;
    }
    return T;
}

// T (or E+ on the last x step): [u][i][c][t]
__device__ __forceinline__ Terms x_terms(const TwArgs& a, long long idx) {
    const int dim = a.P.dim, R = 1 << dim, n = a.P.n;
    const int r_out = a.ax_out.r1 * (dim == 2 ? a.ax_out.r1 : 1);
    const int shiftB = dim * (a.L - a.level);
    int t = (int)(idx % r_out);
    long long rest = idx / r_out;
    int c = (int)(rest % R);
    rest /= R;
    int i = (int)(rest % R);
    long long u = rest / R;
    long long ap = u >> shiftB, b = u & ((1LL << shiftB) - 1);
    int Ac[2], Bc[2], Cc[2];
    Terms T;
    box_coords(ap * R + i, dim, Ac);
    box_coords(b, dim, Bc);
    box_coords(b * R + c, dim, Cc);
    term_point(Ac, a.ax_out, t, dim, T.ix[0]);
    term_center(Cc, n >> (a.L - a.level + 1), dim, T.jx[0]);
    T.count = 1;
    if (!a.writes_lambda) {
        term_copy(T.ix[0], dim, T.ix[1]);
        term_center(Bc, n >> (a.L - a.level), dim, T.jx[1]);
        T.count = 2;
    }
    return T;
}

// S: [p][t][s]
__device__ __forceinline__ Terms switch_terms(const TwArgs& a,
                                              long long idx) {
    const int dim = a.P.dim, n = a.P.n;
    const int r_in = a.ax_in.r1 * (dim == 2 ? a.ax_in.r1 : 1);
    const int r_out = a.ax_out.r1 * (dim == 2 ? a.ax_out.r1 : 1);
    const int shiftB = dim * (a.L - a.level);
    int s = (int)(idx % r_in);
    long long rest = idx / r_in;
    int t = (int)(rest % r_out);
    long long p = rest / r_out;
    long long am = p >> shiftB, bm = p & ((1LL << shiftB) - 1);
    int Ac[2], Bc[2];
    Terms T;
    box_coords(am, dim, Ac);
    box_coords(bm, dim, Bc);
    term_point(Ac, a.ax_out, t, dim, T.ix[0]);
    term_point(Bc, a.ax_in, s, dim, T.jx[0]);
    // the terms present: 0, then 1 unless the step reads f, then 2 unless
    // it writes lambda; slot k holds the k-th present term
    T.count = 1;
    if (!a.reads_f) {
        term_center(Ac, n >> a.level, dim, T.ix[1]);
        term_copy(T.jx[0], dim, T.jx[1]);
        T.count = 2;
    }
    if (!a.writes_lambda) {
        if (T.count == 1) {
            term_copy(T.ix[0], dim, T.ix[1]);
            term_center(Bc, n >> (a.L - a.level), dim, T.jx[1]);
        } else {
            term_copy(T.ix[0], dim, T.ix[2]);
            term_center(Bc, n >> (a.L - a.level), dim, T.jx[2]);
        }
        ++T.count;
    }
    return T;
}

// The entry's phase: FP64 terms, differences before the reduction modulo 1.
__device__ __forceinline__ double terms_phase(const PhaseSpec& P,
                                              const Terms& T) {
    double v = phase_value(P, T.ix[0], T.jx[0]);
#pragma unroll
    for (int k = 1; k < 3; ++k)
        if (k < T.count) v -= phase_value(P, T.ix[k], T.jx[k]);
    return v;
}

// Twiddle entry idx of a step (kind STEP_XI: W, or D+ at the head; STEP_X:
// T, or E+ on the last x step), as stored: exp(2 pi i v), v reduced modulo
// 1 in FP64, rounded to complex64.
__device__ __forceinline__ float2 twiddle_entry(const TwArgs& a, int kind,
                                                long long idx) {
    return expi_frac(terms_phase(
        a.P, kind == STEP_XI ? xi_terms(a, idx) : x_terms(a, idx)));
}

}  // namespace bfi
