// Device-side helpers shared by the library's kernels: box and point index
// math on the dyadic trees (Section 4), the phase functions in FP64, and
// complex arithmetic.
//
// Box numbering: a box at tree level l is named by its per-dimension box
// coordinates; in 2D these are interleaved into a Morton index (first
// coordinate on the odd bits) so that the children of box m are R m + c,
// c = c1 * 2 + c2.  Pairs at level l are stored at p = a * R^(L-l) + b.
#pragma once

#include <hip/hip_runtime.h>

#include "bf_internal.h"

namespace bfi {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__host__ __device__ __forceinline__ unsigned spread_bits(unsigned v) {
    v &= 0x0000ffffu;
    v = (v | (v << 8)) & 0x00ff00ffu;
    v = (v | (v << 4)) & 0x0f0f0f0fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

__host__ __device__ __forceinline__ unsigned compact_bits(unsigned v) {
    v &= 0x55555555u;
    v = (v | (v >> 1)) & 0x33333333u;
    v = (v | (v >> 2)) & 0x0f0f0f0fu;
    v = (v | (v >> 4)) & 0x00ff00ffu;
    v = (v | (v >> 8)) & 0x0000ffffu;
    return v;
}

// box index -> per-dimension box coordinates
__device__ __forceinline__ void box_coords(long long m, int dim, int* c) {
    if (dim == 1) {
        c[0] = (int)m;
    } else {
        c[0] = (int)compact_bits((unsigned)(m >> 1));
        c[1] = (int)compact_bits((unsigned)m);
    }
}

__device__ __forceinline__ long long box_index(const int* c, int dim) {
    if (dim == 1) return c[0];
    return ((long long)spread_bits((unsigned)c[0]) << 1) |
           (long long)spread_bits((unsigned)c[1]);
}

// digit d (0 = first dimension) of a flattened tensor point index
__device__ __forceinline__ int point_digit(int t, int r1, int dim, int d) {
    return dim == 1 ? t : (d == 0 ? t / r1 : t % r1);
}

// grid index of point t of the box with coordinates bc
__device__ __forceinline__ void point_grid(const int* bc, const Axis& ax,
                                           int t, int dim, int* g) {
    for (int d = 0; d < dim; ++d)
        g[d] = bc[d] * ax.side + ax.off[point_digit(t, ax.r1, dim, d)];
}

__device__ __forceinline__ void center_grid(const int* bc, int side, int dim,
                                            int* g) {
    for (int d = 0; d < dim; ++d) g[d] = bc[d] * side + (side - 1) / 2;
}

__device__ __forceinline__ long long user_index(const int* g, int dim,
                                                int n) {
    return dim == 1 ? (long long)g[0] : (long long)g[0] * n + g[1];
}

// Quantities of the phase formula that depend on its x argument alone
// (the coefficient functions c(x), c1(x), c2(x), the x part of a separable
// phase), so that a block of entries sharing x points evaluates them once.
struct XPre {
    double c1, c2;
};

__device__ __forceinline__ XPre phase_xpre(const PhaseSpec& P,
                                           const int* ix) {
    const double invn = P.invn;
    XPre q{0.0, 0.0};
    switch (P.kind) {
        case BF_PHASE_FIO1D:
        case BF_PHASE_FIO1D_WARP:
            q.c1 = (P.p[0] + P.p[1] * sinpi(2.0 * ix[0] * invn)) / P.p[2];
            break;
        case BF_PHASE_RADON2D: {
            double u = 2.0 * ix[0] * invn, v = 2.0 * ix[1] * invn;
            q.c1 = (P.p[0] + P.p[1] * sinpi(u) * sinpi(v)) / P.p[2];
            q.c2 = (P.p[3] + P.p[4] * cospi(u) * cospi(v)) / P.p[5];
            break;
        }
        case BF_PHASE_SEPARABLE: {
            double x2 = P.dim > 1 ? ix[1] * invn : 0.0;
            q.c1 = P.p[0] * sinpi(2.0 * ix[0] * invn) * (1.0 + x2);
            break;
        }
        default:
            break;
    }
    return q;
}

// Phase Phi(x_ix, xi_jx) in FP64 from the x quantities q = phase_xpre(ix),
// for the phase kind KIND.  The bilinear part x . xi = sum_d ix_d (jx_d -
// n/2) / n is reduced modulo 1 exactly in integers: n is a power of two, so
// the products may wrap modulo 2^32 and the sum is reduced with a mask.
// Only the fractional part of Phi is ever used.
template <int KIND>
__device__ __forceinline__ double phase_formula_k(const PhaseSpec& P,
                                                  const XPre& q,
                                                  const int* ix,
                                                  const int* jx) {
    const int n = P.n;
    const int dim = KIND == BF_PHASE_RADON2D ? 2
                    : (KIND == BF_PHASE_FIO1D || KIND == BF_PHASE_FIO1D_WARP)
                        ? 1
                        : P.dim;
    if (KIND == BF_PHASE_LOWRANK) {
        // Algorithm 2's input form: Phi = U(i, :) V(j, :)^T
        const double* u = P.U + user_index(ix, P.dim, n) * P.rank;
        const double* v = P.V + user_index(jx, P.dim, n) * P.rank;
        double s = 0.0;
        for (int k = 0; k < P.rank; ++k) s = fma(u[k], v[k], s);
        return s;
    }
    double bil = 0.0;
    if (KIND != BF_PHASE_SEPARABLE) {
        unsigned acc = 0;
        for (int d = 0; d < dim; ++d)
            acc += (unsigned)ix[d] * (unsigned)(jx[d] - n / 2);
        bil = (double)(acc & (unsigned)(n - 1)) * P.invn;
    }
    if (KIND == BF_PHASE_DFT) return bil;
    if (KIND == BF_PHASE_FIO1D)
        return bil + q.c1 * fabs((double)(jx[0] - n / 2));
    if (KIND == BF_PHASE_FIO1D_WARP)
        return bil + q.c1 * (double)(jx[0] - n / 2);
    if (KIND == BF_PHASE_RADON2D) {
        double x1 = (double)(jx[0] - n / 2), x2 = (double)(jx[1] - n / 2);
        return bil + sqrt(q.c1 * q.c1 * x1 * x1 + q.c2 * q.c2 * x2 * x2);
    }
    // BF_PHASE_SEPARABLE
    double nrm2 = 0.0;
    for (int d = 0; d < dim; ++d) {
        double x = (double)(jx[d] - n / 2);
        nrm2 += x * x;
    }
    return q.c1 + P.p[1] * sqrt(nrm2) + P.p[2] * nrm2 * P.invn;
}

__device__ __forceinline__ double phase_formula_pre(const PhaseSpec& P,
                                                    const XPre& q,
                                                    const int* ix,
                                                    const int* jx) {
    switch (P.kind) {
        case BF_PHASE_DFT:
            return phase_formula_k<BF_PHASE_DFT>(P, q, ix, jx);
        case BF_PHASE_FIO1D:
            return phase_formula_k<BF_PHASE_FIO1D>(P, q, ix, jx);
        case BF_PHASE_FIO1D_WARP:
            return phase_formula_k<BF_PHASE_FIO1D_WARP>(P, q, ix, jx);
        case BF_PHASE_RADON2D:
            return phase_formula_k<BF_PHASE_RADON2D>(P, q, ix, jx);
        case BF_PHASE_LOWRANK:
            return phase_formula_k<BF_PHASE_LOWRANK>(P, q, ix, jx);
        default:
            return phase_formula_k<BF_PHASE_SEPARABLE>(P, q, ix, jx);
    }
}

__device__ __forceinline__ double phase_formula(const PhaseSpec& P,
                                                const int* ix,
                                                const int* jx) {
    return phase_formula_pre(P, phase_xpre(P, ix), ix, jx);
}

// Phase of the factorized kernel at output-tree index ix and input-tree
// index jx.  For K that is Phi(x_ix, xi_jx).  The transposed kernel K^T
// (Scenario 2 of Section 1) has the output on the xi grid and the input on
// the x grid, so its phase is Phi(x_jx, xi_ix); the conjugate kernels
// negate it.  Algorithm 4.1 is otherwise unchanged.
__device__ __forceinline__ double phase_value(const PhaseSpec& P,
                                              const int* ix, const int* jx) {
    const double v = P.transpose ? phase_formula(P, jx, ix)
                                 : phase_formula(P, ix, jx);
    return P.conjugate ? -v : v;
}

// exp(2 pi i v) with v reduced to [-1/2, 1/2] first (FP64), stored FP32
__device__ __forceinline__ float2 expi_frac(double v) {
    double t = v - rint(v);
    double s, c;
    sincospi(2.0 * t, &s, &c);
    return make_float2((float)c, (float)s);
}

}  // namespace bfi
