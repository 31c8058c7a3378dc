// Launch arguments and the input gather shared by the apply kernels.
#pragma once

#include "factor_terms.h"

namespace bfi {

struct StepArgs {
    const float2* in;      // state of the previous step (unused when reads_f)
    float2* out;
    const float2* tw;
    const float* mats;
    const float* amat;     // mats in MFMA A-operand order (Step::amat)
    const uint16_t* a16_hi;  // split parts of mats (Step::a16_hi / a16_lo)
    const uint16_t* a16_lo;
    const float* amat_sep;   // 2D: A tables of the 1D factors (Step)
    int a1, b1;              // 2D: input / output points per dimension
    const float2* S;
    const float2* f;       // vector chunk [nv][N] (when reads_f)
    const float2* bamp;    // b_k [r][N] or nullptr (alpha = 1)
    long long units;       // units (xi, x) or pairs (switch)
    long long N;
    int n, dim, L, level;
    int r_in, r_out;
    int Vc;                // columns in the chunk = nv * r_amp
    int r_amp;
    int reads_f;
    int head_side;         // side of the boxes f is read over
    TwArgs twa;            // the step's twiddle entries as functions of
                           // their index (kernels that generate them)
};

// Twiddle entry idx of the step: read from the stored array, or (TWO)
// evaluated in the apply exactly as the construction kernels store it.
template <bool TWO>
__device__ __forceinline__ float2 step_twiddle(const StepArgs& a, int kind,
                                               long long idx) {
    if constexpr (TWO)
        return twiddle_entry(a.twa, kind, idx);
    else
        return a.tw[idx];
}

struct TailArgs {
    const float2* in;
    float2* g;             // output chunk [nv][N]
    const float2* amp_a;   // a_k [r][N] or nullptr
    long long N, nb;       // nb = R^(L - lend) boxes summed per output
    int n, dim, side, r, Vc, r_amp, nv;
};

// Input of the first computed step: the exact levels below it are copies,
// so lambda^{PC} = f restricted to C (all indices of C are its points), and
// the column (v, k) carries b_k(xi) f_v(xi) (eq. (eqn:tg)).
__device__ __forceinline__ float2 head_value(const StepArgs& a, long long box,
                                             int s, int col) {
    int bc[2], gi[2];
    box_coords(box, a.dim, bc);
    if (a.dim == 1) {
        gi[0] = bc[0] * a.head_side + s;
    } else {
        gi[0] = bc[0] * a.head_side + s / a.head_side;
        gi[1] = bc[1] * a.head_side + s % a.head_side;
    }
    const long long j = user_index(gi, a.dim, a.n);
    const int vl = col / a.r_amp, k = col - vl * a.r_amp;
    const float2 fv = a.f[(size_t)vl * a.N + j];
    return a.bamp ? cmul(a.bamp[(size_t)k * a.N + j], fv) : fv;
}

inline StepArgs make_step_args(const Plan& p, const Step& s, int Vc,
                               const float2* f, const float2* in,
                               float2* out) {
    StepArgs a{};
    a.in = in;
    a.out = out;
    a.tw = s.tw;
    a.mats = s.mats;
    a.amat = s.amat;
    a.a16_hi = s.a16_hi;
    a.a16_lo = s.a16_lo;
    a.amat_sep = s.amat_sep;
    a.a1 = s.ax_in.r1;
    a.b1 = s.ax_out.r1;
    a.S = s.S;
    a.f = f;
    a.bamp = p.has_amp ? p.b_dev : nullptr;
    a.units = s.units;
    a.N = p.N;
    a.n = p.n;
    a.dim = p.dim;
    a.L = p.L;
    a.level = s.level;
    a.r_in = s.r_in;
    a.r_out = s.r_out;
    a.Vc = Vc;
    a.r_amp = p.r_amp;
    a.reads_f = s.reads_f ? 1 : 0;
    a.head_side = p.head_step_side;
    a.twa.P = p.phase;
    a.twa.L = p.L;
    a.twa.ax_in = s.ax_in;
    a.twa.ax_out = s.ax_out;
    a.twa.level = s.level;
    a.twa.reads_f = s.reads_f ? 1 : 0;
    a.twa.writes_lambda = s.writes_lambda ? 1 : 0;
    return a;
}

inline TailArgs make_tail_args(const Plan& p, int nv, const float2* in,
                               float2* g) {
    TailArgs t{};
    t.in = in;
    t.g = g;
    t.amp_a = p.has_amp ? p.a_dev : nullptr;
    t.N = p.N;
    t.nb = 1LL << (p.dim * (p.L - p.lend));
    t.n = p.n;
    t.dim = p.dim;
    t.side = p.tail_side;
    t.r = p.steps.back().r_out;
    t.Vc = nv * p.r_amp;
    t.r_amp = p.r_amp;
    t.nv = nv;
    return t;
}

std::string run_basic(Plan& p, int nv, const float2* f, float2* g,
                      float2* buf0, float2* buf1, hipStream_t st);

}  // namespace bfi
