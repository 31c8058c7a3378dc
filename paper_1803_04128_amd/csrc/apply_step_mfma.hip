// One launch per computed step with the contractions on MFMA: the per-level
// form for plans whose ranks are too large for the fused passes (2D boxes of
// up to 8 x 8 points, 64 coefficients per pair).
//
// Each kernel multiplies real (or complex) r_out x r_in blocks into panels of
// 16 columns with v_mfma_f32_16x16x4f32.  Operand layout (checked by an
// in-bounds probe): A lane l = A[l % 16][l / 16], B lane l = B[l / 16][l % 16],
// D lane l holds D[4 (l / 16) + j][l % 16], j < 4.  The shared Lagrange
// matrices come pre-arranged in the A order (Step::amat), so every A load is
// one coalesced 256-byte read; the input panel of a unit is staged in LDS.
// The state layout and the unit / pair index math are those of the vector
// ALU per-step kernels.
#include "apply_common.h"

namespace bfi {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ floatx4 mma(float a, float b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

constexpr int kCols = 16;      // panel columns per block
constexpr int kMaxMT = 4;      // row tiles: r_out <= 64

__device__ __forceinline__ floatx4 zero4() {
    floatx4 z = {0.f, 0.f, 0.f, 0.f};
    return z;
}

}  // namespace

// xi step (eq. (eqn:2) regrouped), block = (unit, 16-column tile); WPC waves
// per output child i share its row tiles (wave h takes tiles h, h + WPC,
// ...): D_i = sum_c M_c (W_{i,c} . X_c).
template <int R, int WPC, bool TWO>
__global__ void __launch_bounds__(R * 64 * WPC) xi_step_mfma(StepArgs a) {
    constexpr int NT = kMaxMT / WPC;                    // tiles per wave
    extern __shared__ float2 lds_step[];
    float2* xs = lds_step;                              // [R][r_in][16]
    float2* ws = xs + (size_t)R * a.r_in * kCols;       // [R][R][r_in]
    const int nct = (a.Vc + kCols - 1) / kCols;
    const long long u = (long long)blockIdx.x / nct;
    const int col0 = (int)((long long)blockIdx.x - u * nct) * kCols;
    const int shiftB = a.dim * (a.L - a.level);
    const long long ap = u >> shiftB, b = u & ((1LL << shiftB) - 1);
    const int nin = R * a.r_in * kCols;
    for (int e = threadIdx.x; e < nin; e += R * 64 * WPC) {
        const int n = e % kCols, cs = e / kCols;
        const int c = cs / a.r_in, s = cs - c * a.r_in;
        const int col = col0 + n;
        float2 v = make_float2(0.f, 0.f);
        if (col < a.Vc) {
            if (a.reads_f) {
                v = head_value(a, b * R + c, s, col);
            } else {
                const long long pin = (ap << (shiftB + a.dim)) + (b << a.dim) + c;
                v = a.in[(pin * a.r_in + s) * a.Vc + col];
            }
        }
        xs[e] = v;
    }
    const int ntw = R * R * a.r_in;
    for (int e = threadIdx.x; e < ntw; e += R * 64 * WPC)
        ws[e] = step_twiddle<TWO>(a, STEP_XI, u * ntw + e);
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = wave / WPC, h = wave - i * WPC;
    const int kq = lane >> 4, n = lane & 15;
    const int MT = (a.r_out + 15) >> 4, KS = (a.r_in + 3) >> 2;
    floatx4 accr[NT], acci[NT];
#pragma unroll
    for (int q = 0; q < NT; ++q) accr[q] = acci[q] = zero4();
    for (int c = 0; c < R; ++c) {
        const float* am = a.amat + (size_t)c * MT * KS * 64 + lane;
        const float2* w = ws + (i * R + c) * a.r_in;
        const float2* x = xs + (size_t)c * a.r_in * kCols + n;
        // the next K step's A operands are read while this one multiplies
        float an[NT];
#pragma unroll
        for (int q = 0; q < NT; ++q) {
            const int m = h + q * WPC;
            an[q] = m < MT ? am[m * KS * 64] : 0.f;
        }
        for (int ks = 0; ks < KS; ++ks) {
            float ac[NT];
#pragma unroll
            for (int q = 0; q < NT; ++q) ac[q] = an[q];
            if (ks + 1 < KS) {
#pragma unroll
                for (int q = 0; q < NT; ++q) {
                    const int m = h + q * WPC;
                    if (m < MT) an[q] = am[(m * KS + ks + 1) * 64];
                }
            }
            const int s = 4 * ks + kq;
            float2 z = make_float2(0.f, 0.f);
            if (s < a.r_in) z = cmul(w[s], x[s * kCols]);
#pragma unroll
            for (int q = 0; q < NT; ++q) {
                if (h + q * WPC < MT) {                 // uniform
                    accr[q] = mma(ac[q], z.x, accr[q]);
                    acci[q] = mma(ac[q], z.y, acci[q]);
                }
            }
        }
    }
    const int col = col0 + n;
    if (col >= a.Vc) return;
    const long long pout = ((ap * R + i) << shiftB) + b;
    float2* o = a.out + pout * a.r_out * a.Vc + col;
#pragma unroll
    for (int q = 0; q < NT; ++q) {
        const int m = h + q * WPC;
        if (m < MT) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int t = 16 * m + 4 * kq + j;
                if (t < a.r_out)
                    o[(size_t)t * a.Vc] = make_float2(accr[q][j], acci[q][j]);
            }
        }
    }
}

// x step (eq. (eqn:3) regrouped), block = (unit, 16-column tile); WPC waves
// per output child i share its row tiles (wave h takes tiles h, h + WPC,
// ...): D_i = sum_c T_{i,c} . (M_i X_c).
template <int R, int WPC, bool TWO>
__global__ void __launch_bounds__(R * 64 * WPC) x_step_mfma(StepArgs a) {
    constexpr int NT = kMaxMT / WPC;                    // tiles per wave
    extern __shared__ float2 lds_step[];
    float2* xs = lds_step;                              // [R][r_in][16]
    float2* ts = xs + (size_t)R * a.r_in * kCols;       // [R][R][r_out]
    const int nct = (a.Vc + kCols - 1) / kCols;
    const long long u = (long long)blockIdx.x / nct;
    const int col0 = (int)((long long)blockIdx.x - u * nct) * kCols;
    const int shiftB = a.dim * (a.L - a.level);
    const long long ap = u >> shiftB, b = u & ((1LL << shiftB) - 1);
    const int nin = R * a.r_in * kCols;
    for (int e = threadIdx.x; e < nin; e += R * 64 * WPC) {
        const int n = e % kCols, cs = e / kCols;
        const int c = cs / a.r_in, s = cs - c * a.r_in;
        const int col = col0 + n;
        float2 v = make_float2(0.f, 0.f);
        if (col < a.Vc) {
            const long long pin = (ap << (shiftB + a.dim)) + (b << a.dim) + c;
            v = a.in[(pin * a.r_in + s) * a.Vc + col];
        }
        xs[e] = v;
    }
    const int ntw = R * R * a.r_out;
    for (int e = threadIdx.x; e < ntw; e += R * 64 * WPC)
        ts[e] = step_twiddle<TWO>(a, STEP_X, u * ntw + e);
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = wave / WPC, h = wave - i * WPC;
    const int kq = lane >> 4, n = lane & 15;
    const int MT = (a.r_out + 15) >> 4, KS = (a.r_in + 3) >> 2;
    const float* am = a.amat + (size_t)i * MT * KS * 64 + lane;
    floatx4 accr[NT], acci[NT];
#pragma unroll
    for (int q = 0; q < NT; ++q) accr[q] = acci[q] = zero4();
    for (int c = 0; c < R; ++c) {
        floatx4 yr[NT], yi[NT];
#pragma unroll
        for (int q = 0; q < NT; ++q) yr[q] = yi[q] = zero4();
        const float2* x = xs + (size_t)c * a.r_in * kCols + n;
        // the next K step's A operands are read while this one multiplies
        float an[NT];
#pragma unroll
        for (int q = 0; q < NT; ++q) {
            const int m = h + q * WPC;
            an[q] = m < MT ? am[m * KS * 64] : 0.f;
        }
        for (int ks = 0; ks < KS; ++ks) {
            float ac[NT];
#pragma unroll
            for (int q = 0; q < NT; ++q) ac[q] = an[q];
            if (ks + 1 < KS) {
#pragma unroll
                for (int q = 0; q < NT; ++q) {
                    const int m = h + q * WPC;
                    if (m < MT) an[q] = am[(m * KS + ks + 1) * 64];
                }
            }
            const int s = 4 * ks + kq;
            const float2 xv = s < a.r_in ? x[s * kCols] : make_float2(0.f, 0.f);
#pragma unroll
            for (int q = 0; q < NT; ++q) {
                if (h + q * WPC < MT) {                 // uniform
                    yr[q] = mma(ac[q], xv.x, yr[q]);
                    yi[q] = mma(ac[q], xv.y, yi[q]);
                }
            }
        }
        const float2* tw = ts + (i * R + c) * a.r_out;
#pragma unroll
        for (int q = 0; q < NT; ++q) {
            const int m = h + q * WPC;
            if (m < MT) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int t = 16 * m + 4 * kq + j;
                    const float2 T = t < a.r_out ? tw[t] : make_float2(0.f, 0.f);
                    accr[q][j] += T.x * yr[q][j] - T.y * yi[q][j];
                    acci[q][j] += T.x * yi[q][j] + T.y * yr[q][j];
                }
            }
        }
    }
    const int col = col0 + n;
    if (col >= a.Vc) return;
    const long long pout = ((ap * R + i) << shiftB) + b;
    float2* o = a.out + pout * a.r_out * a.Vc + col;
#pragma unroll
    for (int q = 0; q < NT; ++q) {
        const int m = h + q * WPC;
        if (m < MT) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int t = 16 * m + 4 * kq + j;
                if (t < a.r_out)
                    o[(size_t)t * a.Vc] = make_float2(accr[q][j], acci[q][j]);
            }
        }
    }
}

// Switch (Algorithm 4.1 step 4 regrouped), block = (pair, 16-column tile),
// wave m = row tile m of nu = S mu.  The complex block S enters as two real
// A operands (Re S, Im S) read straight from HBM in the A layout (each lane
// its row and four consecutive K columns), all K steps issued before the
// input panel is staged in LDS, so that the reads overlap the staging and
// the small LDS footprint lets many blocks stream S at once.
__global__ void __launch_bounds__(kMaxMT * 64) switch_step_mfma(StepArgs a) {
    extern __shared__ float2 lds_step[];
    float2* xs = lds_step;                              // [r_in][16]
    const int nct = (a.Vc + kCols - 1) / kCols;
    const long long p = (long long)blockIdx.x / nct;
    const int col0 = (int)((long long)blockIdx.x - p * nct) * kCols;
    const int shiftB = a.dim * (a.L - a.level);
    const long long bm = p & ((1LL << shiftB) - 1);
    const int m = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int kq = lane >> 4, n = lane & 15;
    const int KS = (a.r_in + 3) >> 2;
    const int row = 16 * m + n;
    const float2* S = a.S + p * a.r_out * a.r_in + (size_t)row * a.r_in;
    float2 sv[16];
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) {
        const int s = 4 * ks + kq;
        sv[ks] = (ks < KS && row < a.r_out && s < a.r_in) ? S[s]
                                                        : make_float2(0.f, 0.f);
    }
    const int nthr = blockDim.x;
    for (int e = threadIdx.x; e < a.r_in * kCols; e += nthr) {
        const int nn = e % kCols, s = e / kCols;
        const int col = col0 + nn;
        float2 v = make_float2(0.f, 0.f);
        if (col < a.Vc)
            v = a.reads_f ? head_value(a, bm, s, col)
                          : a.in[(p * a.r_in + s) * a.Vc + col];
        xs[e] = v;
    }
    __syncthreads();
    floatx4 p1 = zero4(), p2 = zero4(), p3 = zero4(), p4 = zero4();
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) {
        if (ks < KS) {                                  // uniform
            const int s = 4 * ks + kq;
            const float2 xv = s < a.r_in ? xs[s * kCols + n]
                                         : make_float2(0.f, 0.f);
            p1 = mma(sv[ks].x, xv.x, p1);
            p2 = mma(sv[ks].y, xv.y, p2);
            p3 = mma(sv[ks].x, xv.y, p3);
            p4 = mma(sv[ks].y, xv.x, p4);
        }
    }
    const int col = col0 + n;
    if (col >= a.Vc) return;
    float2* o = a.out + p * a.r_out * a.Vc + col;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int t = 16 * m + 4 * kq + j;
        if (t < a.r_out)
            o[(size_t)t * a.Vc] = make_float2(p1[j] - p2[j], p3[j] + p4[j]);
    }
}

// Switch step with its block generated in registers instead of read from
// HBM (the factor construction's S, computed during the apply): one block
// per pair (A, B) of the switch level.  The phase terms that depend on one
// side only, Phi(c_A, xi_s) and Phi(x_t, c_B), and the x quantities of the
// phase formula are evaluated once per pair in FP64 into LDS; each lane then
// forms its A-operand entries
//   S[t][s] = exp(2 pi i [Phi(x_t, xi_s) - Phi(c_A, xi_s) - Phi(x_t, c_B)])
// with the phase difference in FP64, reduced modulo 1, then an FP32
// sincospi, and the block is applied to every 16-column tile of the pair.
struct OtfArgs {
    StepArgs s;
    PhaseSpec P;
    Axis ax_in, ax_out;
    int writes_lambda;
};

constexpr int kOtfRank = kMaxMT * 16;

__device__ __forceinline__ float2 expi_frac32(double v) {
    const float t = (float)(v - rint(v));
    float sn, cs;
    sincospif(2.0f * t, &sn, &cs);
    return make_float2(cs, sn);
}

template <int KIND>
__global__ void __launch_bounds__(kMaxMT * 64) switch_otf_mfma(OtfArgs o) {
    const StepArgs& a = o.s;
    extern __shared__ float2 lds_step[];
    float2* xs = lds_step;                              // [r_in][16]
    double* phs = (double*)(xs + (size_t)a.r_in * kCols);  // [r_in]
    double* pht = phs + kOtfRank;                       // [r_out]
    XPre* xq = (XPre*)(pht + kOtfRank);                 // [r_out] or [r_in]
    int2* xig = (int2*)(xq + kOtfRank);                 // [r_in] grid of xi_s
    const long long p = blockIdx.x;
    const int shiftB = a.dim * (a.L - a.level);
    const long long am = p >> shiftB, bm = p & ((1LL << shiftB) - 1);
    int Ac[2], Bc[2], cA[2], cB[2];
    box_coords(am, a.dim, Ac);
    box_coords(bm, a.dim, Bc);
    center_grid(Ac, a.n >> a.level, a.dim, cA);
    center_grid(Bc, a.n >> (a.L - a.level), a.dim, cB);
    // the formula's x argument is the output point x_t, or for K^T the
    // input point xi_s
    const bool tr = o.P.transpose != 0;
    for (int e = threadIdx.x; e < a.r_in; e += blockDim.x) {
        int xi[2];
        point_grid(Bc, o.ax_in, e, a.dim, xi);
        phs[e] = a.reads_f ? 0.0 : phase_value(o.P, cA, xi);
        if (tr) xq[e] = phase_xpre(o.P, xi);
        xig[e] = make_int2(xi[0], a.dim > 1 ? xi[1] : 0);
    }
    for (int e = threadIdx.x; e < a.r_out; e += blockDim.x) {
        int x[2];
        point_grid(Ac, o.ax_out, e, a.dim, x);
        pht[e] = o.writes_lambda ? 0.0 : phase_value(o.P, x, cB);
        if (!tr) xq[e] = phase_xpre(o.P, x);
    }
    __syncthreads();
    const int m = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int kq = lane >> 4, n = lane & 15;
    const int KS = (a.r_in + 3) >> 2;
    const int row = 16 * m + n;
    const double sg = o.P.conjugate ? -1.0 : 1.0;
    int x[2] = {0, 0};
    XPre qrow{0.0, 0.0};
    double prow = 0.0;
    if (row < a.r_out) {
        point_grid(Ac, o.ax_out, row, a.dim, x);
        if (!tr) qrow = xq[row];
        prow = pht[row];
    }
    float2 sv[16];
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) {
        const int s = 4 * ks + kq;
        sv[ks] = make_float2(0.f, 0.f);
        if (ks < KS && row < a.r_out && s < a.r_in) {
            const int2 g = xig[s];
            const int xi[2] = {g.x, g.y};
            double v = tr ? phase_formula_k<KIND>(o.P, xq[s], xi, x)
                          : phase_formula_k<KIND>(o.P, qrow, x, xi);
            v = sg * v - phs[s];
            v -= prow;
            sv[ks] = expi_frac32(v);
        }
    }
    const int nct = (a.Vc + kCols - 1) / kCols;
    for (int ct = 0; ct < nct; ++ct) {
        const int col0 = ct * kCols;
        if (ct > 0) __syncthreads();                    // tile ct-1 read
        for (int e = threadIdx.x; e < a.r_in * kCols; e += blockDim.x) {
            const int nn = e % kCols, s = e / kCols;
            const int col = col0 + nn;
            float2 v = make_float2(0.f, 0.f);
            if (col < a.Vc)
                v = a.reads_f ? head_value(a, bm, s, col)
                              : a.in[(p * a.r_in + s) * a.Vc + col];
            xs[e] = v;
        }
        __syncthreads();
        floatx4 p1 = zero4(), p2 = zero4(), p3 = zero4(), p4 = zero4();
#pragma unroll
        for (int ks = 0; ks < 16; ++ks) {
            if (ks < KS) {                              // uniform
                const int s = 4 * ks + kq;
                const float2 xv = s < a.r_in ? xs[s * kCols + n]
                                             : make_float2(0.f, 0.f);
                p1 = mma(sv[ks].x, xv.x, p1);
                p2 = mma(sv[ks].y, xv.y, p2);
                p3 = mma(sv[ks].x, xv.y, p3);
                p4 = mma(sv[ks].y, xv.x, p4);
            }
        }
        const int col = col0 + n;
        if (col < a.Vc) {
            float2* out = a.out + p * a.r_out * a.Vc + col;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int t = 16 * m + 4 * kq + j;
                if (t < a.r_out)
                    out[(size_t)t * a.Vc] =
                        make_float2(p1[j] - p2[j], p3[j] + p4[j]);
            }
        }
    }
}

static size_t otf_lds(const Step& s) {
    return (size_t)s.r_in * kCols * sizeof(float2) +
           2 * kOtfRank * sizeof(double) + kOtfRank * sizeof(XPre) +
           kOtfRank * sizeof(int2);
}

// LDS bytes of one block of the step's kernel.
size_t step_mfma_lds(const Plan& p, const Step& s) {
    if (s.kind == STEP_SWITCH)
        return p.switch_otf ? otf_lds(s)
                            : (size_t)s.r_in * kCols * sizeof(float2);
    const int rt = s.kind == STEP_XI ? s.r_in : s.r_out;
    return ((size_t)p.R * s.r_in * kCols + (size_t)p.R * p.R * rt) *
           sizeof(float2);
}

void init_step_mfma_attrs() {
    static bool done = false;
    if (done) return;
    const void* fns[] = {(const void*)xi_step_mfma<2, 1, false>,
                         (const void*)xi_step_mfma<4, 2, false>,
                         (const void*)x_step_mfma<2, 1, false>,
                         (const void*)x_step_mfma<4, 2, false>,
                         (const void*)xi_step_mfma<2, 1, true>,
                         (const void*)xi_step_mfma<4, 2, true>,
                         (const void*)x_step_mfma<2, 1, true>,
                         (const void*)x_step_mfma<4, 2, true>,
                         (const void*)switch_step_mfma,
                         (const void*)switch_otf_mfma<BF_PHASE_DFT>,
                         (const void*)switch_otf_mfma<BF_PHASE_FIO1D>,
                         (const void*)switch_otf_mfma<BF_PHASE_RADON2D>,
                         (const void*)switch_otf_mfma<BF_PHASE_SEPARABLE>,
                         (const void*)switch_otf_mfma<BF_PHASE_FIO1D_WARP>,
                         (const void*)switch_otf_mfma<BF_PHASE_LOWRANK>};
    for (const void* fn : fns)
        (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  160 * 1024);
    done = true;
}

// Launches one step; "" on success.
std::string launch_step_sep(const Plan& p, const Step& s, StepArgs a,
                            hipStream_t st);

std::string launch_step_mfma(const Plan& p, const Step& s, const StepArgs& a,
                             hipStream_t st) {
    if (s.r_out > kMaxMT * 16) return "step rank above 64";
    const long long nct = (a.Vc + kCols - 1) / kCols;
    const size_t lds = step_mfma_lds(p, s);
    if (lds > 160 * 1024) return "step does not fit in LDS";
    init_step_mfma_attrs();
    if (s.kind == STEP_SWITCH && p.switch_otf) {
        if (s.units > 0x7fffffffLL) return "switch grid too large";
        if (s.r_in > kOtfRank) return "switch rank above 64";
        const int MT = (s.r_out + 15) / 16;
        OtfArgs o{};
        o.s = a;
        o.P = p.phase;
        o.ax_in = s.ax_in;
        o.ax_out = s.ax_out;
        o.writes_lambda = s.writes_lambda ? 1 : 0;
        const dim3 grid((unsigned)s.units), block(64 * MT);
        switch (p.phase.kind) {
            case BF_PHASE_DFT:
                hipLaunchKernelGGL(switch_otf_mfma<BF_PHASE_DFT>, grid, block,
                                   lds, st, o);
                break;
            case BF_PHASE_FIO1D:
                hipLaunchKernelGGL(switch_otf_mfma<BF_PHASE_FIO1D>, grid,
                                   block, lds, st, o);
                break;
            case BF_PHASE_RADON2D:
                hipLaunchKernelGGL(switch_otf_mfma<BF_PHASE_RADON2D>, grid,
                                   block, lds, st, o);
                break;
            case BF_PHASE_SEPARABLE:
                hipLaunchKernelGGL(switch_otf_mfma<BF_PHASE_SEPARABLE>, grid,
                                   block, lds, st, o);
                break;
            case BF_PHASE_FIO1D_WARP:
                hipLaunchKernelGGL(switch_otf_mfma<BF_PHASE_FIO1D_WARP>, grid,
                                   block, lds, st, o);
                break;
            case BF_PHASE_LOWRANK:
                hipLaunchKernelGGL(switch_otf_mfma<BF_PHASE_LOWRANK>, grid,
                                   block, lds, st, o);
                break;
            default:
                return "unknown phase kind";
        }
    } else if (s.kind == STEP_SWITCH) {
        const long long nb = s.units * nct;
        if (nb > 0x7fffffffLL) return "switch grid too large";
        const int MT = (s.r_out + 15) / 16;
        hipLaunchKernelGGL(switch_step_mfma, dim3((unsigned)nb), dim3(64 * MT),
                           lds, st, a);
    } else if (step_sep_ok(p, s)) {
        return launch_step_sep(p, s, a, st);
    } else {
        const long long nb = s.units * nct;
        if (nb > 0x7fffffffLL) return "step grid too large";
        const dim3 grid((unsigned)nb);
        const bool xi = s.kind == STEP_XI;
        if (p.R == 2 && p.twiddle_otf) {
            if (xi)
                hipLaunchKernelGGL((xi_step_mfma<2, 1, true>), grid, dim3(128),
                                   lds, st, a);
            else
                hipLaunchKernelGGL((x_step_mfma<2, 1, true>), grid, dim3(128),
                                   lds, st, a);
        } else if (p.R == 2) {
            if (xi)
                hipLaunchKernelGGL((xi_step_mfma<2, 1, false>), grid,
                                   dim3(128), lds, st, a);
            else
                hipLaunchKernelGGL((x_step_mfma<2, 1, false>), grid,
                                   dim3(128), lds, st, a);
        } else if (p.twiddle_otf) {
            if (xi)
                hipLaunchKernelGGL((xi_step_mfma<4, 2, true>), grid, dim3(512),
                                   lds, st, a);
            else
                hipLaunchKernelGGL((x_step_mfma<4, 2, true>), grid, dim3(512),
                                   lds, st, a);
        } else {
            if (xi)
                hipLaunchKernelGGL((xi_step_mfma<4, 2, false>), grid,
                                   dim3(512), lds, st, a);
            else
                hipLaunchKernelGGL((x_step_mfma<4, 2, false>), grid,
                                   dim3(512), lds, st, a);
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return std::string("step launch: ") + hipGetErrorString(e);
    return "";
}

}  // namespace bfi
