// 2D per-step levels with the shared matrices contracted one dimension at a
// time (FP32 MFMA).  In 2D the Lagrange matrix of a child is the Kronecker
// product of 1D matrices, M_{(c1,c2)} = L^{c1} (x) L^{c2} (b x a each: b
// output, a input points per dimension; boxes are square, so both
// dimensions share L^0 and L^1).  Per unit and 16-column tile:
//   xi level (eq. (eqn:2) regrouped), output child i:
//     Z_{c1}[s1][t2] = sum_{c2, s2} L^{c2}[t2][s2] (W_{i,c} . X_c)[s1, s2]
//     Y_i[t1][t2]    = sum_{c1, s1} L^{c1}[t1][s1] Z_{c1}[s1][t2]
//   (the second-dimension children summed before the first dimension's
//   matrix: 4 a^2 b + 2 a b^2 multiply-adds per output child and column);
//   x level (eq. (eqn:3) regrouped), input child c:
//     Z_c[i2][s1][t2] = sum_{s2} L^{i2}[t2][s2] X_c[s1, s2]
//     Y_{i,c}[t1][t2] = sum_{s1} L^{i1}[t1][s1] Z_c[i2][s1][t2]
//     D_i += T_{i,c} . Y_{i,c}
//   (the second-dimension products formed once for both first-dimension
//   children: 2 a^2 b + 4 a b^2 per input child and column).
// Both stages run on v_mfma_f32_16x16x4f32 with the 1D matrices as A: the
// xi stages stack the two children along K (rows t, K = (child, s) <= 16),
// the x stages stack them along the rows (rows (child, t) <= 16, K = s);
// the two stages of a level meet in LDS.  Operand layout: A lane l =
// A[l % 16][l / 16], B lane l = B[l / 16][l % 16], D lane l holds
// D[4 (l / 16) + j][l % 16].
#include "apply_common.h"

namespace bfi {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kCols = 16;
constexpr int kSepWaves = 8;      // waves per block (two blocks share a CU)

__device__ __forceinline__ floatx4 mma(float a, float b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ floatx4 zero4() {
    floatx4 z = {0.f, 0.f, 0.f, 0.f};
    return z;
}

}  // namespace

// The switch of Algorithm 4.1 (step 4) fused behind the last xi level: the
// level's four output pairs (A_i, B) stay in LDS and each is multiplied by
// its block S_{A_i B} (read from HBM in the A layout of the switch step), so
// the level's output and the switch's input never go through HBM.
struct SwFuse {
    const float2* S;     // switch blocks [pair][r_out][r_in], r_in = xi r_out
    int r_out;           // switch output coefficients per pair
    int ys_off;          // LDS offset (float2) of the level's output Y
};

// Units per block of the per-step kernels: the units run one after the
// other, the next unit's input panel and twiddles read into registers while
// the current one computes.
constexpr int kSepUnits = 4;
constexpr int kSepPreX = 8;      // panel entries per thread: 4 r_in 16 <= 4096
constexpr int kSepPreT = 2;      // twiddles per thread: 16 r <= 1024

// xi step, block = (kSepUnits consecutive units, or one with SW, 16-column
// tile), kSepWaves waves: kSepWaves / 4 per output child i.  LDS: X
// [4][r_in][16], W [4][4][r_in], Z [4][2][a][b][16]; with SW, Y
// [4][r_out][16] at sw.ys_off (over X and W once they are read, or past Z).
// MODE: kSepPlain (kSepUnits units per block, pipelined), kSepHead (a level
// that reads f: one unit per block, f gathered straight into LDS, few
// registers so that four blocks share a CU), kSepSwitch (the switch fused
// behind the level, one unit per block).
enum { kSepPlain = 0, kSepHead = 1, kSepSwitch = 2 };

template <int MODE, bool TWO>
__global__ void __launch_bounds__(kSepWaves * 64) xi_step_sep(StepArgs a,
                                                              SwFuse sw) {
    constexpr bool SW = MODE == kSepSwitch;
    constexpr int UPB = MODE == kSepPlain ? kSepUnits : 1;
    extern __shared__ float2 lds_step[];
    const int A1 = a.a1, B1 = a.b1;
    float2* xs = lds_step;
    float2* ws = xs + (size_t)4 * a.r_in * kCols;
    float2* zs = ws + (size_t)16 * a.r_in;
    const int nct = (a.Vc + kCols - 1) / kCols;
    const long long grp = (long long)blockIdx.x / nct;
    const int col0 = (int)((long long)blockIdx.x - grp * nct) * kCols;
    const long long u0 = grp * UPB;
    // (the grid covers the units exactly when UPB = 1)
    const long long u1 = UPB == 1 ? u0 + 1
                                  : (u0 + UPB < a.units ? u0 + UPB : a.units);
    const int shiftB = 2 * (a.L - a.level);
    const int nthr = kSepWaves * 64;
    // switch: jobs (output child, 16-row tile of S), one wave each; the
    // first two jobs' block entries are read now, ahead of the level's work
    // (all of them for blocks of up to 64 S rows: 4 children x 4 row tiles
    // over 8 waves)
    const int MT = SW ? (sw.r_out + 15) >> 4 : 0;
    const int KS = (a.r_out + 3) >> 2;
    float2 sv0[16], sv1[16];
    if constexpr (SW) {
        const long long ap = u0 >> shiftB, b = u0 & ((1LL << shiftB) - 1);
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        const int row0 = lane & 15, g = lane >> 4;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int job = wave + q * kSepWaves;
            const int ii = job / MT, m = job - ii * MT;
            const int row = 16 * m + row0;
            const bool ok = job < 4 * MT && row < sw.r_out;
            const long long p = ((ap * 4 + ii) << shiftB) + b;
            const float2* Sp =
                sw.S + ((size_t)p * sw.r_out + row) * a.r_out;
#pragma unroll
            for (int ks = 0; ks < 16; ++ks) {
                const int s = 4 * ks + g;
                const float2 v = (ok && ks < KS && s < a.r_out)
                                     ? Sp[s]
                                     : make_float2(0.f, 0.f);
                if (q == 0) sv0[ks] = v; else sv1[ks] = v;
            }
        }
    }
    // input panel rows (child, point) of this thread: row0 + (nthr / 16) m,
    // its column fixed; the row steps without a division
    const int rows = 4 * a.r_in, nw = 16 * a.r_in;
    const int n16 = threadIdx.x & (kCols - 1), pcol = col0 + n16;
    const int prow0 = threadIdx.x >> 4;
    float2 px[kSepPreX], pw[kSepPreT];
    auto issue = [&](long long uu) {
        const long long apu = uu >> shiftB, bu = uu & ((1LL << shiftB) - 1);
        const long long pin0 = (apu << (shiftB + 2)) + (bu << 2);
        int c = prow0 / a.r_in, s = prow0 - c * a.r_in;
#pragma unroll
        for (int m = 0; m < kSepPreX; ++m) {
            px[m] = make_float2(0.f, 0.f);
            if (c < 4 && pcol < a.Vc)
                px[m] = a.reads_f
                            ? head_value(a, bu * 4 + c, s, pcol)
                            : a.in[((pin0 + c) * a.r_in + s) * a.Vc + pcol];
            s += nthr / kCols;
            while (s >= a.r_in) {
                s -= a.r_in;
                ++c;
            }
        }
#pragma unroll
        for (int m = 0; m < kSepPreT; ++m) {
            const int e = threadIdx.x + m * nthr;
            if (e < nw) pw[m] = step_twiddle<TWO>(a, STEP_XI, uu * nw + e);
        }
    };
    auto put = [&]() {
#pragma unroll
        for (int m = 0; m < kSepPreX; ++m) {
            const int row = prow0 + m * (nthr / kCols);
            if (row < rows) xs[row * kCols + n16] = px[m];
        }
#pragma unroll
        for (int m = 0; m < kSepPreT; ++m) {
            const int e = threadIdx.x + m * nthr;
            if (e < nw) ws[e] = pw[m];
        }
    };
    if constexpr (MODE == kSepHead) {
        // the head level: f gathered straight into LDS
        const long long bu = u0 & ((1LL << shiftB) - 1);
        int row = prow0, c = row / a.r_in, s = row - c * a.r_in;
        for (; c < 4; row += nthr / kCols) {
            xs[row * kCols + n16] = pcol < a.Vc
                                        ? head_value(a, bu * 4 + c, s, pcol)
                                        : make_float2(0.f, 0.f);
            s += nthr / kCols;
            while (s >= a.r_in) {
                s -= a.r_in;
                ++c;
            }
        }
        for (int e = threadIdx.x; e < nw; e += nthr)
            ws[e] = step_twiddle<TWO>(a, STEP_XI, u0 * nw + e);
    } else {
        issue(u0);
        put();
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    constexpr int WPC = kSepWaves / 4;            // waves per output child
    const int i = wave / WPC, h = wave % WPC;
    const int g = lane >> 4, n = lane & 15;
    const int nks = (2 * A1 + 3) >> 2;
    float am[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) am[ks] = a.amat_sep[ks * 64 + lane];
    // this lane's K entries (child, point) per K step, k = 4 ks + g: their
    // offsets in X and W (-1 past 2a)
    int kx[4], kw[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
        const int k = 4 * ks + g;
        const int c2 = k / A1, s2 = k - c2 * A1;
        const bool ok = k < 2 * A1;
        kx[ks] = ok ? (c2 * a.r_in + s2) * kCols + n : -1;
        kw[ks] = ok ? (i * 4 + c2) * a.r_in + s2 : -1;
    }
    // stage-2 K entries (c1, s1) of this lane: offsets in Z (-1 past 2a)
    int kz[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
        const int k = 4 * ks + g;
        kz[ks] = k < 2 * A1 ? ((i * 2 * A1 + k) * B1) * kCols + n : -1;
    }
    const int col = col0 + n;
    float2* ys = lds_step + sw.ys_off;
    for (long long u = u0; u < u1; ++u) {
        const long long ap = u >> shiftB, b = u & ((1LL << shiftB) - 1);
        __syncthreads();                    // X and W of unit u in LDS
        if constexpr (UPB > 1)
            if (u + 1 < u1) issue(u + 1);
        // stage 1: combos (c1, s1), split over the child's waves
        for (int cb = h; cb < 2 * A1; cb += WPC) {
            const int c1 = cb / A1, s1 = cb - c1 * A1;
            const int dx = (2 * c1 * a.r_in + s1 * A1) * kCols;
            const int dw = 2 * c1 * a.r_in + s1 * A1;
            floatx4 zr = zero4(), zi = zero4();
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                if (ks < nks) {                         // uniform
                    float2 z = make_float2(0.f, 0.f);
                    if (kx[ks] >= 0)
                        z = cmul(ws[kw[ks] + dw], xs[kx[ks] + dx]);
                    zr = mma(am[ks], z.x, zr);
                    zi = mma(am[ks], z.y, zi);
                }
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int t2 = 4 * g + j;
                if (t2 < B1)
                    zs[((((size_t)i * 2 + c1) * A1 + s1) * B1 + t2) * kCols +
                       n] = make_float2(zr[j], zi[j]);
            }
        }
        __syncthreads();
        // stage 2: one t2 per wave at a time
        const long long pout = ((ap * 4 + i) << shiftB) + b;
        float2* o = a.out + pout * a.r_out * a.Vc + col;
        for (int t2 = h; t2 < B1; t2 += WPC) {
            floatx4 yr = zero4(), yi = zero4();
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                if (ks < nks) {                         // uniform
                    float2 z = make_float2(0.f, 0.f);
                    if (kz[ks] >= 0) z = zs[kz[ks] + t2 * kCols];
                    yr = mma(am[ks], z.x, yr);
                    yi = mma(am[ks], z.y, yi);
                }
            }
            if constexpr (SW) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int t1 = 4 * g + j;
                    if (t1 < B1)
                        ys[((size_t)i * a.r_out + t1 * B1 + t2) * kCols + n] =
                            make_float2(yr[j], yi[j]);
                }
            } else if (col < a.Vc) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int t1 = 4 * g + j;
                    if (t1 < B1)
                        o[(size_t)(t1 * B1 + t2) * a.Vc] =
                            make_float2(yr[j], yi[j]);
                }
            }
        }
        if constexpr (SW) {
            // nu^{A_i B} = S_{A_i B} mu^{A_i B}: rows t of S (16 per job),
            // K = s, complex products as four real chains (Re S Re Y,
            // Im S Im Y, Re S Im Y, Im S Re Y)
            __syncthreads();
            for (int job = wave; job < 4 * MT; job += kSepWaves) {
                const int ii = job / MT, m = job - ii * MT;
                const long long p = ((ap * 4 + ii) << shiftB) + b;
                float2 sv[16];
                if (job == wave) {
#pragma unroll
                    for (int ks = 0; ks < 16; ++ks) sv[ks] = sv0[ks];
                } else if (job == wave + kSepWaves) {
#pragma unroll
                    for (int ks = 0; ks < 16; ++ks) sv[ks] = sv1[ks];
                } else {
                    const int row = 16 * m + n;
                    const float2* Sp =
                        sw.S + ((size_t)p * sw.r_out + row) * a.r_out;
#pragma unroll
                    for (int ks = 0; ks < 16; ++ks) {
                        const int s = 4 * ks + g;
                        sv[ks] = (row < sw.r_out && ks < KS && s < a.r_out)
                                     ? Sp[s]
                                     : make_float2(0.f, 0.f);
                    }
                }
                floatx4 p1 = zero4(), p2 = zero4(), p3 = zero4(), p4 = zero4();
#pragma unroll
                for (int ks = 0; ks < 16; ++ks) {
                    if (ks < KS) {                      // uniform
                        const int s = 4 * ks + g;
                        const float2 yv =
                            s < a.r_out
                                ? ys[((size_t)ii * a.r_out + s) * kCols + n]
                                : make_float2(0.f, 0.f);
                        p1 = mma(sv[ks].x, yv.x, p1);
                        p2 = mma(sv[ks].y, yv.y, p2);
                        p3 = mma(sv[ks].x, yv.y, p3);
                        p4 = mma(sv[ks].y, yv.x, p4);
                    }
                }
                if (col < a.Vc) {
                    float2* os = a.out + p * sw.r_out * a.Vc + col;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int t = 16 * m + 4 * g + j;
                        if (t < sw.r_out)
                            os[(size_t)t * a.Vc] =
                                make_float2(p1[j] - p2[j], p3[j] + p4[j]);
                    }
                }
            }
        }
        if constexpr (UPB > 1) {
            if (u + 1 < u1) {
                __syncthreads();            // X, W and Z of unit u are read
                put();
            }
        }
    }
}

// x step, block = (kSepUnits consecutive units, 16-column tile).  LDS: X
// [4][r_in][16], T [4][4][r_out], Z [4][2][a][b][16].
template <bool TWO>
__global__ void __launch_bounds__(kSepWaves * 64) x_step_sep(StepArgs a) {
    extern __shared__ float2 lds_step[];
    const int A1 = a.a1, B1 = a.b1;
    float2* xs = lds_step;
    float2* ts = xs + (size_t)4 * a.r_in * kCols;
    float2* zs = ts + (size_t)16 * a.r_out;
    const int nct = (a.Vc + kCols - 1) / kCols;
    const long long grp = (long long)blockIdx.x / nct;
    const int col0 = (int)((long long)blockIdx.x - grp * nct) * kCols;
    const long long u0 = grp * kSepUnits;
    const long long u1 = u0 + kSepUnits < a.units ? u0 + kSepUnits : a.units;
    const int shiftB = 2 * (a.L - a.level);
    const int nthr = kSepWaves * 64;
    const int rows = 4 * a.r_in, nt = 16 * a.r_out;
    // panel rows (child, point) of this thread: row0 + (nthr / 16) m
    const int n16 = threadIdx.x & (kCols - 1), pcol = col0 + n16;
    const int row0 = threadIdx.x >> 4;
    float2 px[kSepPreX], pt[kSepPreT];
    auto issue = [&](long long uu) {
        const long long apu = uu >> shiftB, bu = uu & ((1LL << shiftB) - 1);
        const long long pin0 = (apu << (shiftB + 2)) + (bu << 2);
        int c = row0 / a.r_in, s = row0 - c * a.r_in;
#pragma unroll
        for (int m = 0; m < kSepPreX; ++m) {
            px[m] = make_float2(0.f, 0.f);
            if (c < 4 && pcol < a.Vc)
                px[m] = a.in[((pin0 + c) * a.r_in + s) * a.Vc + pcol];
            s += nthr / kCols;
            while (s >= a.r_in) {
                s -= a.r_in;
                ++c;
            }
        }
#pragma unroll
        for (int m = 0; m < kSepPreT; ++m) {
            const int e = threadIdx.x + m * nthr;
            if (e < nt) pt[m] = step_twiddle<TWO>(a, STEP_X, uu * nt + e);
        }
    };
    auto put = [&]() {
#pragma unroll
        for (int m = 0; m < kSepPreX; ++m) {
            const int row = row0 + m * (nthr / kCols);
            if (row < rows) xs[row * kCols + n16] = px[m];
        }
#pragma unroll
        for (int m = 0; m < kSepPreT; ++m) {
            const int e = threadIdx.x + m * nthr;
            if (e < nt) ts[e] = pt[m];
        }
    };
    issue(u0);
    put();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane >> 4, n = lane & 15;
    const int nks = (A1 + 3) >> 2;
    float am[2];
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) am[ks] = a.amat_sep[ks * 64 + lane];
    // this lane's D rows 4 g + j = (child, point) of both stages: stage 1
    // writes Z at (i2, t2) = that split (offset rz, -1 past 2b), stage 2
    // reads the same split as (i1, t1)
    int rz[4], ri1[4], rt1[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int row = 4 * g + j;
        const int ch = row / B1, pt1 = row - ch * B1;
        const bool ok = row < 2 * B1;
        rz[j] = ok ? (ch * A1 * B1 + pt1) * kCols + n : -1;
        ri1[j] = ok ? ch : -1;
        rt1[j] = ok ? pt1 : 0;
    }
    const int col = col0 + n;
    for (long long u = u0; u < u1; ++u) {
        const long long ap = u >> shiftB, b = u & ((1LL << shiftB) - 1);
        __syncthreads();                    // X and T of unit u in LDS
        if (u + 1 < u1) issue(u + 1);       // in flight during the stages
        // stage 1: combos (c, s1); rows (i2, t2)
        for (int cb = wave; cb < 4 * A1; cb += kSepWaves) {
            const int c = cb / A1, s1 = cb - c * A1;
            floatx4 zr = zero4(), zi = zero4();
            const int xb = (c * a.r_in + s1 * A1 + g) * kCols + n;
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
                if (ks < nks) {                         // uniform
                    const int s2 = 4 * ks + g;
                    const float2 x = s2 < A1 ? xs[xb + 4 * ks * kCols]
                                             : make_float2(0.f, 0.f);
                    zr = mma(am[ks], x.x, zr);
                    zi = mma(am[ks], x.y, zi);
                }
            }
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (rz[j] >= 0)
                    zs[rz[j] + (c * 2 * A1 + s1) * B1 * kCols] =
                        make_float2(zr[j], zi[j]);
        }
        __syncthreads();
        // stage 2 and the twiddles: combos (i2, t2); rows (i1, t1); sum
        // over c
        for (int cb = wave; cb < 2 * B1; cb += kSepWaves) {
            const int i2 = cb / B1, t2 = cb - i2 * B1;
            // this lane's output rows (i1, t1): child ii, coefficient t
            int ii[4], tt[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                ii[j] = ri1[j] < 0 ? -1 : ri1[j] * 2 + i2;
                tt[j] = rt1[j] * B1 + t2;
            }
            floatx4 dr = zero4(), di = zero4();
            for (int c = 0; c < 4; ++c) {
                floatx4 yr = zero4(), yi = zero4();
                const int zb = (((c * 2 + i2) * A1) * B1 + t2) * kCols + n;
#pragma unroll
                for (int ks = 0; ks < 2; ++ks) {
                    if (ks < nks) {                     // uniform
                        const int s1 = 4 * ks + g;
                        const float2 z = s1 < A1 ? zs[zb + s1 * B1 * kCols]
                                                 : make_float2(0.f, 0.f);
                        yr = mma(am[ks], z.x, yr);
                        yi = mma(am[ks], z.y, yi);
                    }
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (ii[j] >= 0) {
                        const float2 T = ts[(ii[j] * 4 + c) * a.r_out + tt[j]];
                        dr[j] += T.x * yr[j] - T.y * yi[j];
                        di[j] += T.x * yi[j] + T.y * yr[j];
                    }
                }
            }
            if (col < a.Vc) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (ii[j] >= 0) {
                        const long long pout = ((ap * 4 + ii[j]) << shiftB) + b;
                        a.out[(pout * a.r_out + tt[j]) * a.Vc + col] =
                            make_float2(dr[j], di[j]);
                    }
                }
            }
        }
        if (u + 1 < u1) {
            __syncthreads();                // X, Z and T of unit u are read
            put();
        }
    }
}

size_t step_sep_lds(const Step& s) {
    const int a1 = s.ax_in.r1, b1 = s.ax_out.r1;
    const int rt = s.kind == STEP_XI ? s.r_in : s.r_out;
    return ((size_t)4 * s.r_in * kCols + (size_t)16 * rt +
            (size_t)8 * a1 * b1 * kCols) * sizeof(float2);
}

// LDS of the xi level with the switch fused: Y over X and W where it fits
// there (both are read before stage 2 starts), else past Z.
static void sep_switch_lds(const Step& s, size_t* bytes, int* ys_off) {
    const size_t xw = (size_t)4 * s.r_in * kCols + (size_t)16 * s.r_in;
    const size_t y = (size_t)4 * s.r_out * kCols;
    const size_t base = step_sep_lds(s) / sizeof(float2);
    *ys_off = y <= xw ? 0 : (int)base;
    *bytes = (y <= xw ? base : base + y) * sizeof(float2);
}

bool sep_switch_ok(const Plan& p, const Step& xi, const Step& sw) {
    if (!(p.sep_switch && p.mfma && p.precision == BF_FP32 && !p.switch_otf))
        return false;
    if (xi.kind != STEP_XI || sw.kind != STEP_SWITCH || !step_sep_ok(p, xi))
        return false;
    if (!sw.S || sw.r_in != xi.r_out || sw.level != xi.level || sw.r_out > 64)
        return false;
    size_t bytes;
    int off;
    sep_switch_lds(xi, &bytes, &off);
    return bytes <= 160 * 1024;
}

// The separable form applies to 2D steps whose stacked children fit one
// 16-row / 16-deep MFMA operand (points per dimension <= 8).
bool step_sep_ok(const Plan& p, const Step& s) {
    return p.dim == 2 && s.kind != STEP_SWITCH && s.amat_sep &&
           s.ax_in.r1 <= 8 && s.ax_out.r1 <= 8;
}

void init_step_sep_attrs() {
    const void* fns[] = {(const void*)xi_step_sep<kSepPlain, false>,
                         (const void*)xi_step_sep<kSepHead, false>,
                         (const void*)xi_step_sep<kSepSwitch, false>,
                         (const void*)x_step_sep<false>,
                         (const void*)xi_step_sep<kSepPlain, true>,
                         (const void*)xi_step_sep<kSepHead, true>,
                         (const void*)xi_step_sep<kSepSwitch, true>,
                         (const void*)x_step_sep<true>};
    for (const void* f : fns)
        (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  160 * 1024);
}

std::string launch_step_sep(const Plan& p, const Step& s, StepArgs a,
                            hipStream_t st) {
    const long long nct = (a.Vc + kCols - 1) / kCols;
    const int upb = s.kind == STEP_XI && s.reads_f ? 1 : kSepUnits;
    const long long groups = (s.units + upb - 1) / upb;
    const long long nb = groups * nct;
    if (nb > 0x7fffffffLL) return "step grid too large";
    const size_t lds = step_sep_lds(s);
    if (lds > 160 * 1024) return "step does not fit in LDS";
    a.a1 = s.ax_in.r1;
    a.b1 = s.ax_out.r1;
    a.amat_sep = s.amat_sep;
    const dim3 grid((unsigned)nb), block(kSepWaves * 64);
    if (p.twiddle_otf) {
        if (s.kind == STEP_XI && s.reads_f)
            hipLaunchKernelGGL((xi_step_sep<kSepHead, true>), grid, block, lds,
                               st, a, SwFuse{});
        else if (s.kind == STEP_XI)
            hipLaunchKernelGGL((xi_step_sep<kSepPlain, true>), grid, block,
                               lds, st, a, SwFuse{});
        else
            hipLaunchKernelGGL((x_step_sep<true>), grid, block, lds, st, a);
    } else {
        if (s.kind == STEP_XI && s.reads_f)
            hipLaunchKernelGGL((xi_step_sep<kSepHead, false>), grid, block,
                               lds, st, a, SwFuse{});
        else if (s.kind == STEP_XI)
            hipLaunchKernelGGL((xi_step_sep<kSepPlain, false>), grid, block,
                               lds, st, a, SwFuse{});
        else
            hipLaunchKernelGGL((x_step_sep<false>), grid, block, lds, st, a);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return std::string("step launch: ") + hipGetErrorString(e);
    return "";
}

// The last xi level and the switch in one launch: out receives the
// switch's output (the pairs of level h after S).
std::string launch_sep_switch(const Plan& p, const Step& xi, const Step& sw,
                              StepArgs a, hipStream_t st) {
    if (!sep_switch_ok(p, xi, sw)) return "fused switch does not apply";
    const long long nct = (a.Vc + kCols - 1) / kCols;
    const long long nb = xi.units * nct;
    if (nb > 0x7fffffffLL) return "step grid too large";
    size_t lds;
    SwFuse f{sw.S, sw.r_out, 0};
    sep_switch_lds(xi, &lds, &f.ys_off);
    a.a1 = xi.ax_in.r1;
    a.b1 = xi.ax_out.r1;
    a.amat_sep = xi.amat_sep;
    if (p.twiddle_otf)
        hipLaunchKernelGGL((xi_step_sep<kSepSwitch, true>), dim3((unsigned)nb),
                           dim3(kSepWaves * 64), lds, st, a, f);
    else
        hipLaunchKernelGGL((xi_step_sep<kSepSwitch, false>), dim3((unsigned)nb),
                           dim3(kSepWaves * 64), lds, st, a, f);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return std::string("step launch: ") + hipGetErrorString(e);
    return "";
}

}  // namespace bfi
