// Split-precision per-step kernels (BF16x3 / FP16x3 on MFMA, FP32
// accumulation): the per-level form of plans whose ranks exceed the fused
// passes (2D boxes of up to 8 x 8 points).  As the FP32 per-step kernels
// (one unit or pair and 16 panel columns per block), with every product
// split x = hi + lo into 16-bit parts and formed as hi*hi + hi*lo + lo*hi on
// v_mfma_f32_16x16x16 (bf16 or f16): A lane l holds A[l % 16][4 (l / 16) +
// e], B lane l holds B[4 (l / 16) + e][l % 16], e < 4, one 16-deep K block
// per instruction.
//   - the Lagrange matrices come split at plan time in that A order
//     (Step::a16_hi / a16_lo: [child][row tile][K block][lane][4]);
//   - the switch blocks of a split plan are stored as their parts (Re hi,
//     Re lo, Im hi, Im lo) per entry, the bytes of one complex64;
//   - the panel is split as it is read; in half precision every panel
//     column of a block is first scaled by a power of two (exact) so that
//     its largest magnitude maps into [0.5, 1), and the products are scaled
//     back.
#include "apply_common.h"
#include "split_common.h"

namespace bfi {

namespace {

constexpr int kCols = 16;      // panel columns per block
constexpr int kMaxMT = 4;      // row tiles: r_out <= 64

__device__ __forceinline__ floatx4 zero4() {
    floatx4 z = {0.f, 0.f, 0.f, 0.f};
    return z;
}

// Per-column scale exponents of a staged panel (half precision only): the
// block's threads fold max |re|, |im| of their entries into cmax[16] (bits
// of non-negative floats order as integers), then every lane takes e with
// cmax = f 2^e, f in [0.5, 1) (e = 0 for a zero column).
__device__ __forceinline__ void fold_max(int* cmax, int col, float2 v) {
    const float m = fmaxf(fabsf(v.x), fabsf(v.y));
    atomicMax(cmax + col, __float_as_int(m));
}

__device__ __forceinline__ int col_exponent(const int* cmax, int col) {
    int e = 0;
    const float m = __int_as_float(cmax[col]);
    if (m > 0.f) (void)frexpf(m, &e);
    return e;
}

template <int PREC>
__device__ __forceinline__ void split4(const float (&v)[4], int ex,
                                       typename Split<PREC>::v4& h,
                                       typename Split<PREC>::v4& l) {
    using SP = Split<PREC>;
#pragma unroll
    for (int e = 0; e < 4; ++e)
        SP::put4(h, l, e, SP::kScaled ? ldexpf(v[e], -ex) : v[e]);
}

template <int PREC>
__device__ __forceinline__ floatx4 mma3(typename Split<PREC>::v4 ah,
                                        typename Split<PREC>::v4 al,
                                        typename Split<PREC>::v4 bh,
                                        typename Split<PREC>::v4 bl,
                                        floatx4 c) {
    using SP = Split<PREC>;
    c = SP::mma16(ah, bh, c);
    c = SP::mma16(ah, bl, c);
    return SP::mma16(al, bh, c);
}

template <int PREC>
__device__ __forceinline__ typename Split<PREC>::v4 load_a(const uint16_t* t,
                                                           size_t idx) {
    return __builtin_bit_cast(typename Split<PREC>::v4,
                              ((const uint2*)t)[idx]);
}

}  // namespace

// xi step (eq. (eqn:2) regrouped), block = (unit, 16-column tile), WPC
// waves per output child i: D_i = sum_c M_c (W_{i,c} . X_c).
template <int R, int WPC, int PREC>
__global__ void __launch_bounds__(R * 64 * WPC) xi_step_split(StepArgs a) {
    constexpr int NT = kMaxMT / WPC;
    extern __shared__ float2 lds_step[];
    float2* xs = lds_step;                              // [R][r_in][16]
    float2* ws = xs + (size_t)R * a.r_in * kCols;       // [R][R][r_in]
    int* cmax = (int*)(ws + (size_t)R * R * a.r_in);    // [16]
    const int nct = (a.Vc + kCols - 1) / kCols;
    const long long u = (long long)blockIdx.x / nct;
    const int col0 = (int)((long long)blockIdx.x - u * nct) * kCols;
    const int shiftB = a.dim * (a.L - a.level);
    const long long ap = u >> shiftB, b = u & ((1LL << shiftB) - 1);
    if (threadIdx.x < kCols) cmax[threadIdx.x] = 0;
    __syncthreads();
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
        // |W x| = |x|: the twiddles do not change the column scale
        if (Split<PREC>::kScaled) fold_max(cmax, n, v);
    }
    const int ntw = R * R * a.r_in;
    for (int e = threadIdx.x; e < ntw; e += R * 64 * WPC)
        ws[e] = a.tw[u * ntw + e];
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = wave / WPC, h = wave - i * WPC;
    const int g = lane >> 4, n = lane & 15;
    const int MT = (a.r_out + 15) >> 4, KB = (a.r_in + 15) >> 4;
    const int ex = Split<PREC>::kScaled ? col_exponent(cmax, n) : 0;
    floatx4 accr[NT], acci[NT];
#pragma unroll
    for (int q = 0; q < NT; ++q) accr[q] = acci[q] = zero4();
    for (int c = 0; c < R; ++c) {
        const float2* w = ws + (i * R + c) * a.r_in;
        const float2* x = xs + (size_t)c * a.r_in * kCols + n;
        for (int kb = 0; kb < KB; ++kb) {
            float vr[4], vi[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int s = 16 * kb + 4 * g + e;
                float2 z = make_float2(0.f, 0.f);
                if (s < a.r_in) z = cmul(w[s], x[s * kCols]);
                vr[e] = z.x;
                vi[e] = z.y;
            }
            typename Split<PREC>::v4 brh, brl, bih, bil;
            split4<PREC>(vr, ex, brh, brl);
            split4<PREC>(vi, ex, bih, bil);
#pragma unroll
            for (int q = 0; q < NT; ++q) {
                const int m = h + q * WPC;
                if (m < MT) {                           // uniform
                    const size_t at = (((size_t)c * MT + m) * KB + kb) * 64 + lane;
                    const auto ah = load_a<PREC>(a.a16_hi, at);
                    const auto al = load_a<PREC>(a.a16_lo, at);
                    accr[q] = mma3<PREC>(ah, al, brh, brl, accr[q]);
                    acci[q] = mma3<PREC>(ah, al, bih, bil, acci[q]);
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
                const int t = 16 * m + 4 * g + j;
                if (t < a.r_out)
                    o[(size_t)t * a.Vc] =
                        make_float2(ldexpf(accr[q][j], ex), ldexpf(acci[q][j], ex));
            }
        }
    }
}

// x step (eq. (eqn:3) regrouped), block = (unit, 16-column tile), WPC
// waves per output child i: D_i = sum_c T_{i,c} . (M_i X_c).
template <int R, int WPC, int PREC>
__global__ void __launch_bounds__(R * 64 * WPC) x_step_split(StepArgs a) {
    constexpr int NT = kMaxMT / WPC;
    extern __shared__ float2 lds_step[];
    float2* xs = lds_step;                              // [R][r_in][16]
    float2* ts = xs + (size_t)R * a.r_in * kCols;       // [R][R][r_out]
    int* cmax = (int*)(ts + (size_t)R * R * a.r_out);   // [16]
    const int nct = (a.Vc + kCols - 1) / kCols;
    const long long u = (long long)blockIdx.x / nct;
    const int col0 = (int)((long long)blockIdx.x - u * nct) * kCols;
    const int shiftB = a.dim * (a.L - a.level);
    const long long ap = u >> shiftB, b = u & ((1LL << shiftB) - 1);
    if (threadIdx.x < kCols) cmax[threadIdx.x] = 0;
    __syncthreads();
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
        if (Split<PREC>::kScaled) fold_max(cmax, n, v);
    }
    const int ntw = R * R * a.r_out;
    for (int e = threadIdx.x; e < ntw; e += R * 64 * WPC)
        ts[e] = a.tw[u * ntw + e];
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = wave / WPC, h = wave - i * WPC;
    const int g = lane >> 4, n = lane & 15;
    const int MT = (a.r_out + 15) >> 4, KB = (a.r_in + 15) >> 4;
    const int ex = Split<PREC>::kScaled ? col_exponent(cmax, n) : 0;
    floatx4 accr[NT], acci[NT];
#pragma unroll
    for (int q = 0; q < NT; ++q) accr[q] = acci[q] = zero4();
    for (int c = 0; c < R; ++c) {
        floatx4 yr[NT], yi[NT];
#pragma unroll
        for (int q = 0; q < NT; ++q) yr[q] = yi[q] = zero4();
        const float2* x = xs + (size_t)c * a.r_in * kCols + n;
        for (int kb = 0; kb < KB; ++kb) {
            float vr[4], vi[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int s = 16 * kb + 4 * g + e;
                const float2 z = s < a.r_in ? x[s * kCols] : make_float2(0.f, 0.f);
                vr[e] = z.x;
                vi[e] = z.y;
            }
            typename Split<PREC>::v4 brh, brl, bih, bil;
            split4<PREC>(vr, ex, brh, brl);
            split4<PREC>(vi, ex, bih, bil);
#pragma unroll
            for (int q = 0; q < NT; ++q) {
                const int m = h + q * WPC;
                if (m < MT) {                           // uniform
                    const size_t at = (((size_t)i * MT + m) * KB + kb) * 64 + lane;
                    const auto ah = load_a<PREC>(a.a16_hi, at);
                    const auto al = load_a<PREC>(a.a16_lo, at);
                    yr[q] = mma3<PREC>(ah, al, brh, brl, yr[q]);
                    yi[q] = mma3<PREC>(ah, al, bih, bil, yi[q]);
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
                    const int t = 16 * m + 4 * g + j;
                    const float2 T = t < a.r_out ? tw[t] : make_float2(0.f, 0.f);
                    const float y0 = ldexpf(yr[q][j], ex), y1 = ldexpf(yi[q][j], ex);
                    accr[q][j] += T.x * y0 - T.y * y1;
                    acci[q][j] += T.x * y1 + T.y * y0;
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
                const int t = 16 * m + 4 * g + j;
                if (t < a.r_out)
                    o[(size_t)t * a.Vc] = make_float2(accr[q][j], acci[q][j]);
            }
        }
    }
}

// Switch (Algorithm 4.1 step 4 regrouped), block = (pair, 16-column tile),
// wave m = row tile m of nu = S mu; the block's split parts are read
// straight from HBM in the A layout (each lane its row and four
// consecutive K columns per K block) before the panel is staged.
template <int PREC>
__global__ void __launch_bounds__(kMaxMT * 64) switch_step_split(StepArgs a) {
    using SP = Split<PREC>;
    using E = typename SP::e4;
    extern __shared__ float2 lds_step[];
    float2* xs = lds_step;                              // [r_in][16]
    int* cmax = (int*)(xs + (size_t)a.r_in * kCols);    // [16]
    const int nct = (a.Vc + kCols - 1) / kCols;
    const long long p = (long long)blockIdx.x / nct;
    const int col0 = (int)((long long)blockIdx.x - p * nct) * kCols;
    const int shiftB = a.dim * (a.L - a.level);
    const long long bm = p & ((1LL << shiftB) - 1);
    const int m = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane >> 4, n = lane & 15;
    const int KB = (a.r_in + 15) >> 4;
    const int row = 16 * m + n;
    const ushort4* S = (const ushort4*)a.S + p * a.r_out * a.r_in +
                       (size_t)row * a.r_in;
    typename SP::v4 rh[4], rl[4], ih[4], il[4];
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int s = 16 * kb + 4 * g + e;
            ushort4 q = make_ushort4(0, 0, 0, 0);
            if (kb < KB && row < a.r_out && s < a.r_in) q = S[s];
            rh[kb][e] = __builtin_bit_cast(E, q.x);
            rl[kb][e] = __builtin_bit_cast(E, q.y);
            ih[kb][e] = __builtin_bit_cast(E, q.z);
            il[kb][e] = __builtin_bit_cast(E, q.w);
        }
    }
    if (threadIdx.x < kCols) cmax[threadIdx.x] = 0;
    __syncthreads();
    const int nthr = blockDim.x;
    for (int e = threadIdx.x; e < a.r_in * kCols; e += nthr) {
        const int nn = e % kCols, s = e / kCols;
        const int col = col0 + nn;
        float2 v = make_float2(0.f, 0.f);
        if (col < a.Vc)
            v = a.reads_f ? head_value(a, bm, s, col)
                          : a.in[(p * a.r_in + s) * a.Vc + col];
        xs[e] = v;
        if (SP::kScaled) fold_max(cmax, nn, v);
    }
    __syncthreads();
    const int ex = SP::kScaled ? col_exponent(cmax, n) : 0;
    floatx4 p1 = zero4(), p2 = zero4(), p3 = zero4(), p4 = zero4();
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
        if (kb < KB) {                                  // uniform
            float vr[4], vi[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int s = 16 * kb + 4 * g + e;
                const float2 z = s < a.r_in ? xs[s * kCols + n]
                                            : make_float2(0.f, 0.f);
                vr[e] = z.x;
                vi[e] = z.y;
            }
            typename SP::v4 brh, brl, bih, bil;
            split4<PREC>(vr, ex, brh, brl);
            split4<PREC>(vi, ex, bih, bil);
            p1 = mma3<PREC>(rh[kb], rl[kb], brh, brl, p1);
            p2 = mma3<PREC>(ih[kb], il[kb], bih, bil, p2);
            p3 = mma3<PREC>(rh[kb], rl[kb], bih, bil, p3);
            p4 = mma3<PREC>(ih[kb], il[kb], brh, brl, p4);
        }
    }
    const int col = col0 + n;
    if (col >= a.Vc) return;
    float2* o = a.out + p * a.r_out * a.Vc + col;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int t = 16 * m + 4 * g + j;
        if (t < a.r_out)
            o[(size_t)t * a.Vc] = make_float2(ldexpf(p1[j] - p2[j], ex),
                                              ldexpf(p3[j] + p4[j], ex));
    }
}

size_t step_split_lds(const Plan& p, const Step& s) {
    const size_t extra = kCols * sizeof(int);
    if (s.kind == STEP_SWITCH)
        return (size_t)s.r_in * kCols * sizeof(float2) + extra;
    const int rt = s.kind == STEP_XI ? s.r_in : s.r_out;
    return ((size_t)p.R * s.r_in * kCols + (size_t)p.R * p.R * rt) *
               sizeof(float2) + extra;
}

template <int PREC>
static void set_split_attrs() {
    static bool done = false;
    if (done) return;
    const void* fns[] = {(const void*)xi_step_split<2, 1, PREC>,
                         (const void*)xi_step_split<4, 2, PREC>,
                         (const void*)x_step_split<2, 1, PREC>,
                         (const void*)x_step_split<4, 2, PREC>,
                         (const void*)switch_step_split<PREC>};
    for (const void* f : fns)
        (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  160 * 1024);
    done = true;
}

void init_step_split_attrs() {
    set_split_attrs<BF_BF16X3>();
    set_split_attrs<BF_FP16X3>();
}

template <int PREC>
static std::string launch_split(const Plan& p, const Step& s,
                                const StepArgs& a, hipStream_t st) {
    const long long nct = (a.Vc + kCols - 1) / kCols;
    const long long nb = s.units * nct;
    if (nb > 0x7fffffffLL) return "step grid too large";
    const size_t lds = step_split_lds(p, s);
    if (lds > 160 * 1024) return "step does not fit in LDS";
    if (s.kind == STEP_SWITCH) {
        const int MT = (s.r_out + 15) / 16;
        hipLaunchKernelGGL(switch_step_split<PREC>, dim3((unsigned)nb),
                           dim3(64 * MT), lds, st, a);
    } else if (p.R == 2) {
        if (s.kind == STEP_XI)
            hipLaunchKernelGGL((xi_step_split<2, 1, PREC>), dim3((unsigned)nb),
                               dim3(128), lds, st, a);
        else
            hipLaunchKernelGGL((x_step_split<2, 1, PREC>), dim3((unsigned)nb),
                               dim3(128), lds, st, a);
    } else {
        if (s.kind == STEP_XI)
            hipLaunchKernelGGL((xi_step_split<4, 2, PREC>), dim3((unsigned)nb),
                               dim3(512), lds, st, a);
        else
            hipLaunchKernelGGL((x_step_split<4, 2, PREC>), dim3((unsigned)nb),
                               dim3(512), lds, st, a);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return std::string("step launch: ") + hipGetErrorString(e);
    return "";
}

std::string launch_step_split(const Plan& p, const Step& s, const StepArgs& a,
                              hipStream_t st) {
    if (s.r_out > kMaxMT * 16 || s.r_in > kMaxMT * 16)
        return "step rank above 64";
    if (s.kind != STEP_SWITCH && (!a.a16_hi || !a.a16_lo))
        return "split matrices missing";
    return p.precision == BF_FP16X3 ? launch_split<BF_FP16X3>(p, s, a, st)
                                    : launch_split<BF_BF16X3>(p, s, a, st);
}

}  // namespace bfi
