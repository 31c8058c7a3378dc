// Level-fused passes on MFMA (1D, FP32 in and out).
//
// The contraction with a level's shared real matrices is a dense
// (r_out x K) x (K x panel) product and runs on v_mfma_f32_16x16x4f32.
// A operand: the matrix (the same for every unit of the level, held in
// registers for the whole level).  B operand: the panel, 16 complex columns
// per MFMA tile; the real and imaginary parts run as two MFMA chains against
// the same A, so each lane ends with both halves of its outputs.  Lane
// layout of 16x16x4 f32: A lane l holds A[l%16][l/16], B lane l holds
// B[l/16][l%16], D lane l holds D[4(l/16)+j][l%16], j < 4.
//   xi level (eq. (eqn:2) regrouped): out_i = [M_0 | M_1] [W_{i,0} . x_0 ;
//     W_{i,1} . x_1], K = 2 r_in; the twiddle is applied while building B.
//   x level (eq. (eqn:3) regrouped): y_{i,c} = M_i x_c, K = r_in, both
//     children i from the same B values, then out_i = sum_c T_{i,c} . y_{i,c}
//     in registers.
//   switch (Algorithm 4.1 step 4 regrouped): per pair, A = Re S and A = Im S
//     against 16 real columns (Re mu, Im mu of 8 columns); the other half of
//     each product comes from the neighbouring lane.
// Levels update one LDS tile in place (a unit reads its two slots and
// writes the same two, and all of a unit's columns sit in one wave) and the
// next level's twiddles are staged into the second twiddle buffer while a
// level computes, so a level needs one workgroup barrier.  K steps past the
// end use A = 0 and read valid (finite) data, so the loads need no guards.
// R = 2, r <= 16, VT (columns per tile) in {1, 2, 4, 8}.
#include "fused_common.h"
#include "split_common.h"

namespace bfi {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// Workgroups of 16 waves (four per SIMD, <= 128 VGPRs each) on one LDS tile.
constexpr int kMfmaThreads = 1024;
// x-level MFMA tiles per wave at the largest tile (Gk * VT = 512)
template <int VT>
constexpr int wave_tiles() {
    return kMfmaTileCap / (2 * (kMfmaThreads / 64));
}

__device__ __forceinline__ float lane_swap1(float v) {
    // quad_perm [1, 0, 3, 2]: exchange with the neighbouring lane
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1,
                                                   0xF, 0xF, false));
}

__device__ __forceinline__ floatx4 mfma4(float a, float b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Units of local level j (u < Gk / 2) in slot order: u = bl 2^(j-1) + rv,
// rv the bit-reversed apl, so consecutive units read and write consecutive
// slots of the tile (the lanes of one MFMA tile then spread over the LDS
// banks instead of meeting at power-of-two slot strides).  The staged
// twiddles of a level use the same order ([u][i][c][r]).
struct UnitMap {
    int bl, rv, apl;
};

__device__ __forceinline__ UnitMap unit_map(int u, int j) {
    UnitMap m;
    m.rv = u & ((1 << (j - 1)) - 1);
    m.bl = u >> (j - 1);
    m.apl = digit_rev(m.rv, j - 1, 1);
    return m;
}

// ---- split precision: the Split<PREC> parts and products (split_common.h)

// Exponent e of a power-of-two column scale for the half-precision split:
// m is this lane's largest magnitude; the lanes 16, 32 and 48 apart hold
// the same B column (other K rows), so after the exchange every lane of the
// column has the column maximum M = f 2^e, f in [0.5, 1), and the column
// scaled by 2^-e lies in (-1, 1) (zero columns get e = 0).  The exchange
// uses the row-swapping lane permutes (checked by an in-bounds probe: with
// both operands v, permlane16_swap returns rows {0,0,2,2} and {1,1,3,3} of
// v, permlane32_swap the lower and the upper half of v).
__device__ __forceinline__ int column_exponent(float m) {
    const auto p16 = __builtin_amdgcn_permlane16_swap(
        __float_as_uint(m), __float_as_uint(m), false, false);
    m = fmaxf(__uint_as_float(p16[0]), __uint_as_float(p16[1]));
    const auto p32 = __builtin_amdgcn_permlane32_swap(
        __float_as_uint(m), __float_as_uint(m), false, false);
    m = fmaxf(__uint_as_float(p32[0]), __uint_as_float(p32[1]));
    int e = 0;
    (void)frexpf(m, &e);
    return e;
}

// Twiddles of local level j for the group's units into LDS:
// twl[u][i][c][r], u = bl 2^(j-1) + rv the unit in slot order (unit_map),
// rv the bit-reversed apl.
__device__ __forceinline__ void stage_twiddles(const PassArgs& a, int j,
                                               float2* twl, long long ap_grp,
                                               long long bg, bool xi) {
    const PassLevel& lv = a.lv[j - 1];
    const int rr = xi ? lv.r_in : lv.r_out;
    const int kj = a.k - j;
    const int per_unit = 4 * rr;
    const int total = (a.Gk >> 1) * per_unit;
    const int shiftB = a.L - (a.la + j - 1);
    // unit index u = (apg << shiftB) + bgl < N/2, and u * per_unit < 2^31
    const unsigned apg0 = (unsigned)(ap_grp << (j - 1));
    const unsigned bg0 = (unsigned)(bg << kj);
    Walk2 w(threadIdx.x, per_unit);
    for (int e = threadIdx.x; e < total; e += blockDim.x, w.next()) {
        const UnitMap um = unit_map(w.hi, j);
        const unsigned u = ((apg0 + (unsigned)um.apl) << shiftB) + bg0 +
                           (unsigned)um.bl;
        twl[e] = lv.tw[u * (unsigned)per_unit + (unsigned)w.lo];
    }
}

// The same staging split in two: load() issues the global reads into
// registers (up to NT per thread), store() writes them to LDS, so that the
// reads overlap whatever runs in between (a level's MFMA work); entries past
// NT per thread are copied directly by store().
template <int NT>
struct TwStage {
    float2 v[NT];
    int total, per_unit, jl, shiftB;
    unsigned apg0, bg0;
    const float2* tw;

    __device__ __forceinline__ unsigned src_index(int unit, int lo) const {
        const UnitMap um = unit_map(unit, jl);
        const unsigned u = ((apg0 + (unsigned)um.apl) << shiftB) + bg0 +
                           (unsigned)um.bl;
        return u * (unsigned)per_unit + (unsigned)lo;
    }

    __device__ __forceinline__ void load(const PassArgs& a, int j,
                                         long long ap_grp, long long bg,
                                         bool xi) {
        const PassLevel& lv = a.lv[j - 1];
        const int rr = xi ? lv.r_in : lv.r_out;
        const int kj = a.k - j;
        jl = j;
        per_unit = 4 * rr;
        total = (a.Gk >> 1) * per_unit;
        shiftB = a.L - (a.la + j - 1);
        apg0 = (unsigned)(ap_grp << (j - 1));
        bg0 = (unsigned)(bg << kj);
        tw = lv.tw;
        Walk2 w(threadIdx.x, per_unit);
#pragma unroll
        for (int m = 0; m < NT; ++m) {
            if (threadIdx.x + m * (int)blockDim.x < total)
                v[m] = tw[src_index(w.hi, w.lo)];
            w.next();
        }
    }

    __device__ __forceinline__ void store(float2* twl) const {
#pragma unroll
        for (int m = 0; m < NT; ++m) {
            const int e = threadIdx.x + m * (int)blockDim.x;
            if (e < total) twl[e] = v[m];
        }
        const int e0 = threadIdx.x + NT * (int)blockDim.x;
        if (e0 >= total) return;
        Walk2 w(e0, per_unit);
        for (int e = e0; e < total; e += blockDim.x, w.next())
            twl[e] = tw[src_index(w.hi, w.lo)];
    }
};

// Register-staged twiddle entries per thread: what the largest tile
// (Gk * VT = 512, r <= 16) needs, at most 2 (entries past them are copied
// at the store; holding 4 spilled the width-4 passes to scratch).
template <int VT>
constexpr int tw_regs() {
    return (kMfmaTileCap * 8 / VT) * 32 / kMfmaThreads > 2
               ? 2
               : ((kMfmaTileCap * 8 / VT) * 32 / kMfmaThreads < 1
                      ? 1
                      : (kMfmaTileCap * 8 / VT) * 32 / kMfmaThreads);
}

// Register-staged entries per thread of the next sub-iteration's state tile
// in the x pass: the width-8 tile (5 per thread at Gk = 64, r = 10) is
// read whole; narrower tiles, whose passes hold more twiddle and tail
// registers, read 3 and copy the rest at the store (more would spill).
template <int VT>
constexpr int pre_regs() {
    return VT >= 8 ? 5 : 3;
}

// A operand of an FP32 level, one coalesced load per k step (lv.amat):
// xi levels aM[kk], kk < ceil(r_in / 2); x levels aM[4 i + kk], kk <
// ceil(r_in / 4); zero elsewhere.
__device__ __forceinline__ void load_amat(const PassLevel& lv, bool xi,
                                          float (&aM)[8]) {
    const int lane = threadIdx.x & 63;
    if (xi) {
        const int nks2 = (lv.r_in + 1) >> 1;
#pragma unroll
        for (int kk = 0; kk < 8; ++kk)
            aM[kk] = kk < nks2 ? lv.amat[kk * 64 + lane] : 0.f;
    } else {
        const int nks = (lv.r_in + 3) >> 2;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
                aM[4 * i + kk] =
                    kk < nks ? lv.amat[(i * nks + kk) * 64 + lane] : 0.f;
    }
}

// FP32 tile loop of one xi level with NK K steps (pairs of coefficients).
template <int VT, int NK>
__device__ __forceinline__ void xi_tiles_fp32(const PassArgs& a,
                                              const float2* src, int RS,
                                              float2* dst, const float2* twl,
                                              int j, const float (&aM)[8],
                                              int xoff, int woff,
                                              float2* sink) {
    const PassLevel& lv = a.lv[j - 1];
    const int r_in = lv.r_in, r_out = lv.r_out;
    const int kj = a.k - j;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    const int g = lane >> 4, n = lane & 15;
    constexpr int CPT = 16 / VT;             // (unit, i) combinations per tile
    const int sub = n / VT, col = n & (VT - 1);
    const int ntiles = (a.Gk + CPT - 1) / CPT;
    const int DS = a.rmax * VT;
    for (int tau = wave; tau < ntiles; tau += nwaves) {
        int ui = tau * CPT + sub;
        const bool ok = ui < a.Gk;
        if (!ok) ui = 0;                        // padding column: any valid data
        // both children of a unit in one tile (one wave): the unit's output
        // slots are its input slots, updated in place
        const int unit = ui >> 1, i = ui & 1;
        const UnitMap um = unit_map(unit, j);
        const int bl = um.bl, rv = um.rv;
        const float2* xp = src + (((bl * 2) << (j - 1)) + rv) * RS + xoff;
        const float2* wp = twl + (unit * 4 + i * 2) * r_in + woff;
        float2 xs[NK], ws[NK];
#pragma unroll
        for (int kk = 0; kk < NK; ++kk) {
            xs[kk] = xp[kk * 2 * VT];
            ws[kk] = wp[2 * kk];
        }
        floatx4 accr = {0.f, 0.f, 0.f, 0.f}, acci = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < NK; ++kk) {
            const float2 x = xs[kk], w = ws[kk];
            accr = mfma4(aM[kk], w.x * x.x - w.y * x.y, accr);
            acci = mfma4(aM[kk], w.x * x.y + w.y * x.x, acci);
        }
        // rows t >= r_out (exactly zero: A is zero there) and padding
        // columns go to this lane's slot of the pass's pad instead of
        // branching around the stores
        float2* op = dst + (((bl * 2 + i) << (j - 1)) + rv) * DS + col;
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int t = 4 * g + jj;
            float2* p = (ok && t < r_out) ? op + t * VT : sink + lane;
            *p = make_float2(accr[jj], acci[jj]);
        }
    }
}

// One xi level: src (stride src_r coefficients per slot) -> dst.
template <int VT, int PREC>
__device__ __forceinline__ void mfma_xi_level(const PassArgs& a,
                                              const float2* src, int src_r,
                                              float2* dst, const float2* twl,
                                              int j, const float (&aMin)[8],
                                              float2* sink) {
    const PassLevel& lv = a.lv[j - 1];
    const int r_in = lv.r_in, r_out = lv.r_out;
    const int K = 2 * r_in, nks = (K + 3) / 4;
    const int kj = a.k - j;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    const int g = lane >> 4, tA = lane & 15;
    const int n = lane & 15;
    constexpr int CPT = 16 / VT;             // (unit, i) combinations per tile
    const int sub = n / VT, col = n & (VT - 1);
    const int RS = src_r * VT;               // source slot stride
    // the two children's slots differ by 2^(j-1) slots whatever the unit,
    // so x offsets fold the child in: xo = c 2^(j-1) RS + s VT + col
    const int cstride = (1 << (j - 1)) * RS;
    if constexpr (PREC != BF_FP32) {
        // K = 2 r_in <= 32: one 16x16x32 product per (chain, split term).
        // Lane l holds k = 8 g + e ordered with the child fastest: child
        // c = e % 2, coefficient s = 4 g + e / 2, so x and w sit at a fixed
        // lane base plus compile-time (and uniform child) offsets; the hi/lo
        // A parts come pre-arranged, 8 per lane (lv.ahi, lv.alo).
        using SP = Split<PREC>;
        const typename SP::v8 ahi =
            __builtin_bit_cast(typename SP::v8, ((const uint4*)lv.ahi)[lane]);
        const typename SP::v8 alo =
            __builtin_bit_cast(typename SP::v8, ((const uint4*)lv.alo)[lane]);
        const int xbase = 4 * g * VT + col, wbase = 4 * g;
        const int ntiles = (a.Gk + CPT - 1) / CPT;
        const int DS = a.rmax * VT;
        for (int tau = wave; tau < ntiles; tau += nwaves) {
            int ui = tau * CPT + sub;
            const bool ok = ui < a.Gk;
            if (!ok) ui = 0;
            const int unit = ui >> 1, i = ui & 1;
            const UnitMap um = unit_map(unit, j);
            const int bl = um.bl, rv = um.rv;
            const float2* xp = src + (((bl * 2) << (j - 1)) + rv) * RS + xbase;
            const float2* wp = twl + (unit * 4 + i * 2) * r_in + wbase;
            float zr[8], zi[8];
            float zmax = 0.f;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const float2 x = xp[(e & 1) * cstride + (e >> 1) * VT];
                const float2 w = wp[(e & 1) * r_in + (e >> 1)];
                // K rows past r_in read other data and meet A = 0; with the
                // half scaling they are zeroed so that they neither set the
                // scale nor overflow
                const bool kv = !SP::kScaled || wbase + (e >> 1) < r_in;
                zr[e] = kv ? w.x * x.x - w.y * x.y : 0.f;
                zi[e] = kv ? w.x * x.y + w.y * x.x : 0.f;
                if constexpr (SP::kScaled)
                    zmax = fmaxf(zmax, fmaxf(fabsf(zr[e]), fabsf(zi[e])));
            }
            // half: the column scaled into (-1, 1) by a power of two (exact)
            int ex = 0;
            if constexpr (SP::kScaled) ex = column_exponent(zmax);
            typename SP::v8 rh, rl, ih, il;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                SP::put8(rh, rl, e, SP::kScaled ? ldexpf(zr[e], -ex) : zr[e]);
                SP::put8(ih, il, e, SP::kScaled ? ldexpf(zi[e], -ex) : zi[e]);
            }
            floatx4 accr = {0.f, 0.f, 0.f, 0.f}, acci = {0.f, 0.f, 0.f, 0.f};
            accr = SP::mma32(ahi, rh, accr);
            acci = SP::mma32(ahi, ih, acci);
            accr = SP::mma32(ahi, rl, accr);
            acci = SP::mma32(ahi, il, acci);
            accr = SP::mma32(alo, rh, accr);
            acci = SP::mma32(alo, ih, acci);
            if constexpr (SP::kScaled) {
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    accr[jj] = ldexpf(accr[jj], ex);
                    acci[jj] = ldexpf(acci[jj], ex);
                }
            }
            // rows past r_out (zero A rows) and padding columns: the pad
            float2* op = dst + (((bl * 2 + i) << (j - 1)) + rv) * DS + col;
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const int t = 4 * g + jj;
                float2* p = (ok && t < r_out) ? op + t * VT : sink + lane;
                *p = make_float2(accr[jj], acci[jj]);
            }
        }
        return;
    }
    // FP32: K = 2 r_in ordered with the child fastest, k = 4 kk + g ->
    // child c = g % 2, coefficient s = 2 kk + g / 2.  Every lane then reads
    // x and w at a fixed base plus a compile-time step per kk, and A comes
    // pre-arranged in this order (lv.amat, zero past r_in and r_out).  Steps
    // past r_in read finite data: the pass zeroes its LDS before use.  The
    // tile loop is instantiated per number of K steps so that a level runs
    // straight-line code.
    (void)K;
    (void)tA;
    const int nks2 = (r_in + 1) >> 1;
    const int cg = g & 1, sg = g >> 1;
    const int xoff = cg * cstride + sg * VT + col;
    const int woff = cg * r_in + sg;
    switch (nks2) {
#define BF_XI_CASE(NK)                                                     \
        case NK:                                                           \
            xi_tiles_fp32<VT, NK>(a, src, RS, dst, twl, j, aMin, xoff,     \
                                  woff, sink);                             \
            break;
        BF_XI_CASE(1) BF_XI_CASE(2) BF_XI_CASE(3) BF_XI_CASE(4)
        BF_XI_CASE(5) BF_XI_CASE(6) BF_XI_CASE(7) default: BF_XI_CASE(8)
#undef BF_XI_CASE
    }
}

// FP32 tile loop of one x level with NK K steps.
template <int VT, int NK>
__device__ __forceinline__ void x_tiles_fp32(const PassArgs& a,
                                             const float2* src, float2* dst,
                                             const float2* twl, int j,
                                             bool to_tail, floatx4* tacc,
                                             const float (&aM)[8],
                                             float2* sink) {
    const PassLevel& lv = a.lv[j - 1];
    const int r_out = lv.r_out;
    const int kj = a.k - j;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    const int g = lane >> 4, n = lane & 15;
    constexpr int UPT = 16 / VT;             // units per tile
    const int sub = n / VT, col = n & (VT - 1);
    const int RS = a.rmax * VT;
    const int xoff = g * VT + col;
    const int nunits = a.Gk >> 1;
    const int ntiles = (nunits + UPT - 1) / UPT;
#pragma unroll
    for (int m = 0; m < wave_tiles<VT>() / 2; ++m) {
        const int tau = wave + m * nwaves;
        if (tau >= ntiles) break;
        int unit = tau * UPT + sub;
        const bool ok = unit < nunits;
        if (!ok) unit = 0;
        const UnitMap um = unit_map(unit, j);
        const int bl = um.bl, rv = um.rv;
        const float2* xp0 = src + (((bl * 2) << (j - 1)) + rv) * RS + xoff;
        const float2* xp1 = xp0 + ((1 << (j - 1)) * RS);
        float2 x0[NK], x1[NK];
#pragma unroll
        for (int kk = 0; kk < NK; ++kk) {
            x0[kk] = xp0[kk * 4 * VT];
            x1[kk] = xp1[kk * 4 * VT];
        }
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            floatx4 y0r = {0.f, 0.f, 0.f, 0.f}, y0i = y0r, y1r = y0r, y1i = y0r;
#pragma unroll
            for (int kk = 0; kk < NK; ++kk) {
                const float am = aM[4 * i + kk];
                y0r = mfma4(am, x0[kk].x, y0r);
                y0i = mfma4(am, x0[kk].y, y0i);
                y1r = mfma4(am, x1[kk].x, y1r);
                y1i = mfma4(am, x1[kk].y, y1i);
            }
            // rows t >= r_out read finite (zeroed or stale) twiddles and are
            // never stored
            const float2* tp = twl + (unit * 4 + i * 2) * r_out + 4 * g;
            floatx4 orr, oii;
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const float2 T0 = tp[jj];
                const float2 T1 = tp[r_out + jj];
                orr[jj] = T0.x * y0r[jj] - T0.y * y0i[jj] + T1.x * y1r[jj] - T1.y * y1i[jj];
                oii[jj] = T0.x * y0i[jj] + T0.y * y0r[jj] + T1.x * y1i[jj] + T1.y * y1r[jj];
            }
            if (to_tail) {
                // fixed (tau, lane) -> (A box, point, column) across subs
                tacc[4 * m + 2 * i] += orr;
                tacc[4 * m + 2 * i + 1] += oii;
            } else {
                // rows t >= r_out (finite: zero A rows times twiddles) and
                // padding units go to this lane's slot of the pass's pad
                float2* op = dst + (((bl * 2 + i) << (j - 1)) + rv) * RS + col;
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const int t = 4 * g + jj;
                    float2* p = (ok && t < r_out) ? op + t * VT : sink + lane;
                    *p = make_float2(orr[jj], oii[jj]);
                }
            }
        }
    }
}

// One x level: src -> dst, or (last level of a tail pass) added into tacc,
// whose lane mapping is the same on every sub-iteration.
template <int VT, int PREC>
__device__ __forceinline__ void mfma_x_level(const PassArgs& a,
                                             const float2* src, float2* dst,
                                             const float2* twl, int j,
                                             bool to_tail, floatx4* tacc,
                                             const float (&aMin)[8],
                                             float2* sink) {
    const PassLevel& lv = a.lv[j - 1];
    const int r_in = lv.r_in, r_out = lv.r_out;
    const int nks = (r_in + 3) / 4;
    const int kj = a.k - j;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    const int g = lane >> 4, tA = lane & 15;
    const int n = lane & 15;
    constexpr int UPT = 16 / VT;             // units per tile
    const int sub = n / VT, col = n & (VT - 1);
    const int RS = a.rmax * VT;
    if constexpr (PREC != BF_FP32) {
        // K = r_in <= 16: one 16x16x16 product per (child i, chain, term);
        // lane l holds s = 4 g + e, and the hi/lo A parts of M_i come
        // pre-arranged, 4 per lane (lv.ahi, lv.alo)
        using SP = Split<PREC>;
        typename SP::v4 ahi[2], alo[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            ahi[i] = __builtin_bit_cast(typename SP::v4,
                                        ((const uint2*)lv.ahi)[i * 64 + lane]);
            alo[i] = __builtin_bit_cast(typename SP::v4,
                                        ((const uint2*)lv.alo)[i * 64 + lane]);
        }
        const int xbase = 4 * g * VT + col;
        const int nunits = a.Gk >> 1;
        const int ntiles = (nunits + UPT - 1) / UPT;
#pragma unroll
        for (int m = 0; m < wave_tiles<VT>() / 2; ++m) {
            const int tau = wave + m * nwaves;
            if (tau >= ntiles) break;
            int unit = tau * UPT + sub;
            const bool ok = unit < nunits;
            if (!ok) unit = 0;
            const UnitMap um = unit_map(unit, j);
            const int bl = um.bl, rv = um.rv;
            const float2* xp0 = src + (((bl * 2) << (j - 1)) + rv) * RS;
            const float2* xp1 = xp0 + ((1 << (j - 1)) * RS);
            float2 x0[4], x1[4];
            float m0 = 0.f, m1 = 0.f;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                // rows past r_in meet A = 0; with the half scaling they are
                // zeroed (no scale, no overflow)
                const bool kv = !SP::kScaled || 4 * g + e < r_in;
                const float2 z = make_float2(0.f, 0.f);
                x0[e] = kv ? xp0[xbase + e * VT] : z;
                x1[e] = kv ? xp1[xbase + e * VT] : z;
                if constexpr (SP::kScaled) {
                    m0 = fmaxf(m0, fmaxf(fabsf(x0[e].x), fabsf(x0[e].y)));
                    m1 = fmaxf(m1, fmaxf(fabsf(x1[e].x), fabsf(x1[e].y)));
                }
            }
            // half: each child's columns scaled into (-1, 1) by a power of 2
            int e0 = 0, e1 = 0;
            if constexpr (SP::kScaled) {
                e0 = column_exponent(m0);
                e1 = column_exponent(m1);
            }
            typename SP::v4 r0h, r0l, i0h, i0l, r1h, r1l, i1h, i1l;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                SP::put4(r0h, r0l, e, SP::kScaled ? ldexpf(x0[e].x, -e0) : x0[e].x);
                SP::put4(i0h, i0l, e, SP::kScaled ? ldexpf(x0[e].y, -e0) : x0[e].y);
                SP::put4(r1h, r1l, e, SP::kScaled ? ldexpf(x1[e].x, -e1) : x1[e].x);
                SP::put4(i1h, i1l, e, SP::kScaled ? ldexpf(x1[e].y, -e1) : x1[e].y);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const floatx4 z = {0.f, 0.f, 0.f, 0.f};
                floatx4 y0r = SP::mma16(ahi[i], r0h, z), y0i = SP::mma16(ahi[i], i0h, z);
                floatx4 y1r = SP::mma16(ahi[i], r1h, z), y1i = SP::mma16(ahi[i], i1h, z);
                y0r = SP::mma16(ahi[i], r0l, y0r);
                y0i = SP::mma16(ahi[i], i0l, y0i);
                y1r = SP::mma16(ahi[i], r1l, y1r);
                y1i = SP::mma16(ahi[i], i1l, y1i);
                y0r = SP::mma16(alo[i], r0h, y0r);
                y0i = SP::mma16(alo[i], i0h, y0i);
                y1r = SP::mma16(alo[i], r1h, y1r);
                y1i = SP::mma16(alo[i], i1h, y1i);
                if constexpr (SP::kScaled) {
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) {
                        y0r[jj] = ldexpf(y0r[jj], e0);
                        y0i[jj] = ldexpf(y0i[jj], e0);
                        y1r[jj] = ldexpf(y1r[jj], e1);
                        y1i[jj] = ldexpf(y1i[jj], e1);
                    }
                }
                // rows t >= r_out read finite twiddles and are not stored
                const float2* tp = twl + (unit * 4 + i * 2) * r_out + 4 * g;
                floatx4 orr, oii;
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const float2 T0 = tp[jj];
                    const float2 T1 = tp[r_out + jj];
                    orr[jj] = T0.x * y0r[jj] - T0.y * y0i[jj] + T1.x * y1r[jj] - T1.y * y1i[jj];
                    oii[jj] = T0.x * y0i[jj] + T0.y * y0r[jj] + T1.x * y1i[jj] + T1.y * y1r[jj];
                }
                if (to_tail) {
                    tacc[4 * m + 2 * i] += orr;
                    tacc[4 * m + 2 * i + 1] += oii;
                } else {
                    // rows past r_out and padding units: the pad
                    float2* op = dst + (((bl * 2 + i) << (j - 1)) + rv) * RS + col;
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) {
                        const int t = 4 * g + jj;
                        float2* p = (ok && t < r_out) ? op + t * VT : sink + lane;
                        *p = make_float2(orr[jj], oii[jj]);
                    }
                }
            }
        }
        return;
    }
    // FP32: coefficient s = 4 kk + g, so each lane reads x at a fixed base
    // plus a compile-time step per kk; A comes pre-arranged (lv.amat, zero
    // past r_in and r_out) and steps past r_in read finite (zeroed) LDS.
    // The tile loop is instantiated per number of K steps.
    (void)tA;
    switch (nks) {
#define BF_X_CASE(NK)                                                      \
        case NK:                                                           \
            x_tiles_fp32<VT, NK>(a, src, dst, twl, j, to_tail, tacc, aMin, \
                                 sink);                                    \
            break;
        BF_X_CASE(1) BF_X_CASE(2) BF_X_CASE(3) default: BF_X_CASE(4)
#undef BF_X_CASE
    }
}

// Switch blocks of one round of pairs (NP per wave) in registers, in the
// A-operand layout of the switch's MFMAs: lane l holds S[l % 16][4 kk +
// l / 16] of each of its wave's pairs (zero past the ranks).
template <int NP>
struct SwRound {
    float2 v[NP][4];
};

// Rounds of the switch: the FP32 passes take two pairs per wave and round
// and read each round's blocks at its start; the split-precision passes,
// whose levels leave more registers free, take one pair per round and read
// the next round's blocks ahead (the first round's during the last level).
template <int PREC>
constexpr int sw_pairs() { return PREC == BF_FP32 ? 2 : 1; }
template <int PREC>
constexpr bool sw_ahead() { return PREC != BF_FP32; }

// Issue the reads of the round starting at slot r0 (group of the pass whose
// switch pairs are (a0 + rev_k(slot), bfix)).
template <int NP>
__device__ __forceinline__ void sw_load(const PassArgs& a, long long a0,
                                        long long bfix, int r0,
                                        SwRound<NP>& R) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    const int r_in = a.sw_r_in, r_out = a.sw_r_out;
    const int nks = (r_in + 3) / 4;
    const int shiftB = a.L - (a.la - 1 + a.k);
    const int g = lane >> 4, tA = lane & 15;
    const float2* S0 = a.S + (size_t)((a0 << shiftB) + bfix) * r_out * r_in;
#pragma unroll
    for (int m = 0; m < NP; ++m) {
        const int slot = r0 + wave + m * nwaves;
        if (slot >= a.Gk) break;
        const unsigned dA = (unsigned)digit_rev(slot, a.k, 1);
        const float2* S = S0 + (dA << shiftB) * (unsigned)(r_out * r_in);
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            if (kk >= nks) break;
            const int s = 4 * kk + g;
            R.v[m][kk] = (s < r_in && tA < r_out) ? S[tA * r_in + s]
                                                  : make_float2(0.f, 0.f);
        }
    }
}

// nu = S mu per pair, in place (pairs are independent, so each wave reads
// its pair's slot and writes it back without a workgroup barrier between).
// 16 real columns: n = (column, re|im), Re nu = Re S Re mu - Im S Im mu and
// Im nu = Re S Im mu + Im S Re mu with the cross term from lane n ^ 1.
// AHEAD: first holds the first round's blocks, read by the caller ahead of
// time, and each round issues the next round's reads before its own MFMA
// work; otherwise each round reads its blocks at its start.
template <int VT, int NP, bool AHEAD>
__device__ __forceinline__ void mfma_switch(const PassArgs& a, float2* tile,
                                            long long a0, long long bfix,
                                            const SwRound<NP>& first) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    const int r_in = a.sw_r_in, r_out = a.sw_r_out;
    const int nks = (r_in + 3) / 4;
    const int g = lane >> 4;
    const int n = lane & 15;
    const int col = n >> 1, reim = n & 1;
    const int colc = col < VT ? col : 0;
    float* tf = (float*)tile;
    int so[4];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
        const int s = 4 * kk + g;
        so[kk] = ((s < r_in ? s : 0) * VT + colc) * 2 + reim;
    }
    const int step = NP * nwaves;
    SwRound<NP> cur = first;
    for (int r0 = 0; r0 < a.Gk; r0 += step) {   // rounds of pairs
        SwRound<NP> nxt;
        if constexpr (AHEAD) {
            if (r0 + step < a.Gk) sw_load(a, a0, bfix, r0 + step, nxt);
        } else {
            sw_load(a, a0, bfix, r0, cur);
        }
#pragma unroll
        for (int m = 0; m < NP; ++m) {
            const int slot = r0 + wave + m * nwaves;
            if (slot >= a.Gk) break;
            const int base = slot * a.rmax * VT * 2;
            float bv[4];
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                if (kk >= nks) break;
                bv[kk] = tf[base + so[kk]];
            }
            floatx4 ar = {0.f, 0.f, 0.f, 0.f}, ai = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                if (kk >= nks) break;
                ar = mfma4(cur.v[m][kk].x, bv[kk], ar);
                ai = mfma4(cur.v[m][kk].y, bv[kk], ai);
            }
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const float p = lane_swap1(ai[jj]);
                const float v = reim ? ar[jj] + p : ar[jj] - p;
                const int t = 4 * g + jj;
                if (col < VT && t < r_out) tf[base + (t * VT + col) * 2 + reim] = v;
            }
        }
        if constexpr (AHEAD) cur = nxt;
    }
    __syncthreads();
}

// Split-precision switch (BF16x3 / FP16x3).  The stored blocks of a split
// plan hold, per entry, the 16-bit parts (Re hi, Re lo, Im hi, Im lo) of
// S_{AB}[t][s] (split once at plan time), so a block streams the same bytes
// as in FP32.  One pair per wave and round, r_in <= 16: a single 16x16x16
// product per part, lane l holding A[l % 16][4 (l / 16) + e] and
// B[4 (l / 16) + e][l % 16], e < 4.  Re nu and Im nu come from A = Re S and
// A = Im S, each as hi*hi + hi*lo + lo*hi on the split panel (FP16: each
// column scaled by a power of two first), with the cross term from the
// neighbouring lane as in FP32.
template <int PREC>
struct SwRoundSplit {
    typename Split<PREC>::v4 rh, rl, ih, il;
};

template <int PREC>
__device__ __forceinline__ void sw_load_split(const PassArgs& a, long long a0,
                                              long long bfix, int r0,
                                              SwRoundSplit<PREC>& R) {
    using V = typename Split<PREC>::v4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r_in = a.sw_r_in, r_out = a.sw_r_out;
    const int shiftB = a.L - (a.la - 1 + a.k);
    const int g = lane >> 4, tA = lane & 15;
    const int slot = r0 + wave;
    R.rh = R.rl = R.ih = R.il = V{};
    if (slot >= a.Gk || tA >= r_out) return;
    const unsigned dA = (unsigned)digit_rev(slot, a.k, 1);
    const ushort4* S = (const ushort4*)a.S +
                       (size_t)((a0 << shiftB) + bfix) * r_out * r_in +
                       (size_t)(dA << shiftB) * (unsigned)(r_out * r_in) +
                       (size_t)tA * r_in;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int sx = 4 * g + e;
        ushort4 q = make_ushort4(0, 0, 0, 0);
        if (sx < r_in) q = S[sx];
        using E = typename Split<PREC>::e4;
        R.rh[e] = __builtin_bit_cast(E, q.x);
        R.rl[e] = __builtin_bit_cast(E, q.y);
        R.ih[e] = __builtin_bit_cast(E, q.z);
        R.il[e] = __builtin_bit_cast(E, q.w);
    }
}

template <int VT, int PREC>
__device__ __forceinline__ void mfma_switch_split(
    const PassArgs& a, float2* tile, long long a0, long long bfix,
    const SwRoundSplit<PREC>& first) {
    using SP = Split<PREC>;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    const int r_in = a.sw_r_in, r_out = a.sw_r_out;
    const int g = lane >> 4;
    const int n = lane & 15;
    const int col = n >> 1, reim = n & 1;
    const int colc = col < VT ? col : 0;
    float* tf = (float*)tile;
    SwRoundSplit<PREC> cur = first;
    for (int r0 = 0; r0 < a.Gk; r0 += nwaves) {   // rounds of pairs
        SwRoundSplit<PREC> nxt;
        if (r0 + nwaves < a.Gk) sw_load_split<PREC>(a, a0, bfix, r0 + nwaves, nxt);
        const int slot = r0 + wave;
        if (slot < a.Gk) {
            const int base = slot * a.rmax * VT * 2;
            float bv[4];
            float m = 0.f;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int sx = 4 * g + e;
                // rows past r_in meet A = 0; zeroed so that they set no scale
                bv[e] = (sx < r_in && col < VT)
                            ? tf[base + (sx * VT + colc) * 2 + reim] : 0.f;
                if constexpr (SP::kScaled) m = fmaxf(m, fabsf(bv[e]));
            }
            int ex = 0;
            if constexpr (SP::kScaled) ex = column_exponent(m);
            typename SP::v4 bh, bl;
#pragma unroll
            for (int e = 0; e < 4; ++e)
                SP::put4(bh, bl, e, SP::kScaled ? ldexpf(bv[e], -ex) : bv[e]);
            const floatx4 z = {0.f, 0.f, 0.f, 0.f};
            floatx4 ar = SP::mma16(cur.rh, bh, z), ai = SP::mma16(cur.ih, bh, z);
            ar = SP::mma16(cur.rh, bl, ar);
            ai = SP::mma16(cur.ih, bl, ai);
            ar = SP::mma16(cur.rl, bh, ar);
            ai = SP::mma16(cur.il, bh, ai);
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                if constexpr (SP::kScaled) {
                    ar[jj] = ldexpf(ar[jj], ex);
                    ai[jj] = ldexpf(ai[jj], ex);
                }
                const float p = lane_swap1(ai[jj]);
                const float v = reim ? ar[jj] + p : ar[jj] - p;
                const int t = 4 * g + jj;
                if (col < VT && t < r_out) tf[base + (t * VT + col) * 2 + reim] = v;
            }
        }
        cur = nxt;
    }
    __syncthreads();
}

// A operand of level j from a pass's per-workgroup LDS copy.
__device__ __forceinline__ void read_amat(const float* AX, int j,
                                          float (&aM)[8]) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < 8; ++q) aM[q] = AX[(j - 1) * 512 + q * 64 + lane];
}

// Zero the tiles, the twiddle buffers and the trailing pad of a pass (the
// f tile is written whole before use), so that K steps past a level's rank
// and rows past r_out read finite values, which then meet zero A entries or
// are never stored.
__device__ __forceinline__ void zero_pass_lds(float2* lds, int n_front,
                                              float2* pad) {
    for (int e = threadIdx.x; e < n_front; e += blockDim.x)
        lds[e] = make_float2(0.f, 0.f);
    if (threadIdx.x < kMfmaLdsPad) pad[threadIdx.x] = make_float2(0.f, 0.f);
    __syncthreads();
}

// LDS of an MFMA pass: the tile (Gk x rmax x VT), two twiddle buffers
// (2 Gk rmax each), the f tile (Gk x head_r x VT) when the pass starts from
// f, then a zeroed pad of kMfmaLdsPad entries.  Levels update the tile in
// place: a unit reads its two slots and writes the same two slots, and all
// of a unit's columns sit in one wave, so no other wave touches them within
// the level.
//
// HIN (a.head_inplace): the head is gathered into T at every sub-iteration.
template <int VT, int PREC, bool HIN>
__global__ void __launch_bounds__((kMfmaThreads))
xi_pass_mfma(PassArgs a) {
    extern __shared__ float2 lds[];
    // every LDS pointer below is lds + offset (not read from an array of
    // pointers) so the compiler keeps them in the LDS address space and
    // emits ds_read / ds_write
    const int tsz = a.Gk * a.rmax * VT, wsz = 2 * a.Gk * a.rmax;
    // two twiddle buffers (the next level's written while a level runs), or
    // one (written after a barrier) where that lets two workgroups share a
    // CU
    const int nw = (HIN && a.tw_single) ? 1 : 2;
    float2* const T = lds;
    float2* const W0 = lds + tsz;
    float2* const W1 = lds + tsz + (nw - 1) * wsz;
    float2* const ftile = lds + tsz + nw * wsz;
    // the head in a tile of its own (kept for all sub-iterations), or
    // gathered into T at the tile's slot stride for each sub-iteration, so
    // that level 1 runs in place like the others
    const bool fsep = !HIN && a.has_head;
    long long spatial;
    int chunk;
    block_coords(a, spatial, chunk);
    if (spatial >= a.nspatial) return;
    // zeroed pad after the tiles: reads past a level's rank land here, and
    // stores of rows past r_out and of padding columns go here (finite)
    float2* const pad = fsep ? ftile + a.Gk * a.head_r * VT : ftile;
    // in-place head (FP32): the A operands of every level are staged in LDS
    // once (AX[(j - 1) 512 + q 64 + lane] = aM[q] of level j, the order of
    // load_amat), which leaves the registers to hold the gathered head
    constexpr bool kAX = HIN && PREC == BF_FP32;
    float* const AX = (float*)(pad + kMfmaLdsPad);
    if constexpr (kAX) {
        for (int e = threadIdx.x; e < a.k * 512; e += blockDim.x) {
            const int j = e >> 9, q = (e >> 6) & 7, ln = e & 63;
            const PassLevel& lv = a.lv[j];
            AX[e] = q < ((lv.r_in + 1) >> 1) ? lv.amat[q * 64 + ln] : 0.f;
        }
    }
    zero_pass_lds(lds, tsz + nw * wsz, pad);
    const int part = (int)(spatial % a.sub_split);
    spatial /= a.sub_split;
    const long long bg = spatial % a.nbg;
    const long long ap_base = spatial / a.nbg;
    // the f tile is shared by the sub-iterations of the workgroup (the T_X
    // boxes at level l0 - 1 all see the same input): kept in LDS, or (in
    // place, FP32) in registers and written into T at every sub-iteration
    if (fsep) load_head(a, ftile, bg * a.Gk, chunk);
    HeadRegs<8> hreg;
    const bool hkeep = kAX && hreg.fits(a);
    if (hkeep) hreg.load(a, bg * a.Gk, chunk);
    for (int si = 0; si < a.n_sub; ++si) {
        const int sub = part * a.n_sub + si;
        const long long ap_grp = a.has_head ? sub : ap_base;
        if (!a.has_head) {
            const long long p0 = (ap_grp << (a.L - a.la + 1)) + bg * a.Gk;
            load_tile(a, T, p0, a.lv[0].r_in, chunk);
        } else if constexpr (HIN) {
            if (hkeep)
                hreg.store(a, T, a.rmax);
            else
                load_head(a, T, bg * a.Gk, chunk, a.rmax);
        }
        stage_twiddles(a, 1, W0, ap_grp, bg, true);
        float aM[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if constexpr (PREC == BF_FP32 && !kAX) load_amat(a.lv[0], true, aM);
        __syncthreads();
        // level j uses W0 (j odd) or W1; the next level's A operand and
        // twiddles are read from global memory before the level's MFMA work
        // and the twiddles written to the other buffer after it, so the
        // reads overlap the work; level 1 of a head pass reads the f tile
        for (int j = 1; j < a.k; ++j) {
            const bool odd = (j & 1) != 0;
            float aMn[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            TwStage<tw_regs<VT>()> next;
            if constexpr (PREC == BF_FP32 && !kAX) load_amat(a.lv[j], true, aMn);
            next.load(a, j + 1, ap_grp, bg, true);
            if constexpr (kAX) read_amat(AX, j, aM);
            const bool from_f = j == 1 && fsep;
            mfma_xi_level<VT, PREC>(a, from_f ? ftile : T,
                                    from_f ? a.head_r : a.rmax, T,
                                    odd ? W0 : W1, j, aM, pad);
            if (nw == 1) __syncthreads();   // the level's twiddles are read
            next.store(odd ? W1 : W0);
            __syncthreads();
            if constexpr (!kAX) {
#pragma unroll
                for (int q = 0; q < 8; ++q) aM[q] = aMn[q];
            }
        }
        {
            // the last level reads the switch's first blocks ahead
            const int j = a.k;
            if constexpr (kAX) read_amat(AX, j, aM);
            SwRound<sw_pairs<PREC>()> sw0;
            SwRoundSplit<PREC == BF_FP32 ? BF_BF16X3 : PREC> sws0;
            if constexpr (PREC != BF_FP32)
                if (a.has_switch) sw_load_split<PREC>(a, ap_grp * a.Gk, bg, 0, sws0);
            const bool from_f = j == 1 && fsep;
            mfma_xi_level<VT, PREC>(a, from_f ? ftile : T,
                                    from_f ? a.head_r : a.rmax, T,
                                    (j & 1) ? W0 : W1, j, aM, pad);
            __syncthreads();
            if (a.has_switch) {
                if constexpr (PREC == BF_FP32)
                    mfma_switch<VT, sw_pairs<PREC>(), sw_ahead<PREC>()>(
                        a, T, ap_grp * a.Gk, bg, sw0);
                else
                    mfma_switch_split<VT, PREC>(a, T, ap_grp * a.Gk, bg, sws0);
            }
        }
        store_tile(a, T, ap_grp * a.Gk, bg, chunk);
        __syncthreads();
    }
}

// The FP32 A operands of all levels are staged in LDS once per workgroup
// (AX[(j - 1) 512 + q 64 + lane] = aM[q] of level j, the order of
// load_amat): they are shared by every unit of a level, and reading them
// from LDS per level keeps them (and the next level's) out of the
// registers.
template <int VT, int PREC>
__global__ void __launch_bounds__((kMfmaThreads))
x_pass_mfma(PassArgs a) {
    extern __shared__ float2 lds[];
    const int tsz = a.Gk * a.rmax * VT, wsz = 2 * a.Gk * a.rmax;
    float2* const T = lds;
    float2* const W0 = lds + tsz;
    float2* const W1 = lds + tsz + wsz;
    long long spatial;
    int chunk;
    block_coords(a, spatial, chunk);
    if (spatial >= a.nspatial) return;
    float2* const pad = lds + tsz + 2 * wsz;
    float* const AX = (float*)(pad + kMfmaLdsPad);
    if constexpr (PREC == BF_FP32) {
        for (int e = threadIdx.x; e < a.k * 512; e += blockDim.x) {
            const int j = e >> 9, q = (e >> 6) & 7, ln = e & 63;
            const PassLevel& lv = a.lv[j];
            const int nks = (lv.r_in + 3) >> 2, i = q >> 2, kk = q & 3;
            AX[e] = kk < nks ? lv.amat[(i * nks + kk) * 64 + ln] : 0.f;
        }
    }
    zero_pass_lds(lds, tsz + 2 * wsz, pad);
    // with x_split > 1 the workgroup takes part `part` of the B groups
    const int part = (int)(spatial % a.x_split);
    spatial /= a.x_split;
    const long long ap_grp = a.has_tail ? spatial : spatial / a.nbg;
    const long long bg0 = a.has_tail ? 0 : spatial % a.nbg;
    floatx4 tacc[2 * wave_tiles<VT>()];
#pragma unroll
    for (int m = 0; m < 2 * wave_tiles<VT>(); ++m) tacc[m] = floatx4{0.f, 0.f, 0.f, 0.f};
    // the next sub-iteration's tile and level-1 twiddles are read during
    // the current one's last level and written at the next one's start
    // (not in FP16x3, whose x levels leave no registers for them)
    constexpr bool kPre = PREC != BF_FP16X3;
    TileLoad<pre_regs<VT>()> pre;
    TwStage<tw_regs<VT>()> pre_tw;
    for (int si = 0; si < a.n_sub; ++si) {
        const int sub = part * a.n_sub + si;
        const long long bg = a.has_tail ? sub : bg0;
        if (si == 0 || !kPre) {
            const long long p0 = (ap_grp << (a.L - a.la + 1)) + bg * a.Gk;
            load_tile(a, T, p0, a.lv[0].r_in, chunk);
            stage_twiddles(a, 1, W0, ap_grp, bg, false);
        } else {
            pre.store(a, T, a.lv[0].r_in);
            pre_tw.store(W0);
        }
        __syncthreads();
        for (int j = 1; j <= a.k; ++j) {
            const bool odd = (j & 1) != 0;
            float aM[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            TwStage<tw_regs<VT>()> next;
            if (j < a.k) {
                next.load(a, j + 1, ap_grp, bg, false);
            } else if (kPre && si + 1 < a.n_sub) {
                const long long bgn = a.has_tail ? sub + 1 : bg0;
                pre.load(a, (ap_grp << (a.L - a.la + 1)) + bgn * a.Gk,
                         a.lv[0].r_in, chunk);
                pre_tw.load(a, 1, ap_grp, bgn, false);
            }
            if constexpr (PREC == BF_FP32) read_amat(AX, j, aM);
            mfma_x_level<VT, PREC>(a, T, T, odd ? W0 : W1, j,
                                   a.has_tail && j == a.k, tacc, aM, pad);
            if (j < a.k) next.store(odd ? W1 : W0);
            __syncthreads();
        }
        if (!a.has_tail) {
            store_tile(a, T, ap_grp * a.Gk, bg, chunk);
            __syncthreads();
        }
    }
    if (!a.has_tail) return;
    // final coefficients of the Gk boxes A to LDS as [a_loc][t][VT], then
    // g_v(x) = sum_k a_k(x) lambda_k(x) (eq. (eqn:tg))
    float2* fin = T;
    {
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        const int nwaves = blockDim.x >> 6;
        const int r_out = a.lv[a.k - 1].r_out;
        constexpr int UPT = 16 / VT;
        const int nunits = a.Gk >> 1;
        const int ntiles = (nunits + UPT - 1) / UPT;
        const int n = lane & 15, g = lane >> 4;
        const int sub = n / VT, col = n & (VT - 1);
#pragma unroll
        for (int m = 0; m < wave_tiles<VT>() / 2; ++m) {
            const int tau = wave + m * nwaves;
            if (tau >= ntiles) break;
            const int unit = tau * UPT + sub;
            if (unit >= nunits) continue;
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                // last level (j = k): the unit's A boxes are its apl's
                const int aloc = unit_map(unit, a.k).apl * 2 + i;
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const int t = 4 * g + jj;
                    if (t < r_out)
                        fin[(aloc * a.tail_r + t) * VT + col] =
                            make_float2(tacc[4 * m + 2 * i][jj],
                                        tacc[4 * m + 2 * i + 1][jj]);
                }
            }
        }
    }
    __syncthreads();
    const int tv = VT / a.r_amp;
    const int total = a.Gk * a.tail_r * tv;
    const int v0 = chunk * tv;
    const int nvs = a.Vs / a.r_amp;
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
        const int t = e % a.tail_r;
        const int rest = e / a.tail_r;
        const int aloc = rest % a.Gk;
        const int vl = rest / a.Gk;
        if (v0 + vl >= nvs) continue;
        const long long x = (ap_grp * a.Gk + aloc) * (long long)a.tail_side + t;
        float2 sum = make_float2(0.f, 0.f);
        for (int kk = 0; kk < a.r_amp; ++kk) {
            const float2 v = fin[(aloc * a.tail_r + t) * VT + vl * a.r_amp + kk];
            if (a.amp_a) {
                const float2 z = cmul(a.amp_a[(size_t)kk * a.N + x], v);
                sum.x += z.x;
                sum.y += z.y;
            } else {
                sum.x += v.x;
                sum.y += v.y;
            }
        }
        if (a.x_split > 1)   // partial sum over this part's B groups
            a.gpart[((size_t)part * nvs + v0 + vl) * a.N + x] = sum;
        else
            a.g[(size_t)(v0 + vl) * a.N + x] = sum;
    }
}

// g[v][x] = sum over the parts of a split tail pass, in part order (the
// same order for every batch size, so results do not depend on it).
__global__ void __launch_bounds__(256) sum_parts(const float2* part,
                                                 float2* g, int parts,
                                                 long long count) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= count) return;
    float2 s = part[i];
    for (int p = 1; p < parts; ++p) {
        const float2 v = part[(size_t)p * count + i];
        s.x += v.x;
        s.y += v.y;
    }
    g[i] = s;
}

std::string launch_sum_parts(const PassArgs& a, int nv, hipStream_t st) {
    const long long count = (long long)nv * a.N;
    hipLaunchKernelGGL(sum_parts, dim3((unsigned)((count + 255) / 256)),
                       dim3(256), 0, st, a.gpart, a.g, a.x_split, count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return std::string("sum_parts launch: ") + hipGetErrorString(e);
    return "";
}

size_t mfma_pass_lds(const PassArgs& a, bool is_xi) {
    const size_t tsz = (size_t)a.Gk * a.rmax * a.Vt, wsz = (size_t)2 * a.Gk * a.rmax;
    const int nw = (is_xi && a.head_inplace && a.tw_single) ? 1 : 2;
    size_t e = tsz + nw * wsz + kMfmaLdsPad;
    if (is_xi && a.has_head && !a.head_inplace)
        e += (size_t)a.Gk * a.head_r * a.Vt;
    // A operands of the FP32 x passes and in-place head xi passes
    if (a.prec == BF_FP32 && (!is_xi || a.head_inplace)) e += (size_t)a.k * 256;
    return e * sizeof(float2);
}

template <int VT, int PREC>
static void set_attrs() {
    static bool attr = false;
    if (attr) return;
    (void)hipFuncSetAttribute((const void*)xi_pass_mfma<VT, PREC, false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
    (void)hipFuncSetAttribute((const void*)xi_pass_mfma<VT, PREC, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
    (void)hipFuncSetAttribute((const void*)x_pass_mfma<VT, PREC>,
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
    attr = true;
}

template <int PREC>
static void set_attrs_prec() {
    set_attrs<1, PREC>();
    set_attrs<2, PREC>();
    set_attrs<4, PREC>();
    set_attrs<8, PREC>();
}

void init_mfma_attrs() {
    set_attrs_prec<BF_FP32>();
    set_attrs_prec<BF_BF16X3>();
    set_attrs_prec<BF_FP16X3>();
}

// Threads of an MFMA pass workgroup.  A pass whose LDS fits twice in a CU
// runs as workgroups of 512 threads when the grid still has two of them per
// CU (256 CUs): the same 16 waves per CU, in two groups with their own
// barriers, so one group's reads of the next level's factors overlap the
// other's MFMA work (with few columns per group a level mostly waits on
// them).  The xi pass loops over its tiles with any number of waves; the x
// pass gives each wave at most one tile per level, which 8 waves cover only
// for groups of at most half the largest tile (Gk Vt <= 256).
static int pass_threads(const PassArgs& a, bool is_xi, int vt, size_t lds,
                        long long nblocks) {
    const bool two = 2 * lds <= 160 * 1024 && nblocks >= 512;
    const bool covered =
        is_xi || (long long)a.Gk * vt <= (long long)kMfmaTileCap * 8 / 2;
    return two && covered ? kMfmaThreads / 2 : kMfmaThreads;
}

template <int VT, int PREC>
static std::string launch_vt(const PassArgs& a, bool is_xi, size_t lds,
                             hipStream_t st) {
    set_attrs<VT, PREC>();
    const long long nblocks = a.nspatial * a.nchunk;
    const int threads = pass_threads(a, is_xi, VT, lds, nblocks);
    if (is_xi && a.head_inplace)
        hipLaunchKernelGGL((xi_pass_mfma<VT, PREC, true>),
                           dim3((unsigned)nblocks), dim3(threads), lds, st, a);
    else if (is_xi)
        hipLaunchKernelGGL((xi_pass_mfma<VT, PREC, false>),
                           dim3((unsigned)nblocks), dim3(threads), lds, st, a);
    else
        hipLaunchKernelGGL((x_pass_mfma<VT, PREC>), dim3((unsigned)nblocks),
                           dim3(threads), lds, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return std::string("MFMA pass launch: ") + hipGetErrorString(e);
    return "";
}

template <int PREC>
static std::string launch_prec(const PassArgs& a, bool is_xi, size_t lds,
                               hipStream_t st) {
    switch (a.Vt) {
        case 1: return launch_vt<1, PREC>(a, is_xi, lds, st);
        case 2: return launch_vt<2, PREC>(a, is_xi, lds, st);
        case 4: return launch_vt<4, PREC>(a, is_xi, lds, st);
        case 8: return launch_vt<8, PREC>(a, is_xi, lds, st);
        default: return "MFMA pass: tile width must be 1, 2, 4 or 8";
    }
}

std::string launch_mfma_pass(const PassArgs& a, bool is_xi, size_t lds,
                             hipStream_t st) {
    switch (a.prec) {
        case BF_FP32: return launch_prec<BF_FP32>(a, is_xi, lds, st);
        case BF_BF16X3: return launch_prec<BF_BF16X3>(a, is_xi, lds, st);
        case BF_FP16X3: return launch_prec<BF_FP16X3>(a, is_xi, lds, st);
        default: return "MFMA pass: unknown precision";
    }
}

}  // namespace bfi
