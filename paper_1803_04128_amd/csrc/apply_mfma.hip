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
// K steps past the end use A = 0 and read valid (finite) data, so the loads
// need no guards.  R = 2, r <= 16, VT (columns per tile) in {1, 2, 4, 8}.
#include "fused_common.h"

namespace bfi {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// 8 waves per workgroup share one LDS tile (two waves per SIMD)
constexpr int kMfmaThreads = 512;
constexpr int kWaveTiles = kMfmaTileCap / (2 * (kMfmaThreads / 64));

__device__ __forceinline__ float lane_swap1(float v) {
    // quad_perm [1, 0, 3, 2]: exchange with the neighbouring lane
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1,
                                                   0xF, 0xF, false));
}

__device__ __forceinline__ floatx4 mfma4(float a, float b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Twiddles of local level j for the group's units into LDS:
// twl[unit_loc][i][c][r], unit_loc = apl 2^(k-j) + bl, contiguous per apl.
__device__ __forceinline__ void stage_twiddles(const PassArgs& a,
                                               const PassLevel& lv, int rr,
                                               float2* twl, int j,
                                               long long ap_grp,
                                               long long bg) {
    const int kj = a.k - j;
    const int per_unit = 4 * rr;
    const int total = (a.Gk >> 1) * per_unit;
    const int shiftB = a.L - (a.la + j - 1);
    Walk2 w(threadIdx.x, per_unit);
    for (int e = threadIdx.x; e < total; e += blockDim.x, w.next()) {
        const int unit = w.hi;
        const int apl = unit >> kj, bl = unit & ((1 << kj) - 1);
        const long long apg = (ap_grp << (j - 1)) + apl;
        const long long bgl = (bg << kj) + bl;
        const long long u = (apg << shiftB) + bgl;
        twl[e] = lv.tw[u * per_unit + w.lo];
    }
}

template <int VT>
__device__ __forceinline__ void mfma_xi_level(const PassArgs& a, float2* tile,
                                              const float2* ftile, float2* twl,
                                              int j, long long ap_grp,
                                              long long bg) {
    const PassLevel& lv = a.lv[j - 1];
    const int r_in = lv.r_in, r_out = lv.r_out;
    const int K = 2 * r_in, nks = (K + 3) / 4;
    const int kj = a.k - j;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    stage_twiddles(a, lv, r_in, twl, j, ap_grp, bg);
    const int g = lane >> 4, tA = lane & 15;
    const int n = lane & 15;
    constexpr int CPT = 16 / VT;             // (unit, i) combinations per tile
    const int sub = n / VT, col = n & (VT - 1);
    const bool from_f = a.has_head && j == 1;
    const float2* src = from_f ? ftile : tile;
    const int RS = (from_f ? a.head_r : a.rmax) * VT;   // slot stride
    // per-lane K-step tables: k = 4 kk + g -> child kc, point ks; the A
    // operand for the whole level; LDS offsets of x and of the twiddle
    float aM[8];
    int kc[8], xo[8], wo[8];
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
        const int k = 4 * kk + g;
        const bool v = kk < nks && k < K;
        const int c = (v && k >= r_in) ? 1 : 0;
        const int s = v ? k - c * r_in : 0;
        kc[kk] = c;
        xo[kk] = s * VT + col;
        wo[kk] = c * r_in + s;
        aM[kk] = (v && tA < r_out) ? lv.mats[(c * r_out + tA) * r_in + s] : 0.f;
    }
    const int ntiles = (a.Gk + CPT - 1) / CPT;
    __syncthreads();
    floatx4 kr[kWaveTiles], ki[kWaveTiles];
#pragma unroll
    for (int m = 0; m < kWaveTiles; ++m) {
        const int tau = wave + m * nwaves;
        if (tau >= ntiles) break;
        int ui = tau * CPT + sub;
        if (ui >= a.Gk) ui = 0;                 // padding column: any valid data
        const int unit = ui >> 1, i = ui & 1;
        const int apl = unit >> kj, bl = unit & ((1 << kj) - 1);
        const int rv = digit_rev(apl, j - 1, 1);
        const int sb0 = (((bl * 2) << (j - 1)) + rv) * RS;
        const int sb1 = (((bl * 2 + 1) << (j - 1)) + rv) * RS;
        const int twb = (unit * 4 + i * 2) * r_in;
        float2 xs[8], ws[8];
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) {
            if (kk >= nks) break;
            xs[kk] = src[(kc[kk] ? sb1 : sb0) + xo[kk]];
            ws[kk] = twl[twb + wo[kk]];
        }
        floatx4 accr = {0.f, 0.f, 0.f, 0.f}, acci = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) {
            if (kk >= nks) break;
            const float2 x = xs[kk], w = ws[kk];
            const float zr = w.x * x.x - w.y * x.y;
            const float zi = w.x * x.y + w.y * x.x;
            accr = mfma4(aM[kk], zr, accr);
            acci = mfma4(aM[kk], zi, acci);
        }
        kr[m] = accr;
        ki[m] = acci;
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < kWaveTiles; ++m) {
        const int tau = wave + m * nwaves;
        if (tau >= ntiles) break;
        const int ui = tau * CPT + sub;
        if (ui >= a.Gk) continue;
        const int unit = ui >> 1, i = ui & 1;
        const int apl = unit >> kj, bl = unit & ((1 << kj) - 1);
        const int slot_out = ((bl * 2 + i) << (j - 1)) + digit_rev(apl, j - 1, 1);
        const int base = slot_out * a.rmax * VT + col;
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int t = 4 * g + jj;
            if (t < r_out) tile[base + t * VT] = make_float2(kr[m][jj], ki[m][jj]);
        }
    }
    __syncthreads();
}

// x level; on the last level of a tail pass the outputs are added into
// tacc (same lane mapping on every sub-iteration) instead of the tile.
template <int VT>
__device__ __forceinline__ void mfma_x_level(const PassArgs& a, float2* tile,
                                             float2* twl, int j,
                                             long long ap_grp, long long bg,
                                             bool to_tail, floatx4* tacc) {
    const PassLevel& lv = a.lv[j - 1];
    const int r_in = lv.r_in, r_out = lv.r_out;
    const int nks = (r_in + 3) / 4;
    const int kj = a.k - j;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    stage_twiddles(a, lv, r_out, twl, j, ap_grp, bg);
    const int g = lane >> 4, tA = lane & 15;
    const int n = lane & 15;
    constexpr int UPT = 16 / VT;             // units per tile
    const int sub = n / VT, col = n & (VT - 1);
    const int RS = a.rmax * VT;
    float aM[2][4];
    int xo[4];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
        const int s = 4 * kk + g;
        const bool v = kk < nks && s < r_in;
        xo[kk] = (v ? s : 0) * VT + col;
#pragma unroll
        for (int i = 0; i < 2; ++i)
            aM[i][kk] = (v && tA < r_out) ? lv.mats[(i * r_out + tA) * r_in + s]
                                          : 0.f;
    }
    const int nunits = a.Gk >> 1;
    const int ntiles = (nunits + UPT - 1) / UPT;
    __syncthreads();
    // keep[m][i]: (re, im) accumulators of output child i
    floatx4 kr[kWaveTiles / 2][2], ki[kWaveTiles / 2][2];
#pragma unroll
    for (int m = 0; m < kWaveTiles / 2; ++m) {
        const int tau = wave + m * nwaves;
        if (tau >= ntiles) break;
        int unit = tau * UPT + sub;
        const bool ok = unit < nunits;
        if (!ok) unit = 0;
        const int apl = unit >> kj, bl = unit & ((1 << kj) - 1);
        const int rv = digit_rev(apl, j - 1, 1);
        const int sb0 = (((bl * 2) << (j - 1)) + rv) * RS;
        const int sb1 = (((bl * 2 + 1) << (j - 1)) + rv) * RS;
        float2 x0[4], x1[4];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            if (kk >= nks) break;
            x0[kk] = tile[sb0 + xo[kk]];
            x1[kk] = tile[sb1 + xo[kk]];
        }
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            floatx4 y0r = {0.f, 0.f, 0.f, 0.f}, y0i = y0r, y1r = y0r, y1i = y0r;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                if (kk >= nks) break;
                const float am = aM[i][kk];
                y0r = mfma4(am, x0[kk].x, y0r);
                y0i = mfma4(am, x0[kk].y, y0i);
                y1r = mfma4(am, x1[kk].x, y1r);
                y1i = mfma4(am, x1[kk].y, y1i);
            }
            const int twb = (unit * 4 + i * 2) * r_out;
            floatx4 orr, oii;
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                int t = 4 * g + jj;
                if (t >= r_out) t = 0;
                const float2 T0 = twl[twb + t];
                const float2 T1 = twl[twb + r_out + t];
                orr[jj] = T0.x * y0r[jj] - T0.y * y0i[jj] + T1.x * y1r[jj] - T1.y * y1i[jj];
                oii[jj] = T0.x * y0i[jj] + T0.y * y0r[jj] + T1.x * y1i[jj] + T1.y * y1r[jj];
            }
            kr[m][i] = orr;
            ki[m][i] = oii;
        }
    }
    __syncthreads();
    if (to_tail) {
#pragma unroll
        for (int m = 0; m < kWaveTiles / 2; ++m) {
            const int tau = wave + m * nwaves;
            if (tau >= ntiles) break;
            tacc[4 * m + 0] += kr[m][0];
            tacc[4 * m + 1] += ki[m][0];
            tacc[4 * m + 2] += kr[m][1];
            tacc[4 * m + 3] += ki[m][1];
        }
        return;
    }
#pragma unroll
    for (int m = 0; m < kWaveTiles / 2; ++m) {
        const int tau = wave + m * nwaves;
        if (tau >= ntiles) break;
        const int unit = tau * UPT + sub;
        if (unit >= nunits) continue;
        const int apl = unit >> kj, bl = unit & ((1 << kj) - 1);
        const int rv = digit_rev(apl, j - 1, 1);
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int slot_out = ((bl * 2 + i) << (j - 1)) + rv;
            const int base = slot_out * RS + col;
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const int t = 4 * g + jj;
                if (t < r_out) tile[base + t * VT] = make_float2(kr[m][i][jj], ki[m][i][jj]);
            }
        }
    }
    __syncthreads();
}

// nu = S mu per pair, in place (pairs are independent, so each wave reads
// its pair's slot and writes it back without a workgroup barrier between).
// 16 real columns: n = (column, re|im), Re nu = Re S Re mu - Im S Im mu and
// Im nu = Re S Im mu + Im S Re mu with the cross term from lane n ^ 1.
template <int VT>
__device__ __forceinline__ void mfma_switch(const PassArgs& a, float2* tile,
                                            long long a0, long long bfix) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    const int r_in = a.sw_r_in, r_out = a.sw_r_out;
    const int nks = (r_in + 3) / 4;
    const int shiftB = a.L - (a.la - 1 + a.k);
    const int g = lane >> 4, tA = lane & 15;
    const int n = lane & 15;
    const int col = n >> 1, reim = n & 1;
    const int colc = col < VT ? col : 0;
    float* tf = (float*)tile;
    int so[4];
    bool sv_ok[4];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
        const int s = 4 * kk + g;
        sv_ok[kk] = kk < nks && s < r_in && tA < r_out;
        so[kk] = ((s < r_in ? s : 0) * VT + colc) * 2 + reim;
    }
    for (int slot = wave; slot < a.Gk; slot += nwaves) {
        const long long A = a0 + digit_rev(slot, a.k, 1);
        const long long P = (A << shiftB) + bfix;
        const float2* S = a.S + (size_t)P * r_out * r_in;
        const int base = slot * a.rmax * VT * 2;
        float2 sv[4];
        float bv[4];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            if (kk >= nks) break;
            const int s = 4 * kk + g;
            sv[kk] = sv_ok[kk] ? S[tA * r_in + s] : make_float2(0.f, 0.f);
            bv[kk] = tf[base + so[kk]];
        }
        floatx4 ar = {0.f, 0.f, 0.f, 0.f}, ai = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            if (kk >= nks) break;
            ar = mfma4(sv[kk].x, bv[kk], ar);
            ai = mfma4(sv[kk].y, bv[kk], ai);
        }
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const float p = lane_swap1(ai[jj]);
            const float v = reim ? ar[jj] + p : ar[jj] - p;
            const int t = 4 * g + jj;
            if (col < VT && t < r_out) tf[base + (t * VT + col) * 2 + reim] = v;
        }
    }
    __syncthreads();
}

template <int VT>
__global__ void __launch_bounds__(kMfmaThreads) xi_pass_mfma(PassArgs a) {
    extern __shared__ float2 lds[];
    float2* tile = lds;
    float2* twl = lds + (size_t)a.Gk * a.rmax * VT;
    float2* ftile = twl + (size_t)2 * a.Gk * a.rmax;
    long long spatial;
    int chunk;
    block_coords(a, spatial, chunk);
    if (spatial >= a.nspatial) return;
    const long long bg = spatial % a.nbg;
    const long long ap_base = spatial / a.nbg;
    // the f tile is shared by every sub-iteration (the T_X boxes at level
    // l0 - 1 all see the same input); the barrier inside the first level
    // orders these loads before their use
    if (a.has_head) load_head(a, ftile, bg * a.Gk, chunk);
    for (int sub = 0; sub < a.n_sub; ++sub) {
        const long long ap_grp = a.has_head ? sub : ap_base;
        if (!a.has_head) {
            const long long p0 = (ap_grp << (a.L - a.la + 1)) + bg * a.Gk;
            load_tile(a, tile, p0, a.lv[0].r_in, chunk);
        }
        for (int j = 1; j <= a.k; ++j)
            mfma_xi_level<VT>(a, tile, ftile, twl, j, ap_grp, bg);
        if (a.has_switch) mfma_switch<VT>(a, tile, ap_grp * a.Gk, bg);
        store_tile(a, tile, ap_grp * a.Gk, bg, chunk);
        __syncthreads();
    }
}

template <int VT>
__global__ void __launch_bounds__(kMfmaThreads) x_pass_mfma(PassArgs a) {
    extern __shared__ float2 lds[];
    float2* tile = lds;
    float2* twl = lds + (size_t)a.Gk * a.rmax * VT;
    long long spatial;
    int chunk;
    block_coords(a, spatial, chunk);
    if (spatial >= a.nspatial) return;
    const long long ap_grp = a.has_tail ? spatial : spatial / a.nbg;
    const long long bg0 = a.has_tail ? 0 : spatial % a.nbg;
    floatx4 tacc[2 * kWaveTiles];
#pragma unroll
    for (int m = 0; m < 2 * kWaveTiles; ++m) tacc[m] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int sub = 0; sub < a.n_sub; ++sub) {
        const long long bg = a.has_tail ? sub : bg0;
        const long long p0 = (ap_grp << (a.L - a.la + 1)) + bg * a.Gk;
        load_tile(a, tile, p0, a.lv[0].r_in, chunk);
        // (the barrier inside the first level orders the tile loads)
        for (int j = 1; j <= a.k; ++j)
            mfma_x_level<VT>(a, tile, twl, j, ap_grp, bg,
                             a.has_tail && j == a.k, tacc);
        if (!a.has_tail) store_tile(a, tile, ap_grp * a.Gk, bg, chunk);
        __syncthreads();
    }
    if (!a.has_tail) return;
    // final coefficients of the Gk boxes A to LDS as [a_loc][t][VT], then
    // g_v(x) = sum_k a_k(x) lambda_k(x) (eq. (eqn:tg))
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
        for (int m = 0; m < kWaveTiles / 2; ++m) {
            const int tau = wave + m * nwaves;
            if (tau >= ntiles) break;
            const int unit = tau * UPT + sub;
            if (unit >= nunits) continue;
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int aloc = unit * 2 + i;       // last level: unit = apl
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const int t = 4 * g + jj;
                    if (t < r_out)
                        tile[(aloc * a.tail_r + t) * VT + col] =
                            make_float2(tacc[4 * m + 2 * i][jj],
                                        tacc[4 * m + 2 * i + 1][jj]);
                }
            }
        }
    }
    __syncthreads();
    const float2* acc = tile;
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
            const float2 v = acc[(aloc * a.tail_r + t) * VT + vl * a.r_amp + kk];
            if (a.amp_a) {
                const float2 z = cmul(a.amp_a[(size_t)kk * a.N + x], v);
                sum.x += z.x;
                sum.y += z.y;
            } else {
                sum.x += v.x;
                sum.y += v.y;
            }
        }
        a.g[(size_t)(v0 + vl) * a.N + x] = sum;
    }
}

template <int VT>
static std::string launch_vt(const PassArgs& a, bool is_xi, size_t lds,
                             hipStream_t st) {
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void*)xi_pass_mfma<VT>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  160 * 1024);
        (void)hipFuncSetAttribute((const void*)x_pass_mfma<VT>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  160 * 1024);
        attr = true;
    }
    const long long nblocks = a.nspatial * a.nchunk;
    if (is_xi)
        hipLaunchKernelGGL(xi_pass_mfma<VT>, dim3((unsigned)nblocks),
                           dim3(kMfmaThreads), lds, st, a);
    else
        hipLaunchKernelGGL(x_pass_mfma<VT>, dim3((unsigned)nblocks),
                           dim3(kMfmaThreads), lds, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return std::string("MFMA pass launch: ") + hipGetErrorString(e);
    return "";
}

std::string launch_mfma_pass(const PassArgs& a, bool is_xi, size_t lds,
                             hipStream_t st) {
    switch (a.Vt) {
        case 1: return launch_vt<1>(a, is_xi, lds, st);
        case 2: return launch_vt<2>(a, is_xi, lds, st);
        case 4: return launch_vt<4>(a, is_xi, lds, st);
        case 8: return launch_vt<8>(a, is_xi, lds, st);
        default: return "MFMA pass: tile width must be 1, 2, 4 or 8";
    }
}

}  // namespace bfi
