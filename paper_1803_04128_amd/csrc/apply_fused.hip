// Level-fused passes of the regrouped butterfly apply (FP32).
//
// A pass runs k consecutive levels of one kind (recursion in xi, eq. (eqn:2),
// or recursion in x, eq. (eqn:3)) on a tile of R^k pairs held in LDS:
//   - the R^k input pairs (a', b' = bg R^k + m), m < R^k, at level la-1 depend
//     only on each other, and after k levels they have become the R^k pairs
//     (a' R^k + m, bg) at level la+k-1 (the butterfly "radix-R^k group");
//   - levels run in place: the logical pair (a, b) of local level j sits in
//     slot b R^j + rev_j(a), rev_j the base-R digit reversal over j digits,
//     so a unit's R outputs overwrite exactly its R inputs.
// The first xi pass folds the exact copy levels (it reads f, scaled by b_k)
// and loops over the R^(l0-1) T_X boxes that share the same input; the xi
// half ends with the switch on the tile.  The last x pass loops over the
// R^(L-lend) boxes B of the exact sum levels and accumulates their final
// coefficients in LDS, then writes g = sum_k a_k (sum_B lambda) (eq. (eqn:tg)
// and Algorithm 4.1 steps 5-6).
//
// State between passes: complex64 [column chunk][pair][t][Vt], Vt columns
// per tile, so a tile's pairs are one contiguous block.
#include <algorithm>
#include <cstdlib>

#include "fused_common.h"

namespace bfi {

template <int R, int TB, int MAXIT>
__device__ __forceinline__ void tile_xi_level(const PassArgs& a, float2* tile,
                              const float2* ftile, int j, long long ap_grp,
                              long long bg) {
    const PassLevel& lv = a.lv[j - 1];
    const int dim = a.dim;
    const int kj = a.k - j;                       // digits of b_loc
    const int nunits = a.Gk / R;
    const int ntb = (lv.r_out + TB - 1) / TB;
    const int items = nunits * R * ntb * a.Vt;
    const int level = a.la + j - 1;
    const int shiftB = dim * (a.L - level);
    const bool from_f = a.has_head && j == 1;
    float2 keep[MAXIT][TB];
#pragma unroll
    for (int it = 0; it < MAXIT; ++it) {
        const int item = it * kPassThreads + threadIdx.x;
        if (item >= items) break;
        const int col = item % a.Vt;
        int rest = item / a.Vt;
        const int tb = rest % ntb;
        rest /= ntb;
        const int i = rest % R;
        const int unit = rest / R;
        const int apl = unit >> (dim * kj), bl = unit & ((1 << (dim * kj)) - 1);
        const long long apg = (ap_grp << (dim * (j - 1))) + apl;
        const long long bgl = (bg << (dim * kj)) + bl;
        const long long u = (apg << shiftB) + bgl;
        const float2* tw = lv.tw + (u * R + i) * R * lv.r_in;
        const int rv = digit_rev(apl, j - 1, dim);
#pragma unroll
        for (int t = 0; t < TB; ++t) keep[it][t] = make_float2(0.f, 0.f);
        for (int c = 0; c < R; ++c) {
            const int slot_in = ((bl * R + c) << (dim * (j - 1))) + rv;
            const float* m = lv.mats + (size_t)c * lv.r_out * lv.r_in +
                             (size_t)tb * TB * lv.r_in;
            for (int s = 0; s < lv.r_in; ++s) {
                const float2 x =
                    from_f ? ftile[(slot_in * a.head_r + s) * a.Vt + col]
                           : tile[(slot_in * a.rmax + s) * a.Vt + col];
                const float2 z = cmul(tw[c * lv.r_in + s], x);
#pragma unroll
                for (int t = 0; t < TB; ++t) {
                    if (tb * TB + t < lv.r_out) {
                        const float w = m[t * lv.r_in + s];
                        keep[it][t].x += w * z.x;
                        keep[it][t].y += w * z.y;
                    }
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < MAXIT; ++it) {
        const int item = it * kPassThreads + threadIdx.x;
        if (item >= items) break;
        const int col = item % a.Vt;
        int rest = item / a.Vt;
        const int tb = rest % ntb;
        rest /= ntb;
        const int i = rest % R;
        const int unit = rest / R;
        const int apl = unit >> (dim * kj), bl = unit & ((1 << (dim * kj)) - 1);
        const int slot_out = ((bl * R + i) << (dim * (j - 1))) +
                             digit_rev(apl, j - 1, dim);
#pragma unroll
        for (int t = 0; t < TB; ++t) {
            const int tt = tb * TB + t;
            if (tt < lv.r_out) tile[(slot_out * a.rmax + tt) * a.Vt + col] = keep[it][t];
        }
    }
    __syncthreads();
}

// One x level on the tile.  Items are (output child i, unit, t block,
// column), i slowest.
template <int R, int TB, int MAXIT>
__device__ __forceinline__ void tile_x_level(const PassArgs& a, float2* tile, int j,
                             long long ap_grp, long long bg) {
    const PassLevel& lv = a.lv[j - 1];
    const int dim = a.dim;
    const int kj = a.k - j;
    const int nunits = a.Gk / R;
    const int ntb = (lv.r_out + TB - 1) / TB;
    const int items = nunits * R * ntb * a.Vt;
    const int level = a.la + j - 1;
    const int shiftB = dim * (a.L - level);
    float2 keep[MAXIT][TB];
#pragma unroll
    for (int it = 0; it < MAXIT; ++it) {
        const int item = it * kPassThreads + threadIdx.x;
        if (item >= items) break;
        const int col = item % a.Vt;
        int rest = item / a.Vt;
        const int tb = rest % ntb;
        rest /= ntb;
        const int unit = rest % nunits;
        const int i = rest / nunits;
        const int apl = unit >> (dim * kj), bl = unit & ((1 << (dim * kj)) - 1);
        const long long apg = (ap_grp << (dim * (j - 1))) + apl;
        const long long bgl = (bg << (dim * kj)) + bl;
        const long long u = (apg << shiftB) + bgl;
        const int rv = digit_rev(apl, j - 1, dim);
        const float* m = lv.mats + (size_t)i * lv.r_out * lv.r_in +
                         (size_t)tb * TB * lv.r_in;
#pragma unroll
        for (int t = 0; t < TB; ++t) keep[it][t] = make_float2(0.f, 0.f);
        for (int c = 0; c < R; ++c) {
            const int slot_in = ((bl * R + c) << (dim * (j - 1))) + rv;
            float2 y[TB];
#pragma unroll
            for (int t = 0; t < TB; ++t) y[t] = make_float2(0.f, 0.f);
            for (int s = 0; s < lv.r_in; ++s) {
                const float2 x = tile[(slot_in * a.rmax + s) * a.Vt + col];
#pragma unroll
                for (int t = 0; t < TB; ++t) {
                    if (tb * TB + t < lv.r_out) {
                        const float w = m[t * lv.r_in + s];
                        y[t].x += w * x.x;
                        y[t].y += w * x.y;
                    }
                }
            }
            const float2* tw = lv.tw + ((u * R + i) * R + c) * lv.r_out + tb * TB;
#pragma unroll
            for (int t = 0; t < TB; ++t) {
                if (tb * TB + t < lv.r_out) {
                    const float2 z = cmul(tw[t], y[t]);
                    keep[it][t].x += z.x;
                    keep[it][t].y += z.y;
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < MAXIT; ++it) {
        const int item = it * kPassThreads + threadIdx.x;
        if (item >= items) break;
        const int col = item % a.Vt;
        int rest = item / a.Vt;
        const int tb = rest % ntb;
        rest /= ntb;
        const int unit = rest % nunits;
        const int i = rest / nunits;
        const int apl = unit >> (dim * kj), bl = unit & ((1 << (dim * kj)) - 1);
        const int slot_out = ((bl * R + i) << (dim * (j - 1))) +
                             digit_rev(apl, j - 1, dim);
#pragma unroll
        for (int t = 0; t < TB; ++t) {
            const int tt = tb * TB + t;
            if (tt < lv.r_out) tile[(slot_out * a.rmax + tt) * a.Vt + col] = keep[it][t];
        }
    }
    __syncthreads();
}

// Copy the tile's Gk pairs (slot m = logical a_loc digit-reversed) to the
// state at the pass's last level: pair (a0 + a_loc) R^(L-lb) + bfix.
template <int R, int TB, int MAXIT>
__global__ void __launch_bounds__(kPassThreads) xi_pass(PassArgs a) {
    extern __shared__ float2 lds[];
    float2* tile = lds;
    float2* ftile = lds + (size_t)a.Gk * a.rmax * a.Vt;
    long long spatial;
    int chunk;
    block_coords(a, spatial, chunk);
    if (spatial >= a.nspatial) return;
    const int part = (int)(spatial % a.sub_split);
    spatial /= a.sub_split;
    const long long bg = spatial % a.nbg;
    const long long ap_base = spatial / a.nbg;
    if (a.has_head) {
        load_head(a, ftile, bg * a.Gk, chunk);
        __syncthreads();
    }
    for (int si = 0; si < a.n_sub; ++si) {
        const int sub = part * a.n_sub + si;
        const long long ap_grp = a.has_head ? sub : ap_base;
        if (!a.has_head) {
            const long long p0 = (ap_grp << (a.dim * (a.L - a.la + 1))) +
                                 bg * a.Gk;
            load_tile(a, tile, p0, a.lv[0].r_in, chunk);
            __syncthreads();
        }
        for (int j = 1; j <= a.k; ++j)
            tile_xi_level<R, TB, MAXIT>(a, tile, ftile, j, ap_grp, bg);
        if (a.has_switch)
            tile_switch<TB, MAXIT>(a, tile, ap_grp * a.Gk, bg, a.k, tile,
                                   a.rmax);
        store_tile(a, tile, ap_grp * a.Gk, bg, chunk);
        __syncthreads();
    }
}

template <int R, int TB, int MAXIT>
__global__ void __launch_bounds__(kPassThreads) x_pass(PassArgs a) {
    extern __shared__ float2 lds[];
    float2* tile = lds;
    float2* extra = lds + (size_t)a.Gk * a.rmax * a.Vt;   // head or tail
    long long spatial;
    int chunk;
    block_coords(a, spatial, chunk);
    if (spatial >= a.nspatial) return;
    const long long ap_grp = a.has_tail ? spatial : spatial / a.nbg;
    const long long bg0 = a.has_tail ? 0 : spatial % a.nbg;
    if (a.has_tail) {
        for (int e = threadIdx.x; e < a.Gk * a.tail_r * a.Vt; e += blockDim.x)
            extra[e] = make_float2(0.f, 0.f);
    }
    for (int sub = 0; sub < a.n_sub; ++sub) {
        const long long bg = a.has_tail ? sub : bg0;
        if (a.has_head) {
            // no xi level: lambda^{AB} = f restricted to B at level L-h, then
            // the switch in place (pairs a' = ap_grp, b = bg Gk + m)
            float2* hf = extra + (a.has_tail ? (size_t)a.Gk * a.tail_r * a.Vt : 0);
            load_head(a, hf, bg * a.Gk, chunk);
            __syncthreads();
            // slots hold pairs (ap_grp, bg Gk + m): A fixed, B varies
            {
                const int TBs = TB;
                const int nt = (a.sw_r_out + TBs - 1) / TBs;
                const int items = a.Gk * nt * a.Vt;
                const int shiftB = a.dim * (a.L - (a.la - 1));
                for (int item = threadIdx.x; item < items; item += blockDim.x) {
                    const int col = item % a.Vt;
                    const int rest = item / a.Vt;
                    const int tb = rest % nt;
                    const int m = rest / nt;
                    const long long P = (ap_grp << shiftB) + bg * a.Gk + m;
                    const float2* S = a.S + (size_t)P * a.sw_r_out * a.sw_r_in;
                    float2 acc[TB];
#pragma unroll
                    for (int t = 0; t < TB; ++t) acc[t] = make_float2(0.f, 0.f);
                    for (int s = 0; s < a.sw_r_in; ++s) {
                        const float2 x = hf[(m * a.head_r + s) * a.Vt + col];
#pragma unroll
                        for (int t = 0; t < TB; ++t) {
                            const int tt = tb * TB + t;
                            if (tt < a.sw_r_out) {
                                const float2 z = cmul(S[tt * a.sw_r_in + s], x);
                                acc[t].x += z.x;
                                acc[t].y += z.y;
                            }
                        }
                    }
#pragma unroll
                    for (int t = 0; t < TB; ++t) {
                        const int tt = tb * TB + t;
                        if (tt < a.sw_r_out) tile[(m * a.rmax + tt) * a.Vt + col] = acc[t];
                    }
                }
            }
            __syncthreads();
        } else {
            const long long p0 = (ap_grp << (a.dim * (a.L - a.la + 1))) +
                                 bg * a.Gk;
            const int r_in = a.k > 0 ? a.lv[0].r_in : a.tail_r;
            load_tile(a, tile, p0, r_in, chunk);
            __syncthreads();
        }
        for (int j = 1; j <= a.k; ++j)
            tile_x_level<R, TB, MAXIT>(a, tile, j, ap_grp, bg);
        if (a.has_tail) {
            // lambda of the pairs (A = ap_grp Gk + a_loc, bg): accumulate
            const int total = a.Gk * a.tail_r * a.Vt;
            for (int e = threadIdx.x; e < total; e += blockDim.x) {
                const int col = e % a.Vt;
                const int rest = e / a.Vt;
                const int t = rest % a.tail_r;
                const int aloc = rest / a.tail_r;
                const int slot = digit_rev(aloc, a.k, a.dim);
                const float2 v = tile[(slot * a.rmax + t) * a.Vt + col];
                extra[e].x += v.x;
                extra[e].y += v.y;
            }
        } else {
            store_tile(a, tile, ap_grp * a.Gk, bg, chunk);
        }
        __syncthreads();
    }
    if (a.has_tail) {
        // g_v(x) = sum_k a_k(x) acc_k(x) for the points of the Gk boxes A
        const int tv = a.Vt / a.r_amp;
        const int total = a.Gk * a.tail_r * tv;
        const int v0 = chunk * tv;
        const int nvs = a.Vs / a.r_amp;
        for (int e = threadIdx.x; e < total; e += blockDim.x) {
            const int t = e % a.tail_r;
            const int rest = e / a.tail_r;
            const int aloc = rest % a.Gk;
            const int vl = rest / a.Gk;
            if (v0 + vl >= nvs) continue;
            int Ac[2], gi[2];
            box_coords(ap_grp * a.Gk + aloc, a.dim, Ac);
            if (a.dim == 1) {
                gi[0] = Ac[0] * a.tail_side + t;
            } else {
                gi[0] = Ac[0] * a.tail_side + t / a.tail_side;
                gi[1] = Ac[1] * a.tail_side + t % a.tail_side;
            }
            const long long x = user_index(gi, a.dim, a.n);
            float2 sum = make_float2(0.f, 0.f);
            for (int kk = 0; kk < a.r_amp; ++kk) {
                const float2 v = extra[(aloc * a.tail_r + t) * a.Vt +
                                       vl * a.r_amp + kk];
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
}

// ----------------------------------------------------------- host planning

constexpr size_t kLdsBudget = 96 * 1024;
constexpr size_t kMfmaLdsBudget = 150 * 1024;

struct Tiling {
    int TB, MAXIT;
};

static Tiling tiling_for(int dim) { return dim == 1 ? Tiling{16, 2} : Tiling{32, 2}; }

static bool pow2_le8(int v) { return v == 1 || v == 2 || v == 4 || v == 8; }

static int count_kind(const Plan& p, int kind) {
    int c = 0;
    for (const auto& s : p.steps) c += s.kind == kind;
    return c;
}

// MFMA passes serve 1D plans whose tile width is a power of two <= 8
// (a plan configured without MFMA uses the vector-ALU passes).
static bool mfma_mode(const Plan& p, int Vt) {
    return p.mfma && p.dim == 1 && pow2_le8(Vt) && pow2_le8(p.r_amp);
}

// Levels of the next pass when the n levels left of a half are split into
// equal passes of at most d levels (d = 0: one pass); a single level is never
// left over for a pass of its own (the pass before takes it).
static int split_levels(int n, int d) {
    if (d <= 0 || n <= d) return n;
    const int parts = (n + d - 1) / d;
    const int take = (n + parts - 1) / parts;
    return n - take == 1 ? n : take;
}

// Columns per tile: a multiple of the amplitude rank (the final sums
// recombine the r terms of a vector inside one workgroup), about 8.  For the
// MFMA passes the width is a power of two, lowered (not below r) until the
// larger half's passes fit (Gk * Vt <= 512; one pass per half unless the
// fusion depth is capped).
int fused_tile_cols(const Plan& p, int Vs) {
    // a configured width (a multiple of r) replaces the default of about 8
    int tv = std::max(1, 8 / p.r_amp);
    if (p.tile_cols >= p.r_amp) tv = p.tile_cols / p.r_amp;
    int vt = std::min(tv * p.r_amp, Vs);
    if (p.dim == 1 && pow2_le8(p.r_amp)) {
        int v2 = 1;
        while (v2 * 2 <= vt) v2 *= 2;
        vt = v2;
        const int m = split_levels(
            std::max(count_kind(p, STEP_XI), count_kind(p, STEP_X)),
            p.max_pass_levels);
        while (vt > p.r_amp && (1LL << m) * vt > 512) vt /= 2;
    }
    return vt;
}

static int rank_max(const Plan& p, int s0, int s1) {
    int r = 1;
    for (int k = s0; k <= s1; ++k)
        r = std::max(r, std::max(p.steps[k].r_in, p.steps[k].r_out));
    return r;
}

static bool pass_fits(const Plan& p, int s0, int s1, int Vt, bool head,
                      bool tail) {
    const int k = s1 - s0 + 1;
    const Tiling tl = tiling_for(p.dim);
    const long long Gk = 1LL << (p.dim * k);
    // a xi pass that ends the xi half also carries the switch
    if (p.steps[s1].kind == STEP_XI && s1 + 1 < (int)p.steps.size() &&
        p.steps[s1 + 1].kind == STEP_SWITCH)
        ++s1;
    const int rmax = rank_max(p, s0, s1);
    if (k > kMaxPassLevels) return false;
    if (mfma_mode(p, Vt) && p.steps[s0].kind != STEP_SWITCH) {
        const int hr1 = p.head_step_side;
        // the tile (updated in place), two twiddle buffers, the f tile of
        // the head pass and, in an FP32 x pass, every level's A operand
        const bool x_amat =
            p.steps[s0].kind == STEP_X && p.precision == BF_FP32;
        const size_t lds = (size_t)Gk * rmax * Vt * 8 + (size_t)4 * Gk * rmax * 8 +
                           (head ? (size_t)Gk * hr1 * Vt * 8 : 0) + kMfmaLdsPad * 8 +
                           (x_amat ? (size_t)k * 256 * 8 : 0);
        return lds <= kMfmaLdsBudget && Gk * Vt <= (long long)kMfmaTileCap * 8;
    }
    size_t lds = (size_t)Gk * rmax * Vt * 8;
    const int hr = p.head_step_side == 1 ? 1 :
                   (p.dim == 1 ? p.head_step_side
                               : p.head_step_side * p.head_step_side);
    const int tr = p.dim == 1 ? p.tail_side : p.tail_side * p.tail_side;
    if (head) lds += (size_t)Gk * hr * Vt * 8;
    if (tail) lds += (size_t)Gk * tr * Vt * 8;
    if (lds > kLdsBudget) return false;
    for (int q = s0; q <= s1; ++q) {
        const int ntb = (p.steps[q].r_out + tl.TB - 1) / tl.TB;
        if (Gk * ntb * Vt > (long long)kPassThreads * tl.MAXIT) return false;
    }
    return true;
}

// Split the computed steps into passes.  Step indices: xi levels occupy
// [0, nxi), the switch is nxi, x levels (nxi, nsteps).
std::vector<Pass> plan_passes(const Plan& p, int Vt) {
    std::vector<Pass> out;
    const int nsteps = (int)p.steps.size();
    int nxi = 0;
    while (nxi < nsteps && p.steps[nxi].kind == STEP_XI) ++nxi;
    const int sw = nxi;
    // xi half: passes over [0, nxi) ; the switch rides on the last one.
    // With a fusion-depth cap the remaining levels are split into equal
    // passes of at most that many; every pass is then shortened until it
    // fits.
    if (nxi > 0) {
        int s0 = 0;
        while (s0 < nxi) {
            int s1 = s0 + split_levels(nxi - s0, p.max_pass_levels) - 1;
            while (s1 > s0 && !pass_fits(p, s0, s1, Vt, s0 == 0, false)) --s1;
            Pass ps{};
            ps.first = s0;
            ps.last = s1;
            ps.tail = false;
            out.push_back(ps);
            s0 = s1 + 1;
        }
    }
    // x half: passes over (sw, nsteps); the last one has the tail; with no
    // xi level the first x pass starts with the switch on f.
    int s0 = sw + 1;
    if (s0 >= nsteps) {
        Pass ps{};
        ps.first = nxi > 0 ? nsteps : sw;   // empty x pass (tail only)
        ps.last = nxi > 0 ? nsteps - 1 : sw;
        ps.tail = true;
        out.push_back(ps);
        return out;
    }
    bool first_x = true;
    while (s0 < nsteps) {
        int s1 = s0 + split_levels(nsteps - s0, p.max_pass_levels) - 1;
        while (s1 > s0 &&
               !pass_fits(p, s0, s1, Vt, first_x && nxi == 0, s1 == nsteps - 1))
            --s1;
        Pass ps{};
        ps.first = (first_x && nxi == 0) ? sw : s0;
        ps.last = s1;
        ps.tail = (s1 == nsteps - 1);
        out.push_back(ps);
        s0 = s1 + 1;
        first_x = false;
    }
    return out;
}

int fused_pass_count(const Plan& p, int Vs) {
    return (int)plan_passes(p, fused_tile_cols(p, Vs)).size();
}

size_t fused_state_bytes(const Plan& p, int Vs) {
    const int Vt = fused_tile_cols(p, Vs);
    const int nchunk = (Vs + Vt - 1) / Vt;
    return (size_t)p.N * p.max_rank * (size_t)nchunk * Vt * sizeof(float2);
}

void init_mfma_attrs();

template <int R, int TB, int MAXIT>
static void set_lds_limit() {
    static bool done = false;
    if (done) return;
    (void)hipFuncSetAttribute((const void*)xi_pass<R, TB, MAXIT>,
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
    (void)hipFuncSetAttribute((const void*)x_pass<R, TB, MAXIT>,
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
    done = true;
}

// Raise the dynamic LDS limit of every pass kernel once, before any launch
// (so that a graph capture records launches only).
void init_kernel_attrs() {
    set_lds_limit<2, 16, 2>();
    set_lds_limit<4, 32, 2>();
    init_mfma_attrs();
    init_step_split_attrs();
    init_step_sep_attrs();
}

// dry: check every pass of the configuration (LDS, tile caps, grid) and
// launch nothing.
std::string run_fused(Plan& p, int nv, const float2* f, float2* g,
                      float2* buf0, float2* buf1, hipStream_t st, bool dry) {
    const int Vs = nv * p.r_amp;
    const int Vt = fused_tile_cols(p, Vs);
    const int nchunk = (Vs + Vt - 1) / Vt;
    const std::vector<Pass> passes = plan_passes(p, Vt);
    const int nsteps = (int)p.steps.size();
    int nxi = 0;
    while (nxi < nsteps && p.steps[nxi].kind == STEP_XI) ++nxi;
    const Step& swst = p.steps[nxi];
    const int hr = p.dim == 1 ? p.head_step_side
                              : p.head_step_side * p.head_step_side;
    const int tr = p.dim == 1 ? p.tail_side : p.tail_side * p.tail_side;
    const float2* cur = nullptr;
    float2* bufs[2] = {buf0, buf1};
    int which = 0;
    const double N = (double)p.N;
    for (size_t pi = 0; pi < passes.size(); ++pi) {
        const Pass& ps = passes[pi];
        PassArgs a{};
        const bool is_xi = ps.first < nxi;
        // levels of the pass (the switch is not a level)
        int k = 0;
        double flops = 0, fbytes = 0;
        int rmax = 1;
        for (int q = ps.first; q <= ps.last && q < nsteps; ++q) {
            const Step& s = p.steps[q];
            rmax = std::max(rmax, std::max(s.r_in, s.r_out));
            if (s.kind == STEP_SWITCH) continue;
            a.lv[k].tw = s.tw;
            a.lv[k].mats = s.mats;
            a.lv[k].amat = s.kind == STEP_XI ? s.amat_xi : s.amat;
            a.lv[k].ahi = s.asplit_hi;
            a.lv[k].alo = s.asplit_lo;
            a.lv[k].r_in = s.r_in;
            a.lv[k].r_out = s.r_out;
            a.lv[k].level = s.level;
            ++k;
            fbytes += s.tw_elems * 8.0 + s.mat_elems * 4.0;
            flops += step_alg_flops(p, s, Vs);
        }
        a.k = k;
        a.prec = p.precision;
        a.Gk = 1 << (p.dim * k);
        a.L = p.L;
        a.n = p.n;
        a.dim = p.dim;
        a.N = p.N;
        a.Vs = Vs;
        a.Vt = Vt;
        a.nchunk = nchunk;
        a.r_amp = p.r_amp;
        a.in = cur;
        a.out = bufs[which];
        a.f = f;
        a.bamp = p.has_amp ? p.b_dev : nullptr;
        a.head_side = p.head_step_side;
        a.head_r = hr;
        a.S = swst.S;
        a.sw_r_in = swst.r_in;
        a.sw_r_out = swst.r_out;
        a.g = g;
        a.amp_a = p.has_amp ? p.a_dev : nullptr;
        a.tail_side = p.tail_side;
        a.tail_r = tr;
        double in_bytes = 0, out_bytes = 0, state_bytes = 0;
        size_t lds = 0;
        if (is_xi) {
            a.la = p.steps[ps.first].level;
            a.has_head = ps.first == 0;
            a.has_switch = ps.last == nxi - 1;
            a.rmax = std::max(rmax, a.has_switch ? std::max(swst.r_in, swst.r_out) : 1);
            a.r_state_out = a.has_switch ? swst.r_out : p.steps[ps.last].r_out;
            a.nbg = 1LL << (p.dim * (p.L - a.la + 1 - k));
            if (a.has_head) {
                a.nspatial = a.nbg;
                a.n_sub = 1 << (p.dim * (a.la - 1));
            } else {
                a.nspatial = (1LL << (p.dim * (a.la - 1))) * a.nbg;
                a.n_sub = 1;
            }
            lds = (size_t)a.Gk * a.rmax * Vt * 8 +
                  (a.has_head ? (size_t)a.Gk * hr * Vt * 8 : 0);
            in_bytes = a.has_head ? N * nv * 8.0 + (p.has_amp ? N * p.r_amp * 8.0 : 0)
                                  : 0.0;
            state_bytes = (a.has_head ? 0.0 : N * a.lv[0].r_in * Vs * 8.0) +
                          N * a.r_state_out * Vs * 8.0;
            if (a.has_switch) {
                fbytes += swst.S_elems * 8.0;
                flops += N * Vs * swst.r_out * (double)swst.r_in * 8.0;
            }
        } else {
            const bool head_sw = ps.first == nxi && nxi == 0;   // switch on f
            a.la = k > 0 ? a.lv[0].level : p.h + 1;
            a.has_head = head_sw;
            a.has_switch = head_sw;
            a.has_tail = ps.tail;
            a.rmax = std::max(rmax, std::max(tr, head_sw ? swst.r_out : 1));
            a.r_state_out = k > 0 ? a.lv[k - 1].r_out : tr;
            a.nbg = 1LL << (p.dim * (p.L - a.la + 1 - k));
            if (a.has_tail) {
                a.nspatial = 1LL << (p.dim * (a.la - 1));
                a.n_sub = (int)a.nbg;
            } else {
                a.nspatial = (1LL << (p.dim * (a.la - 1))) * a.nbg;
                a.n_sub = 1;
            }
            lds = (size_t)a.Gk * a.rmax * Vt * 8 +
                  (a.has_tail ? (size_t)a.Gk * tr * Vt * 8 : 0) +
                  (head_sw ? (size_t)a.Gk * hr * Vt * 8 : 0);
            in_bytes = head_sw ? N * nv * 8.0 + (p.has_amp ? N * p.r_amp * 8.0 : 0)
                               : 0.0;
            out_bytes = a.has_tail ? N * nv * 8.0 + (p.has_amp ? N * p.r_amp * 8.0 : 0)
                                   : 0.0;
            state_bytes = (head_sw ? 0.0
                                   : N * (k > 0 ? a.lv[0].r_in : swst.r_out) *
                                         Vs * 8.0) +
                          (a.has_tail ? 0.0 : N * a.r_state_out * Vs * 8.0);
            if (head_sw) {
                fbytes += swst.S_elems * 8.0;
                flops += N * Vs * swst.r_out * (double)swst.r_in * 8.0;
            }
            if (a.has_tail)
                flops += N * Vs * (double)(1LL << (p.dim * (p.L - p.lend))) * 2.0 +
                         N * nv * p.r_amp * 8.0;
        }
        // a head pass with few workgroups spreads its sub-iterations over
        // more of them (each reloads the f tile) to fill the chip
        a.sub_split = 1;
        if (is_xi && a.has_head)
            while (a.sub_split < a.n_sub &&
                   a.nspatial * nchunk * a.sub_split < 512)
                a.sub_split *= 2;
        a.n_sub /= a.sub_split;
        a.nspatial *= a.sub_split;
        // a tail pass with few A groups splits its B groups over more
        // workgroups; the split depends on the plan only (not on the batch
        // size), so the summation order is the same for every batch, and
        // the partial outputs fit the state buffer this pass does not use
        a.x_split = 1;
        a.gpart = bufs[which];
        if (!is_xi && a.has_tail && mfma_mode(p, Vt) && k > 0 && !a.has_head &&
            (long long)a.Gk * Vt <= (long long)kMfmaTileCap * 8)   // MFMA pass
            while (a.x_split < a.n_sub && a.nspatial * a.x_split < 256 &&
                   2 * a.x_split <= p.max_rank * p.r_amp)
                a.x_split *= 2;
        a.n_sub /= a.x_split;
        a.nspatial *= a.x_split;
        a.xcd_map = (a.nspatial % 8 == 0) ? 1 : 0;
        if (lds > 160 * 1024) return "fused pass does not fit in LDS";
        {
            // every level (and the switch) must fit the per-thread item cap
            const Tiling tl = tiling_for(p.dim);
            const long long cap = (long long)kPassThreads * tl.MAXIT;
            for (int q = 0; q < k; ++q) {
                const int ntb = (a.lv[q].r_out + tl.TB - 1) / tl.TB;
                if ((long long)a.Gk * ntb * Vt > cap) return "fused tile too large";
            }
            const int ntbs = (swst.r_out + tl.TB - 1) / tl.TB;
            if (a.has_switch && (long long)a.Gk * ntbs * Vt > cap)
                return "fused tile too large for the switch";
        }
        const long long nblocks = a.nspatial * nchunk;
        if (nblocks > 0x7fffffffLL) return "fused pass grid too large";
        const bool use_mfma =
            mfma_mode(p, Vt) && (is_xi || (k > 0 && !a.has_head)) &&
            (long long)a.Gk * Vt <= (long long)kMfmaTileCap * 8;
        // the split precisions exist only on the MFMA passes; never compute
        // a requested BF16/FP16 apply in FP32 silently
        if (p.precision != BF_FP32 && !use_mfma)
            return "split precision needs the 1D MFMA passes (power-of-two "
                   "tile width, r in {1, 2, 4, 8}, a level in every pass)";
        // a head xi pass whose own f tile keeps it at one workgroup per CU
        // writes the head into the state tile at every sub-iteration
        // instead (from registers in FP32, else gathered again) when that
        // lets two workgroups of 512 threads share a CU; they then overlap
        // each other's factor reads and barriers
        // (with one twiddle buffer where two do not fit twice)
        a.head_inplace = 0;
        a.tw_single = 0;
        if (use_mfma && is_xi && a.has_head && a.head_r <= a.rmax) {
            const size_t keep = mfma_pass_lds(a, true);
            a.head_inplace = 1;
            const size_t in = mfma_pass_lds(a, true);
            a.tw_single = 1;
            const size_t in1 = mfma_pass_lds(a, true);
            const bool want = 2 * keep > 160 * 1024 && nblocks >= 512;
            a.head_inplace = want && 2 * in1 <= 160 * 1024 ? 1 : 0;
            a.tw_single = a.head_inplace && 2 * in > 160 * 1024 ? 1 : 0;
        }
        if (use_mfma) {
            lds = mfma_pass_lds(a, is_xi);
            if (lds > 160 * 1024) return "MFMA pass does not fit in LDS";
        }
        if (dry) continue;
        ProfScope prof(p, st);
        const char* name;
        if (use_mfma) {
            std::string err = launch_mfma_pass(a, is_xi, lds, st);
            if (!err.empty()) return err;
            name = is_xi ? "xi_pass_mfma" : "x_pass_mfma";
        } else if (p.dim == 1) {
            set_lds_limit<2, 16, 2>();
            if (is_xi)
                hipLaunchKernelGGL((xi_pass<2, 16, 2>), dim3((unsigned)nblocks),
                                   dim3(kPassThreads), lds, st, a);
            else
                hipLaunchKernelGGL((x_pass<2, 16, 2>), dim3((unsigned)nblocks),
                                   dim3(kPassThreads), lds, st, a);
            name = is_xi ? "xi_pass<2>" : "x_pass<2>";
        } else {
            set_lds_limit<4, 32, 2>();
            if (is_xi)
                hipLaunchKernelGGL((xi_pass<4, 32, 2>), dim3((unsigned)nblocks),
                                   dim3(kPassThreads), lds, st, a);
            else
                hipLaunchKernelGGL((x_pass<4, 32, 2>), dim3((unsigned)nblocks),
                                   dim3(kPassThreads), lds, st, a);
            name = is_xi ? "xi_pass<4>" : "x_pass<4>";
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return std::string("fused pass launch: ") + hipGetErrorString(e);
        if (a.x_split > 1 && a.has_tail) {
            // the tail pass writes x_split partial sums, summed into g below
            out_bytes = 0.0;
            state_bytes += a.x_split * (double)nv * N * 8.0;
        }
        prof.end(name, in_bytes + out_bytes + fbytes, flops, state_bytes);
        if (a.x_split > 1) {
            ProfScope ps2(p, st);
            std::string err = launch_sum_parts(a, nv, st);
            if (!err.empty()) return err;
            ps2.end("sum_parts", nv * N * 8.0,
                    (double)(a.x_split - 1) * nv * N * 2.0,
                    a.x_split * (double)nv * N * 8.0);
        }
        cur = bufs[which];
        which ^= 1;
    }
    return "";
}

}  // namespace bfi
