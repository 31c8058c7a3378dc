// Shared pieces of the level-fused passes: launch arguments, block ->
// (spatial group, column chunk) mapping, and the tile copies between HBM and
// LDS.  Copy loops step through their index spaces incrementally (no integer
// division per element).
//
// A pass runs k consecutive levels of one kind (recursion in xi, eq. (eqn:2),
// or recursion in x, eq. (eqn:3)) on a tile of R^k pairs held in LDS:
//   - the R^k input pairs (a', b' = bg R^k + m), m < R^k, at level la-1 depend
//     only on each other, and after k levels they have become the R^k pairs
//     (a' R^k + m, bg) at level la+k-1 (a radix-R^k butterfly group);
//   - levels run in place: the logical pair (a, b) of local level j sits in
//     slot b R^j + rev_j(a), rev_j the base-R digit reversal over j digits,
//     so a unit's R outputs overwrite exactly its R inputs.
// State between passes: complex64 [column chunk][pair][t][Vt], Vt columns
// per tile, so a tile's pairs are one contiguous block.
#pragma once

#include "apply_common.h"

namespace bfi {

constexpr int kMaxPassLevels = 12;
constexpr int kPassThreads = 256;
// MFMA tiles (16 panel columns each) a workgroup holds per level
constexpr int kMfmaTileCap = 64;
constexpr int kMfmaLdsPad = 128;  // zeroed float2 entries after an MFMA pass's LDS

struct PassLevel {
    const float2* tw;
    const float* mats;
    const float* amat;         // mats in the MFMA A order of the level
                               // (Step::amat_xi for xi levels, Step::amat
                               // for x levels)
    const uint16_t* ahi;       // 16-bit hi/lo A parts (split precisions,
    const uint16_t* alo;       // Step::asplit_hi / asplit_lo)
    int r_in, r_out, level;
};

struct PassArgs {
    PassLevel lv[kMaxPassLevels];
    int k, Gk, la, L, n, dim;
    int prec;                 // BF_FP32, BF_BF16X3 or BF_FP16X3
    long long N;
    int Vs, Vt, nchunk, r_amp;
    int rmax;                 // coefficient slots per pair in the tile
    const float2* in;
    float2* out;
    int r_state_out;          // coefficients per pair written out
    // head: the input is f restricted to the input boxes (times b_k)
    int has_head;
    const float2* f;
    const float2* bamp;
    int head_side, head_r;
    int head_inplace;         // xi MFMA passes: 1 = the head is gathered
                              // into the state tile (slot stride rmax) at
                              // every sub-iteration instead of being kept
                              // in a tile of its own for all of them
    int tw_single;            // in-place head xi passes: 1 = one twiddle
                              // buffer (the next level's twiddles written
                              // after a barrier) instead of two
    int n_sub;                // sub-iterations per workgroup
    int x_split;              // tail x passes: workgroups sharing the
                              // sub-iterations (B groups) of one A group;
                              // each writes its partial g to gpart
    float2* gpart;            // [x_split][nv][N] partial outputs
    int sub_split;            // xi head passes: workgroups sharing the
                              // sub-iterations of one spatial group (the
                              // block index carries the part)
    long long nbg;            // groups along T_Omega at the output level
    long long nspatial;
    int xcd_map;              // 1: XCD-aware block -> (spatial, chunk)
    // switch on the tile (end of the xi half, or start of an x pass that
    // reads f because there is no xi level)
    int has_switch;
    const float2* S;
    int sw_r_in, sw_r_out;
    // tail: final sums and amplitude
    int has_tail;
    float2* g;
    const float2* amp_a;
    int tail_side, tail_r;
};

__device__ __forceinline__ int digit_rev(int x, int j, int dim) {
    if (j == 0) return 0;
    if (dim == 1) return (int)(__brev((unsigned)x) >> (32 - j));
    int r = 0;
    for (int q = 0; q < j; ++q) {
        r = (r << dim) | (x & ((1 << dim) - 1));
        x >>= dim;
    }
    return r;
}

__device__ __forceinline__ void block_coords(const PassArgs& a,
                                             long long& spatial, int& chunk) {
    const long long bid = blockIdx.x;
    if (a.xcd_map) {
        // blocks are dealt round-robin to 8 XCDs: keep the column chunks of
        // one spatial group on one XCD, consecutively, so its factors are
        // read from HBM once and then hit that XCD's L2
        const long long xcd = bid & 7, slot = bid >> 3;
        chunk = (int)(slot % a.nchunk);
        spatial = (slot / a.nchunk) * 8 + xcd;
    } else {
        chunk = (int)(bid % a.nchunk);
        spatial = bid / a.nchunk;
    }
}

// Incremental decode of e = hi * n_lo + lo while e advances by blockDim.x.
struct Walk2 {
    int hi, lo, dhi, dlo, n_lo;
    __device__ __forceinline__ Walk2(int e, int n) : n_lo(n) {
        hi = e / n;
        lo = e - hi * n;
        dhi = (int)blockDim.x / n;
        dlo = (int)blockDim.x - dhi * n;
    }
    __device__ __forceinline__ void next() {
        hi += dhi;
        lo += dlo;
        if (lo >= n_lo) {
            lo -= n_lo;
            ++hi;
        }
    }
};

// Head value of input box `box` (side head_side, all of its indices),
// index s within it, panel column gc: b_k(xi) f_v(xi), zero past the
// panel's columns.
__device__ __forceinline__ float2 head_entry(const PassArgs& a, long long box,
                                             int s, int gc) {
    float2 v = make_float2(0.f, 0.f);
    if (gc < a.Vs) {
        int bc[2], gi[2];
        box_coords(box, a.dim, bc);
        if (a.dim == 1) {
            gi[0] = bc[0] * a.head_side + s;
        } else {
            const int s1 = s / a.head_side;
            gi[0] = bc[0] * a.head_side + s1;
            gi[1] = bc[1] * a.head_side + (s - s1 * a.head_side);
        }
        const long long j = user_index(gi, a.dim, a.n);
        const int vl = gc / a.r_amp, kk = gc - vl * a.r_amp;
        const float2 fv = a.f[(size_t)vl * a.N + j];
        v = a.bamp ? cmul(a.bamp[(size_t)kk * a.N + j], fv) : fv;
    }
    return v;
}

// Gather of the head into dst[(m * rs + s) * Vt + col], rs = head_r unless
// given: input box box0 + m and column col of the chunk.
__device__ __forceinline__ void load_head(const PassArgs& a, float2* dst,
                                          long long box0, int chunk,
                                          int rs = 0) {
    // rows head_r..rs-1 of each box are skipped: element e lands at
    // e + m (rs - head_r) Vt
    const int gap = rs > a.head_r ? (rs - a.head_r) * a.Vt : 0;
    const int total = a.Gk * a.head_r * a.Vt;
    const int e0 = threadIdx.x;
    Walk2 rc(e0, a.Vt);                  // (row, col), row = m * head_r + s
    Walk2 ms(rc.hi, a.head_r);           // (m, s)
    // the row advances by rc.dhi or rc.dhi + 1 per step
    const int q0 = rc.dhi / a.head_r, r0 = rc.dhi - q0 * a.head_r;
    const int q1 = (rc.dhi + 1) / a.head_r, r1 = rc.dhi + 1 - q1 * a.head_r;
    for (int e = e0; e < total; e += blockDim.x) {
        const int col = rc.lo, m = ms.hi, s = ms.lo;
        dst[e + m * gap] = head_entry(a, box0 + m, s, chunk * a.Vt + col);
        const int old_row = rc.hi;
        rc.next();
        const bool plus = (rc.hi - old_row) != rc.dhi;
        ms.hi += plus ? q1 : q0;
        ms.lo += plus ? r1 : r0;
        if (ms.lo >= a.head_r) {
            ms.lo -= a.head_r;
            ++ms.hi;
        }
    }
}

// The head gathered once into registers (NR entries per thread, in the
// order of load_head) and written to LDS as often as needed; covers heads
// of at most NR * blockDim entries (fits()).
template <int NR>
struct HeadRegs {
    float2 v[NR];

    __device__ __forceinline__ bool fits(const PassArgs& a) const {
        return a.Gk * a.head_r * a.Vt <= NR * (int)blockDim.x;
    }
    __device__ __forceinline__ void load(const PassArgs& a, long long box0,
                                         int chunk) {
        const int per_box = a.head_r * a.Vt;
        const int total = a.Gk * per_box;
#pragma unroll
        for (int m = 0; m < NR; ++m) {
            const int e = threadIdx.x + m * (int)blockDim.x;
            v[m] = make_float2(0.f, 0.f);
            if (e < total) {
                const int box = e / per_box, rem = e - box * per_box;
                const int s = rem / a.Vt, col = rem - s * a.Vt;
                v[m] = head_entry(a, box0 + box, s, chunk * a.Vt + col);
            }
        }
    }
    __device__ __forceinline__ void store(const PassArgs& a, float2* dst,
                                          int rs) const {
        const int per_box = a.head_r * a.Vt;
        const int total = a.Gk * per_box;
        const int gap = (rs - a.head_r) * a.Vt;
        Walk2 w(threadIdx.x, per_box);
#pragma unroll
        for (int m = 0; m < NR; ++m) {
            const int e = threadIdx.x + m * (int)blockDim.x;
            if (e < total) dst[e + w.hi * gap] = v[m];
            w.next();
        }
    }
};

// Copy the tile's Gk pairs (slot = digit-reversed logical a_loc) to the
// state at the pass's last level lb: pair (a0 + a_loc) R^(L-lb) + bfix.
__device__ __forceinline__ void store_tile(const PassArgs& a,
                                           const float2* tile, long long a0,
                                           long long bfix, int chunk) {
    const int lb = a.la - 1 + a.k;
    const int shiftB = a.dim * (a.L - lb);
    const int per_pair = a.r_state_out * a.Vt;
    const int lds_pair = a.rmax * a.Vt;
    const int total = a.Gk * per_pair;
    // pair offsets within one column chunk stay below N * per_pair < 2^31
    float2* base = a.out + (size_t)chunk * a.N * per_pair +
                   (size_t)((a0 << shiftB) + bfix) * per_pair;
    Walk2 w(threadIdx.x, per_pair);      // (slot, t * Vt + col)
    for (int e = threadIdx.x; e < total; e += blockDim.x, w.next()) {
        const unsigned dA = (unsigned)digit_rev(w.hi, a.k, a.dim);
        base[(dA << shiftB) * (unsigned)per_pair + (unsigned)w.lo] =
            tile[w.hi * lds_pair + w.lo];
    }
}

// Load the Gk consecutive pairs p0 .. p0+Gk-1 of the input state into slots.
// load_tile in two halves: load() issues the global reads of the tile into
// registers (up to NR per thread), store() writes them to LDS and copies
// any entries past NR per thread directly, so that the reads overlap the
// work in between.
template <int NR>
struct TileLoad {
    float2 v[NR];
    const float2* base;
    int total;

    __device__ __forceinline__ void load(const PassArgs& a, long long p0,
                                         int r_in, int chunk) {
        const int per_pair = r_in * a.Vt;
        total = a.Gk * per_pair;
        base = a.in + (size_t)chunk * a.N * per_pair + (size_t)p0 * per_pair;
#pragma unroll
        for (int m = 0; m < NR; ++m) {
            const int e = threadIdx.x + m * (int)blockDim.x;
            if (e < total) v[m] = base[e];
        }
    }

    __device__ __forceinline__ void store(const PassArgs& a, float2* tile,
                                          int r_in) const {
        const int per_pair = r_in * a.Vt;
        const int lds_pair = a.rmax * a.Vt;
        Walk2 w(threadIdx.x, per_pair);
#pragma unroll
        for (int m = 0; m < NR; ++m) {
            const int e = threadIdx.x + m * (int)blockDim.x;
            if (e < total) tile[w.hi * lds_pair + w.lo] = v[m];
            w.next();
        }
        for (int e = threadIdx.x + NR * (int)blockDim.x; e < total;
             e += blockDim.x, w.next())
            tile[w.hi * lds_pair + w.lo] = base[e];
    }
};

__device__ __forceinline__ void load_tile(const PassArgs& a, float2* tile,
                                          long long p0, int r_in, int chunk) {
    const int per_pair = r_in * a.Vt;
    const int lds_pair = a.rmax * a.Vt;
    const int total = a.Gk * per_pair;
    const float2* base = a.in + (size_t)chunk * a.N * per_pair +
                         (size_t)p0 * per_pair;
    Walk2 w(threadIdx.x, per_pair);
    for (int e = threadIdx.x; e < total; e += blockDim.x, w.next())
        tile[w.hi * lds_pair + w.lo] = base[e];
}

// The switch on a tile (vector ALU): slots hold the pairs (A = a0 +
// rev_k(slot), B = bfix) at level h, global pair P = A R^(L-h) + bfix.
template <int TB, int MAXIT>
__device__ __forceinline__ void tile_switch(const PassArgs& a, float2* tile,
                                            long long a0, long long bfix,
                                            int kdig, const float2* src,
                                            int src_stride_r) {
    const int ntb = (a.sw_r_out + TB - 1) / TB;
    const int items = a.Gk * ntb * a.Vt;
    const int shiftB = a.dim * (a.L - (a.la - 1 + a.k));
    float2 keep[MAXIT][TB];
#pragma unroll
    for (int it = 0; it < MAXIT; ++it) {
        const int item = it * kPassThreads + threadIdx.x;
        if (item >= items) break;
        const int col = item % a.Vt;
        const int rest = item / a.Vt;
        const int tb = rest % ntb;
        const int slot = rest / ntb;
        const long long A = a0 + digit_rev(slot, kdig, a.dim);
        const long long P = (A << shiftB) + bfix;
        const float2* S = a.S + (size_t)P * a.sw_r_out * a.sw_r_in;
#pragma unroll
        for (int t = 0; t < TB; ++t) keep[it][t] = make_float2(0.f, 0.f);
        for (int s = 0; s < a.sw_r_in; ++s) {
            const float2 x = src[(slot * src_stride_r + s) * a.Vt + col];
#pragma unroll
            for (int t = 0; t < TB; ++t) {
                const int tt = tb * TB + t;
                if (tt < a.sw_r_out) {
                    const float2 z = cmul(S[tt * a.sw_r_in + s], x);
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
        const int rest = item / a.Vt;
        const int tb = rest % ntb;
        const int slot = rest / ntb;
#pragma unroll
        for (int t = 0; t < TB; ++t) {
            const int tt = tb * TB + t;
            if (tt < a.sw_r_out)
                tile[(slot * a.rmax + tt) * a.Vt + col] = keep[it][t];
        }
    }
    __syncthreads();
}

// MFMA passes (apply_mfma.hip): launch one pass; "" on success.
std::string launch_mfma_pass(const PassArgs& a, bool is_xi, size_t lds,
                             hipStream_t st);
// Dynamic LDS bytes of an MFMA pass with these arguments.
size_t mfma_pass_lds(const PassArgs& a, bool is_xi);
std::string launch_sum_parts(const PassArgs& a, int nv, hipStream_t st);

}  // namespace bfi
