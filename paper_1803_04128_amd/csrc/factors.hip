// Factor construction on the device, FP64 phase arithmetic.
//
// Kernel entries at interpolation points (Algorithm 2; Algorithm 4.1, eqs.
// (eqn:1), (eqn:2), the switch step and eq. (eqn:3)) regrouped so that each
// level stores unit-modulus diagonals (twiddles) and one real Lagrange
// matrix per child position:
//   xi level l:  W_{A,C}[s] = exp(2 pi i [Phi(c_A, xi_s^C) - Phi(c_P, xi_s^C)])
//   switch:      S_{AB}[t][s] = exp(2 pi i [Phi(x_t^A, xi_s^B)
//                               - Phi(c_A, xi_s^B) - Phi(x_t^A, c_B)])
//   x level l:   T_{A,C}[t] = exp(2 pi i [Phi(x_t^A, c_C) - Phi(x_t^A, c_B)])
// Each phase is evaluated in FP64, the difference is reduced modulo 1 and
// only then passed to sincospi; the result is stored as FP32 complex.
#include <cstring>
#include <vector>

#include <hip/hip_fp16.h>

#include "factor_terms.h"

namespace bfi {

constexpr int kFactorBlock = 256;

#define HIPCHK(x)                                                       \
    do {                                                                \
        hipError_t e_ = (x);                                            \
        if (e_ != hipSuccess)                                           \
            return std::string(#x ": ") + hipGetErrorString(e_);        \
    } while (0)

// Stored switch blocks of a split-precision plan: each complex64 entry is
// replaced in place by its 16-bit parts (Re hi, Re lo, Im hi, Im lo), the
// same 8 bytes, in bfloat16 (round to nearest even) or half.
__global__ void split_switch_blocks(float2* S, long long count, int use_half) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
         i < count; i += (long long)gridDim.x * blockDim.x) {
        const float2 v = S[i];
        unsigned short h[4];
        const float parts[2] = {v.x, v.y};
        for (int c = 0; c < 2; ++c) {
            const float x = parts[c];
            if (use_half) {
                const __half hi = __float2half_rn(x);
                const __half lo = __float2half_rn(x - __half2float(hi));
                h[2 * c] = __half_as_ushort(hi);
                h[2 * c + 1] = __half_as_ushort(lo);
            } else {
                const unsigned u = __float_as_uint(x);
                const unsigned hb = (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u;
                const float r = x - __uint_as_float(hb);
                const unsigned ul = __float_as_uint(r);
                const unsigned lb = (ul + 0x7fffu + ((ul >> 16) & 1u)) >> 16;
                h[2 * c] = (unsigned short)(hb >> 16);
                h[2 * c + 1] = (unsigned short)lb;
            }
        }
        ((ushort4*)S)[i] = make_ushort4(h[0], h[1], h[2], h[3]);
    }
}

// hi + lo of a split entry (read-back of split plans)
__device__ __forceinline__ float2 join_split(float2 raw, int split) {
    const ushort4 q = __builtin_bit_cast(ushort4, raw);
    if (split == BF_FP16X3)
        return make_float2(__half2float(__ushort_as_half(q.x)) +
                               __half2float(__ushort_as_half(q.y)),
                           __half2float(__ushort_as_half(q.z)) +
                               __half2float(__ushort_as_half(q.w)));
    return make_float2(__uint_as_float((unsigned)q.x << 16) +
                           __uint_as_float((unsigned)q.y << 16),
                       __uint_as_float((unsigned)q.z << 16) +
                           __uint_as_float((unsigned)q.w << 16));
}

__global__ void xi_twiddles(TwArgs a) {
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
         idx < a.total; idx += (long long)gridDim.x * blockDim.x)
        a.out[idx] = expi_frac(terms_phase(a.P, xi_terms(a, idx)));
}

__global__ void x_twiddles(TwArgs a) {
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
         idx < a.total; idx += (long long)gridDim.x * blockDim.x)
        a.out[idx] = expi_frac(terms_phase(a.P, x_terms(a, idx)));
}

__global__ void switch_blocks(TwArgs a) {
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
         idx < a.total; idx += (long long)gridDim.x * blockDim.x)
        a.out[idx] = expi_frac(terms_phase(a.P, switch_terms(a, idx)));
}

// Diagnostic read-back of stored entries: for each requested entry index,
// the user indices of its phase terms (-1 past the term count) and the
// stored value.  kind: STEP_XI / STEP_X (twiddles) or STEP_SWITCH (blocks).
__global__ void factor_entries(TwArgs a, int kind, const float2* src,
                               const long long* idx, int count,
                               long long* xo, long long* jo, float2* val,
                               int split) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    const long long e = idx[k];
    const Terms T = kind == STEP_XI ? xi_terms(a, e)
                    : kind == STEP_X ? x_terms(a, e)
                                     : switch_terms(a, e);
    for (int t = 0; t < 3; ++t) {
        xo[3 * k + t] = t < T.count ? user_index(T.ix[t], a.P.dim, a.P.n) : -1;
        jo[3 * k + t] = t < T.count ? user_index(T.jx[t], a.P.dim, a.P.n) : -1;
    }
    val[k] = split ? join_split(src[e], split) : src[e];
}

std::string read_factor_entries(const Plan& p, int step, int which,
                                const long long* idx, int count,
                                long long* x_out, long long* xi_out,
                                float* val_out) {
    const Step& s = p.steps[step];
    const float2* src = which == 0 ? s.tw : s.S;
    const size_t total = which == 0 ? s.tw_elems : s.S_elems;
    if (!src || total == 0)
        return which == 0 ? "the step stores no twiddles"
                          : "the step stores no switch blocks";
    for (int k = 0; k < count; ++k)
        if (idx[k] < 0 || (size_t)idx[k] >= total)
            return "entry index out of range";
    TwArgs t{};
    t.P = p.phase;
    t.L = p.L;
    t.ax_in = s.ax_in;
    t.ax_out = s.ax_out;
    t.level = s.level;
    t.reads_f = s.reads_f;
    t.writes_lambda = s.writes_lambda;
    void* mem = nullptr;
    const size_t bi = (size_t)count * sizeof(long long);
    HIPCHK(hipMalloc(&mem, bi * 7 + (size_t)count * sizeof(float2)));
    long long* di = (long long*)mem;
    long long* dx = di + count;
    long long* dj = dx + 3 * (size_t)count;
    float2* dv = (float2*)(dj + 3 * (size_t)count);
    std::string err;
    hipError_t e = hipMemcpy(di, idx, bi, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(factor_entries, dim3((count + 255) / 256),
                           dim3(256), 0, 0, t, s.kind, src, di, count, dx, dj,
                           dv,
                           which == 1 && p.precision != BF_FP32 ? p.precision : 0);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(x_out, dx, 3 * bi, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(xi_out, dj, 3 * bi, hipMemcpyDeviceToHost);
    if (e == hipSuccess)
        e = hipMemcpy(val_out, dv, (size_t)count * sizeof(float2),
                      hipMemcpyDeviceToHost);
    if (e != hipSuccess) err = std::string("factor read-back: ") + hipGetErrorString(e);
    (void)hipFree(mem);
    return err;
}

// complex128 host amplitude factors -> complex64 device (conjugated for
// the conjugate kernels)
__global__ void narrow_complex(const double2* in, float2* out, long long m,
                               int conj) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
         i < m; i += (long long)gridDim.x * blockDim.x)
        out[i] = make_float2((float)in[i].x,
                             conj ? -(float)in[i].y : (float)in[i].y);
}

// 16-bit hi/lo split of the FP32 Lagrange matrices (bfloat16 or half).
__global__ void split_matrices(const float* m, uint16_t* hi, uint16_t* lo,
                               long long count, int use_half) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
         i < count; i += (long long)gridDim.x * blockDim.x) {
        float v = m[i];
        if (use_half) {
            __half h = __float2half_rn(v);
            float r = v - __half2float(h);
            __half l = __float2half_rn(r);
            hi[i] = __half_as_ushort(h);
            lo[i] = __half_as_ushort(l);
        } else {
            // round-to-nearest-even bfloat16
            unsigned u = __float_as_uint(v);
            unsigned rh = u + 0x7fffu + ((u >> 16) & 1u);
            unsigned hb = rh & 0xffff0000u;
            float r = v - __uint_as_float(hb);
            unsigned ul = __float_as_uint(r);
            unsigned rl = ul + 0x7fffu + ((ul >> 16) & 1u);
            hi[i] = (uint16_t)(hb >> 16);
            lo[i] = (uint16_t)(rl >> 16);
        }
    }
}

static int grid_for(long long total) {
    long long g = (total + kFactorBlock - 1) / kFactorBlock;
    return (int)(g < 65536 ? (g < 1 ? 1 : g) : 65536);
}

static size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }


// Offsets of every factor array inside the plan arena.
struct ArenaLayout {
    std::vector<size_t> off_tw, off_m, off_hi, off_lo, off_am, off_ax, off_af;
    std::vector<size_t> off_2f, off_2h, off_2l;   // 2D split tables
    std::vector<size_t> off_sep;                  // 2D separable A tables
    size_t off_a = 0, off_b = 0, bytes = 0;
};

static ArenaLayout arena_layout(Plan& p) {
    ArenaLayout A;
    size_t bytes = 0;
    const bool split = p.precision != BF_FP32;
    auto& off_tw = A.off_tw;
    auto& off_m = A.off_m;
    auto& off_hi = A.off_hi;
    auto& off_lo = A.off_lo;
    auto& off_am = A.off_am;
    auto& off_ax = A.off_ax;
    auto& off_af = A.off_af;
    for (auto& s : p.steps) {
        off_am.push_back(bytes);
        bytes = align_up(bytes + s.amat_elems * sizeof(float));
        off_ax.push_back(bytes);
        bytes = align_up(bytes + s.amat_xi_elems * sizeof(float));
        off_tw.push_back(bytes);
        if (p.tw_stored) bytes = align_up(bytes + s.tw_elems * sizeof(float2));
        off_m.push_back(bytes);
        bytes = align_up(bytes + s.mat_elems * sizeof(float));
        // split precisions: the arranged FP32 table, then its hi and lo parts
        if (split && s.mat_elems && p.dim == 1 && s.r_out <= 16)
            s.asplit_elems = 512;
        off_af.push_back(bytes);
        bytes = align_up(bytes + s.asplit_elems * sizeof(float));
        off_hi.push_back(bytes);
        bytes = align_up(bytes + s.asplit_elems * 2);
        off_lo.push_back(bytes);
        bytes = align_up(bytes + s.asplit_elems * 2);
        // split plans of the per-step form: the 16x16x16 A tables
        s.a16_elems = 0;
        if (split && s.mat_elems && p.dim == 2)
            s.a16_elems = (size_t)p.R * ((s.r_out + 15) / 16) *
                          ((s.r_in + 15) / 16) * 256;
        A.off_2f.push_back(bytes);
        bytes = align_up(bytes + s.a16_elems * sizeof(float));
        A.off_2h.push_back(bytes);
        bytes = align_up(bytes + s.a16_elems * 2);
        A.off_2l.push_back(bytes);
        bytes = align_up(bytes + s.a16_elems * 2);
        s.sep_elems = (p.dim == 2 && !s.lag1_host.empty())
                          ? (s.kind == STEP_XI ? 256 : 128) : 0;
        A.off_sep.push_back(bytes);
        bytes = align_up(bytes + s.sep_elems * sizeof(float));
    }
    A.off_a = bytes;
    if (p.has_amp) bytes = align_up(bytes + (size_t)p.r_amp * p.N * sizeof(float2));
    A.off_b = bytes;
    if (p.has_amp) bytes = align_up(bytes + (size_t)p.r_amp * p.N * sizeof(float2));
    A.bytes = bytes;
    return A;
}

size_t factor_arena_bytes(Plan& p) { return arena_layout(p).bytes; }

std::string build_factors(Plan& p) {
    const ArenaLayout A = arena_layout(p);
    const auto& off_tw = A.off_tw;
    const auto& off_m = A.off_m;
    const auto& off_hi = A.off_hi;
    const auto& off_lo = A.off_lo;
    const auto& off_am = A.off_am;
    const auto& off_ax = A.off_ax;
    const auto& off_af = A.off_af;
    const size_t off_a = A.off_a, off_b = A.off_b, bytes = A.bytes;
    const bool has_amp = p.has_amp;
    p.arena_bytes = bytes;
    HIPCHK(hipMalloc(&p.arena, bytes > 0 ? bytes : 256));
    char* base = (char*)p.arena;

    TwArgs t{};
    t.P = p.phase;
    t.L = p.L;
    for (size_t k = 0; k < p.steps.size(); ++k) {
        Step& s = p.steps[k];
        s.tw = s.tw_elems && p.tw_stored ? (float2*)(base + off_tw[k])
                                         : nullptr;
        s.S = nullptr;   // build_switch_blocks
        s.mats = s.mat_elems ? (float*)(base + off_m[k]) : nullptr;
        s.amat = s.amat_elems ? (float*)(base + off_am[k]) : nullptr;
        s.amat_xi = s.amat_xi_elems ? (float*)(base + off_ax[k]) : nullptr;
        if (s.asplit_elems) {
            s.asplit_hi = (uint16_t*)(base + off_hi[k]);
            s.asplit_lo = (uint16_t*)(base + off_lo[k]);
        }
        t.ax_in = s.ax_in;
        t.ax_out = s.ax_out;
        t.level = s.level;
        t.reads_f = s.reads_f;
        t.writes_lambda = s.writes_lambda;
        if (s.kind == STEP_SWITCH || !s.tw) {
            // stored switch blocks are built by build_switch_blocks; a plan
            // built without stored twiddles evaluates them in the apply
        } else if (s.kind == STEP_XI) {
            t.total = (long long)s.tw_elems;
            t.out = s.tw;
            hipLaunchKernelGGL(xi_twiddles, dim3(grid_for(t.total)),
                               dim3(kFactorBlock), 0, 0, t);
        } else if (s.kind == STEP_X) {
            t.total = (long long)s.tw_elems;
            t.out = s.tw;
            hipLaunchKernelGGL(x_twiddles, dim3(grid_for(t.total)),
                               dim3(kFactorBlock), 0, 0, t);
        }
        HIPCHK(hipGetLastError());
        if (s.mat_elems) {
            std::vector<float> mf(s.mat_elems);
            for (size_t e = 0; e < s.mat_elems; ++e)
                mf[e] = (float)s.mats_host[e];
            HIPCHK(hipMemcpy(s.mats, mf.data(), s.mat_elems * sizeof(float),
                             hipMemcpyHostToDevice));
            // the same matrices in MFMA A-operand order
            const int MT = (s.r_out + 15) / 16, KS = (s.r_in + 3) / 4;
            std::vector<float> am(s.amat_elems, 0.f);
            for (int c = 0; c < p.R; ++c)
                for (int mt = 0; mt < MT; ++mt)
                    for (int ks = 0; ks < KS; ++ks)
                        for (int l = 0; l < 64; ++l) {
                            const int t = 16 * mt + l % 16, sx = 4 * ks + l / 16;
                            if (t < s.r_out && sx < s.r_in)
                                am[(((size_t)c * MT + mt) * KS + ks) * 64 + l] =
                                    mf[((size_t)c * s.r_out + t) * s.r_in + sx];
                        }
            HIPCHK(hipMemcpy(s.amat, am.data(), s.amat_elems * sizeof(float),
                             hipMemcpyHostToDevice));
            if (s.amat_xi_elems) {
                // xi order of the fused 1D passes: k = 4 kk + g, child
                // c = g % 2, coefficient 2 kk + g / 2
                std::vector<float> ax(s.amat_xi_elems, 0.f);
                const int nk = (s.r_in + 1) / 2;
                for (int kk = 0; kk < nk; ++kk)
                    for (int l = 0; l < 64; ++l) {
                        const int t = l % 16, g = l / 16;
                        const int c = g % 2, sx = 2 * kk + g / 2;
                        if (t < s.r_out && sx < s.r_in)
                            ax[(size_t)kk * 64 + l] =
                                mf[((size_t)c * s.r_out + t) * s.r_in + sx];
                    }
                HIPCHK(hipMemcpy(s.amat_xi, ax.data(),
                                 s.amat_xi_elems * sizeof(float),
                                 hipMemcpyHostToDevice));
            }
            if (s.sep_elems) {
                // A tables of the one-dimension-at-a-time 2D contractions
                const int a1 = s.ax_in.r1, b1 = s.ax_out.r1;
                std::vector<float> sp(s.sep_elems, 0.f);
                for (int l = 0; l < 64; ++l) {
                    const int row = l % 16, kq = l / 16;
                    if (s.kind == STEP_XI) {
                        for (int ks = 0; ks < 4; ++ks) {
                            const int k = 4 * ks + kq;
                            const int c = k / a1, sx = k - c * a1;
                            if (row < b1 && k < 2 * a1)
                                sp[(size_t)ks * 64 + l] = (float)
                                    s.lag1_host[((size_t)c * b1 + row) * a1 + sx];
                        }
                    } else {
                        for (int ks = 0; ks < 2; ++ks) {
                            const int sx = 4 * ks + kq;
                            const int i = row / b1, t = row - i * b1;
                            if (row < 2 * b1 && sx < a1)
                                sp[(size_t)ks * 64 + l] = (float)
                                    s.lag1_host[((size_t)i * b1 + t) * a1 + sx];
                        }
                    }
                }
                s.amat_sep = (float*)(base + A.off_sep[k]);
                HIPCHK(hipMemcpy(s.amat_sep, sp.data(), sp.size() * sizeof(float),
                                 hipMemcpyHostToDevice));
            }
            if (s.a16_elems) {
                // 16x16x16 A tables of the per-step split kernels, arranged
                // in FP32, then split into hi and lo parts on the device
                const int MTs = (s.r_out + 15) / 16, KB = (s.r_in + 15) / 16;
                std::vector<float> af(s.a16_elems, 0.f);
                for (int c = 0; c < p.R; ++c)
                    for (int mt = 0; mt < MTs; ++mt)
                        for (int kb = 0; kb < KB; ++kb)
                            for (int l = 0; l < 64; ++l)
                                for (int e = 0; e < 4; ++e) {
                                    const int t = 16 * mt + l % 16;
                                    const int sx = 16 * kb + 4 * (l / 16) + e;
                                    if (t < s.r_out && sx < s.r_in)
                                        af[((((size_t)c * MTs + mt) * KB + kb) * 64 + l) * 4 + e] =
                                            mf[((size_t)c * s.r_out + t) * s.r_in + sx];
                                }
                float* dev = (float*)(base + A.off_2f[k]);
                s.a16_hi = (uint16_t*)(base + A.off_2h[k]);
                s.a16_lo = (uint16_t*)(base + A.off_2l[k]);
                HIPCHK(hipMemcpy(dev, af.data(), af.size() * sizeof(float),
                                 hipMemcpyHostToDevice));
                hipLaunchKernelGGL(split_matrices,
                                   dim3(grid_for((long long)s.a16_elems)),
                                   dim3(kFactorBlock), 0, 0, dev, s.a16_hi,
                                   s.a16_lo, (long long)s.a16_elems,
                                   p.precision == BF_FP16X3 ? 1 : 0);
                HIPCHK(hipGetLastError());
            }
            if (s.asplit_elems) {
                // A operands of the split products, arranged per lane, then
                // split into hi and lo parts on the device
                std::vector<float> af(s.asplit_elems, 0.f);
                for (int l = 0; l < 64; ++l) {
                    const int t = l % 16, g = l / 16;
                    if (t >= s.r_out) continue;
                    if (s.kind == STEP_XI) {
                        for (int e = 0; e < 8; ++e) {
                            const int c = e % 2, sx = 4 * g + e / 2;
                            if (sx < s.r_in)
                                af[(size_t)l * 8 + e] =
                                    mf[((size_t)c * s.r_out + t) * s.r_in + sx];
                        }
                    } else {
                        for (int i = 0; i < 2; ++i)
                            for (int e = 0; e < 4; ++e) {
                                const int sx = 4 * g + e;
                                if (sx < s.r_in)
                                    af[((size_t)i * 64 + l) * 4 + e] =
                                        mf[((size_t)i * s.r_out + t) * s.r_in + sx];
                            }
                    }
                }
                float* dev = (float*)(base + off_af[k]);
                HIPCHK(hipMemcpy(dev, af.data(), af.size() * sizeof(float),
                                 hipMemcpyHostToDevice));
                hipLaunchKernelGGL(split_matrices,
                                   dim3(grid_for((long long)s.asplit_elems)),
                                   dim3(kFactorBlock), 0, 0, dev,
                                   s.asplit_hi, s.asplit_lo,
                                   (long long)s.asplit_elems,
                                   p.precision == BF_FP16X3 ? 1 : 0);
                HIPCHK(hipGetLastError());
            }
        }
    }
    HIPCHK(hipDeviceSynchronize());
    if (has_amp) {
        p.a_dev = (float2*)(base + off_a);
        p.b_dev = (float2*)(base + off_b);
    }
    return "";
}

// Upload and narrow the amplitude factors (host complex128 [r][N]).
// The switch blocks S of every switch step in an allocation of their own:
// built when the plan's execution form reads them (all forms but the
// per-step MFMA form with on-the-fly blocks), kept until bf_destroy.
static size_t switch_layout(const Plan& p, std::vector<size_t>& off) {
    size_t bytes = 0;
    for (auto& s : p.steps) {
        off.push_back(bytes);
        bytes = align_up(bytes + s.S_elems * sizeof(float2));
    }
    return bytes;
}

size_t switch_block_bytes(const Plan& p) {
    std::vector<size_t> off;
    return switch_layout(p, off);
}

std::string build_switch_blocks(Plan& p) {
    if (p.S_arena) return "";
    std::vector<size_t> off;
    const size_t bytes = switch_layout(p, off);
    if (bytes == 0) return "";
    void* mem = nullptr;
    HIPCHK(hipMalloc(&mem, bytes));
    TwArgs t{};
    t.P = p.phase;
    t.L = p.L;
    for (size_t k = 0; k < p.steps.size(); ++k) {
        Step& s = p.steps[k];
        if (s.kind != STEP_SWITCH || !s.S_elems) continue;
        s.S = (float2*)((char*)mem + off[k]);
        t.ax_in = s.ax_in;
        t.ax_out = s.ax_out;
        t.level = s.level;
        t.reads_f = s.reads_f;
        t.writes_lambda = s.writes_lambda;
        t.total = (long long)s.S_elems;
        t.out = s.S;
        hipLaunchKernelGGL(switch_blocks, dim3(grid_for(t.total)),
                           dim3(kFactorBlock), 0, 0, t);
    }
    // split-precision plans read the blocks only in the split MFMA switch
    if (p.precision != BF_FP32)
        hipLaunchKernelGGL(split_switch_blocks,
                           dim3(grid_for((long long)(bytes / sizeof(float2)))),
                           dim3(kFactorBlock), 0, 0, (float2*)mem,
                           (long long)(bytes / sizeof(float2)),
                           p.precision == BF_FP16X3 ? 1 : 0);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        for (auto& s : p.steps) s.S = nullptr;
        (void)hipFree(mem);
        return std::string("switch blocks: ") + hipGetErrorString(e);
    }
    p.S_arena = mem;
    p.S_bytes = bytes;
    return "";
}

std::string upload_amplitude(Plan& p, const double* a, const double* b) {
    const long long m = (long long)p.r_amp * p.N;
    void* tmp = nullptr;
    HIPCHK(hipMalloc(&tmp, (size_t)m * sizeof(double2)));
    // a_k weights the output and b_k the input of K; K^T has its output on
    // the xi grid, so there the b_k weight the output and the a_k the input
    const bool tr = (p.op & BF_OP_T) != 0;
    const double* src[2] = {tr ? b : a, tr ? a : b};
    float2* dst[2] = {p.a_dev, p.b_dev};
    const int conj = (p.op & BF_OP_C) != 0;
    for (int k = 0; k < 2; ++k) {
        hipError_t e = hipMemcpy(tmp, src[k], (size_t)m * sizeof(double2),
                                 hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(tmp);
            return std::string("hipMemcpy amplitude: ") + hipGetErrorString(e);
        }
        hipLaunchKernelGGL(narrow_complex, dim3(grid_for(m)),
                           dim3(kFactorBlock), 0, 0, (const double2*)tmp,
                           dst[k], m, conj);
        e = hipDeviceSynchronize();
        if (e != hipSuccess) {
            (void)hipFree(tmp);
            return std::string("narrow amplitude: ") + hipGetErrorString(e);
        }
    }
    HIPCHK(hipFree(tmp));
    return "";
}

}  // namespace bfi
