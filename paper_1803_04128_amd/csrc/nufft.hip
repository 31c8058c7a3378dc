// NUFFT by dimension lifting on the device (Section 3, eq. (eqn:tg3)):
//   g_v(x_i) = sum_k a_k(x_i) sum_j exp(2 pi i P_i . Q_j) b_k(xi_j) f_v(xi_j),
// r_eps r-dimensional type-3 NUFFTs (r = 1 or 2) from the sources s_j = Q_j
// to the targets t_i = P_i, for every vector and amplitude term.
//
// Type 3 through two Gaussian griddings, per dimension (centers sbar, tbar,
// half-widths S, X of the shifted points s' = s - sbar, t' = t - tbar):
//   sum_j c_j e^{2 pi i t.s_j} = e^{2 pi i t.sbar} sum_j [c_j e^{2 pi i tbar.s'_j}]
//                                e^{2 pi i t'.s'_j};
//   spreading the shifted sources with phi(u) = exp(-(u/h)^2 / (4 b)) onto
//   the grid u = m h (h = 1 / (4 X): twice the Nyquist rate of the targets)
//   turns the sum into (1 / phihat(t')) h sum_m F_m e^{2 pi i m theta},
//   theta = t' h, |theta| <= 1/4; that Fourier series is evaluated by the
//   second gridding: coefficients h F_m / psihat_m on an oversampled FFT
//   grid of Mr points, a power of two of at least 4 Mh (63/64) (modes
//   |m| <= Mh), one FFT with the positive
//   exponent, and the Gaussian psi(theta) = exp(-(theta Mr)^2 / (4 b)) at
//   each target, divided by Mr.
// Both Gaussians use b = W / (4 pi sqrt(1/2)) and 2 W grid points per
// dimension, which balances the truncation error exp(-W^2 / (4 b)) against
// the aliasing error at oversampling 2 (about 1e-7 relative at W = 7).
// Point positions are split on the host (FP64) into an integer grid index
// and a fraction in [0, 1), and the phase factors are computed in FP64, so
// the device arithmetic (FP32) only forms Gaussian weights of fractions.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "apply_common.h"

namespace bfi {

namespace {

constexpr int kW = 7;                 // stencil half-width (2 kW points)
constexpr int kFftMax = 4096;         // longest FFT held in one workgroup
// 2D spreading gathers while its contribution lists (N (2 kW)^2 entries of
// 8 bytes) stay within 2 GiB, and spreads by atomics past that
constexpr long long kMaxGatherEntries = 1LL << 28;
constexpr int kNufftThreads = 256;
constexpr int kFftLds = 80 * 1024;    // FFT workgroup LDS (two per CU)
constexpr int kFftThreads = 1024;     // FFT workgroup (16 waves)
constexpr double kPi = 3.141592653589793238462643383279502884;

struct NuArgs {
    int r, K, nv;                     // dims, amplitude terms, vectors
    long long N;
    int Mr[2], Mh[2];
    long long cells;
    float b4;                         // 4 b
    const int* sbase;
    const float* sfrac;
    const float2* pre;
    const int* tbase;
    const float* tfrac;
    const float2* post;
    const float* dec0;
    const float* dec1;
    // the sources' contributions by grid cell (CSR, built at plan time):
    // cell m takes entries cptr[m] .. cptr[m + 1] - 1, each a source index
    // and its Gaussian weight times the cell's deconvolution factor (the
    // products over the dimensions in 2D); null where 2D spreads by atomics
    const int* cptr;
    const int* cidx;
    const float* cwt;
    const float2* a;
    const float2* b;                  // gather: [N][kp]; atomics: [K][N]
    int kp;                           // gather: terms per source row of b
    const float2* f;                  // [nv][N] chunk
    float2* g;
    float2* grid;                     // [nv * K][cells]
};

__global__ void __launch_bounds__(kNufftThreads)
nufft_zero(float2* p, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
         i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = make_float2(0.f, 0.f);
}

// Gaussian weights of the 2 kW grid points m0 - kW + 1 + e around a point at
// grid position m0 + frac.
__device__ __forceinline__ void gauss(float frac, float b4, float (&w)[2 * kW]) {
#pragma unroll
    for (int e = 0; e < 2 * kW; ++e) {
        const float d = (float)(e - kW + 1) - frac;
        w[e] = expf(-d * d / b4);
    }
}

__device__ __forceinline__ int wrap(int m, int M) {
    m %= M;
    return m < 0 ? m + M : m;
}

// Sources to the grid: thread per source, every column of the chunk.
// Column c = v K + k carries b_k(xi_j) f_v(xi_j) times the source phase;
// each grid point gets phi times h / psihat of its mode.
template <int R>
__global__ void __launch_bounds__(kNufftThreads) nufft_spread(NuArgs a) {
    for (long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x;
         j < a.N; j += (long long)gridDim.x * blockDim.x) {
        float w0[2 * kW], w1[2 * kW];
        int c0[2 * kW], c1[2 * kW];
        {
            const int m0 = a.sbase[j * R];
            gauss(a.sfrac[j * R], a.b4, w0);
#pragma unroll
            for (int e = 0; e < 2 * kW; ++e) {
                const int m = m0 - kW + 1 + e;
                w0[e] *= a.dec0[m + a.Mh[0]];
                c0[e] = wrap(m, a.Mr[0]);
            }
        }
        if (R == 2) {
            const int m0 = a.sbase[j * R + 1];
            gauss(a.sfrac[j * R + 1], a.b4, w1);
#pragma unroll
            for (int e = 0; e < 2 * kW; ++e) {
                const int m = m0 - kW + 1 + e;
                w1[e] *= a.dec1[m + a.Mh[1]];
                c1[e] = wrap(m, a.Mr[1]);
            }
        }
        const float2 pj = a.pre[j];
        for (int v = 0; v < a.nv; ++v) {
            const float2 fv = cmul(a.f[(size_t)v * a.N + j], pj);
            for (int k = 0; k < a.K; ++k) {
                const float2 val = cmul(a.b[(size_t)k * a.N + j], fv);
                float2* gc = a.grid + (size_t)(v * a.K + k) * a.cells;
                if (R == 1) {
#pragma unroll
                    for (int e = 0; e < 2 * kW; ++e) {
                        atomicAdd(&gc[c0[e]].x, w0[e] * val.x);
                        atomicAdd(&gc[c0[e]].y, w0[e] * val.y);
                    }
                } else {
                    for (int e = 0; e < 2 * kW; ++e) {
                        float2* row = gc + (size_t)c0[e] * a.Mr[1];
                        const float vx = w0[e] * val.x, vy = w0[e] * val.y;
#pragma unroll
                        for (int e1 = 0; e1 < 2 * kW; ++e1) {
                            atomicAdd(&row[c1[e1]].x, w1[e1] * vx);
                            atomicAdd(&row[c1[e1]].y, w1[e1] * vy);
                        }
                    }
                }
            }
        }
    }
}

// Spreading as a gather: thread per (grid cell, vector, group of G
// amplitude terms) sums the contributions listed for its cell, in source
// order, and writes every cell (no atomics, no zeroing, a deterministic
// sum; cells in row-major order in 2D).  Column c = v K + k carries
// b_k(xi_j) f_v(xi_j) times the source phase, as in nufft_spread.  b is
// stored by source, b[j kp + k] with kp = G times the groups (zero past
// K), so that a contribution's G terms come in 16-byte reads and its
// index, weight, f and phase reads serve all G.
template <int G>
__global__ void __launch_bounds__(kNufftThreads) nufft_gather(NuArgs a) {
    const int ngrp = a.kp / G;
    const long long M = a.cells;
    const long long total = M * a.nv * ngrp;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
         e < total; e += (long long)gridDim.x * blockDim.x) {
        const long long m = e % M;
        const long long rest = e / M;
        const int grp = (int)(rest % ngrp), v = (int)(rest / ngrp);
        const int k0 = grp * G;
        float2 acc[G];
#pragma unroll
        for (int kk = 0; kk < G; ++kk) acc[kk] = make_float2(0.f, 0.f);
        const int t1 = a.cptr[m + 1];
        for (int t = a.cptr[m]; t < t1; ++t) {
            const int j = a.cidx[t];
            const float w = a.cwt[t];
            const float2 fp = cmul(a.f[(size_t)v * a.N + j], a.pre[j]);
            const float2 wf = make_float2(w * fp.x, w * fp.y);
            const float4* bp =
                (const float4*)(a.b + (size_t)j * a.kp + k0);
#pragma unroll
            for (int h = 0; h < G / 2; ++h) {
                const float4 b2 = bp[h];
                const float2 z0 = cmul(make_float2(b2.x, b2.y), wf);
                const float2 z1 = cmul(make_float2(b2.z, b2.w), wf);
                acc[2 * h].x += z0.x;
                acc[2 * h].y += z0.y;
                acc[2 * h + 1].x += z1.x;
                acc[2 * h + 1].y += z1.y;
            }
        }
#pragma unroll
        for (int kk = 0; kk < G; ++kk)
            if (k0 + kk < a.K)
                a.grid[(size_t)(v * a.K + k0 + kk) * a.cells + m] = acc[kk];
    }
}

// Terms per gather group: all K when K <= 32 (rounded up to 8), else 32.
int gather_group(int K) {
    return K >= 32 ? 32 : ((K + 7) / 8) * 8;
}

// Batched power-of-two FFT with the positive exponent, `batch` sequences per
// workgroup held in LDS: y_k = sum_t x_t exp(2 pi i t k / n).  Element t of
// sequence s in column col is read at src + col col_dist + s seq_dist +
// t stride, and output k is written at dst + col ocol_dist + s oseq_dist +
// k ostride (dst = src with the same addressing transforms in place: a
// workgroup reads all of its sequences before it writes any).  The
// sequences of a workgroup are consecutive (s0 .. s0 + batch - 1), so where
// a side is strided (adjacent sequences adjacent in memory) its element
// loop runs across the batch and each element index moves as `batch`
// contiguous entries.  Decimation in time after a bit-reversed load: the
// radix-2 stages are taken two at a time (one radix-4 pass over LDS, the
// same butterflies and table twiddles as the two stages), with a single
// stage first when log2 n is odd, and the twiddle table of the length is
// staged in LDS.  That single stage (odd lengths) or the first radix-4
// pass (even lengths) is formed as the entries are read, and the last
// radix-4 pass writes its outputs from registers, so the entries cross LDS
// two times fewer.  In LDS, entry i of sequence b sits at b P + i + i / 16
// (P = fft_pitch(n)): one pad entry every 16 entries and one more per
// sequence spread the bit-reversed stores, the batch-fastest element loops
// and the short butterfly spans over the banks.  With total > 0 (first step
// of a four-step transform of length total, a power of two), output k of
// sequence s is multiplied by exp(2 pi i s k / total).
struct FftArgs {
    const float2* src;
    float2* dst;
    const float2* tw;       // exp(2 pi i k / n), k < n / 2
    int logn;
    long long stride, seq_dist, col_dist;
    long long ostride, oseq_dist, ocol_dist;
    long long nseq;         // sequences per column (a multiple of batch)
    long long total;
    float tscale;           // 2 / total (exact), 0 without the twiddle
    int batch;              // sequences per workgroup (power of two)
    int logb;               // log2 batch
};

// LDS entries per sequence of an n-point FFT workgroup (see above).
__host__ __device__ constexpr long long fft_pitch(long long n) {
    return n + n / 16 + 1;
}

__device__ __forceinline__ int fft_ix(int b, int P, int i) {
    return b * P + i + (i >> 4);
}

__device__ __forceinline__ float2 cadd(float2 a, float2 b) {
    return make_float2(a.x + b.x, a.y + b.y);
}

__device__ __forceinline__ float2 csub(float2 a, float2 b) {
    return make_float2(a.x - b.x, a.y - b.y);
}

__global__ void __launch_bounds__(kFftThreads) fft_lds(FftArgs a) {
    extern __shared__ float2 lds_fft[];
    const int n = 1 << a.logn, B = a.batch;
    const int P = (int)fft_pitch(n);
    float2* x = lds_fft;                        // [batch][P]
    float2* tws = lds_fft + (size_t)B * P;      // [n / 2]
    const long long groups = a.nseq / B;
    const long long col = (long long)blockIdx.x / groups;
    const long long s0 = ((long long)blockIdx.x - col * groups) * B;
    const float2* in = a.src + col * a.col_dist + s0 * a.seq_dist;
    const bool bin = a.stride != 1;
    int lh = 0;
    if (a.logn & 1) {
        // odd length: the span-1 stage (pairs t, t + n/2 of the natural
        // order, adjacent after the bit reversal, twiddle 1) as they are
        // read
        for (int pe = threadIdx.x; pe < (n / 2) * B; pe += blockDim.x) {
            const int t = bin ? pe >> a.logb : (pe & (n / 2 - 1));
            const int b = bin ? pe & (B - 1) : (pe >> (a.logn - 1));
            const int rv = (int)(__brev((unsigned)t) >> (32 - a.logn));
            const float2* src = in + (long long)t * a.stride + b * a.seq_dist;
            const float2 u = src[0];
            const float2 v = src[(long long)(n / 2) * a.stride];
            const int i0 = fft_ix(b, P, rv);    // rv even: i0 + 1 is rv + 1
            x[i0] = cadd(u, v);
            x[i0 + 1] = csub(u, v);
        }
        lh = 1;
    } else {
        // even length: the first radix-4 pass (stages 0 and 1 on the
        // entries t, t + n/2, t + n/4, t + 3n/4 of the natural order, which
        // sit at rv .. rv + 3 after the bit reversal) as they are read, with
        // the table's twiddles 0 and n/4 (read from the table itself: the
        // LDS copy is not staged yet)
        const float2 w0 = a.tw[0], wq = a.tw[n / 4];
        for (int pe = threadIdx.x; pe < (n / 4) * B; pe += blockDim.x) {
            const int t = bin ? pe >> a.logb : (pe & (n / 4 - 1));
            const int b = bin ? pe & (B - 1) : (pe >> (a.logn - 2));
            const int rv = (int)(__brev((unsigned)t) >> (32 - a.logn));
            const float2* src = in + (long long)t * a.stride + b * a.seq_dist;
            const long long qs = (long long)(n / 4) * a.stride;
            const float2 u0 = src[0], v0 = cmul(src[2 * qs], w0);
            const float2 u1 = src[qs], v1 = cmul(src[3 * qs], w0);
            const float2 b0 = cadd(u0, v0), b1 = csub(u0, v0);
            const float2 c2 = cmul(cadd(u1, v1), w0);
            const float2 c3 = cmul(csub(u1, v1), wq);
            const int i0 = fft_ix(b, P, rv);    // rv % 4 = 0: i0 + c is rv + c
            x[i0] = cadd(b0, c2);
            x[i0 + 2] = csub(b0, c2);
            x[i0 + 1] = cadd(b1, c3);
            x[i0 + 3] = csub(b1, c3);
        }
        lh = 2;
    }
    for (int e = threadIdx.x; e < n / 2; e += blockDim.x) tws[e] = a.tw[e];
    __syncthreads();
    // radix-4 passes: stages lh (span half) and lh + 1 (span 2 half) on the
    // four entries j0 + {0, 1, 2, 3} half; the last (lh = logn - 2) writes
    // the output from registers
    for (; lh + 2 < a.logn; lh += 2) {
        const int half = 1 << lh;
        const int ts1 = n >> (lh + 1), ts2 = n >> (lh + 2);
        for (int qq = threadIdx.x; qq < (n / 4) * B; qq += blockDim.x) {
            const int b = qq >> (a.logn - 2), q = qq & (n / 4 - 1);
            const int grp = q >> lh, jj = q & (half - 1);
            const int j0 = (grp << (lh + 2)) + jj;
            const int i0 = fft_ix(b, P, j0), i1 = fft_ix(b, P, j0 + half);
            const int i2 = fft_ix(b, P, j0 + 2 * half);
            const int i3 = fft_ix(b, P, j0 + 3 * half);
            const float2 w1 = tws[jj * ts1];
            const float2 u0 = x[i0], v0 = cmul(x[i1], w1);
            const float2 u1 = x[i2], v1 = cmul(x[i3], w1);
            const float2 b0 = cadd(u0, v0), b1 = csub(u0, v0);
            const float2 c2 = cmul(cadd(u1, v1), tws[jj * ts2]);
            const float2 c3 = cmul(csub(u1, v1), tws[(jj + half) * ts2]);
            x[i0] = cadd(b0, c2);
            x[i2] = csub(b0, c2);
            x[i1] = cadd(b1, c3);
            x[i3] = csub(b1, c3);
        }
        __syncthreads();
    }
    float2* out = a.dst + col * a.ocol_dist + s0 * a.oseq_dist;
    const bool bout = a.ostride != 1;
    // output t of sequence b (with the four-step twiddle exp(2 pi i s t /
    // total), the product reduced exactly first; p < total <= 2^24, so
    // 2 p / total is exact in FP32)
    auto put = [&](int b, int t, float2 y) {
        if (a.total > 0) {
            const long long p = ((s0 + b) * t) & (a.total - 1);
            float sn, cs;
            sincospif((float)p * a.tscale, &sn, &cs);
            y = cmul(y, make_float2(cs, sn));
        }
        out[(long long)t * a.ostride + b * a.oseq_dist] = y;
    };
    if (lh + 2 == a.logn) {
        // the last radix-4 pass (half = n/4, one group): entries q + c n/4
        // are the outputs t = q, q + n/4, q + n/2, q + 3n/4; on a strided
        // output side the sequence index runs fastest across the lanes so
        // that the writes move in runs
        const int half = n / 4;
        for (int qq = threadIdx.x; qq < (n / 4) * B; qq += blockDim.x) {
            const int b = bout ? qq & (B - 1) : qq >> (a.logn - 2);
            const int q = bout ? qq >> a.logb : qq & (n / 4 - 1);
            const int i0 = fft_ix(b, P, q), i1 = fft_ix(b, P, q + half);
            const int i2 = fft_ix(b, P, q + 2 * half);
            const int i3 = fft_ix(b, P, q + 3 * half);
            const float2 w1 = tws[q * 2];
            const float2 u0 = x[i0], v0 = cmul(x[i1], w1);
            const float2 u1 = x[i2], v1 = cmul(x[i3], w1);
            const float2 b0 = cadd(u0, v0), b1 = csub(u0, v0);
            const float2 c2 = cmul(cadd(u1, v1), tws[q]);
            const float2 c3 = cmul(csub(u1, v1), tws[q + half]);
            put(b, q, cadd(b0, c2));
            put(b, q + half, cadd(b1, c3));
            put(b, q + 2 * half, csub(b0, c2));
            put(b, q + 3 * half, csub(b1, c3));
        }
    } else {
        // lengths 2 and 4: the stages formed at the read were all of them
        for (int e = threadIdx.x; e < n * B; e += blockDim.x) {
            const int t = bout ? e >> a.logb : (e & (n - 1));
            const int b = bout ? e & (B - 1) : (e >> a.logn);
            put(b, t, x[fft_ix(b, P, t)]);
        }
    }
}

// Grid to targets: thread per (target, vector); the Gaussian psi over the
// 2 kW points around theta Mr in each dimension, for every amplitude term,
// recombined with a_k and the target factor (phase, 1 / (phihat Mr)).
template <int R>
__global__ void __launch_bounds__(kNufftThreads) nufft_interp(NuArgs a) {
    const long long total = a.N * a.nv;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
         e < total; e += (long long)gridDim.x * blockDim.x) {
        const int v = (int)(e / a.N);
        const long long i = e - (long long)v * a.N;
        float w0[2 * kW], w1[2 * kW];
        int p0[2 * kW], p1[2 * kW];
        {
            const int m0 = a.tbase[i * R];
            gauss(a.tfrac[i * R], a.b4, w0);
#pragma unroll
            for (int q = 0; q < 2 * kW; ++q) {
                p0[q] = wrap(m0 - kW + 1 + q, a.Mr[0]);
            }
        }
        if (R == 2) {
            const int m0 = a.tbase[i * R + 1];
            gauss(a.tfrac[i * R + 1], a.b4, w1);
#pragma unroll
            for (int q = 0; q < 2 * kW; ++q) p1[q] = wrap(m0 - kW + 1 + q, a.Mr[1]);
        }
        float2 acc = make_float2(0.f, 0.f);
        for (int k = 0; k < a.K; ++k) {
            const float2* gc = a.grid + (size_t)(v * a.K + k) * a.cells;
            float2 s = make_float2(0.f, 0.f);
            if (R == 1) {
#pragma unroll
                for (int q = 0; q < 2 * kW; ++q) {
                    const float2 h = gc[p0[q]];
                    s.x += w0[q] * h.x;
                    s.y += w0[q] * h.y;
                }
            } else {
                for (int q = 0; q < 2 * kW; ++q) {
                    const float2* row = gc + (size_t)p0[q] * a.Mr[1];
                    float2 t = make_float2(0.f, 0.f);
#pragma unroll
                    for (int q1 = 0; q1 < 2 * kW; ++q1) {
                        const float2 h = row[p1[q1]];
                        t.x += w1[q1] * h.x;
                        t.y += w1[q1] * h.y;
                    }
                    s.x += w0[q] * t.x;
                    s.y += w0[q] * t.y;
                }
            }
            const float2 z = cmul(a.a[(size_t)k * a.N + i], s);
            acc.x += z.x;
            acc.y += z.y;
        }
        a.g[(size_t)v * a.N + i] = cmul(acc, a.post[i]);
    }
}

int blocks_for_n(long long n) {
    long long b = (n + kNufftThreads - 1) / kNufftThreads;
    return (int)std::max<long long>(1, std::min<long long>(b, 65536));
}

int ilog2i(long long v) {
    int l = 0;
    while ((1LL << l) < v) ++l;
    return l;
}

long long next_pow2(long long v) {
    long long p = 1;
    while (p < v) p <<= 1;
    return p;
}

}  // namespace

struct NufftPlan {
    int r = 1, K = 1;
    long long N = 0;
    int Mr[2] = {1, 1}, Mh[2] = {0, 0};
    long long cells = 1;
    int n1 = 0, n2 = 0;
    double b = 0;
    void* arena = nullptr;
    size_t arena_bytes = 0;
    int* sbase = nullptr;
    float* sfrac = nullptr;
    float2* pre = nullptr;
    int* tbase = nullptr;
    float* tfrac = nullptr;
    float2* post = nullptr;
    float* dec[2] = {nullptr, nullptr};
    float2* a = nullptr;
    float2* bb = nullptr;     // NuArgs::b
    int kp = 0;
    bool gather = false;      // spreading by the CSR gather (else atomics)
    int* cptr = nullptr;      // 1D gather CSR (NuArgs)
    int* cidx = nullptr;
    float* cwt = nullptr;
    // FFT twiddle tables by log2 length
    std::vector<std::pair<int, float2*>> tw;
    const float2* twiddles(int logn) const {
        for (auto& t : tw)
            if (t.first == logn) return t.second;
        return nullptr;
    }
};

void nufft_free(NufftPlan* q) {
    if (!q) return;
    if (q->arena) (void)hipFree(q->arena);
    delete q;
}

// The grid of nv vectors, twice over for a four-step transform (its second
// step writes the spectrum to a buffer of its own, in natural order).
size_t nufft_grid_bytes(const NufftPlan& q, int nv) {
    return (q.n1 ? 2 : 1) * (size_t)nv * q.K * q.cells * sizeof(float2);
}

// FP64 host planning (see the head of this file).
std::string nufft_build(Plan& p, int r, const double* P, const double* Q,
                        int K, const double* a, const double* b) {
    // batched FFT workgroups take up to kFftLds bytes of LDS
    (void)hipFuncSetAttribute((const void*)fft_lds,
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              kFftLds);
    NufftPlan* q = new (std::nothrow) NufftPlan();
    if (!q) return "host allocation";
    const long long N = p.N;
    q->r = r;
    q->K = K;
    q->N = N;
    q->b = kW / (4.0 * kPi * std::sqrt(0.5));
    double sbar[2], tbar[2], h[2];
    for (int d = 0; d < r; ++d) {
        double smin = Q[d], smax = Q[d], tmin = P[d], tmax = P[d];
        for (long long j = 0; j < N; ++j) {
            smin = std::min(smin, Q[j * r + d]);
            smax = std::max(smax, Q[j * r + d]);
            tmin = std::min(tmin, P[j * r + d]);
            tmax = std::max(tmax, P[j * r + d]);
        }
        sbar[d] = 0.5 * (smin + smax);
        tbar[d] = 0.5 * (tmin + tmax);
        const double S = 0.5 * (smax - smin), X = 0.5 * (tmax - tmin);
        // twice the Nyquist rate of the targets; a dimension whose targets
        // barely spread takes a grid of about the sources' width
        h[d] = X > 0 ? std::min(1.0 / (4.0 * X), std::max(S, 1.0))
                     : std::max(S, 1.0);
        q->Mh[d] = (int)std::ceil(S / h[d]) + kW + 1;
        // Mr >= 4 Mh, or half the power of two when that still keeps 4 Mh
        // within 64/63 of it (the second gridding's oversampling then at
        // least 1.97: its aliasing term at the highest mode goes from
        // exp(-15.55) to at most exp(-15.30)); a grid of 4 (N/2 + kW + 1)
        // cells otherwise doubles to the next power of two
        long long mr = std::max<long long>(16, next_pow2(4LL * q->Mh[d]));
        if (mr > 16 && 4LL * q->Mh[d] * 63 <= (mr / 2) * 64) mr /= 2;
        if (mr > (r == 1 ? (1LL << 24) : (long long)kFftMax)) {
            delete q;
            return "the lifted grid is too large (space-bandwidth product)";
        }
        q->Mr[d] = (int)mr;
    }
    q->cells = (long long)q->Mr[0] * (r == 2 ? q->Mr[1] : 1);
    if (q->cells > (1LL << 24)) {
        delete q;
        return "the lifted grid is too large (space-bandwidth product)";
    }
    if (r == 1 && q->Mr[0] > kFftMax) {
        const int l = ilog2i(q->Mr[0]);
        q->n1 = 1 << ((l + 1) / 2);
        q->n2 = q->Mr[0] / q->n1;
    }
    // host arrays
    std::vector<int> sbase((size_t)N * r), tbase((size_t)N * r);
    std::vector<float> sfrac((size_t)N * r), tfrac((size_t)N * r);
    std::vector<float2> pre(N), post(N), av((size_t)K * N), bv((size_t)K * N);
    const double b4 = 4.0 * q->b;
    for (long long j = 0; j < N; ++j) {
        double ph = 0;
        for (int d = 0; d < r; ++d) {
            const double sp = Q[j * r + d] - sbar[d];
            const double u = sp / h[d];
            const double fl = std::floor(u);
            sbase[j * r + d] = (int)fl;
            sfrac[j * r + d] = (float)(u - fl);
            ph += tbar[d] * sp;
        }
        ph -= std::nearbyint(ph);
        pre[j] = make_float2((float)std::cos(2 * kPi * ph),
                             (float)std::sin(2 * kPi * ph));
    }
    for (long long i = 0; i < N; ++i) {
        double ph = 0, mag = 1;
        for (int d = 0; d < r; ++d) {
            const double tp = P[i * r + d] - tbar[d];
            const double th = tp * h[d] * q->Mr[d];
            const double fl = std::floor(th);
            tbase[i * r + d] = (int)fl;
            tfrac[i * r + d] = (float)(th - fl);
            ph += P[i * r + d] * sbar[d];
            // 1 / (phihat(t') Mr), phihat(t) = h sqrt(4 pi b) e^{-4 pi^2 b h^2 t^2}
            const double phihat = h[d] * std::sqrt(4 * kPi * q->b) *
                                  std::exp(-4 * kPi * kPi * q->b * h[d] * h[d] * tp * tp);
            mag /= phihat * q->Mr[d];
        }
        ph -= std::nearbyint(ph);
        post[i] = make_float2((float)(mag * std::cos(2 * kPi * ph)),
                              (float)(mag * std::sin(2 * kPi * ph)));
    }
    for (long long e = 0; e < (long long)K * N; ++e)
        av[e] = make_float2((float)a[2 * e], (float)a[2 * e + 1]);
    long long per_source = 2 * kW;
    if (r == 2) per_source *= 2 * kW;
    // BF_NUFFT_ATOMICS=1 at plan time: 2D spreads by atomics at any size
    const char* aenv = std::getenv("BF_NUFFT_ATOMICS");
    const bool atomics = r == 2 && aenv && std::atoi(aenv) == 1;
    q->gather = r == 1 || (!atomics && N * per_source <= kMaxGatherEntries);
    if (q->gather) {
        // for the gather: by source, kp terms a row (it reads a source's
        // terms together), zero past K
        const int G = gather_group(K);
        q->kp = (K + G - 1) / G * G;
        bv.assign((size_t)N * q->kp, make_float2(0.f, 0.f));
        for (int k = 0; k < K; ++k)
            for (long long j = 0; j < N; ++j) {
                const long long e = (long long)k * N + j;
                bv[(size_t)j * q->kp + k] =
                    make_float2((float)b[2 * e], (float)b[2 * e + 1]);
            }
    } else {
        for (long long e = 0; e < (long long)K * N; ++e)
            bv[e] = make_float2((float)b[2 * e], (float)b[2 * e + 1]);
    }
    std::vector<float> dec[2];
    for (int d = 0; d < r; ++d) {
        const int Mh = q->Mh[d];
        dec[d].resize(2 * Mh);
        for (int m = -Mh; m < Mh; ++m) {
            // h / psihat_m, psihat_m = sqrt(4 pi b) / Mr e^{-4 pi^2 b m^2 / Mr^2}
            const double x = (double)m / q->Mr[d];
            dec[d][m + Mh] = (float)(h[d] * q->Mr[d] / std::sqrt(4 * kPi * q->b) *
                                     std::exp(4 * kPi * kPi * q->b * x * x));
        }
    }
    // 1D: every source's 2 kW contributions listed by grid cell (CSR),
    // each weight the Gaussian of the source's offset times the cell's
    // deconvolution factor (FP64, stored FP32)
    std::vector<int> cptr, cidx;
    std::vector<float> cwt;
    if (q->gather) {
        // the grid point (mode) of contribution e of source j in dimension
        // d, its cell index and its FP64 weight (Gaussian of the offset
        // times the deconvolution factor)
        auto mode = [&](long long j, int d, int e) -> long long {
            return (long long)sbase[j * r + d] - kW + 1 + e;
        };
        auto cell_d = [&](long long m, int d) -> long long {
            const long long M = q->Mr[d];
            const long long c = m % M;
            return c < 0 ? c + M : c;
        };
        auto weight = [&](long long j, int d, int e) -> double {
            const double dd = (double)(e - kW + 1) - (double)sfrac[j * r + d];
            return std::exp(-dd * dd / b4) *
                   (double)dec[d][mode(j, d, e) + q->Mh[d]];
        };
        for (long long j = 0; j < N; ++j)
            for (int d = 0; d < r; ++d)
                for (int e = 0; e < 2 * kW; ++e) {
                    const long long m = mode(j, d, e);
                    if (m + q->Mh[d] < 0 || m + q->Mh[d] >= 2LL * q->Mh[d]) {
                        delete q;
                        return "a source falls outside the lifted grid";
                    }
                }
        const int E1 = r == 2 ? 2 * kW : 1;     // entries of the 2nd dim
        auto cell_of = [&](long long j, int e0, int e1) -> long long {
            const long long c0 = cell_d(mode(j, 0, e0), 0);
            return r == 1 ? c0
                          : c0 * q->Mr[1] + cell_d(mode(j, 1, e1), 1);
        };
        cptr.assign((size_t)q->cells + 1, 0);
        for (long long j = 0; j < N; ++j)
            for (int e0 = 0; e0 < 2 * kW; ++e0)
                for (int e1 = 0; e1 < E1; ++e1)
                    ++cptr[(size_t)cell_of(j, e0, e1) + 1];
        for (long long m = 0; m < q->cells; ++m) cptr[m + 1] += cptr[m];
        std::vector<int> fill(cptr.begin(), cptr.end() - 1);
        cidx.resize((size_t)(N * per_source));
        cwt.resize((size_t)(N * per_source));
        for (long long j = 0; j < N; ++j) {
            double w1[2 * kW];
            for (int e1 = 0; e1 < E1; ++e1)
                w1[e1] = r == 2 ? weight(j, 1, e1) : 1.0;
            for (int e0 = 0; e0 < 2 * kW; ++e0) {
                const double w0 = weight(j, 0, e0);
                for (int e1 = 0; e1 < E1; ++e1) {
                    const int pos = fill[(size_t)cell_of(j, e0, e1)]++;
                    cidx[pos] = (int)j;
                    cwt[pos] = (float)(r == 1 ? w0 : w0 * w1[e1]);
                }
            }
        }
    }
    // FFT twiddles for every length the transforms use
    std::vector<int> lens;
    if (r == 1) {
        if (q->n1) {
            lens.push_back(ilog2i(q->n1));
            lens.push_back(ilog2i(q->n2));
        } else {
            lens.push_back(ilog2i(q->Mr[0]));
        }
    } else {
        lens.push_back(ilog2i(q->Mr[0]));
        lens.push_back(ilog2i(q->Mr[1]));
    }
    std::sort(lens.begin(), lens.end());
    lens.erase(std::unique(lens.begin(), lens.end()), lens.end());
    // arena layout
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    size_t off = 0;
    const size_t o_sb = off; off = al(off + sbase.size() * 4);
    const size_t o_sf = off; off = al(off + sfrac.size() * 4);
    const size_t o_pre = off; off = al(off + pre.size() * 8);
    const size_t o_tb = off; off = al(off + tbase.size() * 4);
    const size_t o_tf = off; off = al(off + tfrac.size() * 4);
    const size_t o_post = off; off = al(off + post.size() * 8);
    size_t o_dec[2] = {0, 0};
    for (int d = 0; d < r; ++d) {
        o_dec[d] = off;
        off = al(off + dec[d].size() * 4);
    }
    const size_t o_a = off; off = al(off + av.size() * 8);
    const size_t o_b = off; off = al(off + bv.size() * 8);
    const size_t o_cp = off; off = al(off + cptr.size() * 4);
    const size_t o_ci = off; off = al(off + cidx.size() * 4);
    const size_t o_cw = off; off = al(off + cwt.size() * 4);
    std::vector<size_t> o_tw;
    for (int l : lens) {
        o_tw.push_back(off);
        off = al(off + (size_t)std::max(1, (1 << l) / 2) * 8);
    }
    if (hipMalloc(&q->arena, off) != hipSuccess) {
        q->arena = nullptr;
        delete q;
        return "hipMalloc nufft arena";
    }
    q->arena_bytes = off;
    char* base = (char*)q->arena;
    q->sbase = (int*)(base + o_sb);
    q->sfrac = (float*)(base + o_sf);
    q->pre = (float2*)(base + o_pre);
    q->tbase = (int*)(base + o_tb);
    q->tfrac = (float*)(base + o_tf);
    q->post = (float2*)(base + o_post);
    for (int d = 0; d < r; ++d) q->dec[d] = (float*)(base + o_dec[d]);
    q->a = (float2*)(base + o_a);
    q->bb = (float2*)(base + o_b);
    q->cptr = (int*)(base + o_cp);
    q->cidx = (int*)(base + o_ci);
    q->cwt = (float*)(base + o_cw);
    hipError_t e = hipSuccess;
    auto up = [&](void* dst, const void* src, size_t n) {
        if (e == hipSuccess && n) e = hipMemcpy(dst, src, n, hipMemcpyHostToDevice);
    };
    up(q->sbase, sbase.data(), sbase.size() * 4);
    up(q->sfrac, sfrac.data(), sfrac.size() * 4);
    up(q->pre, pre.data(), pre.size() * 8);
    up(q->tbase, tbase.data(), tbase.size() * 4);
    up(q->tfrac, tfrac.data(), tfrac.size() * 4);
    up(q->post, post.data(), post.size() * 8);
    for (int d = 0; d < r; ++d) up(q->dec[d], dec[d].data(), dec[d].size() * 4);
    up(q->a, av.data(), av.size() * 8);
    up(q->bb, bv.data(), bv.size() * 8);
    up(q->cptr, cptr.data(), cptr.size() * 4);
    up(q->cidx, cidx.data(), cidx.size() * 4);
    up(q->cwt, cwt.data(), cwt.size() * 4);
    for (size_t t = 0; t < lens.size(); ++t) {
        const int n = 1 << lens[t];
        std::vector<float2> w(std::max(1, n / 2));
        for (int k = 0; k < n / 2; ++k)
            w[k] = make_float2((float)std::cos(2 * kPi * k / n),
                               (float)std::sin(2 * kPi * k / n));
        float2* dst = (float2*)(base + o_tw[t]);
        up(dst, w.data(), w.size() * 8);
        q->tw.push_back({lens[t], dst});
    }
    if (e != hipSuccess) {
        nufft_free(q);
        return std::string("nufft upload: ") + hipGetErrorString(e);
    }
    p.nufft = q;
    return "";
}

size_t nufft_factor_bytes(const NufftPlan& q) { return q.arena_bytes; }

// FFTs of every column of the grid; a four-step transform writes its
// spectrum to out in natural order (elsewhere out = data).
static std::string launch_fft(const NufftPlan& q, float2* data, float2* out,
                              int ncols, hipStream_t st) {
    auto run = [&](float2* src, float2* dst, int logn, long long stride,
                   long long seq_dist, long long ostride, long long oseq_dist,
                   long long nseq, long long total) -> std::string {
        // where one side is strided (adjacent sequences adjacent in
        // memory), up to 16 sequences share a workgroup so that its reads
        // or writes move as runs of contiguous entries (batching the
        // contiguous side alone measured no faster)
        const long long n = 1LL << logn, P = fft_pitch(n);
        int batch = 1, logb = 0;
        if (seq_dist == 1 || oseq_dist == 1)
            while (batch < 16 &&
                   ((long long)batch * 2 * P + n / 2) * 8 <= kFftLds &&
                   nseq % (batch * 2) == 0) {
                batch *= 2;
                ++logb;
            }
        const float tscale =
            total > 0 ? (float)std::ldexp(1.0, 1 - ilog2i(total)) : 0.f;
        FftArgs f{src, dst, q.twiddles(logn), logn, stride, seq_dist,
                  q.cells, ostride, oseq_dist, q.cells, nseq, total,
                  tscale, batch, logb};
        if (!f.tw) return "missing FFT twiddles";
        const size_t lds = ((size_t)batch * P + n / 2) * sizeof(float2);
        if (lds > (size_t)kFftLds) return "FFT does not fit in LDS";
        const long long blocks = nseq / batch * ncols;
        if (blocks > 0x7fffffffLL) return "FFT grid too large";
        hipLaunchKernelGGL(fft_lds, dim3((unsigned)blocks),
                           dim3(kFftThreads), lds, st, f);
        return "";
    };
    std::string err;
    if (q.r == 1) {
        if (q.n1) {
            // four-step over j = j1 n2 + j2: n1-point transforms over j1
            // (stride n2) in place, twiddle exp(2 pi i j2 k1 / Mr), then
            // n2-point transforms over j2 (contiguous rows k1); frequency
            // k1 + n1 k2 is written to out at that index
            err = run(data, data, ilog2i(q.n1), q.n2, 1, q.n2, 1, q.n2,
                      q.Mr[0]);
            if (err.empty())
                err = run(data, out, ilog2i(q.n2), 1, q.n2, q.n1, 1, q.n1, 0);
        } else {
            err = run(data, data, ilog2i(q.Mr[0]), 1, 0, 1, 0, 1, 0);
        }
    } else {
        err = run(data, data, ilog2i(q.Mr[1]), 1, q.Mr[1], 1, q.Mr[1],
                  q.Mr[0], 0);                                    // rows
        if (err.empty())
            err = run(data, data, ilog2i(q.Mr[0]), q.Mr[1], 1, q.Mr[1], 1,
                      q.Mr[1], 0);                                // columns
    }
    return err;
}

std::string launch_nufft(Plan& p, int nvec, const float2* f, float2* g,
                         void* ws, size_t ws_bytes, hipStream_t st) {
    const NufftPlan& q = *p.nufft;
    int chunk = std::min(nvec, p.chunk_nvec);
    while (chunk > 1 && nufft_grid_bytes(q, chunk) > ws_bytes) --chunk;
    if (nufft_grid_bytes(q, chunk) > ws_bytes)
        return "workspace too small for one vector";
    const double N = (double)q.N;
    const double stencil = std::pow(2.0 * kW, q.r);
    for (int v0 = 0; v0 < nvec; v0 += chunk) {
        const int nv = std::min(chunk, nvec - v0);
        NuArgs a{};
        a.r = q.r;
        a.K = q.K;
        a.nv = nv;
        a.N = q.N;
        for (int d = 0; d < 2; ++d) {
            a.Mr[d] = q.Mr[d];
            a.Mh[d] = q.Mh[d];
        }
        a.cells = q.cells;
        a.b4 = (float)(4.0 * q.b);
        a.sbase = q.sbase;
        a.sfrac = q.sfrac;
        a.pre = q.pre;
        a.tbase = q.tbase;
        a.tfrac = q.tfrac;
        a.post = q.post;
        a.dec0 = q.dec[0];
        a.dec1 = q.dec[1];
        a.a = q.a;
        a.b = q.bb;
        a.kp = q.kp;
        a.cptr = q.cptr;
        a.cidx = q.cidx;
        a.cwt = q.cwt;
        a.f = f + (size_t)v0 * q.N;
        a.g = g + (size_t)v0 * q.N;
        a.grid = (float2*)ws;
        const long long ncols = (long long)nv * q.K;
        const long long gcells = ncols * q.cells;
        // the spectrum: in place, or (four-step) the second half of ws
        float2* const spec = q.n1 ? a.grid + gcells : a.grid;
        if (!q.gather) {
            ProfScope ps(p, st);
            hipLaunchKernelGGL(nufft_zero, dim3(blocks_for_n(gcells)),
                               dim3(kNufftThreads), 0, st, a.grid, gcells);
            ps.end("nufft_zero", 0.0, 0.0, gcells * 8.0);
        }
        {
            ProfScope ps(p, st);
            if (q.gather) {
                const int G = gather_group(q.K);
                const dim3 grid(blocks_for_n(q.cells * nv * (q.kp / G)));
                switch (G) {
                    case 8:
                        hipLaunchKernelGGL(nufft_gather<8>, grid,
                                           dim3(kNufftThreads), 0, st, a);
                        break;
                    case 16:
                        hipLaunchKernelGGL(nufft_gather<16>, grid,
                                           dim3(kNufftThreads), 0, st, a);
                        break;
                    case 24:
                        hipLaunchKernelGGL(nufft_gather<24>, grid,
                                           dim3(kNufftThreads), 0, st, a);
                        break;
                    default:
                        hipLaunchKernelGGL(nufft_gather<32>, grid,
                                           dim3(kNufftThreads), 0, st, a);
                        break;
                }
            } else
                hipLaunchKernelGGL(nufft_spread<2>, dim3(blocks_for_n(q.N)),
                                   dim3(kNufftThreads), 0, st, a);
            ps.end("nufft_spread", N * nv * 8.0 + N * q.K * 8.0 + N * 16.0,
                   N * ncols * (stencil * 4.0 + 12.0), N * ncols * stencil * 8.0);
        }
        {
            ProfScope ps(p, st);
            std::string err = launch_fft(q, a.grid, spec, (int)ncols, st);
            if (!err.empty()) return err;
            const double passes = q.r == 2 || q.n1 ? 2.0 : 1.0;
            ps.end("nufft_fft", 0.0,
                   5.0 * gcells * std::log2((double)q.cells),
                   2.0 * passes * gcells * 8.0);
        }
        {
            ProfScope ps(p, st);
            a.grid = spec;
            const long long nt = q.N * nv;
            if (q.r == 1)
                hipLaunchKernelGGL(nufft_interp<1>, dim3(blocks_for_n(nt)),
                                   dim3(kNufftThreads), 0, st, a);
            else
                hipLaunchKernelGGL(nufft_interp<2>, dim3(blocks_for_n(nt)),
                                   dim3(kNufftThreads), 0, st, a);
            ps.end("nufft_interp", N * nv * 8.0 + N * q.K * 8.0 + N * 16.0,
                   N * ncols * (stencil * 4.0 + 8.0), N * ncols * stencil * 8.0);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return std::string("nufft launch: ") + hipGetErrorString(e);
    }
    return "";
}

}  // namespace bfi
