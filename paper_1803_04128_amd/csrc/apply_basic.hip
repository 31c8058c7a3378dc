// One launch per computed step: the plain FP32 apply of the regrouped
// butterfly (Algorithm 4.1, steps 2-6, with the exact copy and sum levels
// folded into the index math of the first step and of the final sums).
//
// State layout between launches: complex64 [pair p][coefficient t][column],
// p = a * R^(L-l) + b for the pair (A = a, B = b) at level l; a column is
// (vector v, amplitude term k) at v * r_amp + k inside the vector chunk.
// A unit (a', b) reads the R consecutive pairs a' R^(L-l+1) + R b + c and
// writes pairs (R a' + i) R^(L-l) + b: the butterfly permutation is this
// index math.
#include "apply_common.h"

namespace bfi {

// xi step (eq. (eqn:2) regrouped): thread = (unit, output child i, column).
template <int R, int RM>
__global__ void __launch_bounds__(256) xi_step_basic(StepArgs a) {
    const long long gid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long total = a.units * R * a.Vc;
    if (gid >= total) return;
    const int col = (int)(gid % a.Vc);
    const long long rest = gid / a.Vc;
    const int i = (int)(rest % R);
    const long long u = rest / R;
    const int shiftB = a.dim * (a.L - a.level);
    const long long ap = u >> shiftB, b = u & ((1LL << shiftB) - 1);
    float2 acc[RM];
#pragma unroll
    for (int t = 0; t < RM; ++t) acc[t] = make_float2(0.f, 0.f);
    const float2* tw = a.tw + (u * R + i) * R * a.r_in;
    for (int c = 0; c < R; ++c) {
        const long long pin = (ap << (shiftB + a.dim)) + (b << a.dim) + c;
        for (int s = 0; s < a.r_in; ++s) {
            float2 x = a.reads_f ? head_value(a, b * R + c, s, col)
                                 : a.in[(pin * a.r_in + s) * a.Vc + col];
            const float2 z = cmul(tw[c * a.r_in + s], x);
            const float* m = a.mats + (size_t)c * a.r_out * a.r_in + s;
#pragma unroll
            for (int t = 0; t < RM; ++t) {
                if (t < a.r_out) {
                    const float w = m[t * a.r_in];
                    acc[t].x += w * z.x;
                    acc[t].y += w * z.y;
                }
            }
        }
    }
    const long long pout = ((ap * R + i) << shiftB) + b;
#pragma unroll
    for (int t = 0; t < RM; ++t)
        if (t < a.r_out) a.out[(pout * a.r_out + t) * a.Vc + col] = acc[t];
}

// x step (eq. (eqn:3) regrouped): thread = (unit, output child i, column).
template <int R, int RM>
__global__ void __launch_bounds__(256) x_step_basic(StepArgs a) {
    const long long gid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long total = a.units * R * a.Vc;
    if (gid >= total) return;
    const int col = (int)(gid % a.Vc);
    const long long rest = gid / a.Vc;
    const int i = (int)(rest % R);
    const long long u = rest / R;
    const int shiftB = a.dim * (a.L - a.level);
    const long long ap = u >> shiftB, b = u & ((1LL << shiftB) - 1);
    float2 acc[RM];
#pragma unroll
    for (int t = 0; t < RM; ++t) acc[t] = make_float2(0.f, 0.f);
    const float* mi = a.mats + (size_t)i * a.r_out * a.r_in;
    for (int c = 0; c < R; ++c) {
        const long long pin = (ap << (shiftB + a.dim)) + (b << a.dim) + c;
        float2 y[RM];
#pragma unroll
        for (int t = 0; t < RM; ++t) y[t] = make_float2(0.f, 0.f);
        for (int s = 0; s < a.r_in; ++s) {
            const float2 x = a.in[(pin * a.r_in + s) * a.Vc + col];
#pragma unroll
            for (int t = 0; t < RM; ++t) {
                if (t < a.r_out) {
                    const float w = mi[t * a.r_in + s];
                    y[t].x += w * x.x;
                    y[t].y += w * x.y;
                }
            }
        }
        const float2* tw = a.tw + ((u * R + i) * R + c) * a.r_out;
#pragma unroll
        for (int t = 0; t < RM; ++t) {
            if (t < a.r_out) {
                const float2 z = cmul(tw[t], y[t]);
                acc[t].x += z.x;
                acc[t].y += z.y;
            }
        }
    }
    const long long pout = ((ap * R + i) << shiftB) + b;
#pragma unroll
    for (int t = 0; t < RM; ++t)
        if (t < a.r_out) a.out[(pout * a.r_out + t) * a.Vc + col] = acc[t];
}

// switch (Algorithm 4.1 step 4 regrouped): thread = (pair, column).
template <int RM>
__global__ void __launch_bounds__(256) switch_basic(StepArgs a) {
    const long long gid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long total = a.units * a.Vc;
    if (gid >= total) return;
    const int col = (int)(gid % a.Vc);
    const long long p = gid / a.Vc;
    const int shiftB = a.dim * (a.L - a.level);
    const long long bm = p & ((1LL << shiftB) - 1);
    float2 acc[RM];
#pragma unroll
    for (int t = 0; t < RM; ++t) acc[t] = make_float2(0.f, 0.f);
    const float2* S = a.S + (size_t)p * a.r_out * a.r_in;
    for (int s = 0; s < a.r_in; ++s) {
        const float2 x = a.reads_f ? head_value(a, bm, s, col)
                                   : a.in[(p * a.r_in + s) * a.Vc + col];
#pragma unroll
        for (int t = 0; t < RM; ++t) {
            if (t < a.r_out) {
                const float2 z = cmul(S[t * a.r_in + s], x);
                acc[t].x += z.x;
                acc[t].y += z.y;
            }
        }
    }
#pragma unroll
    for (int t = 0; t < RM; ++t)
        if (t < a.r_out) a.out[(p * a.r_out + t) * a.Vc + col] = acc[t];
}

// Final sums (Algorithm 4.1 steps 5-6 at the exact levels) and the amplitude
// (eq. (eqn:tg)): g_v(x) = sum_k a_k(x) sum_B lambda_k^{A(x), B}(x), the
// inner sum over the R^(L-lend) boxes B at level L-lend.
// Thread = (output index x, vector), the vector fastest so that
// neighbouring threads read neighbouring state columns.
__global__ void __launch_bounds__(256) tail_basic(TailArgs a) {
    const long long gid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (gid >= a.N * a.nv) return;
    const int vl = (int)(gid % a.nv);
    const long long x = gid / a.nv;
    int g[2], Ac[2], tdig[2];
    if (a.dim == 1) {
        g[0] = (int)x;
    } else {
        g[0] = (int)(x / a.n);
        g[1] = (int)(x % a.n);
    }
    for (int d = 0; d < a.dim; ++d) {
        Ac[d] = g[d] / a.side;
        tdig[d] = g[d] % a.side;
    }
    const int t = a.dim == 1 ? tdig[0] : tdig[0] * a.side + tdig[1];
    const long long am = box_index(Ac, a.dim);
    float2 sum = make_float2(0.f, 0.f);
    for (int k = 0; k < a.r_amp; ++k) {
        const int col = vl * a.r_amp + k;
        float2 s = make_float2(0.f, 0.f);
        for (long long bb = 0; bb < a.nb; ++bb) {
            const float2 v = a.in[((am * a.nb + bb) * a.r + t) * a.Vc + col];
            s.x += v.x;
            s.y += v.y;
        }
        if (a.amp_a) {
            const float2 z = cmul(a.amp_a[(size_t)k * a.N + x], s);
            sum.x += z.x;
            sum.y += z.y;
        } else {
            sum.x += s.x;
            sum.y += s.y;
        }
    }
    a.g[(size_t)vl * a.N + x] = sum;
}

static unsigned blocks_for(long long total) {
    return (unsigned)((total + 255) / 256);
}

template <int R, int RM>
static void launch_step_basic(const Step& s, const StepArgs& a,
                              hipStream_t st) {
    if (s.kind == STEP_XI)
        hipLaunchKernelGGL((xi_step_basic<R, RM>),
                           dim3(blocks_for(a.units * R * a.Vc)), dim3(256), 0,
                           st, a);
    else if (s.kind == STEP_X)
        hipLaunchKernelGGL((x_step_basic<R, RM>),
                           dim3(blocks_for(a.units * R * a.Vc)), dim3(256), 0,
                           st, a);
    else
        hipLaunchKernelGGL((switch_basic<RM>), dim3(blocks_for(a.units * a.Vc)),
                           dim3(256), 0, st, a);
}

std::string launch_step_mfma(const Plan& p, const Step& s, const StepArgs& a,
                             hipStream_t st);

std::string launch_step_split(const Plan& p, const Step& s,
                              const StepArgs& a, hipStream_t st);

std::string launch_sep_switch(const Plan& p, const Step& xi, const Step& sw,
                              StepArgs a, hipStream_t st);

std::string run_basic(Plan& p, int nv, const float2* f, float2* g,
                      float2* buf0, float2* buf1, hipStream_t st) {
    const int Vc = nv * p.r_amp;
    const float2* cur = nullptr;
    float2* bufs[2] = {buf0, buf1};
    int which = 0;
    const double N = (double)p.N, c8 = 8.0 * Vc;
    const double head_bytes = N * nv * 8.0 + (p.has_amp ? N * p.r_amp * 8.0 : 0);
    for (size_t k = 0; k < p.steps.size(); ++k) {
        const Step& s = p.steps[k];
        StepArgs a = make_step_args(p, s, Vc, f, cur, bufs[which]);
        const bool otf = p.mfma && p.switch_otf && s.kind == STEP_SWITCH;
        double bytes = (s.reads_f ? head_bytes : 0.0) +
                       (p.twiddle_otf ? 0.0 : s.tw_elems * 8.0) +
                       (otf ? 0.0 : s.S_elems * 8.0) + s.mat_elems * 4.0;
        double sbytes = (s.reads_f ? 0.0 : N * s.r_in * c8) +
                        N * s.r_out * c8;
        double flops = step_alg_flops(p, s, Vc);
        const char* name = s.kind == STEP_XI ? "xi_step_basic"
                           : s.kind == STEP_X ? "x_step_basic"
                                              : "switch_basic";
        ProfScope ps(p, st);
        if (k + 1 < p.steps.size() && sep_switch_ok(p, s, p.steps[k + 1])) {
            // the last xi level and the switch in one launch
            const Step& sw = p.steps[k + 1];
            std::string err = launch_sep_switch(p, s, sw, a, st);
            if (!err.empty()) return err;
            name = "xi_sep_switch";
            bytes += sw.S_elems * 8.0;
            flops += step_alg_flops(p, sw, Vc);
            sbytes += N * (double)(sw.r_out - s.r_out) * c8;
            ++k;
        } else if (p.mfma && p.precision != BF_FP32) {
            // split-precision contractions on MFMA
            std::string err = launch_step_split(p, s, a, st);
            if (!err.empty()) return err;
            name = s.kind == STEP_XI ? "xi_step_split"
                   : s.kind == STEP_X ? "x_step_split"
                                      : "switch_step_split";
        } else if (p.mfma) {
            // contractions on MFMA (one launch per step)
            std::string err = launch_step_mfma(p, s, a, st);
            if (!err.empty()) return err;
            const bool sep = step_sep_ok(p, s);
            name = s.kind == STEP_XI ? (sep ? "xi_step_sep" : "xi_step_mfma")
                   : s.kind == STEP_X ? (sep ? "x_step_sep" : "x_step_mfma")
                   : otf              ? "switch_otf_mfma"
                                      : "switch_step_mfma";
        } else if (p.dim == 1) {
            if (p.max_rank <= 16) launch_step_basic<2, 16>(s, a, st);
            else return "1D rank above 16";
        } else {
            if (p.max_rank <= 16) launch_step_basic<4, 16>(s, a, st);
            else if (p.max_rank <= 36) launch_step_basic<4, 36>(s, a, st);
            else launch_step_basic<4, 64>(s, a, st);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return std::string("step launch: ") + hipGetErrorString(e);
        ps.end(name, bytes, flops, sbytes);
        cur = bufs[which];
        which ^= 1;
    }
    TailArgs t = make_tail_args(p, nv, cur, g);
    ProfScope ps(p, st);
    hipLaunchKernelGGL(tail_basic, dim3(blocks_for(p.N * nv)), dim3(256), 0,
                       st, t);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return std::string("tail launch: ") + hipGetErrorString(e);
    ps.end("tail_basic", N * nv * 8.0 + (p.has_amp ? N * p.r_amp * 8.0 : 0),
           N * Vc * (double)t.nb * 2.0 + N * nv * p.r_amp * 8.0,
           N * t.r * c8);
    return "";
}

}  // namespace bfi
